"""ctypes front-end of the plain C oracle (``ej_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by the
CPU-baseline leg of the benchmark.  The product package never imports it.

``build()`` compiles ``ej_oracle.c`` with gcc into ``liboracle.so`` next to
this file; every other function loads that library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ej_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

P61 = (1 << 61) - 1
GAMMA = 0x9E3779B97F4A7C15

_lib = None


def build(force: bool = True) -> str:
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall",
                               "-Wno-unused-function", SRC, "-o", tmp])
        os.replace(tmp, LIB)
    return LIB


class _Result(ctypes.Structure):
    _fields_ = [
        ("sigma", ctypes.c_uint32), ("L", ctypes.c_uint32),
        ("n_raw", ctypes.c_uint64), ("n_cand", ctypes.c_uint64), ("cand", ctypes.POINTER(ctypes.c_uint64)),
        ("cand_dist", ctypes.POINTER(ctypes.c_uint32)),
        ("n_out", ctypes.c_uint64), ("out", ctypes.POINTER(ctypes.c_uint64)),
        ("out_dist", ctypes.POINTER(ctypes.c_uint32)),
        ("keys", ctypes.POINTER(ctypes.c_uint64)),
        ("sig", ctypes.POINTER(ctypes.c_uint8)),
    ]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build(force=False)
        L = ctypes.CDLL(LIB)
        u8p = ctypes.POINTER(ctypes.c_uint8)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        i32p = ctypes.POINTER(ctypes.c_int32)
        L.ejo_mix64.restype = ctypes.c_uint64
        L.ejo_mix64.argtypes = [ctypes.c_uint64]
        L.ejo_word.restype = ctypes.c_uint64
        L.ejo_word.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        L.ejo_stream_key.restype = ctypes.c_uint64
        L.ejo_stream_key.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32]
        L.ejo_splitmix64_stream.restype = None
        L.ejo_splitmix64_stream.argtypes = [ctypes.c_uint64, ctypes.c_uint64, u64p]
        L.ejo_draw.restype = None
        L.ejo_draw.argtypes = [ctypes.c_uint64] + [ctypes.c_uint32] * 5 + [u8p, u32p, u64p]
        L.ejo_alphabet.restype = ctypes.c_int
        L.ejo_alphabet.argtypes = [u8p, ctypes.c_uint64, i32p]
        L.ejo_cgk_embed.restype = None
        L.ejo_cgk_embed.argtypes = [u8p, ctypes.c_uint32, u8p, ctypes.c_uint32,
                                    ctypes.c_uint32, u8p]
        L.ejo_key.restype = ctypes.c_uint64
        L.ejo_key.argtypes = [u8p, u32p, u64p, ctypes.c_uint32]
        L.ejo_ed_full.restype = ctypes.c_uint32
        L.ejo_ed_full.argtypes = [u8p, ctypes.c_uint32, u8p, ctypes.c_uint32]
        L.ejo_ed_banded.restype = ctypes.c_uint32
        L.ejo_ed_banded.argtypes = [u8p, ctypes.c_uint32, u8p, ctypes.c_uint32, ctypes.c_uint32]
        L.ejo_effective_L.restype = ctypes.c_uint32
        L.ejo_effective_L.argtypes = [u64p, ctypes.c_uint32, ctypes.c_uint32]
        L.ejo_join.restype = ctypes.c_int
        L.ejo_join.argtypes = [u8p, u64p, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                               ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                               ctypes.c_uint64, u8p, u32p, u64p, ctypes.POINTER(_Result)]
        L.ejo_join_opts.restype = ctypes.c_int
        L.ejo_join_opts.argtypes = [u8p, u64p, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                    ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                    ctypes.c_uint64, u8p, u32p, u64p, ctypes.c_uint32,
                                    ctypes.POINTER(_Result)]
        L.ejo_result_free.restype = None
        L.ejo_result_free.argtypes = [ctypes.POINTER(_Result)]
        L.ejo_verify_pairs.restype = None
        L.ejo_verify_pairs.argtypes = [u8p, u64p, u64p, ctypes.c_uint64, ctypes.c_uint32, u32p]
        L.ejo_query.restype = ctypes.c_int64
        L.ejo_query.argtypes = [u8p, u64p, ctypes.c_uint32, u8p, u64p, ctypes.c_uint32, u32p,
                                ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                ctypes.c_uint64, u64p, u32p, u32p, ctypes.c_uint64]
        L.ejo_join_plus.restype = ctypes.c_int
        L.ejo_join_plus.argtypes = [u8p, u64p] + [ctypes.c_uint32] * 6 + [ctypes.c_uint64] + \
            [ctypes.c_uint32] * 3 + [ctypes.POINTER(_Result)]
        L.ejo_plus_kappa.restype = ctypes.c_uint32
        L.ejo_plus_kappa.argtypes = [ctypes.c_uint32, ctypes.c_uint32]
        L.ejo_plus_default_T.restype = ctypes.c_uint32
        L.ejo_plus_default_T.argtypes = [ctypes.c_uint32, ctypes.c_uint32]
        L.ejo_embed_hamming.restype = ctypes.c_int
        L.ejo_embed_hamming.argtypes = [u8p, u64p, ctypes.c_uint32, ctypes.c_uint32,
                                        ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint32,
                                        ctypes.c_uint32, u64p, ctypes.c_uint64, u32p]
        L.ejo_join_grouped.restype = ctypes.c_int
        L.ejo_join_grouped.argtypes = [u8p, u64p] + [ctypes.c_uint32] * 6 + [ctypes.c_uint64] + \
            [ctypes.POINTER(_Result)]
        L.ejo_keys.restype = ctypes.c_int
        L.ejo_keys.argtypes = [u8p, u64p, ctypes.c_uint32, u8p, u64p, ctypes.c_uint32,
                               ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                               ctypes.c_uint32, ctypes.c_uint64, u64p]
        L.ejo_exact_short.restype = ctypes.c_int
        L.ejo_exact_short.argtypes = [u8p, u64p, ctypes.c_uint32, ctypes.c_uint32,
                                      ctypes.c_uint32, ctypes.POINTER(_Result)]
        L.ejo_brute_join.restype = ctypes.c_uint64
        L.ejo_brute_join.argtypes = [u8p, u64p, ctypes.c_uint32, ctypes.c_uint32,
                                     u64p, u32p, ctypes.c_uint64, ctypes.c_int]
        _lib = L
    return _lib


def _ptr(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def _u8(b) -> np.ndarray:
    if isinstance(b, (bytes, bytearray)):
        return np.frombuffer(bytes(b) + b"\0", dtype=np.uint8)[:len(b)].copy()
    return np.ascontiguousarray(b, dtype=np.uint8)


# ------------------------------------------------------------------- RNG --

def mix64(z: int) -> int:
    return int(lib().ejo_mix64(z))


def word(key: int, c: int) -> int:
    return int(lib().ejo_word(key, c))


def stream_key(seed: int, tag: int, idx: int) -> int:
    return int(lib().ejo_stream_key(seed, tag, idx))


def splitmix64(seed: int, count: int) -> np.ndarray:
    out = np.zeros(max(count, 1), dtype=np.uint64)
    lib().ejo_splitmix64_stream(seed, count, _ptr(out, ctypes.c_uint64))
    return out[:count]


def draw(seed: int, r: int, z: int, m: int, L: int, sigma: int):
    """Returns (Rbits[r, L*sigma] 0/1, pos[r, z, m], v[r, z, m])."""
    Rb = np.zeros(max(r * L * sigma, 1), dtype=np.uint8)
    pos = np.zeros(r * z * m, dtype=np.uint32)
    v = np.zeros(r * z * m, dtype=np.uint64)
    lib().ejo_draw(seed, r, z, m, L, sigma, _ptr(Rb, ctypes.c_uint8),
                   _ptr(pos, ctypes.c_uint32), _ptr(v, ctypes.c_uint64))
    return Rb[:r * L * sigma].reshape(r, L * sigma), pos.reshape(r, z, m), v.reshape(r, z, m)


# ----------------------------------------------------------- primitives --

def alphabet(chars) -> tuple[int, np.ndarray]:
    c = _u8(chars)
    lut = np.zeros(256, dtype=np.int32)
    s = lib().ejo_alphabet(_ptr(c, ctypes.c_uint8), c.shape[0], _ptr(lut, ctypes.c_int32))
    return int(s), lut


def cgk_embed(codes, Rbits_l, sigma: int, L: int) -> np.ndarray:
    x = _u8(codes)
    R = np.ascontiguousarray(Rbits_l, dtype=np.uint8)
    out = np.zeros(max(L, 1), dtype=np.uint8)
    lib().ejo_cgk_embed(_ptr(x, ctypes.c_uint8), x.shape[0], _ptr(R, ctypes.c_uint8),
                        sigma, L, _ptr(out, ctypes.c_uint8))
    return out[:L]


def key(t, pos, v) -> int:
    t = _u8(t)
    pos = np.ascontiguousarray(pos, dtype=np.uint32)
    v = np.ascontiguousarray(v, dtype=np.uint64)
    return int(lib().ejo_key(_ptr(t, ctypes.c_uint8), _ptr(pos, ctypes.c_uint32),
                             _ptr(v, ctypes.c_uint64), pos.shape[0]))


def ed_full(x, y) -> int:
    x, y = _u8(x), _u8(y)
    return int(lib().ejo_ed_full(_ptr(x, ctypes.c_uint8), x.shape[0],
                                 _ptr(y, ctypes.c_uint8), y.shape[0]))


def ed_banded(x, y, K: int) -> int:
    x, y = _u8(x), _u8(y)
    return int(lib().ejo_ed_banded(_ptr(x, ctypes.c_uint8), x.shape[0],
                                   _ptr(y, ctypes.c_uint8), y.shape[0], K))


def effective_L(offsets, L_req: int) -> int:
    off = np.ascontiguousarray(offsets, dtype=np.uint64)
    return int(lib().ejo_effective_L(_ptr(off, ctypes.c_uint64), off.shape[0] - 1, L_req))


# -------------------------------------------------------------- the join --

STOP_AFTER_CANDIDATES = 1
NO_SIG = 2


def _arr(ptr, count):
    if not ptr or count == 0:
        return None
    return np.ctypeslib.as_array(ptr, (count,)).copy()


class JoinResult:
    def __init__(self, res: _Result, n: int, r: int, z: int, m: int, key_cols: int | None = None):
        self.sigma = int(res.sigma)
        self.L = int(res.L)
        self.n_raw = int(res.n_raw)
        nc, no = int(res.n_cand), int(res.n_out)
        T = r * z
        empty = np.zeros(0, dtype=np.uint64)
        self.cand = _arr(res.cand, nc) if nc else empty
        cd = _arr(res.cand_dist, nc)
        self.cand_dist = cd if cd is not None else np.zeros(0, dtype=np.uint32)
        self.out = _arr(res.out, no) if no else empty
        od = _arr(res.out_dist, no)
        self.out_dist = od if od is not None else np.zeros(0, dtype=np.uint32)
        kc = n if key_cols is None else key_cols
        keys = _arr(res.keys, T * kc)
        self.keys = keys.reshape(T, kc) if keys is not None else np.zeros((T, kc), np.uint64)
        sig = _arr(res.sig, n * T * m)
        self.sig = sig.reshape(n, r, z, m) if sig is not None else None

    @staticmethod
    def pairs(codes: np.ndarray) -> np.ndarray:
        codes = np.asarray(codes, dtype=np.uint64)
        return np.stack([(codes >> np.uint64(32)).astype(np.int64),
                         (codes & np.uint64(0xFFFFFFFF)).astype(np.int64)], 1)

    @property
    def cand_pairs(self):
        return self.pairs(self.cand)

    @property
    def out_pairs(self):
        return self.pairs(self.out)


def _exact_short(c, off, n, K, S, res):
    """ejo_exact_short on a result in place (S = 0: nothing)."""
    if S and lib().ejo_exact_short(_ptr(c, ctypes.c_uint8) if c.size else None,
                                   _ptr(off, ctypes.c_uint64), n, K, S, ctypes.byref(res)) != 0:
        lib().ejo_result_free(ctypes.byref(res))
        raise MemoryError("oracle short-string pass: allocation failed")


def join(chars, offsets, K: int, r: int, z: int, m: int, seed: int = 0, L: int = 0,
         explicit_R=None, explicit_pos=None, explicit_v=None, opts: int = 0,
         exact_len: int = 0) -> JoinResult:
    """The oracle's EmbedJoin.  opts: STOP_AFTER_CANDIDATES (the candidate set
    only, `cand_dist`/`out` empty), NO_SIG (no sampled symbols kept).
    exact_len > 0 adds every pair of strings no longer than exact_len whose
    lengths differ by at most K to the candidates (ejo_exact_short)."""
    c = _u8(chars)
    off = np.ascontiguousarray(offsets, dtype=np.uint64)
    n = off.shape[0] - 1
    res = _Result()
    eR = None if explicit_R is None else np.ascontiguousarray(explicit_R, dtype=np.uint8)
    eP = None if explicit_pos is None else np.ascontiguousarray(explicit_pos, dtype=np.uint32)
    eV = None if explicit_v is None else np.ascontiguousarray(explicit_v, dtype=np.uint64)
    rc = lib().ejo_join_opts(_ptr(c, ctypes.c_uint8) if c.size else None,
                             _ptr(off, ctypes.c_uint64), n, K, r, z, m, L, seed,
                             None if eR is None else _ptr(eR, ctypes.c_uint8),
                             None if eP is None else _ptr(eP, ctypes.c_uint32),
                             None if eV is None else _ptr(eV, ctypes.c_uint64),
                             opts, ctypes.byref(res))
    if rc == -2:
        raise ValueError("all 256 byte values occur: no code is left for the padding symbol")
    if rc != 0:
        raise ValueError(f"oracle join rejected its arguments (rc={rc})")
    _exact_short(c, off, n, K, exact_len, res)
    try:
        return JoinResult(res, n, r, z, m)
    finally:
        lib().ejo_result_free(ctypes.byref(res))


def plus_kappa(K: int, delta: int) -> int:
    return int(lib().ejo_plus_kappa(K, delta))


def plus_default_T(K: int, delta: int) -> int:
    return int(lib().ejo_plus_default_T(K, delta))


def join_plus(chars, offsets, K: int, r: int, z: int, m: int, delta: int, T: int = 0,
              seed: int = 0, L: int = 0, opts: int = 0, exact_len: int = 0) -> JoinResult:
    """The oracle's EmbedJoin+ (Algorithms 4-5): ceil(K/delta) suffixes per
    string, a pair is a candidate when one of its suffix pairs collides in at
    least T tables (T = 0: 2 if there is more than one suffix, else 1).
    keys are [r*z, n*kappa] (suffix k of string i at column i*kappa + k)."""
    c = _u8(chars)
    off = np.ascontiguousarray(offsets, dtype=np.uint64)
    n = off.shape[0] - 1
    if T == 0:
        T = plus_default_T(K, delta)
    res = _Result()
    rc = lib().ejo_join_plus(_ptr(c, ctypes.c_uint8) if c.size else None,
                             _ptr(off, ctypes.c_uint64), n, K, r, z, m, L, seed, delta, T, opts,
                             ctypes.byref(res))
    if rc == -2:
        raise ValueError("all 256 byte values occur: no code is left for the padding symbol")
    if rc != 0:
        raise ValueError(f"oracle join_plus rejected its arguments (rc={rc})")
    _exact_short(c, off, n, K, exact_len, res)
    try:
        return JoinResult(res, n, r, z, m, key_cols=n * plus_kappa(K, delta))
    finally:
        lib().ejo_result_free(ctypes.byref(res))


def join_grouped(chars, offsets, K: int, r: int, z: int, m: int, seed: int = 0,
                 L: int = 0, exact_len: int = 0) -> JoinResult:
    """The oracle's grouping variant (Section 4.1): EmbedJoin on each length
    group ((g)K, (g+2)K] on its own (L = 3 x the group's longest string unless
    L > 0), the union of the groups' candidates and outputs."""
    c = _u8(chars)
    off = np.ascontiguousarray(offsets, dtype=np.uint64)
    n = off.shape[0] - 1
    res = _Result()
    rc = lib().ejo_join_grouped(_ptr(c, ctypes.c_uint8) if c.size else None,
                                _ptr(off, ctypes.c_uint64), n, K, r, z, m, L, seed,
                                ctypes.byref(res))
    if rc != 0:
        raise ValueError(f"oracle join_grouped rejected its arguments (rc={rc})")
    _exact_short(c, off, n, K, exact_len, res)
    try:
        return JoinResult(res, n, r, z, m, key_cols=0)
    finally:
        lib().ejo_result_free(ctypes.byref(res))


def candidates(chars, offsets, K: int, r: int, z: int, m: int, seed: int = 0, L: int = 0):
    """Algorithm 3's candidate set C (sorted codes i << 32 | j) and the number of
    pairs the tables found before de-duplication, from the same loop as join()
    stopped before verification."""
    res = join(chars, offsets, K, r, z, m, seed=seed, L=L, opts=STOP_AFTER_CANDIDATES | NO_SIG)
    return res.cand, res.n_raw


def verify_pairs(chars, offsets, pairs, K: int) -> np.ndarray:
    c = _u8(chars)
    off = np.ascontiguousarray(offsets, dtype=np.uint64)
    p = np.ascontiguousarray(pairs, dtype=np.uint64)
    d = np.zeros(max(p.shape[0], 1), dtype=np.uint32)
    lib().ejo_verify_pairs(_ptr(c, ctypes.c_uint8) if c.size else None,
                           _ptr(off, ctypes.c_uint64), _ptr(p, ctypes.c_uint64),
                           p.shape[0], K, _ptr(d, ctypes.c_uint32))
    return d[:p.shape[0]]


def brute_join(chars, offsets, K: int, full: bool = False):
    """Exact join over all pairs: (pairs[i<j] as uint64 codes, dist).  full=True
    uses textbook Wagner-Fischer, else Ukkonen's threshold DP."""
    c = _u8(chars)
    off = np.ascontiguousarray(offsets, dtype=np.uint64)
    n = off.shape[0] - 1
    cap = 1 << 16
    while True:
        out = np.zeros(cap, dtype=np.uint64)
        d = np.zeros(cap, dtype=np.uint32)
        cnt = int(lib().ejo_brute_join(_ptr(c, ctypes.c_uint8) if c.size else None,
                                       _ptr(off, ctypes.c_uint64), n, K,
                                       _ptr(out, ctypes.c_uint64), _ptr(d, ctypes.c_uint32), cap,
                                       1 if full else 0))
        if cnt <= cap:
            return out[:cnt], d[:cnt]
        cap = cnt


def embed_hamming(chars, offsets, pairs, r: int, L: int = 0, seed: int = 0, K: int = 0,
                  delta: int = 0) -> np.ndarray:
    """Hamming distance [count, r] between the L-symbol embeddings of each
    pair's strings under each seed (with delta > 0: the minimum over the
    ceil(K/delta)^2 suffix pairs)."""
    c = _u8(chars)
    off = np.ascontiguousarray(offsets, dtype=np.uint64)
    p = np.ascontiguousarray(pairs, dtype=np.uint64)
    out = np.zeros(max(p.shape[0] * r, 1), dtype=np.uint32)
    rc = lib().ejo_embed_hamming(_ptr(c, ctypes.c_uint8) if c.size else None,
                                 _ptr(off, ctypes.c_uint64), off.shape[0] - 1, r, L, seed, K,
                                 delta, _ptr(p, ctypes.c_uint64), p.shape[0],
                                 _ptr(out, ctypes.c_uint32))
    if rc != 0:
        raise ValueError(f"invalid arguments (rc={rc})")
    return out[:p.shape[0] * r].reshape(p.shape[0], r)


def keys(index_chars, index_offsets, x_chars, x_offsets, r: int, z: int, m: int, seed: int = 0,
         L: int = 0) -> np.ndarray:
    """Bucket keys [nx, r*z] of the strings x under the alphabet, truncation
    and random streams of the index set (x may be the index itself)."""
    ic, xc = _u8(index_chars), _u8(x_chars)
    io = np.ascontiguousarray(index_offsets, dtype=np.uint64)
    xo = np.ascontiguousarray(x_offsets, dtype=np.uint64)
    n, nx = io.shape[0] - 1, xo.shape[0] - 1
    out = np.zeros(max(nx * r * z, 1), dtype=np.uint64)
    rc = lib().ejo_keys(_ptr(ic, ctypes.c_uint8) if ic.size else None, _ptr(io, ctypes.c_uint64), n,
                        _ptr(xc, ctypes.c_uint8) if xc.size else None, _ptr(xo, ctypes.c_uint64),
                        nx, r, z, m, L, seed, _ptr(out, ctypes.c_uint64))
    if rc == -2:
        raise ValueError("a byte outside the index alphabet")
    if rc != 0:
        raise ValueError(f"invalid key arguments (rc={rc})")
    return out[:nx * r * z].reshape(nx, r * z)


def query(index_chars, index_offsets, q_chars, q_offsets, Kq, r: int, z: int, m: int,
          seed: int = 0, L: int = 0):
    """Serving semantics: per query, the index positions sharing a key with
    it in some table, within K_q in length and in edit distance, sorted.
    Returns (offsets[nq+1], ids, dist); raises ValueError for a query byte
    outside the index alphabet."""
    ic, qc = _u8(index_chars), _u8(q_chars)
    io = np.ascontiguousarray(index_offsets, dtype=np.uint64)
    qo = np.ascontiguousarray(q_offsets, dtype=np.uint64)
    K = np.ascontiguousarray(Kq, dtype=np.uint32)
    n, nq = io.shape[0] - 1, qo.shape[0] - 1
    cap = 1 << 12
    while True:
        off = np.zeros(nq + 1, dtype=np.uint64)
        ids = np.zeros(cap, dtype=np.uint32)
        d = np.zeros(cap, dtype=np.uint32)
        cnt = int(lib().ejo_query(_ptr(ic, ctypes.c_uint8) if ic.size else None,
                                  _ptr(io, ctypes.c_uint64), n,
                                  _ptr(qc, ctypes.c_uint8) if qc.size else None,
                                  _ptr(qo, ctypes.c_uint64), nq,
                                  _ptr(K, ctypes.c_uint32) if K.size else None, r, z, m, L, seed,
                                  _ptr(off, ctypes.c_uint64), _ptr(ids, ctypes.c_uint32),
                                  _ptr(d, ctypes.c_uint32), cap))
        if cnt == -2:
            raise ValueError("query byte outside the index alphabet")
        if cnt == -3:
            raise ValueError("all 256 byte values occur in the index")
        if cnt < 0:
            raise ValueError("invalid query arguments")
        if cnt <= cap:
            return off, ids[:cnt], d[:cnt]
        cap = cnt
