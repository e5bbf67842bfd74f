"""MI355X (gfx950) implementation of the EmbedJoin hot path.

Thin ctypes binding over ``libembedjoin.so`` (C ABI in ``include/embedjoin.h``).
Every step of the join runs in the library's HIP kernels; this module only
marshals arguments.  PyTorch provides device memory and streams.  Importing
works without a GPU, but every call needs the built library and a device: a
missing library raises ``ImportError`` when the first call is made -- there is
no fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libembedjoin.so")

EJ_OK, EJ_EINVAL, EJ_EALPHABET, EJ_ENOMEM, EJ_ECAPACITY, EJ_EHIP, EJ_EUNSUPPORTED = range(7)
STATUS_NAMES = {0: "EJ_OK", 1: "EJ_EINVAL", 2: "EJ_EALPHABET", 3: "EJ_ENOMEM",
                4: "EJ_ECAPACITY", 5: "EJ_EHIP", 6: "EJ_EUNSUPPORTED"}
FLAG_PLAIN, FLAG_GRAPH, FLAG_TIMING, FLAG_DEVICE_OUT = 0, 1, 2, 4

# Every symbol declared in include/embedjoin.h.
EXPORTS = [
    "ej_create", "ej_destroy", "ej_last_error", "ej_version", "ej_workspace_bytes",
    "ej_tune_set", "ej_tune_get",
    "ej_join", "ej_join_ex", "ej_join_device", "ej_join_plus", "ej_join_plus_device",
    "ej_join_grouped", "ej_join_grouped_device",
    "ej_result_free", "ej_autotune",
    "ej_embed", "ej_lsh_bucket", "ej_candidates", "ej_verify", "ej_verify_static",
    "ej_set_explicit_randomness", "ej_embed_hamming", "ej_calibrate", "ej_probe_valu",
    "ej_index_build", "ej_index_insert", "ej_query_batch", "ej_query_workspace_estimate", "ej_index_set_hbm_limit",
    "ej_index_size", "ej_qresult_free", "ej_index_free",
]


class EmbedJoinError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class Params(ctypes.Structure):
    _fields_ = [("K", ctypes.c_uint32), ("r", ctypes.c_uint32), ("z", ctypes.c_uint32),
                ("m", ctypes.c_uint32), ("L", ctypes.c_uint32), ("flags", ctypes.c_uint32),
                ("seed", ctypes.c_uint64), ("exact_len", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32)]


class _Result(ctypes.Structure):
    _fields_ = [("count", ctypes.c_uint64), ("pairs", ctypes.POINTER(ctypes.c_uint32)),
                ("dist", ctypes.POINTER(ctypes.c_int32)), ("n_candidates", ctypes.c_uint64),
                ("n_raw", ctypes.c_uint64), ("sigma", ctypes.c_uint32), ("L", ctypes.c_uint32),
                ("ms_prep", ctypes.c_float), ("ms_embed", ctypes.c_float),
                ("ms_bucket", ctypes.c_float), ("ms_candidates", ctypes.c_float),
                ("ms_verify", ctypes.c_float), ("ms_output", ctypes.c_float),
                ("walk_steps", ctypes.c_uint64), ("verify_columns", ctypes.c_uint64),
                ("ms_verify_kernel", ctypes.c_float), ("verify_launches", ctypes.c_uint32),
                ("verify_form", ctypes.c_uint32), ("on_device", ctypes.c_uint32),
                ("graph", ctypes.c_uint32)]


class CalibOpts(ctypes.Structure):
    _fields_ = [("K", ctypes.c_uint32), ("delta", ctypes.c_uint32), ("T", ctypes.c_uint32),
                ("r_max", ctypes.c_uint32), ("z_list", ctypes.POINTER(ctypes.c_uint32)),
                ("nz", ctypes.c_uint32), ("m_list", ctypes.POINTER(ctypes.c_uint32)),
                ("nm", ctypes.c_uint32), ("L_list", ctypes.POINTER(ctypes.c_uint32)),
                ("nL", ctypes.c_uint32), ("target_recall", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("exact_len", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32)]


class CalibResult(ctypes.Structure):
    _fields_ = [("r", ctypes.c_uint32), ("z", ctypes.c_uint32), ("m", ctypes.c_uint32),
                ("L", ctypes.c_uint32), ("recall", ctypes.c_double),
                ("false_rate", ctypes.c_double), ("work", ctypes.c_double),
                ("n_similar", ctypes.c_uint64), ("n_dissimilar", ctypes.c_uint64),
                ("best_recall", ctypes.c_double)]


class _QResult(ctypes.Structure):
    _fields_ = [("nq", ctypes.c_uint32), ("offsets", ctypes.POINTER(ctypes.c_uint64)),
                ("ids", ctypes.POINTER(ctypes.c_uint32)), ("dist", ctypes.POINTER(ctypes.c_int32)),
                ("n_candidates", ctypes.c_uint64), ("ms_total", ctypes.c_float),
                ("workspace_bytes", ctypes.c_uint64)]


_lib = None


def lib():
    """Loads libembedjoin.so (raises ImportError if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_1702_00093_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, u8p, u32p, u64p, i32p = (ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint8),
                                 ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_uint64),
                                 ctypes.POINTER(ctypes.c_int32))
    u32, u64, c_int = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
    sig = {
        "ej_create": (c_int, [ctypes.POINTER(vp), c_int, vp]),
        "ej_destroy": (None, [vp]),
        "ej_last_error": (ctypes.c_char_p, [vp]),
        "ej_version": (c_int, []),
        "ej_workspace_bytes": (u64, [vp]),
        "ej_tune_set": (c_int, [vp, ctypes.c_char_p, u32]),
        "ej_tune_get": (c_int, [vp, ctypes.c_char_p, u32p]),
        "ej_join": (c_int, [vp, vp, vp, u32, u32, u32, u32, u32, u64, ctypes.POINTER(_Result)]),
        "ej_join_ex": (c_int, [vp, vp, vp, u32, ctypes.POINTER(Params), ctypes.POINTER(_Result)]),
        "ej_join_device": (c_int, [vp, vp, vp, u32, ctypes.POINTER(Params),
                                   ctypes.POINTER(_Result)]),
        "ej_join_plus": (c_int, [vp, vp, vp, u32, ctypes.POINTER(Params), u32, u32,
                                 ctypes.POINTER(_Result)]),
        "ej_join_plus_device": (c_int, [vp, vp, vp, u32, ctypes.POINTER(Params), u32, u32,
                                        ctypes.POINTER(_Result)]),
        "ej_join_grouped": (c_int, [vp, vp, vp, u32, ctypes.POINTER(Params),
                                    ctypes.POINTER(_Result)]),
        "ej_join_grouped_device": (c_int, [vp, vp, vp, u32, ctypes.POINTER(Params),
                                           ctypes.POINTER(_Result)]),
        "ej_result_free": (None, [ctypes.POINTER(_Result)]),
        "ej_autotune": (c_int, [vp, vp, vp, u32, ctypes.POINTER(Params), u32,
                                ctypes.POINTER(ctypes.c_float)]),
        "ej_embed": (c_int, [vp, vp, vp, u32, ctypes.POINTER(Params), vp, vp, u32p, u32p]),
        "ej_lsh_bucket": (c_int, [vp, vp, vp, u32, u32, u32, vp, vp, u64p]),
        "ej_candidates": (c_int, [vp, vp, vp, vp, u64, vp, u32, u32, u32, vp, u64, u64p, u64p]),
        "ej_verify": (c_int, [vp, vp, vp, u32, vp, u64, u32, vp, vp]),
        "ej_verify_static": (c_int, [vp, vp, vp, u32, vp, u64, u32, vp, vp]),
        "ej_set_explicit_randomness": (c_int, [vp, u32, u32, u32, u32, u32, vp, vp, vp]),
        "ej_embed_hamming": (c_int, [vp, vp, vp, u32, ctypes.POINTER(Params), u32, vp, u64, vp]),
        "ej_calibrate": (c_int, [vp, vp, vp, u32, vp, u64, ctypes.POINTER(CalibOpts),
                                 ctypes.POINTER(CalibResult), vp]),
        "ej_probe_valu": (c_int, [vp, u32, u32, u32, ctypes.POINTER(ctypes.c_double),
                                  ctypes.POINTER(ctypes.c_float)]),
        "ej_index_build": (c_int, [vp, vp, vp, u32, ctypes.POINTER(Params), c_int,
                                   ctypes.POINTER(vp)]),
        "ej_index_insert": (c_int, [vp, vp, vp, u32, c_int]),
        "ej_query_batch": (c_int, [vp, vp, vp, u32, vp, ctypes.POINTER(_QResult)]),
        "ej_query_workspace_estimate": (u64, [vp, vp, u32, vp]),
        "ej_index_set_hbm_limit": (None, [vp, u64]),
        "ej_index_size": (u32, [vp]),
        "ej_qresult_free": (None, [ctypes.POINTER(_QResult)]),
        "ej_index_free": (None, [vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


# ---------------------------------------------------------------- helpers --

def _torch():
    import torch
    return torch


def _ptr(x):
    """Address of a numpy array or torch tensor (None -> NULL)."""
    if x is None:
        return None
    if isinstance(x, np.ndarray):
        return x.ctypes.data
    return x.data_ptr()


def _host_u8(chars) -> np.ndarray:
    if isinstance(chars, (bytes, bytearray, memoryview)):
        return np.frombuffer(bytes(chars), dtype=np.uint8)
    if hasattr(chars, "detach"):
        chars = chars.detach().cpu().numpy()
    return np.ascontiguousarray(chars, dtype=np.uint8)


def _host_u64(offsets) -> np.ndarray:
    if hasattr(offsets, "detach"):
        offsets = offsets.detach().cpu().numpy()
    return np.ascontiguousarray(offsets, dtype=np.uint64)


def _is_device(x) -> bool:
    return hasattr(x, "is_cuda") and x.is_cuda


def _torch_stream_done():
    """The library runs on its own stream: device buffers that torch's current
    stream writes (or will reuse) must be settled before a call."""
    _torch().cuda.current_stream().synchronize()


class _DeviceArray:
    """A device buffer described by the CUDA array interface, so that torch
    can take it over without a copy through the host."""

    def __init__(self, ptr: int, shape, typestr: str):
        self.__cuda_array_interface__ = {"shape": tuple(shape), "typestr": typestr,
                                         "data": (ptr, False), "version": 3, "strides": None}


@dataclass
class JoinResult:
    """Output pairs (i < j, sorted) with their distances.  With
    FLAG_DEVICE_OUT the result is in device memory (`pairs_device` [count, 2]
    int32 and `dist_device` torch tensors, owned by torch); `pairs`/`dist`
    copy it to the host when first read."""
    pairs_host: np.ndarray | None
    dist_host: np.ndarray | None
    n_candidates: int
    n_raw: int
    sigma: int
    L: int
    ms: dict
    walk_steps: int = 0
    verify_columns: int = 0
    ms_verify_kernel: float = 0.0
    verify_launches: int = 0
    verify_form: int = 0       # 0 two-pass, 1 persistent groups, 2 one pair per lane, 3 split,
    #                            4 grouped by pattern, 5 two-pass with 2 or 4 words per lane
    pairs_device: object = None
    dist_device: object = None
    graph: int = 0             # 0 host-sized, 1 device-sized uncaptured, 2 graph replay

    @property
    def pairs(self) -> np.ndarray:       # [count, 2] int64
        if self.pairs_host is None:
            self.pairs_host = self.pairs_device.cpu().numpy().astype(np.uint32) \
                .astype(np.int64)
        return self.pairs_host

    @property
    def dist(self) -> np.ndarray:        # [count] int32
        if self.dist_host is None:
            self.dist_host = self.dist_device.cpu().numpy()
        return self.dist_host

    @property
    def count(self) -> int:
        return int(self.pairs_device.shape[0]) if self.pairs_host is None else \
            int(self.pairs_host.shape[0])

    @property
    def codes(self) -> np.ndarray:
        return (self.pairs[:, 0].astype(np.uint64) << np.uint64(32)) | \
            self.pairs[:, 1].astype(np.uint64)


class Context:
    """A library context bound to one device and one HIP stream."""

    def __init__(self, device: int = 0, stream=None):
        # torch carries a HIP runtime of its own besides the one this library
        # links; torch's must start first or it finds no device afterwards
        _torch().cuda.init()
        L = lib()
        self._h = ctypes.c_void_p()
        st = L.ej_create(ctypes.byref(self._h), device, stream)
        if st != EJ_OK:
            raise EmbedJoinError(st, "ej_create failed")
        self.device = device

    def close(self):
        if self._h:
            lib().ej_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st: int):
        if st != EJ_OK:
            msg = lib().ej_last_error(self._h)
            raise EmbedJoinError(st, msg.decode() if msg else "")

    def tune_set(self, name: str, value: int):
        self._check(lib().ej_tune_set(self._h, name.encode(), int(value)))

    def tune_get(self, name: str) -> int:
        v = ctypes.c_uint32()
        self._check(lib().ej_tune_get(self._h, name.encode(), ctypes.byref(v)))
        return int(v.value)

    @property
    def workspace_bytes(self) -> int:
        return int(lib().ej_workspace_bytes(self._h))

    # ----------------------------------------------------------- the join --
    def join(self, chars, offsets, K: int, r: int, z: int, m: int, seed: int = 0, L: int = 0,
             flags: int = 0, exact_len: int = 0) -> JoinResult:
        """EmbedJoin self-join.  Host inputs (bytes / numpy / CPU tensors) go
        through ej_join_ex; CUDA tensors (uint8 chars, int64 offsets) go
        through ej_join_device.  exact_len > 0: every pair of strings no
        longer than exact_len whose lengths differ by at most K is a
        candidate too."""
        return self._join(chars, offsets, Params(K, r, z, m, L, flags, seed, exact_len), None)

    def join_plus(self, chars, offsets, K: int, r: int, z: int, m: int, delta: int = 0,
                  T: int = 0, seed: int = 0, L: int = 0, flags: int = 0,
                  exact_len: int = 0) -> JoinResult:
        """EmbedJoin+ (ej_join_plus / ej_join_plus_device): ceil(K/delta)
        suffixes per string, tuple threshold T (0: the paper's rule)."""
        return self._join(chars, offsets, Params(K, r, z, m, L, flags, seed, exact_len),
                          (delta, T))

    def join_grouped(self, chars, offsets, K: int, r: int, z: int, m: int, seed: int = 0,
                     L: int = 0, flags: int = 0, exact_len: int = 0) -> JoinResult:
        """EmbedJoin with grouping instead of truncation (ej_join_grouped /
        ej_join_grouped_device)."""
        return self._join(chars, offsets, Params(K, r, z, m, L, flags, seed, exact_len),
                          "grouped")

    def _join(self, chars, offsets, p, plus) -> JoinResult:
        res = _Result()
        if _is_device(chars) or _is_device(offsets):
            torch = _torch()
            assert chars.dtype == torch.uint8 and offsets.dtype == torch.int64
            assert chars.is_contiguous() and offsets.is_contiguous()
            n = offsets.numel() - 1
            # the library works on its own stream: inputs written on torch's
            # current stream must be complete first
            torch.cuda.current_stream().synchronize()
            if plus is None:
                st = lib().ej_join_device(self._h, _ptr(chars), _ptr(offsets), n,
                                          ctypes.byref(p), ctypes.byref(res))
            elif plus == "grouped":
                st = lib().ej_join_grouped_device(self._h, _ptr(chars), _ptr(offsets), n,
                                                  ctypes.byref(p), ctypes.byref(res))
            else:
                st = lib().ej_join_plus_device(self._h, _ptr(chars), _ptr(offsets), n,
                                               ctypes.byref(p), plus[0], plus[1],
                                               ctypes.byref(res))
        else:
            c = _host_u8(chars)
            o = _host_u64(offsets)
            n = o.shape[0] - 1
            cp = _ptr(c) if c.size else None
            if plus is None:
                st = lib().ej_join_ex(self._h, cp, _ptr(o), n, ctypes.byref(p), ctypes.byref(res))
            elif plus == "grouped":
                st = lib().ej_join_grouped(self._h, cp, _ptr(o), n, ctypes.byref(p),
                                           ctypes.byref(res))
            else:
                st = lib().ej_join_plus(self._h, cp, _ptr(o), n, ctypes.byref(p), plus[0],
                                        plus[1], ctypes.byref(res))
        self._check(st)
        try:
            cnt = int(res.count)
            ms = dict(prep=res.ms_prep, embed=res.ms_embed, bucket=res.ms_bucket,
                      candidates=res.ms_candidates, verify=res.ms_verify, output=res.ms_output)
            ph = dh = pd = dd = None
            if res.on_device:
                # the library's buffers are reused by its next call: torch copies
                # them into memory of its own (device to device)
                torch = _torch()
                pa = ctypes.cast(res.pairs, ctypes.c_void_p).value or 0
                da = ctypes.cast(res.dist, ctypes.c_void_p).value or 0
                if cnt:
                    pd = torch.as_tensor(_DeviceArray(pa, (cnt, 2), "<i4"), device="cuda").clone()
                    dd = torch.as_tensor(_DeviceArray(da, (cnt,), "<i4"), device="cuda").clone()
                else:
                    pd = torch.zeros((0, 2), dtype=torch.int32, device="cuda")
                    dd = torch.zeros(0, dtype=torch.int32, device="cuda")
            else:
                # astype copies: the arrays stay valid after the result is freed
                ph = np.ctypeslib.as_array(res.pairs, (max(cnt, 1) * 2,))[:2 * cnt] \
                    .reshape(cnt, 2).astype(np.int64)
                dh = np.ctypeslib.as_array(res.dist, (max(cnt, 1),))[:cnt].copy()
            return JoinResult(ph, dh, int(res.n_candidates), int(res.n_raw),
                              int(res.sigma), int(res.L), ms, int(res.walk_steps),
                              int(res.verify_columns), float(res.ms_verify_kernel),
                              int(res.verify_launches), int(res.verify_form), pd, dd,
                              int(res.graph))
        finally:
            lib().ej_result_free(ctypes.byref(res))

    KNOBS = ("verify_mode", "verify_order", "verify_split", "verify_pass1_cols",
             "verify_blocks_per_cu", "verify_ring",
             "verify_lds_budget", "embed_lds_budget", "radix_bits", "bucket_key_bits",
             "dedup_sort", "raw_limit", "verify_wpl", "verify_len_order")

    def knobs(self) -> dict:
        return {k: self.tune_get(k) for k in self.KNOBS}

    def autotune(self, d_chars, d_offsets, K: int, r: int, z: int, m: int, seed: int = 0,
                 L: int = 0, reps: int = 2):
        """ej_autotune on device tensors; returns (best join ms, chosen knobs)."""
        p = Params(K, r, z, m, L, 0, seed)
        best = ctypes.c_float()
        n = d_offsets.numel() - 1
        _torch_stream_done()
        self._check(lib().ej_autotune(self._h, _ptr(d_chars), _ptr(d_offsets), n,
                                      ctypes.byref(p), reps, ctypes.byref(best)))
        return float(best.value), self.knobs()

    # ------------------------------------------------------------- stages --
    def embed(self, d_chars, d_offsets, r: int, z: int, m: int, seed: int = 0, L: int = 0,
              want_sig: bool = False):
        """A1-A2 on device tensors.  Returns (keys [r*z, n] int64, sig [n, r, z, m] uint8 or
        None, L_used, sigma)."""
        torch = _torch()
        n = d_offsets.numel() - 1
        keys = torch.empty((r * z, max(n, 1)), dtype=torch.int64, device=d_offsets.device)
        sig = torch.empty((max(n, 1), r, z, m), dtype=torch.uint8, device=d_offsets.device) \
            if want_sig else None
        p = Params(0, r, z, m, L, 0, seed)
        Lu, sg = ctypes.c_uint32(), ctypes.c_uint32()
        _torch_stream_done()
        self._check(lib().ej_embed(self._h, _ptr(d_chars) if d_chars.numel() else None,
                                   _ptr(d_offsets), n, ctypes.byref(p), _ptr(sig), _ptr(keys),
                                   ctypes.byref(Lu), ctypes.byref(sg)))
        return keys[:, :n], (sig[:n] if sig is not None else None), int(Lu.value), int(sg.value)

    def lsh_bucket(self, d_keys, d_len, key_bits: int = 0):
        """A3.  d_keys [T, n] int64, d_len [n] int32.  Returns (ids [T*n] int32,
        group_start [ngroups+1] int32)."""
        torch = _torch()
        T, n = d_keys.shape
        ids = torch.empty(max(T * n, 1), dtype=torch.int32, device=d_keys.device)
        gs = torch.empty(T * n + 1, dtype=torch.int32, device=d_keys.device)
        ng = ctypes.c_uint64()
        kc = d_keys.contiguous()
        _torch_stream_done()
        self._check(lib().ej_lsh_bucket(self._h, _ptr(kc), _ptr(d_len), n, T,
                                        key_bits, _ptr(ids), _ptr(gs), ctypes.byref(ng)))
        return ids[:T * n], gs[:int(ng.value) + 1]

    def candidates(self, d_keys, d_ids, d_group_start, d_len, K: int, capacity: int | None = None):
        """A4.  Returns (pairs int64 codes (i << 32 | j), n_raw)."""
        torch = _torch()
        T, n = d_keys.shape
        cap = capacity if capacity is not None else 1 << 20
        while True:
            out = torch.empty(max(cap, 1), dtype=torch.int64, device=d_keys.device)
            cnt, raw = ctypes.c_uint64(), ctypes.c_uint64()
            kc = d_keys.contiguous()
            _torch_stream_done()
            st = lib().ej_candidates(self._h, _ptr(kc), _ptr(d_ids),
                                     _ptr(d_group_start), d_group_start.numel() - 1, _ptr(d_len),
                                     n, T, K, _ptr(out), cap, ctypes.byref(cnt), ctypes.byref(raw))
            if st == EJ_ECAPACITY and capacity is None:
                cap = int(cnt.value)
                continue
            self._check(st)
            return out[:int(cnt.value)], int(raw.value)

    def verify(self, d_chars, d_offsets, d_pairs, K: int, d_Kq=None, dist=None,
               no_alloc: bool = False):
        """A5.  Returns int32 distances, min(ED, K+1) per pair.  With
        no_alloc, ej_verify_static (no device allocation inside the library;
        `dist` may be given to avoid torch's allocation too)."""
        torch = _torch()
        n = d_offsets.numel() - 1
        cnt = d_pairs.numel()
        if dist is None:
            dist = torch.empty(max(cnt, 1), dtype=torch.int32, device=d_offsets.device)
        fn = lib().ej_verify_static if no_alloc else lib().ej_verify
        _torch_stream_done()
        self._check(fn(self._h, _ptr(d_chars) if d_chars.numel() else None,
                       _ptr(d_offsets), n, _ptr(d_pairs) if cnt else None, cnt, K,
                       _ptr(d_Kq), _ptr(dist)))
        return dist[:cnt]

    def embed_hamming(self, d_chars, d_offsets, d_pairs, r: int, L: int = 0, seed: int = 0,
                      K: int = 0, delta: int = 0):
        """ej_embed_hamming: [count, r] int32 Hamming distances of the pairs'
        L-symbol embeddings per seed (min over suffix pairs when delta > 0)."""
        torch = _torch()
        n = d_offsets.numel() - 1
        cnt = d_pairs.numel()
        ham = torch.empty((max(cnt, 1), r), dtype=torch.int32, device=d_offsets.device)
        p = Params(K, r, 1, 1, L, 0, seed)
        _torch_stream_done()
        self._check(lib().ej_embed_hamming(self._h, _ptr(d_chars) if d_chars.numel() else None,
                                           _ptr(d_offsets), n, ctypes.byref(p), delta,
                                           _ptr(d_pairs) if cnt else None, cnt, _ptr(ham)))
        return ham[:cnt]

    def calibrate(self, d_chars, d_offsets, d_pairs, K: int, r_max: int, z_list, m_list,
                  L_list, target_recall: float = 0.99, seed: int = 0, delta: int = 0, T: int = 0,
                  want_table: bool = False, exact_len: int = 0):
        """ej_calibrate: returns a dict with the chosen (r, z, m, L) and its
        predictions (and the whole grid as an array [nL, r_max, nz, nm, 3]
        when want_table)."""
        n = d_offsets.numel() - 1
        cnt = d_pairs.numel()
        zs = np.ascontiguousarray(z_list, dtype=np.uint32)
        ms = np.ascontiguousarray(m_list, dtype=np.uint32)
        Ls = np.ascontiguousarray(L_list, dtype=np.uint32)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        o = CalibOpts(K, delta, T, r_max, zs.ctypes.data_as(u32p), len(zs),
                      ms.ctypes.data_as(u32p), len(ms), Ls.ctypes.data_as(u32p), len(Ls),
                      float(target_recall), seed, exact_len, 0)
        res = CalibResult()
        table = np.zeros((len(Ls), r_max, len(zs), len(ms), 3)) if want_table else None
        _torch_stream_done()
        self._check(lib().ej_calibrate(self._h, _ptr(d_chars) if d_chars.numel() else None,
                                       _ptr(d_offsets), n, _ptr(d_pairs) if cnt else None, cnt,
                                       ctypes.byref(o), ctypes.byref(res), _ptr(table)))
        out = {k: getattr(res, k) for k, _ in CalibResult._fields_}
        if want_table:
            out["table"] = table
        return out

    def probe_valu(self, iters: int = 4096, blocks_per_cu: int = 8, mix: int = 0):
        """ej_probe_valu: (achieved int32 lane-ops/s, kernel ms)."""
        ops, ms = ctypes.c_double(), ctypes.c_float()
        self._check(lib().ej_probe_valu(self._h, mix, iters, blocks_per_cu, ctypes.byref(ops),
                                        ctypes.byref(ms)))
        return float(ops.value), float(ms.value)

    def set_explicit_randomness(self, r, z, m, L, sigma, Rbits=None, pos=None, v=None):
        if Rbits is None:
            self._check(lib().ej_set_explicit_randomness(self._h, 0, 0, 0, 0, 0, None, None, None))
            return
        R = np.ascontiguousarray(Rbits, dtype=np.uint8)
        P = np.ascontiguousarray(pos, dtype=np.uint32)
        V = None if v is None else np.ascontiguousarray(v, dtype=np.uint64)
        self._check(lib().ej_set_explicit_randomness(self._h, r, z, m, L, sigma, _ptr(R), _ptr(P),
                                                     _ptr(V)))


_default: dict[int, Context] = {}


@dataclass
class QueryResult:
    offsets: np.ndarray        # [nq + 1] uint64: results of query q are [offsets[q], offsets[q+1])
    ids: np.ndarray            # index positions, sorted within each query
    dist: np.ndarray           # edit distances
    n_candidates: int          # (query, index string) pairs verified
    ms: float                  # device time of the batch
    workspace_bytes: int = 0   # the batch's admission figure (estimate + counted stages)

    def of(self, q: int):
        lo, hi = int(self.offsets[q]), int(self.offsets[q + 1])
        return self.ids[lo:hi], self.dist[lo:hi]


class Index:
    """Device-resident LSH index (ej_index_build / ej_query_batch)."""

    def __init__(self, ctx: Context, chars, offsets, r: int, z: int, m: int, seed: int = 0,
                 L: int = 0):
        self._ctx = ctx
        self._h = None
        p = Params(0, r, z, m, L, 0, seed)
        h = ctypes.c_void_p()
        if _is_device(chars):
            torch = _torch()
            o = offsets if _is_device(offsets) else torch.from_numpy(
                _host_u64(offsets).astype(np.int64)).cuda()
            n = int(o.shape[0]) - 1
            torch.cuda.current_stream().synchronize()
            st = lib().ej_index_build(ctx._h, _ptr(chars), _ptr(o), n, ctypes.byref(p), 1,
                                      ctypes.byref(h))
        else:
            c, o = _host_u8(chars), _host_u64(offsets)
            n = int(o.shape[0]) - 1
            st = lib().ej_index_build(ctx._h, _ptr(c) if c.size else None, _ptr(o), n,
                                      ctypes.byref(p), 0, ctypes.byref(h))
        ctx._check(st)
        self._h = h.value
        self.n = n

    def close(self):
        if self._h is not None:
            lib().ej_index_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def insert(self, chars, offsets):
        """ej_index_insert: adds strings (host arrays or CUDA tensors) at the
        next positions."""
        if _is_device(chars):
            torch = _torch()
            o = offsets if _is_device(offsets) else torch.from_numpy(
                _host_u64(offsets).astype(np.int64)).cuda()
            n = int(o.shape[0]) - 1
            torch.cuda.current_stream().synchronize()
            st = lib().ej_index_insert(self._h, _ptr(chars), _ptr(o), n, 1)
        else:
            c, o = _host_u8(chars), _host_u64(offsets)
            n = int(o.shape[0]) - 1
            st = lib().ej_index_insert(self._h, _ptr(c) if c.size else None, _ptr(o), n, 0)
        self._ctx._check(st)
        self.n += n

    def set_hbm_limit(self, nbytes: int):
        lib().ej_index_set_hbm_limit(self._h, int(nbytes))

    def size(self) -> int:
        return int(lib().ej_index_size(self._h))

    def workspace_estimate(self, q_offsets, Kq) -> int:
        o = _host_u64(q_offsets)
        k = np.ascontiguousarray(Kq, dtype=np.uint32)
        return int(lib().ej_query_workspace_estimate(self._h, _ptr(o), o.shape[0] - 1,
                                                     _ptr(k) if k.size else None))

    def query(self, q_chars, q_offsets, Kq) -> QueryResult:
        c, o = _host_u8(q_chars), _host_u64(q_offsets)
        k = np.ascontiguousarray(Kq, dtype=np.uint32)
        nq = o.shape[0] - 1
        res = _QResult()
        st = lib().ej_query_batch(self._h, _ptr(c) if c.size else None, _ptr(o), nq,
                                  _ptr(k) if k.size else None, ctypes.byref(res))
        self._ctx._check(st)
        try:
            offs = np.ctypeslib.as_array(res.offsets, (nq + 1,)).copy() if nq else \
                np.zeros(1, dtype=np.uint64)
            tot = int(offs[-1])
            ids = np.ctypeslib.as_array(res.ids, (max(tot, 1),))[:tot].copy() if tot else \
                np.zeros(0, dtype=np.uint32)
            dist = np.ctypeslib.as_array(res.dist, (max(tot, 1),))[:tot].copy() if tot else \
                np.zeros(0, dtype=np.int32)
            return QueryResult(offs, ids, dist, int(res.n_candidates), float(res.ms_total),
                               int(res.workspace_bytes))
        finally:
            lib().ej_qresult_free(ctypes.byref(res))


def context(device: int = 0) -> Context:
    if device not in _default:
        _default[device] = Context(device)
    return _default[device]


def join(chars, offsets, K: int, r: int, z: int, m: int, seed: int = 0, L: int = 0,
         flags: int = 0, device: int = 0, exact_len: int = 0) -> JoinResult:
    return context(device).join(chars, offsets, K, r, z, m, seed=seed, L=L, flags=flags,
                                exact_len=exact_len)


def version() -> int:
    return int(lib().ej_version())
