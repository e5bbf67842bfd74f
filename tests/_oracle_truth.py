"""Expected results computed from the oracle alone, spread over host threads
(the oracle is a C library called through ctypes, which releases the GIL):
its distances of many pairs, its keys of many strings, and the serving
definition over a whole index (every index string that shares a key with the
query in some table, is within K_q in length and within K_q in edit distance,
sorted by position).  Test infrastructure; no GPU code is used here."""
from concurrent.futures import ThreadPoolExecutor

import numpy as np

THREADS = 16


def oracle_dist(oracle_lib, col, codes, K):
    """The oracle's min(ED, K+1) of each pair (codes a << 32 | b)."""
    codes = np.asarray(codes, dtype=np.uint64)
    if len(codes) == 0:
        return np.zeros(0, dtype=np.uint32)
    chunks = np.array_split(codes, min(THREADS * 4, len(codes)))
    with ThreadPoolExecutor(THREADS) as ex:
        parts = list(ex.map(lambda c: oracle_lib.verify_pairs(col.chars, col.offsets, c, K),
                            chunks))
    return np.concatenate(parts)


def oracle_keys(oracle_lib, col, x, r, z, m, seed, L):
    """The oracle's keys [x.n, r*z] of the strings of x under col's alphabet,
    truncation and random streams (chunks of x's offsets per thread)."""
    bounds = np.linspace(0, x.n, min(THREADS, max(x.n, 1)) + 1).astype(np.int64)
    with ThreadPoolExecutor(THREADS) as ex:
        parts = list(ex.map(lambda ab: oracle_lib.keys(col.chars, col.offsets, x.chars,
                                                       x.offsets[ab[0]:ab[1] + 1], r, z, m,
                                                       seed=seed, L=L),
                            zip(bounds[:-1], bounds[1:])))
    return np.concatenate(parts)


def serving_truth(oracle_lib, col, q, Kq, r, z, m, seed, L):
    """Per query (ids, dists) of the serving definition over the whole index
    col, and the number of (query, string) pairs sharing a key within the
    length window.  Key matches are found table by table with a sorted copy of
    the index's keys and a binary search (a lookup, no arithmetic of the
    method)."""
    ikeys = oracle_keys(oracle_lib, col, col, r, z, m, seed, L)
    qkeys = oracle_keys(oracle_lib, col, q, r, z, m, seed, L)
    ilen, qlen = col.lengths(), q.lengths()
    shared = [set() for _ in range(q.n)]
    for t in range(r * z):
        order = np.argsort(ikeys[:, t], kind="stable")
        sk = ikeys[order, t]
        lo = np.searchsorted(sk, qkeys[:, t], side="left")
        hi = np.searchsorted(sk, qkeys[:, t], side="right")
        for qi in np.nonzero(hi > lo)[0].tolist():
            shared[qi].update(order[lo[qi]:hi[qi]].tolist())
    del ikeys
    pairs = [(qi, s) for qi in range(q.n) for s in sorted(shared[qi])
             if abs(int(ilen[s]) - int(qlen[qi])) <= int(Kq[qi])]

    def ed(p):
        qi, s = p
        x = col.chars[int(col.offsets[s]):int(col.offsets[s + 1])]
        y = q.chars[int(q.offsets[qi]):int(q.offsets[qi + 1])]
        return oracle_lib.ed_banded(x, y, int(Kq[qi]))

    with ThreadPoolExecutor(THREADS) as ex:
        dists = list(ex.map(ed, pairs, chunksize=64))
    want = [([], []) for _ in range(q.n)]
    for (qi, s), d in zip(pairs, dists):
        if d <= Kq[qi]:
            want[qi][0].append(s)
            want[qi][1].append(d)
    return want, len(pairs)
