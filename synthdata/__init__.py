"""Seeded synthetic string collections shaped like the paper's workloads.

This module is shared by the tests, the benchmark and the oracle drivers.  It
holds no part of the join method itself: it only draws strings (clusters of
mutated copies of random base strings) and returns them in the CSR layout the
library takes -- a flat ``uint8`` byte array plus ``uint64`` offsets of length
``n + 1``.  Cluster labels are returned alongside so that planted similar
pairs can be enumerated for recall estimates.

Edit model for a copy of a base string (fixed here, shared by every config):
the number of edits ``E`` is drawn per copy; each edit is a substitution,
deletion or insertion with probability 1/3 each.  Substitution and deletion
sites are distinct positions of the base string drawn uniformly without
replacement; insertion sites are drawn uniformly with replacement from the
``len + 1`` gaps.  A substituted letter is redrawn from the letter
distribution until it differs from the original; inserted letters are drawn
from the letter distribution.

The paper's datasets (protein, medical text, human genome reads) are not
available, so these collections stand in for them with the same alphabet
sizes, length ranges and collection sizes.
"""
from __future__ import annotations

import dataclasses
import numpy as np

DNA = b"ACGT"
# 25 protein-like letters (the paper's protein alphabet size).
PROTEIN25 = b"ACDEFGHIKLMNPQRSTVWYBZXJU"


@dataclasses.dataclass
class Collection:
    chars: np.ndarray      # uint8, concatenated strings
    offsets: np.ndarray    # uint64, n + 1
    labels: np.ndarray     # int64 cluster id per string (-1: singleton / fresh)
    desc: str = ""

    @property
    def n(self) -> int:
        return int(self.offsets.shape[0] - 1)

    def lengths(self) -> np.ndarray:
        return np.diff(self.offsets).astype(np.int64)

    def string(self, i: int) -> bytes:
        return bytes(self.chars[int(self.offsets[i]):int(self.offsets[i + 1])])

    def strings(self) -> list[bytes]:
        return [self.string(i) for i in range(self.n)]


def from_strings(strings, labels=None, desc="") -> Collection:
    strings = [bytes(s) for s in strings]
    lens = np.array([len(s) for s in strings], dtype=np.uint64)
    offsets = np.zeros(len(strings) + 1, dtype=np.uint64)
    np.cumsum(lens, out=offsets[1:])
    chars = np.frombuffer(b"".join(strings), dtype=np.uint8).copy()
    if labels is None:
        labels = np.full(len(strings), -1, dtype=np.int64)
    return Collection(chars, offsets, np.asarray(labels, dtype=np.int64), desc)


def _draw_letters(rng, letters: np.ndarray, probs, size) -> np.ndarray:
    if probs is None:
        return letters[rng.integers(0, letters.shape[0], size=size)]
    return letters[rng.choice(letters.shape[0], size=size, p=probs)]


def mutate(rng, base: np.ndarray, n_edits: int, letters: np.ndarray,
           probs=None) -> np.ndarray:
    """Apply ``n_edits`` edits (sub/del/ins, 1/3 each) to ``base``."""
    L = base.shape[0]
    if n_edits <= 0:
        return base.copy()
    kinds = rng.integers(0, 3, size=n_edits)
    n_sub = int((kinds == 0).sum())
    n_del = int((kinds == 1).sum())
    n_ins = n_edits - n_sub - n_del
    if L == 0:
        n_ins += n_sub + n_del
        n_sub = n_del = 0
    if n_sub + n_del > L:                       # more site edits than letters
        over = n_sub + n_del - L
        take = min(over, n_del)
        n_del -= take
        n_sub -= over - take
        n_ins += over
    out = base.copy()
    keep = np.ones(L, dtype=bool)
    if n_sub + n_del:
        sites = rng.choice(L, size=n_sub + n_del, replace=False)
        sub_sites, del_sites = sites[:n_sub], sites[n_sub:]
        if n_sub:
            new = _draw_letters(rng, letters, probs, n_sub)
            same = new == out[sub_sites]
            while same.any():
                new[same] = _draw_letters(rng, letters, probs, int(same.sum()))
                same = new == out[sub_sites]
            out[sub_sites] = new
        keep[del_sites] = False
    if n_ins:
        gaps = rng.integers(0, L + 1, size=n_ins)
        ins = _draw_letters(rng, letters, probs, n_ins)
        # np.insert places new letters before the original letter at each gap
        out = np.insert(out, gaps, ins)
        keep = np.insert(keep, gaps, True)
    return out[keep]


def _assemble(rng, pieces, labels, desc, shuffle=True) -> Collection:
    n = len(pieces)
    order = rng.permutation(n) if shuffle else np.arange(n)
    pieces = [pieces[i] for i in order]
    labels = np.asarray(labels, dtype=np.int64)[order]
    lens = np.array([p.shape[0] for p in pieces], dtype=np.uint64)
    offsets = np.zeros(n + 1, dtype=np.uint64)
    np.cumsum(lens, out=offsets[1:])
    chars = np.concatenate(pieces).astype(np.uint8) if n else np.zeros(0, np.uint8)
    return Collection(chars, offsets, labels, desc)


def clusters(seed: int, n_bases: int, copies, base_len, edits, letters=DNA,
             probs=None, include_bases=False, desc="") -> Collection:
    """Generic cluster generator.

    ``copies(rng, b)``  -> number of copies of base ``b``
    ``base_len(rng)``   -> length of a base string
    ``edits(rng, L)``   -> number of edits for one copy of a base of length L
    """
    rng = np.random.default_rng(np.random.SeedSequence([seed, 0xDA7A]))
    let = np.frombuffer(letters, dtype=np.uint8)
    pieces, labels = [], []
    for b in range(n_bases):
        L = int(base_len(rng))
        base = _draw_letters(rng, let, probs, L)
        if include_bases:
            pieces.append(base)
            labels.append(b)
        for _ in range(int(copies(rng, b))):
            pieces.append(mutate(rng, base, int(edits(rng, L)), let, probs))
            labels.append(b)
    return _assemble(rng, pieces, labels, desc)


def random_strings(seed: int, n: int, min_len: int, max_len: int,
                   letters=DNA, probs=None) -> Collection:
    rng = np.random.default_rng(np.random.SeedSequence([seed, 0x5EED]))
    let = np.frombuffer(letters, dtype=np.uint8)
    pieces = [_draw_letters(rng, let, probs, int(rng.integers(min_len, max_len + 1)))
              for _ in range(n)]
    return _assemble(rng, pieces, [-1] * n, f"random n={n}", shuffle=False)


def zipf_probs(k: int, s: float) -> np.ndarray:
    p = np.arange(1, k + 1, dtype=np.float64) ** (-s)
    return p / p.sum()


# ---------------------------------------------------------------------------
# The five workload shapes.  Each returns (Collection, params dict).
# ---------------------------------------------------------------------------

def tiny_dna(seed: int = 0, n_bases: int = 200, copies: int = 10):
    """2,000 DNA strings: 200 random bases of length U{900..1100}, ten copies
    each with Poisson(30) edits.  K=50, r=3, z=7, m=24."""
    col = clusters(seed, n_bases, lambda rng, b: copies,
                   lambda rng: rng.integers(900, 1101),
                   lambda rng, L: rng.poisson(30),
                   desc=f"tiny DNA n={n_bases * copies}")
    return col, dict(K=50, r=3, z=7, m=24)


def medium_dna(seed: int = 0, n_bases: int = 2000, copies: int = 10, K: int = 500):
    """20,000 DNA strings: 2,000 bases of length U{4500..5500}, ten copies
    each with Poisson(0.04 len) edits.  K in {250, 500}, r=3, z=7, m=48."""
    col = clusters(seed, n_bases, lambda rng, b: copies,
                   lambda rng: rng.integers(4500, 5501),
                   lambda rng, L: rng.poisson(0.04 * L),
                   desc=f"medium DNA n={n_bases * copies}")
    return col, dict(K=K, r=3, z=7, m=48)


def uneven_dna(seed: int = 0, n_total: int = 80000):
    """80,000 DNA strings, base lengths log-uniform 500..20,000, cluster sizes
    geometric(p=0.3) resampled above 20, per-copy edit rate U(0, 0.08)."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 0xC0FE]))
    let = np.frombuffer(DNA, dtype=np.uint8)
    pieces, labels = [], []
    b = 0
    while len(pieces) < n_total:
        c = int(rng.geometric(0.3))
        while c > 20:
            c = int(rng.geometric(0.3))
        L = int(round(np.exp(rng.uniform(np.log(500), np.log(20000)))))
        base = _draw_letters(rng, let, None, L)
        for _ in range(min(c, n_total - len(pieces))):
            u = rng.uniform(0.0, 0.08)
            pieces.append(mutate(rng, base, int(rng.poisson(u * L)), let))
            labels.append(b)
        b += 1
    return _assemble(rng, pieces, labels, f"uneven DNA n={n_total}"), dict(K=400, r=3, z=7, m=24)


def protein_like(seed: int = 0, n_total: int = 400000):
    """400,000 strings over 25 letters with Zipf(1.1) frequencies; lengths
    lognormal(median 400, sigma 0.8) clipped to 50..4000; cluster sizes with
    mean 4 (geometric p=0.25); per-copy edit rate U(0.02, 0.15)."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 0xB10]))
    let = np.frombuffer(PROTEIN25, dtype=np.uint8)
    probs = zipf_probs(25, 1.1)
    pieces, labels = [], []
    b = 0
    while len(pieces) < n_total:
        c = int(rng.geometric(0.25))
        L = int(np.clip(round(np.exp(rng.normal(np.log(400), 0.8))), 50, 4000))
        base = _draw_letters(rng, let, probs, L)
        for _ in range(min(c, n_total - len(pieces))):
            u = rng.uniform(0.02, 0.15)
            pieces.append(mutate(rng, base, int(rng.poisson(u * L)), let, probs))
            labels.append(b)
        b += 1
    return (_assemble(rng, pieces, labels, f"protein-like n={n_total}"),
            dict(K=100, r=5, z=10, m=32))


def serving_index(seed: int = 0, n_bases: int = 32000, copies: int = 10):
    """Serving index: bases U{4500..5500}, ten copies with Poisson(0.05 len) edits."""
    col = clusters(seed, n_bases, lambda rng, b: copies,
                   lambda rng: rng.integers(4500, 5501),
                   lambda rng, L: rng.poisson(0.05 * L),
                   desc=f"serving index n={n_bases * copies}")
    return col, dict(r=3, z=7)


def serving_queries(index: Collection, seed: int = 0, n_queries: int = 10000,
                    member_frac: float = 0.7):
    """Queries: 70% re-mutated index members (Poisson(0.05 len) edits), 30%
    fresh random DNA of length U{1000..10000}.  Per-query K is a fraction
    drawn from {2%, 5%, 10%} of the query length.  Returns (Collection, Kq,
    source index or -1)."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 0x9E7]))
    let = np.frombuffer(DNA, dtype=np.uint8)
    pieces, src = [], []
    for _ in range(n_queries):
        if rng.random() < member_frac:
            s = int(rng.integers(0, index.n))
            base = index.chars[int(index.offsets[s]):int(index.offsets[s + 1])]
            pieces.append(mutate(rng, base, int(rng.poisson(0.05 * base.shape[0])), let))
            src.append(s)
        else:
            pieces.append(_draw_letters(rng, let, None, int(rng.integers(1000, 10001))))
            src.append(-1)
    col = _assemble(rng, pieces, src, f"queries n={n_queries}", shuffle=False)
    frac = np.array([0.02, 0.05, 0.10])[rng.integers(0, 3, size=n_queries)]
    Kq = np.floor(frac * col.lengths()).astype(np.uint32)
    return col, Kq, np.asarray(src, dtype=np.int64)


def shifted_reads(seed: int = 0, n_bases: int = 5000, copies: int = 10, base_len=(4500, 5500),
                  shift: int = 60, edit_rate: float = 0.003, letters=DNA):
    """Reads with shifts (the case EmbedJoin+ is built for): every cluster is
    `copies` reads of one random genome segment; a read starts at a uniform
    offset in [0, shift] of the segment (so two reads of a cluster differ by
    leading insertions of up to `shift` letters, and as many at the end),
    has the base length, and carries Poisson(edit_rate * len) edits.
    Default: 50,000 DNA reads of length 4,500..5,500."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 0x5F1F7]))
    let = np.frombuffer(letters, dtype=np.uint8)
    pieces, labels = [], []
    for b in range(n_bases):
        L = int(rng.integers(base_len[0], base_len[1] + 1))
        genome = _draw_letters(rng, let, None, L + shift)
        for _ in range(copies):
            s0 = int(rng.integers(0, shift + 1))
            read = genome[s0:s0 + L]
            pieces.append(mutate(rng, read, int(rng.poisson(edit_rate * L)), let))
            labels.append(b)
    return (_assemble(rng, pieces, labels, f"shifted reads n={n_bases * copies}"),
            dict(K=100, delta=50, T=2))


def planted_pairs(col: Collection) -> np.ndarray:
    """All pairs (i < j) that share a cluster label (label >= 0)."""
    lab = col.labels
    order = np.argsort(lab, kind="stable")
    out = []
    sl = lab[order]
    start = 0
    while start < len(order):
        end = start
        while end < len(order) and sl[end] == sl[start]:
            end += 1
        if sl[start] >= 0 and end - start > 1:
            ids = np.sort(order[start:end])
            a, b = np.triu_indices(len(ids), 1)
            out.append(np.stack([ids[a], ids[b]], 1))
        start = end
    if not out:
        return np.zeros((0, 2), dtype=np.int64)
    return np.concatenate(out).astype(np.int64)
