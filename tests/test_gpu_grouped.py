"""GPU parity of the grouping alternative to truncation (Section 4.1):
EmbedJoin on each length group ((g)K, (g+2)K] as a set of its own, the union
of candidates and outputs; through the C ABI against the oracle's grouped
join, bit for bit."""
import sys

import numpy as np
import pytest

import synthdata as sd
from tests._gpu_util import pairs_to_codes, to_device

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ej():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1702_00093_amd as ej
    ej.lib()
    return ej


@pytest.fixture(scope="module")
def ctx(ej):
    return ej.Context(0)


def _assert_equal(res, ref):
    assert pairs_to_codes(res.pairs).tolist() == ref.out.tolist()
    assert res.dist.tolist() == ref.out_dist.astype(np.int32).tolist()
    assert res.n_candidates == len(ref.cand) and res.n_raw == ref.n_raw


CASES = [
    # seed, n_total or bases, K, r, z, m, L, letters
    (0, "uneven", 400, 3, 7, 24, 0),
    (1, "uneven", 150, 2, 6, 8, 0),
    (2, "uneven", 300, 3, 5, 12, 256),   # a caller's truncation in every group
    (3, "boundary", 10, 1, 1, 4, 0),
    (4, "protein", 60, 3, 6, 6, 0),
    (5, "boundary", 0, 2, 2, 2, 0),      # K = 0: one group per length
]


def _collection(seed, kind):
    if kind == "uneven":
        col, _ = sd.uneven_dna(seed, n_total=1500)
        return col
    if kind == "protein":
        col, _ = sd.protein_like(seed, n_total=1200)
        return col
    rng = np.random.default_rng(seed)
    DNA = np.frombuffer(b"ACGT", np.uint8)
    strings = []
    for L in (0, 1, 9, 10, 11, 20, 21, 30, 31, 50, 0, 10, 20):
        s = bytes(DNA[rng.integers(0, 4, size=L)])
        strings += [s, s, bytes(sd.mutate(rng, np.frombuffer(s, np.uint8), 1, DNA))]
    return sd.from_strings(strings)


@pytest.mark.parametrize("case", CASES, ids=[f"c{c[0]}" for c in CASES])
def test_grouped_matches_oracle(ej, ctx, oracle_lib, case):
    seed, kind, K, r, z, m, L = case
    col = _collection(seed, kind)
    ref = oracle_lib.join_grouped(col.chars, col.offsets, K, r, z, m, seed=seed, L=L)
    _say(f"grouped {kind} n={col.n} K={K} cand={len(ref.cand)} out={len(ref.out)}")
    _assert_equal(ctx.join_grouped(col.chars, col.offsets, K, r, z, m, seed=seed, L=L), ref)
    chars, offs = to_device(col)
    _assert_equal(ctx.join_grouped(chars, offs, K, r, z, m, seed=seed, L=L), ref)
