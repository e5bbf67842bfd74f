"""GPU parity of EmbedJoin+ (Algorithms 4-5): suffix embeddings, tuple counts
against the threshold T, verification; called through the C ABI and compared
bit for bit with the oracle's EmbedJoin+ on the same seeded inputs."""
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
    assert res.n_candidates == len(ref.cand)
    assert res.n_raw == ref.n_raw
    assert (res.L, res.sigma) == (ref.L, ref.sigma)


def test_plus_one_suffix_threshold_one_is_the_join(ej, ctx, oracle_lib):
    col, _ = sd.shifted_reads(1, n_bases=40, copies=5, base_len=(200, 500), shift=20,
                              edit_rate=0.02)
    K, r, z, m, L = 40, 3, 5, 6, 64
    _say("plus with one suffix and T=1")
    got = ctx.join_plus(col.chars, col.offsets, K, r, z, m, delta=40, T=1, seed=2, L=L)
    plain = ctx.join(col.chars, col.offsets, K, r, z, m, seed=2, L=L)
    assert got.pairs.tolist() == plain.pairs.tolist() and got.dist.tolist() == plain.dist.tolist()
    assert got.n_candidates == plain.n_candidates and got.n_raw == plain.n_raw
    _assert_equal(got, oracle_lib.join(col.chars, col.offsets, K, r, z, m, seed=2, L=L))


CASES = [
    # seed, bases, copies, len range, shift, K, delta, T, r, z, m, L
    (0, 40, 5, (200, 500), 30, 60, 20, 2, 3, 6, 8, 64),
    (1, 30, 6, (100, 300), 40, 50, 12, 3, 2, 8, 6, 48),
    (2, 50, 4, (50, 400), 25, 45, 15, 1, 3, 4, 7, 0),     # T=1: any suffix pair in one table
    (3, 25, 8, (20, 90), 10, 30, 7, 2, 2, 6, 4, 32),      # short strings: empty suffixes
    (4, 300, 5, (300, 700), 40, 80, 30, 2, 2, 4, 10, 64),  # 1,500 strings: many tiles
]


@pytest.mark.parametrize("case", CASES, ids=[f"c{c[0]}" for c in CASES])
def test_plus_matches_oracle(ej, ctx, oracle_lib, case):
    seed, nb, cp, lens, shift, K, delta, T, r, z, m, L = case
    col, _ = sd.shifted_reads(seed, n_bases=nb, copies=cp, base_len=lens, shift=shift,
                              edit_rate=0.02)
    ref = oracle_lib.join_plus(col.chars, col.offsets, K, r, z, m, delta=delta, T=T, seed=seed,
                               L=L)
    _say(f"plus case {seed}: n={col.n} K={K} delta={delta} T={T} cand={len(ref.cand)}")
    _assert_equal(ctx.join_plus(col.chars, col.offsets, K, r, z, m, delta=delta, T=T,
                                seed=seed, L=L), ref)
    chars, offs = to_device(col)
    _assert_equal(ctx.join_plus(chars, offs, K, r, z, m, delta=delta, T=T, seed=seed, L=L), ref)


def test_plus_default_delta_and_threshold(ej, ctx, oracle_lib):
    col, _ = sd.shifted_reads(7, n_bases=30, copies=4, base_len=(300, 600), shift=30,
                              edit_rate=0.02)
    K, r, z, m, L = 70, 2, 6, 8, 64
    avg = -(-int(col.offsets[-1]) // col.n)
    delta = int(np.floor(np.sqrt(avg)))
    assert delta * delta <= avg < (delta + 1) * (delta + 1)
    ref = oracle_lib.join_plus(col.chars, col.offsets, K, r, z, m, delta=delta, T=0, seed=3, L=L)
    _say(f"plus default delta={delta}")
    _assert_equal(ctx.join_plus(col.chars, col.offsets, K, r, z, m, delta=0, T=0, seed=3, L=L),
                  ref)


def test_plus_leading_shift_always_found(ej, ctx):
    rng = np.random.default_rng(9)
    DNA = np.frombuffer(b"ACGT", np.uint8)
    strings = []
    for _ in range(20):
        x = bytes(DNA[rng.integers(0, 4, size=300)])
        strings += [x, bytes(DNA[rng.integers(0, 4, size=15)]) + x]
    col = sd.from_strings(strings)
    res = ctx.join_plus(col.chars, col.offsets, 30, 2, 3, 8, delta=15, T=2, seed=11, L=128)
    got = set(map(tuple, res.pairs.tolist()))
    assert all((2 * i, 2 * i + 1) in got for i in range(20))


def test_plus_edge_cases(ej, ctx, oracle_lib):
    for strings, K, delta, T in [([b"ACGT"], 3, 1, 2), ([b"", b"", b"A"], 2, 1, 2),
                                 ([b"AC", b"CA", b"ACA", b""], 0, 1, 1),
                                 ([b"ACGTACGT", b"CGTACGTA", b"GT"], 6, 2, 1)]:
        col = sd.from_strings(strings)
        ref = oracle_lib.join_plus(col.chars, col.offsets, K, 2, 3, 2, delta=delta, T=T,
                                   seed=1, L=8)
        _say(f"plus edge {strings}")
        _assert_equal(ctx.join_plus(col.chars, col.offsets, K, 2, 3, 2, delta=delta, T=T,
                                    seed=1, L=8), ref)
