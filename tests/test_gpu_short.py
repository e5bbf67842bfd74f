"""GPU parity of the exhaustive pass over short strings (ej_params.exact_len):
every pair of strings both no longer than S whose lengths differ by at most K
joins the candidates of EmbedJoin, EmbedJoin+ or the grouping join; through
the C ABI against the oracle's ejo_exact_short, bit for bit (candidate count,
raw count, output pairs and distances)."""
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


def _mixed(seed, n_short=300, short=(0, 160), n_bases=40, long=(300, 900)):
    """Random short strings (some empty, the shortest within K of each other
    by chance) beside clusters of longer mutated copies."""
    rng = np.random.default_rng(seed)
    DNA = np.frombuffer(b"ACGT", np.uint8)
    strings = [bytes(DNA[rng.integers(0, 4, size=int(rng.integers(*short)))])
               for _ in range(n_short)]
    strings += [b"", b""]
    col = sd.clusters(seed, n_bases, lambda rr, b: rr.integers(2, 5),
                      lambda rr: rr.integers(*long), lambda rr, LL: rr.poisson(0.03 * LL))
    strings += [col.string(i) for i in range(col.n)]
    order = rng.permutation(len(strings))
    return sd.from_strings([strings[i] for i in order])


CASES = [
    # seed, K, r, z, m, S
    (0, 60, 3, 6, 16, 160),     # every short string in the pass
    (1, 100, 2, 5, 12, 90),     # a cut inside the short strings
    (2, 0, 2, 4, 8, 40),        # K = 0: equal lengths only
    (3, 40, 2, 4, 10, 100000),  # S above every length: the exact join
]


@pytest.mark.parametrize("case", CASES, ids=[f"c{c[0]}" for c in CASES])
def test_join_with_short_pass_matches_oracle(ej, ctx, oracle_lib, case):
    seed, K, r, z, m, S = case
    col = _mixed(seed, n_short=120 if S >= 100000 else 300)
    ref = oracle_lib.join(col.chars, col.offsets, K, r, z, m, seed=seed, exact_len=S)
    _say(f"join+short n={col.n} K={K} S={S} cand={len(ref.cand)} out={len(ref.out)}")
    _assert_equal(ctx.join(col.chars, col.offsets, K, r, z, m, seed=seed, exact_len=S), ref)
    chars, offs = to_device(col)
    _assert_equal(ctx.join(chars, offs, K, r, z, m, seed=seed, exact_len=S,
                           flags=ej.FLAG_GRAPH), ref)
    if S >= 100000:
        truth, tdist = oracle_lib.brute_join(col.chars, col.offsets, K)
        assert ref.out.tolist() == truth.tolist()


def test_short_pass_many_tiles(ej, ctx, oracle_lib):
    """About 200,000 short pairs: the row scan and the emit kernel span many
    workgroups, rows of very different sizes, the union sort several digits."""
    col = _mixed(7, n_short=650, short=(20, 140), n_bases=20)
    K, S = 70, 140
    ref = oracle_lib.join(col.chars, col.offsets, K, 2, 4, 12, seed=7, exact_len=S)
    _say(f"join+short many tiles n={col.n} cand={len(ref.cand)} out={len(ref.out)}")
    assert len(ref.cand) > 150000
    chars, offs = to_device(col)
    _assert_equal(ctx.join(chars, offs, K, 2, 4, 12, seed=7, exact_len=S), ref)


def test_plus_and_grouped_with_short_pass(ej, ctx, oracle_lib):
    col = _mixed(8, n_short=200)
    K, S = 80, 120
    ref = oracle_lib.join_plus(col.chars, col.offsets, K, 2, 4, 10, delta=30, seed=8,
                               exact_len=S)
    _say(f"plus+short n={col.n} cand={len(ref.cand)}")
    _assert_equal(ctx.join_plus(col.chars, col.offsets, K, 2, 4, 10, delta=30, seed=8,
                                exact_len=S), ref)
    ref = oracle_lib.join_grouped(col.chars, col.offsets, K, 2, 4, 10, seed=8, exact_len=S)
    _say(f"grouped+short n={col.n} cand={len(ref.cand)}")
    _assert_equal(ctx.join_grouped(col.chars, col.offsets, K, 2, 4, 10, seed=8, exact_len=S),
                  ref)


def test_short_pass_degenerate_sets(ej, ctx, oracle_lib):
    """No string short enough, exactly one, only empty strings."""
    for strings, K, S in (([b"ACGTACGT", b"ACGTACGA", b"TTTTTTTTT"], 3, 4),
                          ([b"AC", b"ACGTACGTAA", b"ACGTACGTAC"], 3, 2),
                          ([b"", b"", b""], 0, 1)):
        col = sd.from_strings(strings)
        ref = oracle_lib.join(col.chars, col.offsets, K, 1, 2, 2, seed=1, exact_len=S)
        _assert_equal(ctx.join(col.chars, col.offsets, K, 1, 2, 2, seed=1, exact_len=S), ref)
