"""GPU parity on generated inputs (hypothesis, derandomized so that every run
draws the same examples): small sets of near-copies over DNA or a 20-letter
alphabet, empty strings included, joined and verified through the C ABI and
compared with the oracle bit for bit.  The fixed cases in test_gpu_parity.py
cover sizes and layouts; these cover shapes nobody wrote down."""
import sys
import types

import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

from tests._gpu_util import pairs_to_codes, to_device

pytestmark = pytest.mark.gpu

cases = settings(max_examples=100, deadline=None, derandomize=True,
                 suppress_health_check=[HealthCheck.too_slow])


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ej():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1702_00093_amd as ej
    ej.lib()  # raises if the library is not built
    return ej


@pytest.fixture(scope="module")
def ctx(ej):
    return ej.Context(0)


@st.composite
def families(draw, max_len=60):
    """Random base strings with copies carrying a few edits, plus empty
    strings now and then."""
    letters = draw(st.sampled_from(["ACGT", "ACDEFGHIKLMNPQRSTVWY"]))
    bases = draw(st.lists(st.text(alphabet=letters, min_size=1, max_size=max_len), min_size=1,
                          max_size=5))
    out = []
    for b in bases:
        for _ in range(draw(st.integers(1, 4))):
            s = list(b)
            for _ in range(draw(st.integers(0, 4))):
                i = draw(st.integers(0, max(0, len(s) - 1)))
                op = draw(st.sampled_from("isd"))
                c = draw(st.sampled_from(letters))
                if op == "i":
                    s.insert(i, c)
                elif op == "s" and s:
                    s[i] = c
                elif s:
                    del s[i]
            out.append("".join(s).encode())
    out += [b""] * draw(st.integers(0, 2))
    order = draw(st.permutations(range(len(out))))
    return [out[i] for i in order]


def _set(strings):
    chars = np.frombuffer(b"".join(strings), dtype=np.uint8).copy()
    off = np.zeros(len(strings) + 1, dtype=np.uint64)
    off[1:] = np.cumsum([len(s) for s in strings])
    return types.SimpleNamespace(chars=chars, offsets=off)


@cases
@given(families(), st.integers(0, 12), st.integers(1, 6), st.integers(1, 6), st.integers(1, 6),
       st.integers(0, 2**31))
def test_join_equals_the_oracle(ej, ctx, oracle_lib, strings, K, r, z, m, seed):
    col = _set(strings)
    _say(f"join n={len(strings)} K={K} r={r} z={z} m={m} seed={seed}")
    ref = oracle_lib.join(col.chars, col.offsets, K, r, z, m, seed=seed)
    res = ctx.join(col.chars, col.offsets, K, r, z, m, seed=seed)
    assert pairs_to_codes(res.pairs).tolist() == ref.out.tolist()
    assert res.dist.tolist() == ref.out_dist.astype(np.int32).tolist()
    assert res.n_candidates == len(ref.cand)


@cases
@given(families(max_len=300), st.integers(0, 400), st.randoms(use_true_random=False))
def test_verify_equals_the_oracle_in_every_form(ej, ctx, oracle_lib, strings, K, rnd):
    import torch
    col = _set(strings)
    n = len(strings)
    pairs = [(rnd.randrange(n), rnd.randrange(n)) for _ in range(rnd.randrange(1, 40))]
    codes = np.array([(a << 32) | b for a, b in pairs], dtype=np.uint64)
    want = oracle_lib.verify_pairs(col.chars, col.offsets, codes, K).tolist()
    chars, offs = to_device(col)
    d_codes = torch.from_numpy(codes.astype(np.int64)).cuda()
    old = ctx.tune_get("verify_mode")
    try:
        for mode in (0, 1, 2, 3):
            ctx.tune_set("verify_mode", mode)
            _say(f"verify n={n} pairs={len(pairs)} K={K} mode={mode}")
            got = ctx.verify(chars, offs, d_codes, K)
            assert got.cpu().numpy().astype(np.uint32).tolist() == want
    finally:
        ctx.tune_set("verify_mode", old)


def _assert_same_join(res, ref, shape=True):
    """Output, distances, candidate and raw counts; L and the alphabet size
    too, except for the grouped join (each group takes its own)."""
    assert pairs_to_codes(res.pairs).tolist() == ref.out.tolist()
    assert res.dist.tolist() == ref.out_dist.astype(np.int32).tolist()
    assert res.n_candidates == len(ref.cand)
    assert res.n_raw == ref.n_raw
    if shape:
        assert (res.L, res.sigma) == (ref.L, ref.sigma)


@cases
@given(families(), st.integers(1, 12), st.integers(0, 12), st.integers(0, 3), st.integers(1, 5),
       st.integers(1, 5), st.integers(1, 6), st.integers(0, 2**31))
def test_plus_equals_the_oracle(ej, ctx, oracle_lib, strings, K, delta, T, r, z, m, seed):
    col = _set(strings)
    delta = min(delta, K)
    # delta = 0 asks the library for the paper's step, floor(sqrt(ceil(average
    # length))) and at least 1; the oracle takes the step itself
    n = len(strings)
    avg = -(-int(col.offsets[-1]) // n)
    step = delta if delta else max(1, int(np.floor(np.sqrt(avg))))
    _say(f"plus n={n} K={K} delta={delta} (step {step}) T={T} r={r} z={z} m={m} seed={seed}")
    ref = oracle_lib.join_plus(col.chars, col.offsets, K, r, z, m, delta=step, T=T, seed=seed)
    res = ctx.join_plus(col.chars, col.offsets, K, r, z, m, delta=delta, T=T, seed=seed)
    _assert_same_join(res, ref)


@cases
@given(families(), st.integers(1, 12), st.integers(1, 5), st.integers(1, 5), st.integers(1, 6),
       st.integers(0, 2**31))
def test_grouped_equals_the_oracle(ej, ctx, oracle_lib, strings, K, r, z, m, seed):
    col = _set(strings)
    _say(f"grouped n={len(strings)} K={K} r={r} z={z} m={m} seed={seed}")
    ref = oracle_lib.join_grouped(col.chars, col.offsets, K, r, z, m, seed=seed)
    res = ctx.join_grouped(col.chars, col.offsets, K, r, z, m, seed=seed)
    _assert_same_join(res, ref, shape=False)


@cases
@given(families(), st.integers(0, 12), st.integers(1, 5), st.integers(1, 5), st.integers(1, 6),
       st.integers(0, 70), st.integers(0, 2**31))
def test_short_pass_equals_the_oracle(ej, ctx, oracle_lib, strings, K, r, z, m, S, seed):
    col = _set(strings)
    _say(f"short pass n={len(strings)} K={K} S={S} r={r} z={z} m={m} seed={seed}")
    ref = oracle_lib.join(col.chars, col.offsets, K, r, z, m, seed=seed, exact_len=S)
    res = ctx.join(col.chars, col.offsets, K, r, z, m, seed=seed, exact_len=S)
    assert pairs_to_codes(res.pairs).tolist() == ref.out.tolist()
    assert res.dist.tolist() == ref.out_dist.astype(np.int32).tolist()


@cases
@given(families(), st.integers(1, 4), st.integers(1, 4), st.integers(1, 5),
       st.integers(8, 64), st.integers(0, 2**31), st.randoms(use_true_random=False))
def test_queries_equal_the_oracle(ej, ctx, oracle_lib, strings, r, z, m, L, seed, rnd):
    col = _set(strings)
    letters = sorted(set(b"".join(strings))) or [ord("A")]
    queries = []
    for _ in range(rnd.randrange(1, 12)):
        s = bytearray(strings[rnd.randrange(len(strings))])
        for _ in range(rnd.randrange(0, 4)):
            i = rnd.randrange(len(s) + 1)
            c = letters[rnd.randrange(len(letters))]
            if rnd.random() < 0.5 or not s:
                s.insert(i, c)
            else:
                s[min(i, len(s) - 1)] = c
        queries.append(bytes(s))
    q = _set(queries)
    Kq = np.array([rnd.randrange(0, 13) for _ in queries], dtype=np.uint32)
    _say(f"queries n={len(strings)} nq={len(queries)} r={r} z={z} m={m} L={L} seed={seed}")
    ref_off, ref_ids, ref_dist = oracle_lib.query(col.chars, col.offsets, q.chars, q.offsets,
                                                  Kq, r, z, m, seed=seed, L=L)
    ix = ej.Index(ctx, col.chars, col.offsets, r, z, m, seed=seed, L=L)
    try:
        res = ix.query(q.chars, q.offsets, Kq)
        assert res.offsets.astype(np.uint64).tolist() == ref_off.tolist()
        assert res.ids.astype(np.uint32).tolist() == ref_ids.tolist()
        assert res.dist.astype(np.int64).tolist() == ref_dist.astype(np.int64).tolist()
    finally:
        ix.close()


@settings(max_examples=40, deadline=None, derandomize=True,
          suppress_health_check=[HealthCheck.too_slow])
@given(st.integers(0, 2**31), st.integers(5, 60), st.integers(1, 5), st.integers(40, 400),
       st.integers(0, 800), st.floats(0.0, 0.1), st.integers(0, 150), st.integers(1, 8),
       st.integers(1, 8), st.integers(1, 10), st.sampled_from([0, 32, 64, 128]))
def test_larger_joins_equal_the_oracle(ej, ctx, oracle_lib, seed, n_bases, copies, lo, span,
                                       rate, K, r, z, m, L):
    """Sets of up to 300 strings of up to 1,200 letters: many tiles, ragged
    tails, bands of 1 to 5 words, truncated and untruncated walks."""
    import synthdata as sd
    col = sd.clusters(seed, n_bases, lambda rr, b: rr.integers(1, copies + 1),
                      lambda rr: rr.integers(lo, lo + span + 1),
                      lambda rr, LL: rr.poisson(rate * LL))
    _say(f"larger join n={col.n} K={K} r={r} z={z} m={m} L={L} seed={seed}")
    ref = oracle_lib.join(col.chars, col.offsets, K, r, z, m, seed=seed, L=L)
    res = ctx.join(col.chars, col.offsets, K, r, z, m, seed=seed, L=L)
    assert pairs_to_codes(res.pairs).tolist() == ref.out.tolist()
    assert res.dist.tolist() == ref.out_dist.astype(np.int32).tolist()
    assert res.n_candidates == len(ref.cand)


_graph_states = []


@settings(max_examples=30, deadline=None, derandomize=True,
          suppress_health_check=[HealthCheck.too_slow])
@given(families(), st.integers(0, 12), st.integers(1, 5), st.integers(1, 5), st.integers(1, 6),
       st.integers(0, 2**31))
def test_graph_joins_equal_the_oracle(ej, ctx, oracle_lib, strings, K, r, z, m, seed):
    """Device-resident input with EJ_FLAG_GRAPH: the host-sized join, the
    device-sized one and the captured graph's replay all give the oracle's
    result."""
    col = _set(strings)
    chars, offs = to_device(col)
    _say(f"graph join n={len(strings)} K={K} r={r} z={z} m={m} seed={seed}")
    ref = oracle_lib.join(col.chars, col.offsets, K, r, z, m, seed=seed)
    for _ in range(3):
        res = ctx.join(chars, offs, K, r, z, m, seed=seed, flags=ej.FLAG_GRAPH)
        assert pairs_to_codes(res.pairs).tolist() == ref.out.tolist()
        assert res.dist.tolist() == ref.out_dist.astype(np.int32).tolist()
        assert res.n_candidates == len(ref.cand)
        _graph_states.append(res.graph)


def test_graph_joins_were_replayed():
    """The generated graph joins above reached the replayed graph."""
    if not _graph_states:
        pytest.skip("the generated graph joins did not run")
    assert 2 in _graph_states
