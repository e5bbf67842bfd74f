"""Property tests of the CPU oracle (hypothesis): facts of the mathematics that
hold for every input, checked on many random small inputs.  They complement
the fixed pins in test_oracle_pins.py: edit distance is a metric that moves by
at most one per edit and ignores a common prefix or suffix; the banded
computation equals the full one within the threshold (Ukkonen's band); two
CGK walks on strings that share a prefix, driven by the same random bits,
emit the same symbols while both are inside it (Algorithm 1: the walk's
index advances by at most one per step), and emit only padding once past
the end; the sampled key depends on the sampled positions only; the join's
(and EmbedJoin+'s) output is exactly its candidates within K, with their
exact distances; a serving query returns true matches in index order and
always finds an identical member."""
import numpy as np
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

CODE = {ord("A"): 0, ord("C"): 1, ord("G"): 2, ord("T"): 3}

dna = st.text(alphabet="ACGT", max_size=20).map(str.encode)
small = settings(max_examples=60, deadline=None,
                 suppress_health_check=[HealthCheck.too_slow])


def _codes(b):
    return np.array([CODE[c] for c in b], dtype=np.uint8)


def _set(strings):
    chars = b"".join(strings)
    off = np.zeros(len(strings) + 1, dtype=np.uint64)
    off[1:] = np.cumsum([len(s) for s in strings])
    return chars, off


# ------------------------------------------------------------ edit distance --

@small
@given(dna, dna, dna)
def test_edit_distance_is_a_metric(oracle_lib, x, y, z):
    ed = oracle_lib.ed_full
    assert ed(x, x) == 0
    assert (ed(x, y) == 0) == (x == y)
    assert ed(x, y) == ed(y, x)
    assert ed(x, z) <= ed(x, y) + ed(y, z)
    assert abs(len(x) - len(y)) <= ed(x, y) <= max(len(x), len(y))


@small
@given(dna, dna, st.integers(0, 40), st.sampled_from("ACGT"), st.sampled_from(["ins", "del", "sub"]))
def test_one_edit_moves_the_distance_by_at_most_one(oracle_lib, x, w, at, c, kind):
    i = at % (len(x) + 1)
    if kind == "ins":
        y = x[:i] + c.encode() + x[i:]
    elif kind == "del" and x:
        i = min(i, len(x) - 1)
        y = x[:i] + x[i + 1:]
    elif x:
        i = min(i, len(x) - 1)
        y = x[:i] + c.encode() + x[i + 1:]
    else:
        y = x
    ed = oracle_lib.ed_full
    assert ed(x, y) <= 1
    assert abs(ed(x, w) - ed(y, w)) <= 1


@small
@given(dna, dna, dna, dna)
def test_common_prefix_and_suffix_do_not_count(oracle_lib, p, x, y, s):
    ed = oracle_lib.ed_full
    assert ed(p + x + s, p + y + s) == ed(x, y)


@small
@given(dna, dna, st.integers(0, 30))
def test_banded_distance_equals_the_full_one_within_the_threshold(oracle_lib, x, y, K):
    assert oracle_lib.ed_banded(x, y, K) == min(oracle_lib.ed_full(x, y), K + 1)


@small
@given(st.lists(dna, min_size=2, max_size=8), st.integers(0, 25), st.randoms(use_true_random=False))
def test_verified_pairs_are_the_threshold_distance(oracle_lib, strings, K, rnd):
    chars, off = _set(strings)
    n = len(strings)
    pairs = [(rnd.randrange(n), rnd.randrange(n)) for _ in range(10)]
    codes = np.array([(a << 32) | b for a, b in pairs], dtype=np.uint64)
    got = oracle_lib.verify_pairs(chars, off, codes, K)
    want = [min(oracle_lib.ed_full(strings[a], strings[b]), K + 1) for a, b in pairs]
    assert got.tolist() == want


# ---------------------------------------------------------------- CGK walk --

@small
@given(dna, dna, dna, st.integers(1, 70), st.integers(0, 2**32 - 1))
def test_walks_agree_inside_a_common_prefix(oracle_lib, p, x, y, L, seed):
    rng = np.random.default_rng(seed)
    bits = rng.integers(0, 2, size=L * 4, dtype=np.uint8)
    ex = oracle_lib.cgk_embed(_codes(p + x), bits, 4, L)
    ey = oracle_lib.cgk_embed(_codes(p + y), bits, 4, L)
    k = min(len(p), L)
    assert ex[:k].tolist() == ey[:k].tolist()
    if x == y:
        assert ex.tolist() == ey.tolist()


def _runs(seq):
    out = []
    for c in seq:
        if not out or out[-1] != c:
            out.append(c)
    return out


@small
@given(dna, st.integers(1, 70), st.integers(0, 2**32 - 1))
def test_walk_reads_the_string_left_to_right_then_pads(oracle_lib, x, L, seed):
    """The walk's index starts at 0 and advances by 0 or 1 per step, so the
    symbols it emits are x[0] (one or more times), x[1], ... in order: their
    runs are the runs of a prefix of x, of all of x once the walk has passed
    the end, after which it emits only the padding symbol."""
    rng = np.random.default_rng(seed)
    bits = rng.integers(0, 2, size=L * 4, dtype=np.uint8)
    e = oracle_lib.cgk_embed(_codes(x), bits, 4, L).tolist()
    xs = _codes(x).tolist()
    assert len(e) == L and all(0 <= s <= 4 for s in e)
    if not xs:
        assert all(s == 4 for s in e)
        return
    body = e[:e.index(4)] if 4 in e else e
    assert all(s == 4 for s in e[len(body):])
    if 4 in e:
        assert _runs(body) == _runs(xs)
    else:
        assert any(_runs(body) == _runs(xs[:k]) for k in range(1, len(xs) + 1))


@small
@given(dna, st.integers(1, 6), st.integers(0, 2**32 - 1), st.integers(0, 63))
def test_key_depends_on_the_sampled_positions_only(oracle_lib, x, m, seed, change):
    L = 64
    Rb, pos, v = oracle_lib.draw(seed, 1, 1, m, L, 4)
    t = oracle_lib.cgk_embed(_codes(x), Rb[0], 4, L)
    k0 = oracle_lib.key(t, pos[0, 0], v[0, 0])
    assert 0 <= k0 < (1 << 61) - 1
    t2 = t.copy()
    t2[change] = (t2[change] + 1) % 5
    k1 = oracle_lib.key(t2, pos[0, 0], v[0, 0])
    if change not in pos[0, 0].tolist():
        assert k1 == k0


# --------------------------------------------------------------- the join --

@st.composite
def families(draw):
    """A few random base strings, each with a few copies carrying 0-3 edits:
    sets with pairs inside and outside small thresholds."""
    bases = draw(st.lists(st.text(alphabet="ACGT", min_size=4, max_size=24), min_size=1,
                          max_size=4))
    out = []
    for b in bases:
        for _ in range(draw(st.integers(1, 3))):
            s = list(b)
            for _ in range(draw(st.integers(0, 3))):
                i = draw(st.integers(0, max(0, len(s) - 1)))
                op = draw(st.sampled_from("isd"))
                c = draw(st.sampled_from("ACGT"))
                if op == "i":
                    s.insert(i, c)
                elif op == "s" and s:
                    s[i] = c
                elif s:
                    del s[i]
            out.append("".join(s).encode())
    return out


@settings(max_examples=40, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(families(), st.integers(0, 6), st.integers(1, 4), st.integers(1, 4), st.integers(1, 5),
       st.integers(0, 2**31))
def test_join_outputs_its_candidates_within_K_exactly(oracle_lib, strings, K, r, z, m, seed):
    chars, off = _set(strings)
    res = oracle_lib.join(chars, off, K, r, z, m, seed=seed)
    truth_codes, truth_d = oracle_lib.brute_join(chars, off, K, full=True)
    truth = dict(zip(truth_codes.tolist(), truth_d.tolist()))
    cand = set(res.cand.tolist())
    out = dict(zip(res.out.tolist(), res.out_dist.tolist()))
    assert set(out) == cand & set(truth)
    assert all(out[c] == truth[c] for c in out)
    for c in cand:
        a, b = c >> 32, c & 0xFFFFFFFF
        assert a < b and abs(len(strings[a]) - len(strings[b])) <= K


@settings(max_examples=30, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(families(), st.integers(1, 6), st.integers(0, 2**31))
def test_grouped_join_output_is_exact(oracle_lib, strings, K, seed):
    chars, off = _set(strings)
    res = oracle_lib.join_grouped(chars, off, K, 3, 3, 2, seed=seed)
    truth_codes, truth_d = oracle_lib.brute_join(chars, off, K, full=True)
    truth = dict(zip(truth_codes.tolist(), truth_d.tolist()))
    for c, d in zip(res.out.tolist(), res.out_dist.tolist()):
        assert truth.get(c) == d


@settings(max_examples=30, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(families(), st.integers(1, 6), st.integers(1, 6), st.integers(1, 3), st.integers(0, 2**31))
def test_plus_output_is_exact(oracle_lib, strings, K, delta, T, seed):
    chars, off = _set(strings)
    res = oracle_lib.join_plus(chars, off, K, 3, 3, 2, delta=min(delta, K), T=T, seed=seed)
    truth_codes, truth_d = oracle_lib.brute_join(chars, off, K, full=True)
    truth = dict(zip(truth_codes.tolist(), truth_d.tolist()))
    cand = set(res.cand.tolist())
    out = dict(zip(res.out.tolist(), res.out_dist.tolist()))
    assert set(out) == cand & set(truth)
    assert all(out[c] == truth[c] for c in out)


@settings(max_examples=30, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(families(), st.lists(st.integers(0, 8), min_size=1, max_size=6), st.integers(0, 2**31))
def test_query_results_are_true_matches(oracle_lib, strings, kq, seed):
    """Each query's results are index strings within its threshold, with
    their exact distances, in increasing index order; a query equal to an
    index member finds that member at distance 0."""
    chars, off = _set(strings)
    queries = [strings[i % len(strings)] for i in range(len(kq))]
    qc, qo = _set(queries)
    Kq = np.array(kq, dtype=np.uint32)
    ro, ids, dist = oracle_lib.query(chars, off, qc, qo, Kq, 4, 4, 2, seed=seed, L=32)
    for q in range(len(queries)):
        got = list(zip(ids[ro[q]:ro[q + 1]].tolist(), dist[ro[q]:ro[q + 1]].tolist()))
        assert [i for i, _ in got] == sorted(i for i, _ in got)
        for i, d in got:
            assert d == oracle_lib.ed_full(queries[q], strings[i]) <= Kq[q]
        assert (q % len(strings), 0) in got or any(
            strings[i] == queries[q] and d == 0 for i, d in got)
