"""Pins of the CPU oracle against facts outside itself: the paper's worked
examples, published RNG test vectors, the definition of edit distance checked
by exhaustive search, closed forms of the LSH collision probability, and
brute force on tiny inputs."""
import itertools
import json
import os
from collections import deque

import numpy as np
import pytest

import synthdata as sd

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _load(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


# ------------------------------------------------------------------ RNG --

def test_splitmix64_published_vector(oracle_lib):
    g = _load("splitmix64.json")
    got = oracle_lib.splitmix64(g["seed"], len(g["outputs"]))
    assert [int(x) for x in got] == [int(x) for x in g["outputs"]]


def test_counter_word_is_stream_draw(oracle_lib):
    # W(key, c) is the (c+1)-th draw of the sequential generator seeded with key
    for key in (0, 1, 1234567, 0xDEADBEEFCAFEBABE):
        seq = oracle_lib.splitmix64(key, 40)
        assert [oracle_lib.word(key, c) for c in range(40)] == [int(x) for x in seq]


def test_random_string_bits_balanced(oracle_lib):
    R, pos, v = oracle_lib.draw(7, 3, 4, 8, 4000, 4)
    frac = R.mean()
    # 48000 fair bits: 6 sigma is ~0.014
    assert abs(frac - 0.5) < 0.014
    assert (pos < 4000).all()
    assert (v < oracle_lib.P61).all()


def test_coordinates_uniform(oracle_lib):
    L = 64
    _, pos, _ = oracle_lib.draw(3, 4, 16, 64, L, 4)
    counts = np.bincount(pos.ravel(), minlength=L)
    exp = pos.size / L
    chi2 = ((counts - exp) ** 2 / exp).sum()
    # 63 degrees of freedom: 99.99th percentile is ~ 118
    assert chi2 < 118


class SpecRNG:
    """The randomness layout written out a second time, in plain Python
    integers, from its specification alone: W(key, c) is the (c+1)-th output of
    a SplitMix64 generator seeded with key; stream keys are W(seed, tag << 32 |
    idx) (tag 0: the random string of seed l, idx l; tag 1: coordinates of
    table (l, j), idx l z + j; tag 2: second-level vector of that table); bit b
    of R^l is bit b mod 64 of W(key_R, floor(b / 64)); coordinate k is
    floor(W(key_POS, k) L / 2^64); v_k = (W(key_V, k) >> 3) mod (2^61 - 1).
    The generator is stepped sequentially here (state += gamma, then the
    output mix), not through the oracle's counter form."""

    M64 = (1 << 64) - 1

    @classmethod
    def stream(cls, seed, count):
        out, s = [], seed
        for _ in range(count):
            s = (s + 0x9E3779B97F4A7C15) & cls.M64
            z = s
            z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & cls.M64
            z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & cls.M64
            out.append(z ^ (z >> 31))
        return out

    @classmethod
    def key(cls, seed, tag, idx):
        # word number (tag << 32 | idx) of the seed's stream: step the state
        # that many times at once (a Weyl sequence), then mix
        c = (tag << 32) | idx
        s = (seed + (c + 1) * 0x9E3779B97F4A7C15) & cls.M64
        z = ((s ^ (s >> 30)) * 0xBF58476D1CE4E5B9) & cls.M64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & cls.M64
        return z ^ (z >> 31)

    @classmethod
    def r_bits(cls, seed, l, nbits):
        words = cls.stream(cls.key(seed, 0, l), (nbits + 63) // 64)
        return [(words[b // 64] >> (b % 64)) & 1 for b in range(nbits)]

    @classmethod
    def coords(cls, seed, l, j, z, m, L):
        words = cls.stream(cls.key(seed, 1, l * z + j), m)
        return [(w * L) >> 64 for w in words]

    @classmethod
    def vvec(cls, seed, l, j, z, m):
        words = cls.stream(cls.key(seed, 2, l * z + j), m)
        return [(w >> 3) % ((1 << 61) - 1) for w in words]


def test_spec_rng_reproduces_published_vector():
    # the second implementation is itself pinned to the published outputs
    g = _load("splitmix64.json")
    assert SpecRNG.stream(g["seed"], len(g["outputs"])) == [int(x) for x in g["outputs"]]


@pytest.mark.parametrize("seed,r,z,m,L,sigma", [(0, 2, 3, 5, 40, 4), (0xC0FFEE, 3, 2, 7, 1000, 25),
                                               (1 << 63, 1, 4, 3, 7, 2)])
def test_randomness_layout_matches_its_specification(oracle_lib, seed, r, z, m, L, sigma):
    # catches a swapped stream tag, an MSB-first bit order, v = W mod P, a
    # floor-vs-high-product coordinate, or l*z+j vs j*r+l table numbering
    R, pos, v = oracle_lib.draw(seed, r, z, m, L, sigma)
    for l in range(r):
        assert R[l].tolist() == SpecRNG.r_bits(seed, l, L * sigma), f"R bits of seed {l}"
        for j in range(z):
            assert pos[l, j].tolist() == SpecRNG.coords(seed, l, j, z, m, L), f"pos ({l},{j})"
            assert [int(x) for x in v[l, j]] == SpecRNG.vvec(seed, l, j, z, m), f"v ({l},{j})"


def test_randomness_golden_values(oracle_lib):
    # a few values written out once from the specification by hand-checkable
    # integer arithmetic: the first R word of seed 0 and its low bits
    w0 = SpecRNG.stream(SpecRNG.key(0, 0, 0), 1)[0]
    R, _, _ = oracle_lib.draw(0, 1, 1, 1, 16, 4)
    assert R[0].tolist() == [(w0 >> b) & 1 for b in range(64)]


# ------------------------------------------------------------ truncation --

def _offsets(lengths):
    o = np.zeros(len(lengths) + 1, dtype=np.uint64)
    o[1:] = np.cumsum(lengths)
    return o


@pytest.mark.parametrize("lengths,L_req,expect", [
    ([3, 4], 0, 4),            # average 3.5: the ceiling, not the floor (3)
    ([1, 1, 2], 0, 2),         # average 4/3 -> 2
    ([5, 5], 0, 5),            # an exact average stays
    ([2, 5], 100, 15),         # a requested L above 3N is clamped to 3N = 15
    ([2, 5], 15, 15),          # 3N itself is allowed
    ([2, 5], 7, 7),            # a requested L below 3N is kept
    ([0, 0, 0], 0, 1),         # all empty: 3N = 0, raised to the floor of 1
    ([], 0, 1),                # no strings at all
    ([0, 0], 9, 1),            # a request on empty strings: clamped to 0, then 1
])
def test_effective_truncation(oracle_lib, lengths, L_req, expect):
    assert oracle_lib.effective_L(_offsets(lengths), L_req) == expect


def test_join_uses_effective_truncation(oracle_lib):
    col = sd.from_strings([b"ACG", b"ACGT"])
    assert oracle_lib.join(col.chars, col.offsets, 1, 1, 1, 1).L == 4
    assert oracle_lib.join(col.chars, col.offsets, 1, 1, 1, 1, L=50).L == 12


# ------------------------------------------------------------- alphabet --

def test_full_byte_alphabet_is_rejected(oracle_lib):
    # with all 256 byte values present no code is left for the padding symbol
    col = sd.from_strings([bytes(range(256)), b"AB"])
    with pytest.raises(ValueError):
        oracle_lib.join(col.chars, col.offsets, 2, 1, 1, 1)
    q = sd.from_strings([b"AB"])
    with pytest.raises(ValueError):
        oracle_lib.query(col.chars, col.offsets, q.chars, q.offsets, [1], 1, 1, 1)
    col255 = sd.from_strings([bytes(range(255)), b"AB"])
    assert oracle_lib.join(col255.chars, col255.offsets, 2, 1, 1, 1).sigma == 255


# -------------------------------------------------- running example ----

def _running_example_randomness(g):
    sig = g["alphabet"]
    L, r, z, m = g["L"], g["r"], g["z"], g["m"]
    R = np.zeros((r, L * len(sig)), dtype=np.uint8)
    for l, name in enumerate(["R1", "R2"]):
        for k, ch in enumerate(sig):
            for j, bit in enumerate(g["pi"][name][ch]):
                R[l, j * len(sig) + k] = bit
    coords = g["lsh_coordinates_1based"]
    pos = np.zeros((r, z, m), dtype=np.uint32)
    for l in range(r):
        for j in range(z):
            pos[l, j] = np.array(coords[f"f{j + 1}^{l + 1}"]) - 1
    return R, pos


def test_running_example_embeddings(oracle_lib):
    g = _load("running_example.json")
    R, _ = _running_example_randomness(g)
    sigma, lut = oracle_lib.alphabet(b"".join(s.encode() for s in g["strings"]))
    assert sigma == 4
    letters = np.array([ord(c) for c in g["alphabet"]])
    for i, s in enumerate(g["strings"]):
        codes = lut[np.frombuffer(s.encode(), dtype=np.uint8)].astype(np.uint8)
        for l in range(2):
            t = oracle_lib.cgk_embed(codes, R[l], sigma, g["L"])
            got = "".join(chr(letters[c]) for c in t)
            assert got == g["embeddings_prefix"][f"t{i + 1}^{l + 1}"], (i, l)


def test_running_example_join(oracle_lib):
    g = _load("running_example.json")
    R, pos = _running_example_randomness(g)
    col = sd.from_strings([s.encode() for s in g["strings"]])
    res = oracle_lib.join(col.chars, col.offsets, g["K"], g["r"], g["z"], g["m"],
                          seed=0, L=g["L"], explicit_R=R, explicit_pos=pos)
    letters = g["alphabet"]
    for i in range(4):
        sigs = ["".join(letters[c] for c in res.sig[i, l, j]) for l in range(2) for j in range(2)]
        assert sigs == g["signatures"][str(i + 1)], i
    assert (res.cand_pairs + 1).tolist() == g["candidates_1based"]
    assert (res.out_pairs + 1).tolist() == g["output_1based"]
    assert res.out_dist.tolist() == [2, 3]


# ---------------------------------------------------- intro example ----

def test_intro_example_brute_force(oracle_lib):
    g = _load("intro_example.json")
    col = sd.from_strings([s.encode() for s in g["strings"]])
    codes, d = oracle_lib.brute_join(col.chars, col.offsets, g["K"], full=True)
    S = g["strings"]
    got = sorted(tuple(sorted((S[int(c) >> 32], S[int(c) & 0xFFFFFFFF]))) for c in codes)
    assert got == sorted(tuple(sorted(p)) for p in g["output"])
    # threshold is inclusive: at K=3 four more pairs (distance exactly 3) join
    codes3, d3 = oracle_lib.brute_join(col.chars, col.offsets, 3, full=True)
    assert oracle_lib.brute_join(col.chars, col.offsets, 3)[0].tolist() == codes3.tolist()
    assert len(codes3) == 7 and sorted(d3.tolist()) == [2, 2, 2, 3, 3, 3, 3]


def test_intro_example_embedjoin_fixed_seed(oracle_lib):
    g = _load("intro_example.json")
    col = sd.from_strings([s.encode() for s in g["strings"]])
    res = oracle_lib.join(col.chars, col.offsets, g["K"], r=7, z=7, m=1, seed=0, L=5)
    S = g["strings"]
    got = sorted(tuple(sorted((S[a], S[b]))) for a, b in res.out_pairs)
    assert got == sorted(tuple(sorted(p)) for p in g["output"])


# ------------------------------------------------------ edit distance ----

def _ed_by_search(x: bytes, y: bytes, alphabet: bytes) -> int:
    """Edit distance by its definition: breadth-first search over strings,
    one insertion / deletion / substitution per edge."""
    if x == y:
        return 0
    maxlen = max(len(x), len(y)) + 1
    seen = {x}
    q = deque([(x, 0)])
    while q:
        s, d = q.popleft()
        nbrs = set()
        for i in range(len(s)):
            nbrs.add(s[:i] + s[i + 1:])
            for a in alphabet:
                nbrs.add(s[:i] + bytes([a]) + s[i + 1:])
        if len(s) < maxlen:
            for i in range(len(s) + 1):
                for a in alphabet:
                    nbrs.add(s[:i] + bytes([a]) + s[i:])
        for t in nbrs:
            if t == y:
                return d + 1
            if t not in seen:
                seen.add(t)
                q.append((t, d + 1))
    raise AssertionError("unreachable")


def test_edit_distance_matches_definition(oracle_lib):
    rng = np.random.default_rng(11)
    alpha = b"ab"
    for _ in range(120):
        lx, ly = rng.integers(0, 6, size=2)
        x = bytes(rng.choice(list(alpha), size=lx).tolist())
        y = bytes(rng.choice(list(alpha), size=ly).tolist())
        truth = _ed_by_search(x, y, alpha)
        assert oracle_lib.ed_full(x, y) == truth, (x, y)
        for K in range(0, 6):
            assert oracle_lib.ed_banded(x, y, K) == min(truth, K + 1), (x, y, K)


def test_edit_distance_textbook_values(oracle_lib):
    assert oracle_lib.ed_full(b"kitten", b"sitting") == 3
    assert oracle_lib.ed_full(b"", b"abc") == 3
    assert oracle_lib.ed_full(b"flaw", b"lawn") == 2
    assert oracle_lib.ed_banded(b"kitten", b"sitting", 2) == 3
    assert oracle_lib.ed_banded(b"", b"", 0) == 0


def test_banded_matches_full_on_longer_strings(oracle_lib):
    col = sd.clusters(5, 6, lambda r, b: 4, lambda r: r.integers(150, 260),
                      lambda r, L: r.poisson(15))
    S = col.strings()
    rng = np.random.default_rng(2)
    for a, b in itertools.combinations(range(len(S)), 2):
        full = oracle_lib.ed_full(S[a], S[b])
        for K in (0, 5, int(rng.integers(0, 60)), 120):
            assert oracle_lib.ed_banded(S[a], S[b], K) == min(full, K + 1)


def test_edit_distance_metric_properties(oracle_lib):
    col = sd.random_strings(9, 12, 0, 40, letters=b"ACG")
    S = col.strings()
    for a, b in itertools.combinations(range(len(S)), 2):
        d = oracle_lib.ed_full(S[a], S[b])
        assert d == oracle_lib.ed_full(S[b], S[a])
        assert abs(len(S[a]) - len(S[b])) <= d <= max(len(S[a]), len(S[b]))
        if len(S[a]) == len(S[b]):
            assert d <= sum(p != q for p, q in zip(S[a], S[b]))
    for a, b, c in itertools.combinations(range(len(S)), 3):
        assert oracle_lib.ed_full(S[a], S[c]) <= oracle_lib.ed_full(S[a], S[b]) + \
            oracle_lib.ed_full(S[b], S[c])


# --------------------------------------------------------- embedding ----

def _codes(oracle_lib, strings):
    sigma, lut = oracle_lib.alphabet(b"".join(strings))
    return sigma, [lut[np.frombuffer(s, dtype=np.uint8)].astype(np.uint8) for s in strings]


def test_ed_at_most_hamming_when_walks_finish(oracle_lib):
    """Footnote of the introduction: with bottom padding, ED(x,y) <= Ham of the
    embeddings whenever both walks have consumed their strings."""
    col = sd.clusters(21, 30, lambda r, b: 3, lambda r: r.integers(20, 60),
                      lambda r, L: r.poisson(4))
    S = col.strings()
    sigma, C = _codes(oracle_lib, S)
    L = 3 * max(len(s) for s in S)
    R, _, _ = oracle_lib.draw(4, 6, 1, 1, L, sigma)
    checked = 0
    for l in range(6):
        E = [oracle_lib.cgk_embed(c, R[l], sigma, L) for c in C]
        done = [bool(e[-1] == sigma) or len(s) == 0 for e, s in zip(E, S)]
        for a, b in itertools.combinations(range(len(S)), 2):
            if done[a] and done[b]:
                ham = int((E[a] != E[b]).sum())
                assert oracle_lib.ed_full(S[a], S[b]) <= ham
                checked += 1
    assert checked > 1000


def test_embedding_is_prefix_stable_and_deterministic(oracle_lib):
    S = sd.random_strings(3, 10, 0, 80).strings()
    sigma, C = _codes(oracle_lib, S)
    R, _, _ = oracle_lib.draw(1, 1, 1, 1, 300, sigma)
    for c in C:
        full = oracle_lib.cgk_embed(c, R[0], sigma, 300)
        assert (oracle_lib.cgk_embed(c, R[0], sigma, 100) == full[:100]).all()
        # the walk never skips a character: the embedding, with padding and
        # repeats removed step by step, spells the string
        steps = [int(s) for s in full if s != sigma]
        assert len(steps) >= len(c)


def test_walk_length_about_twice_string_length(oracle_lib):
    """Section 4.1: the number of embedding steps concentrates around 2|x|."""
    S = sd.random_strings(5, 60, 800, 1200).strings()
    sigma, C = _codes(oracle_lib, S)
    L = 3 * max(len(s) for s in S)
    R, _, _ = oracle_lib.draw(9, 2, 1, 1, L, sigma)
    ratios = []
    for l in range(2):
        for c in C:
            t = oracle_lib.cgk_embed(c, R[l], sigma, L)
            end = int(np.argmax(t == sigma)) if (t == sigma).any() else L
            ratios.append(end / len(c))
    assert 1.9 < float(np.mean(ratios)) < 2.1


# ---------------------------------------------------------------- LSH ----

def test_key_is_linear_in_the_signature(oracle_lib):
    """<u, v> mod P: raising one coordinate symbol by one adds v_k mod P."""
    rng = np.random.default_rng(4)
    _, _, v = oracle_lib.draw(2, 1, 1, 24, 100, 5)
    v = v[0, 0]
    pos = np.arange(24, dtype=np.uint32)
    for _ in range(50):
        t = rng.integers(0, 5, size=24).astype(np.uint8)
        k = int(rng.integers(0, 24))
        t2 = t.copy()
        t2[k] += 1
        d = (oracle_lib.key(t2, pos, v) - oracle_lib.key(t, pos, v)) % oracle_lib.P61
        assert d == int(v[k])
    # all-zero codes: u = 1 everywhere, key = sum(v) mod P
    t = np.zeros(24, dtype=np.uint8)
    assert oracle_lib.key(t, pos, v) == sum(int(x) for x in v) % oracle_lib.P61


def test_bit_sampling_collision_probability(oracle_lib):
    """Bit-sampling theorem + AND construction: for embeddings at Hamming
    distance H over L coordinates, a table with m coordinates drawn with
    replacement collides with probability (1 - H/L)^m."""
    rng = np.random.default_rng(8)
    L, m = 40, 3
    a = rng.integers(0, 4, size=L).astype(np.uint8)
    b = a.copy()
    H = 10
    flip = rng.choice(L, size=H, replace=False)
    b[flip] = (b[flip] + 1) % 4
    trials = 0
    hits = 0
    for seed in range(40):
        _, pos, v = oracle_lib.draw(seed, 1, 100, m, L, 4)
        for j in range(100):
            trials += 1
            hits += oracle_lib.key(a, pos[0, j], v[0, j]) == oracle_lib.key(b, pos[0, j], v[0, j])
    p = (1 - H / L) ** m
    sd_ = np.sqrt(p * (1 - p) / trials)
    assert abs(hits / trials - p) < 5 * sd_


# -------------------------------------------------------- whole join ----

def _brute_candidates(col, keys, K):
    n = col.n
    lens = col.lengths()
    out = set()
    for a in range(n):
        for b in range(a + 1, n):
            if abs(lens[a] - lens[b]) <= K and (keys[:, a] == keys[:, b]).any():
                out.add((a, b))
    return out


@pytest.mark.parametrize("seed,K,r,z,m,L", [(0, 12, 3, 4, 2, 0), (1, 30, 2, 5, 3, 40),
                                             (2, 5, 4, 3, 1, 20), (3, 0, 3, 3, 2, 0)])
def test_candidates_equal_definition(oracle_lib, seed, K, r, z, m, L):
    """The hash-table loop with eviction yields exactly the pairs that share a
    bucket in some table and differ in length by at most K."""
    col = sd.clusters(seed, 15, lambda rr, b: rr.integers(1, 5), lambda rr: rr.integers(5, 70),
                      lambda rr, LL: rr.poisson(3))
    res = oracle_lib.join(col.chars, col.offsets, K, r, z, m, seed=seed, L=L)
    assert set(map(tuple, res.cand_pairs.tolist())) == _brute_candidates(col, res.keys, K)
    # pairs found before de-duplication: one per table in which the pair's
    # keys agree (and the lengths are within K)
    lens = col.lengths()
    raw = sum(int((res.keys[:, a] == res.keys[:, b]).sum())
              for a in range(col.n) for b in range(a + 1, col.n) if abs(lens[a] - lens[b]) <= K)
    assert res.n_raw == raw
    # the candidates-only mode is the same loop stopped before verification
    cand, n_raw = oracle_lib.candidates(col.chars, col.offsets, K, r, z, m, seed=seed, L=L)
    assert cand.tolist() == res.cand.tolist() and n_raw == raw


def test_buckets_by_key_equal_buckets_by_signature(oracle_lib):
    col = sd.clusters(6, 20, lambda rr, b: 3, lambda rr: rr.integers(10, 30),
                      lambda rr, L: rr.poisson(2))
    r, z, m = 2, 3, 4
    res = oracle_lib.join(col.chars, col.offsets, 5, r, z, m, seed=6, L=16)
    for l in range(r):
        for j in range(z):
            sig = [bytes(res.sig[i, l, j]) for i in range(col.n)]
            key = res.keys[l * z + j]
            for a, b in itertools.combinations(range(col.n), 2):
                assert (sig[a] == sig[b]) == (key[a] == key[b])


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_output_is_exact_subset_and_precision_one(oracle_lib, seed):
    col = sd.clusters(seed, 25, lambda rr, b: rr.integers(1, 5), lambda rr: rr.integers(30, 90),
                      lambda rr, L: rr.poisson(4))
    K = 8
    truth_codes, truth_d = oracle_lib.brute_join(col.chars, col.offsets, K, full=True)
    truth = dict(zip(truth_codes.tolist(), truth_d.tolist()))
    fast_codes, fast_d = oracle_lib.brute_join(col.chars, col.offsets, K)
    assert fast_codes.tolist() == truth_codes.tolist() and fast_d.tolist() == truth_d.tolist()
    res = oracle_lib.join(col.chars, col.offsets, K, 4, 6, 3, seed=seed, L=0)
    for c, d in zip(res.out.tolist(), res.out_dist.tolist()):
        assert truth[c] == d
    # every candidate that is a true pair is reported
    cand_true = [c for c in res.cand.tolist() if c in truth]
    assert sorted(cand_true) == res.out.tolist()


def test_identical_strings_always_join(oracle_lib):
    S = [b"ACGTTGCA" * 5, b"ACGTTGCA" * 5, b"", b"", b"TTTT", b"TTTT"]
    col = sd.from_strings(S)
    res = oracle_lib.join(col.chars, col.offsets, 0, 1, 1, 4, seed=3, L=0)
    assert res.out_pairs.tolist() == [[0, 1], [2, 3], [4, 5]]
    assert res.out_dist.tolist() == [0, 0, 0]


def test_empty_and_degenerate_inputs(oracle_lib):
    col = sd.from_strings([])
    res = oracle_lib.join(col.chars, col.offsets, 3, 2, 2, 2)
    assert res.out.size == 0 and res.cand.size == 0
    col = sd.from_strings([b"", b"", b""])
    res = oracle_lib.join(col.chars, col.offsets, 0, 2, 2, 2)
    assert res.out_pairs.tolist() == [[0, 1], [0, 2], [1, 2]]
    col = sd.from_strings([b"A"])
    res = oracle_lib.join(col.chars, col.offsets, 3, 2, 2, 2)
    assert res.out.size == 0
    with pytest.raises(ValueError):
        oracle_lib.join(col.chars, col.offsets, 3, 0, 2, 2)


# -------------------------------------------------------------- serving --

@pytest.mark.parametrize("seed,K", [(0, 6), (1, 15), (2, 0)])
def test_query_over_the_set_equals_the_self_join(oracle_lib, seed, K):
    """Serving query of string a against index S (same alphabet, truncation
    and streams) returns exactly a itself and the self-join's partners of a:
    two independent code paths (hash tables in length order vs. a double
    loop over all pairs) for the same set."""
    col = sd.clusters(seed, 20, lambda rr, b: rr.integers(1, 5), lambda rr: rr.integers(20, 70),
                      lambda rr, L: rr.poisson(3))
    r, z, m = 3, 4, 3
    res = oracle_lib.join(col.chars, col.offsets, K, r, z, m, seed=seed, L=0)
    partners = {a: {a: 0} for a in range(col.n)}
    for (a, b), d in zip(res.out_pairs.tolist(), res.out_dist.tolist()):
        partners[a][b] = d
        partners[b][a] = d
    off, ids, dist = oracle_lib.query(col.chars, col.offsets, col.chars, col.offsets,
                                      [K] * col.n, r, z, m, seed=seed, L=0)
    for q in range(col.n):
        lo, hi = int(off[q]), int(off[q + 1])
        got = dict(zip(ids[lo:hi].tolist(), dist[lo:hi].tolist()))
        assert got == partners[q]
        assert ids[lo:hi].tolist() == sorted(got)


def test_query_results_are_true_matches(oracle_lib):
    rng = np.random.default_rng(4)
    col = sd.clusters(4, 15, lambda rr, b: 3, lambda rr: rr.integers(40, 120),
                      lambda rr, L: rr.poisson(5))
    S = col.strings()
    Q, Kq = [], []
    for i in range(12):
        base = S[int(rng.integers(0, col.n))]
        Q.append(base if i % 3 == 0 else bytes(sd.mutate(rng, np.frombuffer(base, np.uint8),
                                                         int(rng.integers(0, 6)),
                                                         np.frombuffer(b"ACGT", np.uint8))))
        Kq.append(int(rng.integers(0, 12)))
    qc = sd.from_strings(Q)
    off, ids, dist = oracle_lib.query(col.chars, col.offsets, qc.chars, qc.offsets, Kq, 4, 6, 2,
                                      seed=9, L=0)
    for q in range(len(Q)):
        lo, hi = int(off[q]), int(off[q + 1])
        for s, d in zip(ids[lo:hi].tolist(), dist[lo:hi].tolist()):
            assert oracle_lib.ed_full(Q[q], S[s]) == d <= Kq[q]
        if q % 3 == 0:   # an exact copy of an index string finds it
            assert 0 in dist[lo:hi].tolist()
    with pytest.raises(ValueError):
        bad = sd.from_strings([b"ACGZ"])
        oracle_lib.query(col.chars, col.offsets, bad.chars, bad.offsets, [1], 2, 2, 2)


def test_keys_of_a_set_equal_the_joins_keys(oracle_lib):
    col = sd.clusters(21, 10, lambda rr, b: 3, lambda rr: rr.integers(5, 60),
                      lambda rr, L: rr.poisson(2))
    res = oracle_lib.join(col.chars, col.offsets, 5, 3, 4, 5, seed=2, L=30)
    k = oracle_lib.keys(col.chars, col.offsets, col.chars, col.offsets, 3, 4, 5, seed=2, L=30)
    assert np.array_equal(k.T, res.keys)
    q = sd.from_strings([b"ACGTTT", b"QQ"])
    with pytest.raises(ValueError):
        oracle_lib.keys(col.chars, col.offsets, q.chars, q.offsets, 3, 4, 5)


def test_serving_truth_equals_the_query_definition(oracle_lib):
    # the threaded, sorted-key form of the serving definition that the
    # full-size GPU test uses equals the oracle's plain double loop
    from tests._oracle_truth import serving_truth
    col, _ = sd.serving_index(3, n_bases=40, copies=4)
    q, Kq, _ = sd.serving_queries(col, 3, n_queries=30)
    want, _ = serving_truth(oracle_lib, col, q, Kq, 6, 4, 6, 1, 40)
    off, ids, dist = oracle_lib.query(col.chars, col.offsets, q.chars, q.offsets, Kq, 6, 4, 6,
                                      seed=1, L=40)
    assert sum(len(w[0]) for w in want) > 0
    for qi in range(q.n):
        lo, hi = int(off[qi]), int(off[qi + 1])
        assert want[qi][0] == ids[lo:hi].tolist() and want[qi][1] == dist[lo:hi].tolist()


# ----------------------------------------------------- EmbedJoin+ (§5) ----

def _brute_plus(col, keys, K, kappa, T):
    """Candidates of Algorithm 5 from their definition: pairs within K in
    length with some suffix pair whose keys agree in at least T tables; and
    the size of the tuple multiset (one tuple per table and agreeing suffix
    pair)."""
    n, lens = col.n, col.lengths()
    cand, raw = set(), 0
    for a in range(n):
        for b in range(a + 1, n):
            if abs(lens[a] - lens[b]) > K:
                continue
            for ka in range(kappa):
                for kb in range(kappa):
                    c = int((keys[:, a * kappa + ka] == keys[:, b * kappa + kb]).sum())
                    raw += c
                    if c >= T:
                        cand.add((a, b))
    return cand, raw


def test_plus_with_one_suffix_and_T1_is_embedjoin(oracle_lib):
    for seed in (0, 1, 2):
        col, _ = sd.shifted_reads(seed, n_bases=12, copies=4, base_len=(60, 120), shift=10,
                                  edit_rate=0.03)
        a = oracle_lib.join(col.chars, col.offsets, 20, 3, 4, 3, seed=seed, L=48)
        b = oracle_lib.join_plus(col.chars, col.offsets, 20, 3, 4, 3, delta=20, T=1, seed=seed,
                                 L=48)
        assert oracle_lib.plus_kappa(20, 20) == 1
        assert b.cand.tolist() == a.cand.tolist() and b.n_raw == a.n_raw
        assert b.out.tolist() == a.out.tolist() and b.out_dist.tolist() == a.out_dist.tolist()
        assert np.array_equal(b.keys, a.keys)


@pytest.mark.parametrize("seed,K,delta,T,r,z,m", [(0, 30, 10, 2, 3, 4, 2), (1, 25, 9, 1, 2, 5, 3),
                                                  (2, 40, 15, 3, 2, 6, 2), (3, 12, 5, 2, 3, 3, 1)])
def test_plus_candidates_equal_definition(oracle_lib, seed, K, delta, T, r, z, m):
    col, _ = sd.shifted_reads(seed, n_bases=8, copies=4, base_len=(20, 70), shift=15,
                              edit_rate=0.05)
    res = oracle_lib.join_plus(col.chars, col.offsets, K, r, z, m, delta=delta, T=T, seed=seed,
                               L=40)
    kappa = oracle_lib.plus_kappa(K, delta)
    assert kappa == -(-K // delta)
    want, raw = _brute_plus(col, res.keys, K, kappa, T)
    assert set(map(tuple, res.cand_pairs.tolist())) == want
    assert res.n_raw == raw
    # suffix keys: suffix k of string i is the embedding of s_i[k*delta:]
    sub = sd.from_strings([col.string(i)[k * delta:] for i in range(col.n) for k in range(kappa)])
    k2 = oracle_lib.keys(col.chars, col.offsets, sub.chars, sub.offsets, r, z, m, seed=seed, L=40)
    assert np.array_equal(k2.T, res.keys)
    # output: the candidates within K, exactly
    d = oracle_lib.verify_pairs(col.chars, col.offsets, res.cand, K)
    assert res.out.tolist() == res.cand[d <= K].tolist()
    cand_only = oracle_lib.join_plus(col.chars, col.offsets, K, r, z, m, delta=delta, T=T,
                                     seed=seed, L=40, opts=oracle_lib.STOP_AFTER_CANDIDATES)
    assert cand_only.cand.tolist() == res.cand.tolist() and cand_only.n_raw == res.n_raw


def test_plus_default_threshold():
    # T = 2 when a string has more than one suffix (K > delta), else 1
    from oracle import oracle
    assert oracle.plus_default_T(100, 50) == 2 and oracle.plus_default_T(50, 50) == 1
    assert oracle.plus_default_T(51, 50) == 2 and oracle.plus_kappa(101, 50) == 3


def test_plus_finds_a_leading_shift_of_delta(oracle_lib):
    """y = P + x with |P| = delta: y's second suffix is x itself, so the pair
    collides in every table and is a candidate at any seed; plain EmbedJoin,
    whose walks start out of step, misses many such pairs."""
    rng = np.random.default_rng(4)
    delta, K = 12, 30
    found_plus = found_plain = 0
    for seed in range(40):
        x = bytes(np.frombuffer(b"ACGT", np.uint8)[rng.integers(0, 4, size=200)])
        P = bytes(np.frombuffer(b"ACGT", np.uint8)[rng.integers(0, 4, size=delta)])
        col = sd.from_strings([x, P + x])
        res = oracle_lib.join_plus(col.chars, col.offsets, K, 2, 3, 8, delta=delta, seed=seed,
                                   L=128)
        assert res.cand.tolist() == [1] and res.out_dist.tolist() == [delta]
        assert res.n_raw >= 2 * 3
        found_plus += 1
        found_plain += len(oracle_lib.join(col.chars, col.offsets, K, 2, 3, 8, seed=seed,
                                           L=128).cand)
    assert found_plus == 40 and found_plain < 40


def test_plus_threshold_probability_closed_form(oracle_lib):
    """Two fixed strings, one suffix, one seed, z functions: given the seed's
    embeddings at Hamming distance H over L, each table's keys agree
    independently with p = (1 - H/L)^m, so the number of agreeing tables is
    Binomial(z, p) and the pair is a candidate with probability
    p_T = 1 - sum_{i<T} C(z,i) p^i (1-p)^(z-i) (Section 5)."""
    from math import comb
    x = b"ACGTTGCAAGCTTACGGATCCATGCA" * 3
    y = x[:20] + b"T" + x[21:40] + x[41:] + b"G"
    col = sd.from_strings([x, y])
    sigma, lut = oracle_lib.alphabet(col.chars)
    L, z, m, T, K = 96, 8, 6, 3, 10
    cx, cy = lut[np.frombuffer(x, np.uint8)], lut[np.frombuffer(y, np.uint8)]
    exp_rate = exp_count = 0.0
    hits = counts = 0
    seeds = 1500
    for seed in range(seeds):
        R, _, _ = oracle_lib.draw(seed, 1, 1, 1, L, sigma)
        tx = oracle_lib.cgk_embed(cx.astype(np.uint8), R[0], sigma, L)
        ty = oracle_lib.cgk_embed(cy.astype(np.uint8), R[0], sigma, L)
        p = (1.0 - float((tx != ty).sum()) / L) ** m
        exp_count += z * p
        exp_rate += 1.0 - sum(comb(z, i) * p ** i * (1 - p) ** (z - i) for i in range(T))
        res = oracle_lib.join_plus(col.chars, col.offsets, K, 1, z, m, delta=K, T=T, seed=seed,
                                   L=L)
        counts += res.n_raw
        hits += len(res.cand)
    exp_rate /= seeds
    exp_count /= seeds
    se = (exp_rate * (1 - exp_rate) / seeds) ** 0.5
    assert 0.1 < exp_rate < 0.9
    assert abs(hits / seeds - exp_rate) < 4.5 * se
    assert abs(counts / seeds - exp_count) < 4.5 * (z / seeds) ** 0.5


# ------------------------------------------ distortion diagnostics ----

def test_embed_hamming_properties(oracle_lib):
    rng = np.random.default_rng(2)
    DNA = np.frombuffer(b"ACGT", np.uint8)
    x = bytes(DNA[rng.integers(0, 4, size=150)])
    y = bytes(sd.mutate(rng, np.frombuffer(x, np.uint8), 6, DNA))
    P = bytes(DNA[rng.integers(0, 4, size=10)])
    col = sd.from_strings([x, x, y, P + x, bytes(DNA[rng.integers(0, 4, size=150)])])
    codes = lambda pr: np.array([(a << 32) | b for a, b in pr], dtype=np.uint64)
    pr = [(0, 1), (0, 2), (2, 0), (0, 3), (0, 4)]
    r, L = 6, 400
    h = oracle_lib.embed_hamming(col.chars, col.offsets, codes(pr), r, L=L, seed=3)
    assert (h[0] == 0).all()                        # identical strings
    assert (h[1] == h[2]).all()                     # symmetric
    assert (h <= L).all()
    ed = oracle_lib.ed_full(x, y)
    assert (h[1] >= ed).all()                       # walks end well within L = 400
    hs = oracle_lib.embed_hamming(col.chars, col.offsets, codes(pr), r, L=L, seed=3, K=30,
                                  delta=10)
    assert (hs <= h).all()                          # the (0, 0) suffix pair is among those
    assert (hs[3] == 0).all() and (h[3] > 0).any()  # P + x: its second suffix is x
    # the random pair is farther than the similar pair under every seed
    assert (h[4] > h[1]).all()


# ------------------------------------------------ grouping (§4.1) ----

def _groups(lens, K):
    """Member lists of the length groups ((g)K, (g+2)K] (group 0 with the
    empty strings; one group per length when K = 0)."""
    N = int(lens.max()) if len(lens) else 0
    if K == 0:
        return [np.nonzero(lens == g)[0] for g in range(N + 1)]
    G = max(1, -(-N // K) - 1)
    return [np.nonzero(((lens > g * K) & (lens <= (g + 2) * K)) | ((g == 0) & (lens == 0)))[0]
            for g in range(G)]


@pytest.mark.parametrize("seed,K,r,z,m", [(0, 40, 3, 4, 3), (1, 25, 2, 5, 2), (2, 0, 2, 3, 1)])
def test_grouped_candidates_equal_definition(oracle_lib, seed, K, r, z, m):
    """A grouped candidate is a pair of one group, within K in length, that
    shares a key in some table of that group's own join (its alphabet,
    L = 3 x its longest string); keys from the oracle's key function."""
    col = sd.clusters(seed, 12, lambda rr, b: rr.integers(2, 5), lambda rr: rr.integers(0, 160),
                      lambda rr, LL: rr.poisson(2))
    res = oracle_lib.join_grouped(col.chars, col.offsets, K, r, z, m, seed=seed)
    lens = col.lengths()
    want = set()
    raw = 0
    for ids in _groups(lens, K):
        if len(ids) < 2:
            continue
        sub = sd.from_strings([col.string(int(i)) for i in ids])
        Lg = max(1, 3 * int(lens[ids].max()))
        k = oracle_lib.keys(sub.chars, sub.offsets, sub.chars, sub.offsets, r, z, m, seed=seed,
                            L=Lg)
        for x in range(len(ids)):
            for y in range(x + 1, len(ids)):
                if abs(int(lens[ids[x]]) - int(lens[ids[y]])) <= K:
                    c = int((k[x] == k[y]).sum())
                    raw += c
                    if c:
                        want.add((int(ids[x]), int(ids[y])))
    assert set(map(tuple, res.cand_pairs.tolist())) == want
    assert res.n_raw == raw
    d = oracle_lib.verify_pairs(col.chars, col.offsets, res.cand, K)
    assert res.out.tolist() == res.cand[d <= K].tolist()
    assert res.out_dist.tolist() == d[d <= K].tolist()


def test_grouping_covers_every_length_pair(oracle_lib):
    """Every pair within K in length shares a group (the paper's premise), at
    the group boundaries too: identical strings of lengths 0, K, 2K, 2K+1,
    3K ... always join (identical strings collide in every table)."""
    K = 10
    DNA = np.frombuffer(b"ACGT", np.uint8)
    rng = np.random.default_rng(6)
    strings = []
    for L in (0, 1, K - 1, K, K + 1, 2 * K, 2 * K + 1, 3 * K, 3 * K + 1, 5 * K):
        s = bytes(DNA[rng.integers(0, 4, size=L)])
        strings += [s, s]
    col = sd.from_strings(strings)
    res = oracle_lib.join_grouped(col.chars, col.offsets, K, 1, 1, 4, seed=2)
    got = set(map(tuple, res.out_pairs.tolist()))
    assert all((2 * i, 2 * i + 1) in got for i in range(len(strings) // 2))
    lens = col.lengths()
    for a in range(col.n):
        for b in range(a + 1, col.n):
            if abs(int(lens[a]) - int(lens[b])) <= K:
                assert any(a in g and b in g for g in _groups(lens, K))


def test_grouping_with_one_group_is_the_join_untruncated(oracle_lib):
    col, _ = sd.tiny_dna(3, n_bases=12)
    K = 3000  # above every length: one group
    g = oracle_lib.join_grouped(col.chars, col.offsets, K, 2, 3, 6, seed=1)
    N = int(col.lengths().max())
    a = oracle_lib.join(col.chars, col.offsets, K, 2, 3, 6, seed=1, L=3 * N)
    assert g.cand.tolist() == a.cand.tolist() and g.n_raw == a.n_raw
    assert g.out.tolist() == a.out.tolist()


# ------------------------------------------------- exhaustive short strings --

def _short_mix(seed):
    """Clusters of mixed lengths (some strings of a few letters, some empty)
    whose short members are within a large K of each other by chance."""
    return sd.clusters(seed, 14, lambda rr, b: rr.integers(1, 4),
                       lambda rr: rr.integers(0, 120), lambda rr, LL: rr.poisson(3))


@pytest.mark.parametrize("seed,K", [(0, 30), (1, 0), (2, 60)])
def test_exact_short_above_every_length_is_the_exact_join(oracle_lib, seed, K):
    """With every string short, the candidates are all pairs that pass the
    length filter, so the output is the exact join: it equals brute force by
    textbook Wagner-Fischer, for the EmbedJoin, EmbedJoin+ and grouping
    results alike."""
    col = _short_mix(seed)
    N = int(col.lengths().max())
    truth, tdist = oracle_lib.brute_join(col.chars, col.offsets, K, full=True)
    for res in (oracle_lib.join(col.chars, col.offsets, K, 2, 2, 6, seed=seed, exact_len=N),
                oracle_lib.join_plus(col.chars, col.offsets, K, 2, 2, 6, delta=20, seed=seed,
                                     exact_len=N),
                oracle_lib.join_grouped(col.chars, col.offsets, K, 2, 2, 6, seed=seed,
                                        exact_len=N)):
        assert res.out.tolist() == truth.tolist()
        assert res.out_dist.tolist() == tdist.tolist()
        lens = col.lengths().astype(np.int64)
        n_len_ok = sum(1 for a in range(col.n) for b in range(a + 1, col.n)
                       if abs(lens[a] - lens[b]) <= K)
        assert len(res.cand) == n_len_ok


def test_exact_short_off_leaves_the_join(oracle_lib):
    col = _short_mix(4)
    a = oracle_lib.join(col.chars, col.offsets, 40, 2, 3, 5, seed=3)
    b = oracle_lib.join(col.chars, col.offsets, 40, 2, 3, 5, seed=3, exact_len=0)
    assert a.cand.tolist() == b.cand.tolist() and a.out.tolist() == b.out.tolist()
    assert a.n_raw == b.n_raw


@pytest.mark.parametrize("S", [1, 25, 70])
def test_exact_short_is_the_join_plus_every_short_true_pair(oracle_lib, S):
    """Between the extremes: the output is the LSH join's output united with
    every true pair (brute force) whose strings are both no longer than S,
    and nothing else; the tables' raw count is unchanged."""
    col = _short_mix(5)
    K = 45
    base = oracle_lib.join(col.chars, col.offsets, K, 2, 3, 5, seed=7)
    res = oracle_lib.join(col.chars, col.offsets, K, 2, 3, 5, seed=7, exact_len=S)
    truth, tdist = oracle_lib.brute_join(col.chars, col.offsets, K, full=True)
    lens = col.lengths()
    a = (truth >> np.uint64(32)).astype(np.int64)
    b = (truth & np.uint64(0xFFFFFFFF)).astype(np.int64)
    short_true = truth[(lens[a] <= S) & (lens[b] <= S)]
    want = np.union1d(base.out, short_true)
    assert res.out.tolist() == want.tolist()
    assert res.out_dist.tolist() == tdist[np.isin(truth, want)].tolist()
    assert res.n_raw == base.n_raw
    assert np.isin(base.cand, res.cand).all()
