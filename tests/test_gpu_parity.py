"""GPU parity: every stage of the HIP path, called through the C ABI, against
the CPU oracle on the same seeded inputs.  All results here are integers, so
the bar is bit-exact equality."""
import json
import os
import sys

import numpy as np
import pytest

import synthdata as sd
from tests._gpu_util import codes_to_set, pairs_to_codes, to_device

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden")


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


def _each_verify_mode(ctx):
    """Runs the body once per verification form (two-pass with one, two and
    four band words per lane, persistent tiles, one pair per lane, grouped by
    pattern); the mode yielded for the two-pass form with W words per lane
    (W > 1) is "0wW"."""
    old = (ctx.tune_get("verify_mode"), ctx.tune_get("verify_wpl"))
    try:
        for mode, wpl in ((0, 1), (0, 2), (0, 4), (1, 1), (2, 1), (3, 1)):
            ctx.tune_set("verify_mode", mode)
            ctx.tune_set("verify_wpl", wpl)
            yield mode if wpl == 1 else f"0w{wpl}"
    finally:
        ctx.tune_set("verify_mode", old[0])
        ctx.tune_set("verify_wpl", old[1])


def _oracle_join(oracle_lib, col, K, r, z, m, seed, L=0):
    return oracle_lib.join(col.chars, col.offsets, K, r, z, m, seed=seed, L=L)


def _assert_join_equal(res, ref):
    got = pairs_to_codes(res.pairs)
    assert got.tolist() == ref.out.tolist()
    assert res.dist.tolist() == ref.out_dist.astype(np.int32).tolist()
    assert res.n_candidates == len(ref.cand)
    assert res.L == ref.L and res.sigma == ref.sigma


# ------------------------------------------------------ paper examples ----

def test_running_example_through_hook(ej, ctx, oracle_lib):
    g = json.load(open(os.path.join(GOLD, "running_example.json")))
    letters = g["alphabet"]
    R = np.zeros((2, g["L"] * 4), dtype=np.uint8)
    for l, name in enumerate(["R1", "R2"]):
        for k, ch in enumerate(letters):
            for j, bit in enumerate(g["pi"][name][ch]):
                R[l, j * 4 + k] = bit
    pos = np.zeros((2, 2, 2), dtype=np.uint32)
    for l in range(2):
        for j in range(2):
            pos[l, j] = np.array(g["lsh_coordinates_1based"][f"f{j + 1}^{l + 1}"]) - 1
    col = sd.from_strings([s.encode() for s in g["strings"]])
    _say("running example (explicit randomness)")
    ctx.set_explicit_randomness(2, 2, 2, g["L"], 4, R, pos)
    try:
        chars, offs = to_device(col)
        keys, sig, L_used, sigma = ctx.embed(chars, offs, 2, 2, 2, seed=0, L=g["L"], want_sig=True)
        sig = sig.cpu().numpy()
        for i in range(4):
            got = ["".join(letters[c] for c in sig[i, l, j]) for l in range(2) for j in range(2)]
            assert got == g["signatures"][str(i + 1)]
        res = ctx.join(col.chars, col.offsets, g["K"], 2, 2, 2, seed=0, L=g["L"])
    finally:
        ctx.set_explicit_randomness(0, 0, 0, 0, 0)
    assert (res.pairs + 1).tolist() == g["output_1based"]
    assert res.dist.tolist() == [2, 3]
    assert res.n_candidates == len(g["candidates_1based"])


def test_intro_example(ej, ctx):
    g = json.load(open(os.path.join(GOLD, "intro_example.json")))
    col = sd.from_strings([s.encode() for s in g["strings"]])
    _say("intro example r=7 z=7 m=1 L=5 seed=0")
    res = ctx.join(col.chars, col.offsets, g["K"], 7, 7, 1, seed=0, L=5)
    S = g["strings"]
    got = sorted(tuple(sorted((S[a], S[b]))) for a, b in res.pairs.tolist())
    assert got == sorted(tuple(sorted(p)) for p in g["output"])


# ------------------------------------------------------ stage by stage ----

STAGE_CASES = [
    # seed, n_bases, len range, edits, K, r, z, m, L, letters
    (0, 40, (50, 300), 6, 12, 3, 4, 6, 0, sd.DNA),
    (1, 30, (100, 700), 20, 40, 2, 7, 12, 0, sd.DNA),
    (2, 25, (10, 90), 3, 5, 4, 3, 3, 24, sd.PROTEIN25),
    (3, 20, (200, 2600), 30, 60, 3, 5, 20, 0, sd.DNA),          # walks span several LDS windows
    (4, 30, (0, 40), 2, 3, 3, 4, 2, 0, b"AB"),                  # empty strings, 2 letters
    (5, 15, (30, 120), 8, 20, 2, 6, 5, 0, bytes(range(65, 65 + 40))),  # 40 letters: generic pi path
]


@pytest.mark.parametrize("case", STAGE_CASES, ids=[f"c{c[0]}" for c in STAGE_CASES])
def test_stages_match_oracle(ej, ctx, oracle_lib, case):
    import torch
    seed, nb, (lo, hi), E, K, r, z, m, L, letters = case
    col = sd.clusters(seed, nb, lambda rr, b: rr.integers(1, 6), lambda rr: rr.integers(lo, hi + 1),
                      lambda rr, LL: rr.poisson(E), letters=letters)
    ref = _oracle_join(oracle_lib, col, K, r, z, m, seed, L)
    chars, offs = to_device(col)
    _say(f"stages case seed={seed} n={col.n} K={K} r={r} z={z} m={m} L={L}")
    keys, sig, L_used, sigma = ctx.embed(chars, offs, r, z, m, seed=seed, L=L, want_sig=True)
    torch.cuda.synchronize()
    assert L_used == ref.L and sigma == ref.sigma
    assert np.array_equal(sig.cpu().numpy(), ref.sig)
    assert np.array_equal(keys.cpu().numpy().astype(np.uint64), ref.keys)
    d_len = torch.from_numpy(col.lengths().astype(np.int32)).cuda()
    ids, gstart = ctx.lsh_bucket(keys, d_len)
    cand, n_raw = ctx.candidates(keys, ids, gstart, d_len, K)
    assert cand.cpu().numpy().astype(np.uint64).tolist() == ref.cand.tolist()
    dist = ctx.verify(chars, offs, cand, K)
    assert dist.cpu().numpy().tolist() == ref.cand_dist.astype(np.int32).tolist()
    res = ctx.join(col.chars, col.offsets, K, r, z, m, seed=seed, L=L)
    _assert_join_equal(res, ref)
    # device-resident form gives the same answer
    res2 = ctx.join(chars, offs, K, r, z, m, seed=seed, L=L)
    _assert_join_equal(res2, ref)


def test_bucket_key_bits_do_not_change_candidates(ej, ctx, oracle_lib):
    import torch
    col = sd.clusters(7, 30, lambda rr, b: 4, lambda rr: rr.integers(40, 80),
                      lambda rr, LL: rr.poisson(3))
    K, r, z, m = 10, 3, 5, 2
    ref = _oracle_join(oracle_lib, col, K, r, z, m, 7, 16)
    chars, offs = to_device(col)
    keys, _, _, _ = ctx.embed(chars, offs, r, z, m, seed=7, L=16)
    d_len = torch.from_numpy(col.lengths().astype(np.int32)).cuda()
    for bits in (0, 1, 3, 8, 17, 32):
        _say(f"bucket key_bits={bits}")
        ids, gstart = ctx.lsh_bucket(keys, d_len, key_bits=bits)
        cand, _ = ctx.candidates(keys, ids, gstart, d_len, K)
        assert cand.cpu().numpy().astype(np.uint64).tolist() == ref.cand.tolist()
    # key_bits = 0: each group is exactly one bucket, groups in increasing key
    # order per table, members in (length, position) order
    ids, gstart = ctx.lsh_bucket(keys, d_len, key_bits=0)
    ids, gstart = ids.cpu().numpy(), gstart.cpu().numpy()
    lens, n = col.lengths(), col.n
    want = 0
    for t in range(r * z):
        kt = ref.keys[t]
        want += len(np.unique(kt))
        order = sorted(range(n), key=lambda i: (int(kt[i]), int(lens[i]), i))
        assert ids[t * n:(t + 1) * n].tolist() == order
    assert len(gstart) - 1 == want
    for g in range(len(gstart) - 1):
        a, b = int(gstart[g]), int(gstart[g + 1])
        t = a // n
        assert b <= (t + 1) * n
        assert len(set(ref.keys[t][ids[a:b]].tolist())) == 1
        if g + 1 < len(gstart) - 1 and b < (t + 1) * n:
            assert ref.keys[t][ids[b]] > ref.keys[t][ids[a]]


# ------------------------------------------------------- verification ----

@pytest.mark.parametrize("K", [0, 1, 7, 15, 16, 29, 30, 31, 50, 63, 100, 250, 400, 500, 1000, 1022, 2046])
def test_verify_matches_ukkonen(ej, ctx, oracle_lib, K):
    import torch
    rng = np.random.default_rng(K)
    col = sd.clusters(100 + K, 12, lambda rr, b: 5,
                      lambda rr: rr.integers(0, 3 * K + 60),
                      lambda rr, LL: rr.poisson(max(1, K // 2)))
    n = col.n
    a = rng.integers(0, n, size=400)
    b = rng.integers(0, n, size=400)
    codes = (a.astype(np.uint64) << np.uint64(32)) | b.astype(np.uint64)
    want = oracle_lib.verify_pairs(col.chars, col.offsets, codes, K)
    chars, offs = to_device(col)
    for mode in _each_verify_mode(ctx):
        _say(f"verify K={K} n={n} mode={mode}")
        got = ctx.verify(chars, offs, torch.from_numpy(codes.astype(np.int64)).cuda(), K)
        assert got.cpu().numpy().astype(np.uint32).tolist() == want.tolist()


def test_verify_per_pair_thresholds(ej, ctx, oracle_lib):
    import torch
    rng = np.random.default_rng(5)
    col = sd.clusters(55, 20, lambda rr, b: 4, lambda rr: rr.integers(100, 1500),
                      lambda rr, LL: rr.poisson(40))
    n = col.n
    a = rng.integers(0, n, size=300)
    b = rng.integers(0, n, size=300)
    Kq = rng.integers(0, 600, size=300).astype(np.uint32)
    codes = (a.astype(np.uint64) << np.uint64(32)) | b.astype(np.uint64)
    want = [int(oracle_lib.verify_pairs(col.chars, col.offsets, codes[i:i + 1], int(Kq[i]))[0])
            for i in range(300)]
    chars, offs = to_device(col)
    for mode in _each_verify_mode(ctx):
        _say(f"verify per-pair thresholds mode={mode}")
        got = ctx.verify(chars, offs, torch.from_numpy(codes.astype(np.int64)).cuda(), 0,
                         d_Kq=torch.from_numpy(Kq.astype(np.int32)).cuda())
        assert got.cpu().numpy().tolist() == want


def test_verify_long_strings_random_and_similar(ej, ctx, oracle_lib):
    import torch
    col = sd.clusters(77, 3, lambda rr, b: 3, lambda rr: rr.integers(4500, 5501),
                      lambda rr, LL: rr.poisson(0.04 * LL))
    n = col.n
    a, b = np.triu_indices(n, 1)
    codes = (a.astype(np.uint64) << np.uint64(32)) | b.astype(np.uint64)
    chars, offs = to_device(col)
    for K in (250, 500):
        want = oracle_lib.verify_pairs(col.chars, col.offsets, codes, K)
        for mode in _each_verify_mode(ctx):
            _say(f"verify long K={K} mode={mode}")
            got = ctx.verify(chars, offs, torch.from_numpy(codes.astype(np.int64)).cuda(), K)
            assert got.cpu().numpy().astype(np.uint32).tolist() == want.tolist()


@pytest.mark.parametrize("K", [40, 100, 254, 300, 500, 700, 1000, 2046])
def test_verify_mask_layouts_agree(ej, ctx, oracle_lib, K):
    """Whole-pattern and ring layouts of the match masks, with one and two
    passes, and the lane form at every split width give the oracle's
    distances (bands of 2 to 64 words)."""
    import torch
    rng = np.random.default_rng(K + 7)
    col = sd.clusters(300 + K, 8, lambda rr, b: 4, lambda rr: rr.integers(K // 2, 2 * K + 400),
                      lambda rr, LL: rr.poisson(max(1, K // 3)))
    n = col.n
    a = rng.integers(0, n, size=120)
    b = rng.integers(0, n, size=120)
    codes = (a.astype(np.uint64) << np.uint64(32)) | b.astype(np.uint64)
    want = oracle_lib.verify_pairs(col.chars, col.offsets, codes, K).tolist()
    chars, offs = to_device(col)
    d_codes = torch.from_numpy(codes.astype(np.int64)).cuda()
    old = (ctx.tune_get("verify_ring"), ctx.tune_get("verify_pass1_cols"),
           ctx.tune_get("verify_mode"), ctx.tune_get("verify_split"),
           ctx.tune_get("verify_wpl"))
    try:
        for ring in (0, 2):
            for mode, c1, wpl in ((0, 0, 1), (0, 64, 1), (0, 1024, 1), (1, 0, 1), (0, 0, 2),
                                  (0, 64, 2), (0, 1024, 2), (0, 0, 4), (0, 64, 4),
                                  (0, 1024, 4)):
                ctx.tune_set("verify_ring", ring)
                ctx.tune_set("verify_pass1_cols", c1)
                ctx.tune_set("verify_mode", mode)
                ctx.tune_set("verify_wpl", wpl)
                _say(f"verify layout K={K} ring={ring} mode={mode} c1={c1} wpl={wpl}")
                got = ctx.verify(chars, offs, d_codes, K)
                assert got.cpu().numpy().astype(np.uint32).tolist() == want
        ctx.tune_set("verify_mode", 2)
        for split in (0, 1, 2, 4, 8, 16):
            ctx.tune_set("verify_split", split)
            _say(f"verify lane form K={K} split={split}")
            got = ctx.verify(chars, offs, d_codes, K)
            assert got.cpu().numpy().astype(np.uint32).tolist() == want
        ctx.tune_set("verify_mode", 3)
        _say(f"verify grouped by pattern K={K}")
        got = ctx.verify(chars, offs, d_codes, K)
        assert got.cpu().numpy().astype(np.uint32).tolist() == want
    finally:
        ctx.tune_set("verify_ring", old[0])
        ctx.tune_set("verify_pass1_cols", old[1])
        ctx.tune_set("verify_mode", old[2])
        ctx.tune_set("verify_split", old[3])
        ctx.tune_set("verify_wpl", old[4])


def test_candidate_groups_with_many_distinct_pairs(ej, ctx, oracle_lib):
    """One cluster of 1,100 near-copies among 2,000 strings: the string
    groups of the 32-bit candidate de-duplication then hold more distinct
    pairs than the LDS table takes, and the join falls back to sorting all
    raw pairs; the result is still the oracle's."""
    rng = np.random.default_rng(77)
    DNA = np.frombuffer(b"ACGT", dtype=np.uint8)
    base = DNA[rng.integers(0, 4, size=40)]
    pieces = [bytes(sd.mutate(rng, base, int(rng.integers(0, 2)), DNA)) for _ in range(1100)]
    pieces += [bytes(DNA[rng.integers(0, 4, size=int(rng.integers(30, 60)))]) for _ in range(900)]
    order = rng.permutation(len(pieces))
    col = sd.from_strings([pieces[i] for i in order])
    K, r, z, m = 3, 2, 3, 2
    ref = _oracle_join(oracle_lib, col, K, r, z, m, 13, 32)
    _say(f"dense cluster n={col.n} candidates={len(ref.cand)}")
    for mode in _each_verify_mode(ctx):
        res = ctx.join(col.chars, col.offsets, K, r, z, m, seed=13, L=32)
        _assert_join_equal(res, ref)
        assert res.n_candidates == len(ref.cand)


def test_candidates_above_65536_strings(ej, ctx, oracle_lib):
    """70,000 strings: pair codes need more than 32 bits, and the grouped
    de-duplication works on the codes' low bits; the join equals the
    oracle's."""
    col = sd.clusters(71, 23000, lambda rr, b: rr.integers(1, 6), lambda rr: rr.integers(12, 31),
                      lambda rr, LL: rr.poisson(1))
    assert col.n > 65536
    K, r, z, m = 2, 1, 3, 16
    ref = _oracle_join(oracle_lib, col, K, r, z, m, 3, 24)
    _say(f"n={col.n} candidates={len(ref.cand)}")
    for mode in (0, 2):
        ctx.tune_set("verify_mode", mode)
        try:
            res = ctx.join(col.chars, col.offsets, K, r, z, m, seed=3, L=24)
        finally:
            ctx.tune_set("verify_mode", 0)
        _assert_join_equal(res, ref)
        assert res.n_candidates == len(ref.cand)



def test_join_top_bit_groups_span_tiles(ej, ctx, oracle_lib):
    """The join's pair walk ends a group where the sorted top key bits change.
    With the bucketing cut to 1, 3 or 8 top bits, groups mix many different
    full keys and a 1-bit group (about 2,100 entries per table) spans several
    1,024-entry workgroup tiles; candidates and results stay the oracle's."""
    col = sd.clusters(19, 1700, lambda rr, b: rr.integers(1, 5), lambda rr: rr.integers(20, 41),
                      lambda rr, LL: rr.poisson(1))
    K, r, z, m = 3, 1, 2, 4
    ref = _oracle_join(oracle_lib, col, K, r, z, m, 19, 16)
    old = ctx.tune_get("bucket_key_bits")
    try:
        for bits in (1, 3, 8, 0):
            _say(f"join bucket_key_bits={bits} n={col.n} candidates={len(ref.cand)}")
            ctx.tune_set("bucket_key_bits", bits)
            res = ctx.join(col.chars, col.offsets, K, r, z, m, seed=19, L=16)
            _assert_join_equal(res, ref)
    finally:
        ctx.tune_set("bucket_key_bits", old)

# ------------------------------------------------------------ edge cases ----

def test_edge_cases(ej, ctx, oracle_lib):
    cases = [
        ("empty set", []),
        ("one string", [b"ACGT"]),
        ("all empty", [b"", b"", b""]),
        ("one letter", [b"AAAA", b"AAA", b"AAAAA", b"", b"A"]),
        ("duplicates", [b"ACGTACGT"] * 5 + [b"ACGAACGT"]),
    ]
    for name, S in cases:
        col = sd.from_strings(S)
        for K in (0, 1, 3):
            ref = _oracle_join(oracle_lib, col, K, 3, 4, 2, 11)
            for mode in _each_verify_mode(ctx):
                _say(f"edge {name} K={K} mode={mode}")
                res = ctx.join(col.chars, col.offsets, K, 3, 4, 2, seed=11)
                _assert_join_equal(res, ref)


def test_invalid_arguments_are_rejected(ej, ctx):
    col = sd.from_strings([b"ACGT", b"ACGA"])
    with pytest.raises(ej.EmbedJoinError) as e:
        ctx.join(col.chars, col.offsets, 2, 0, 4, 4)
    assert e.value.status == ej.EJ_EINVAL
    with pytest.raises(ej.EmbedJoinError) as e:
        ctx.join(col.chars, col.offsets, 3000, 1, 1, 1)
    assert e.value.status == ej.EJ_EUNSUPPORTED
    bad = np.array([0, 4, 2], dtype=np.uint64)
    with pytest.raises(ej.EmbedJoinError) as e:
        ctx.join(col.chars, bad, 2, 1, 1, 1)
    assert e.value.status == ej.EJ_EINVAL
    import torch
    chars, offs = to_device(col)
    with pytest.raises(ej.EmbedJoinError) as e:
        ctx.verify(chars, offs, torch.tensor([(5 << 32) | 1], dtype=torch.int64, device="cuda"), 2)
    assert e.value.status == ej.EJ_EINVAL
    # the context still works after errors
    res = ctx.join(col.chars, col.offsets, 1, 2, 2, 2)
    assert res.pairs.tolist() == [[0, 1]]


# -------------------------------------------------- the tiny workload ----

def test_tiny_dna_workload_full(ej, ctx, oracle_lib):
    """2,000 DNA strings (200 bases x 10 copies, Poisson(30) edits), K=50,
    r=3, z=7, m=24 -- the small configuration, in full."""
    col, prm = sd.tiny_dna(0)
    ref = _oracle_join(oracle_lib, col, prm["K"], prm["r"], prm["z"], prm["m"], 0)
    _say(f"tiny workload n={col.n} candidates={len(ref.cand)}")
    res = ctx.join(col.chars, col.offsets, prm["K"], prm["r"], prm["z"], prm["m"], seed=0)
    _assert_join_equal(res, ref)
    chars, offs = to_device(col)
    for mode in _each_verify_mode(ctx):
        res2 = ctx.join(chars, offs, prm["K"], prm["r"], prm["z"], prm["m"], seed=0)
        _assert_join_equal(res2, ref)


def test_tiny_dna_recall_point(ej, ctx, oracle_lib):
    """A permissive parameter point on the tiny workload: output still equals
    the oracle's, and every output pair is a true pair."""
    col, prm = sd.tiny_dna(0, n_bases=60)
    K = prm["K"]
    ref = _oracle_join(oracle_lib, col, K, 7, 16, 8, 3, 64)
    res = ctx.join(col.chars, col.offsets, K, 7, 16, 8, seed=3, L=64)
    _say(f"tiny recall point candidates={res.n_candidates}")
    _assert_join_equal(res, ref)
    S = col.strings()
    for (a, b), d in zip(res.pairs.tolist(), res.dist.tolist()):
        assert oracle_lib.ed_full(S[a], S[b]) == d <= K


# ------------------------------------------------------- launch knobs ----

@pytest.mark.parametrize("c1", [0, 32, 64, 160])
def test_verify_two_pass_resume(ej, ctx, oracle_lib, c1):
    """Pass 1 stops after c1 columns and pass 2 resumes the undecided pairs
    from their saved state: same distances as one pass and as the oracle."""
    import torch
    rng = np.random.default_rng(c1 + 1)
    col = sd.clusters(200 + c1, 10, lambda rr, b: 4, lambda rr: rr.integers(150, 700),
                      lambda rr, LL: rr.poisson(25))
    n = col.n
    a = rng.integers(0, n, size=300)
    b = rng.integers(0, n, size=300)
    codes = (a.astype(np.uint64) << np.uint64(32)) | b.astype(np.uint64)
    chars, offs = to_device(col)
    old = (ctx.tune_get("verify_pass1_cols"), ctx.tune_get("verify_wpl"))
    try:
        ctx.tune_set("verify_pass1_cols", c1)
        for K in (3, 60, 130, 200):
            want = oracle_lib.verify_pairs(col.chars, col.offsets, codes, K)
            for wpl in (1, 2, 4):
                ctx.tune_set("verify_wpl", wpl)
                _say(f"two-pass c1={c1} K={K} wpl={wpl}")
                got = ctx.verify(chars, offs, torch.from_numpy(codes.astype(np.int64)).cuda(), K)
                assert got.cpu().numpy().astype(np.uint32).tolist() == want.tolist()
    finally:
        ctx.tune_set("verify_pass1_cols", old[0])
        ctx.tune_set("verify_wpl", old[1])


def test_knobs_do_not_change_results(ej, ctx, oracle_lib):
    col = sd.clusters(9, 40, lambda rr, b: rr.integers(1, 5), lambda rr: rr.integers(100, 900),
                      lambda rr, LL: rr.poisson(12))
    K, r, z, m, L = 40, 4, 6, 4, 64
    ref = _oracle_join(oracle_lib, col, K, r, z, m, 5, L)
    knobs = [("radix_bits", 4), ("radix_bits", 11), ("bucket_key_bits", 5),
             ("embed_lds_budget", 8192), ("verify_lds_budget", 4096),
             ("verify_blocks_per_cu", 1), ("verify_pass1_cols", 64), ("verify_ring", 0),
             ("verify_ring", 2), ("verify_mode", 1), ("verify_wpl", 1),
             ("verify_wpl", 4), ("verify_len_order", 0), ("verify_order", 0)]
    # the persistent forms with and without the multiplicity order
    try:
        for mode, split in ((1, 0), (2, 0), (2, 1), (2, 4)):
            ctx.tune_set("verify_mode", mode)
            ctx.tune_set("verify_split", split)
            for order in (0, 1):
                ctx.tune_set("verify_order", order)
                _say(f"persistent verification mode={mode} split={split} order={order}")
                _assert_join_equal(ctx.join(col.chars, col.offsets, K, r, z, m, seed=5, L=L),
                                   ref)
    finally:
        ctx.tune_set("verify_mode", 0)
        ctx.tune_set("verify_order", 1)
        ctx.tune_set("verify_split", 0)
    for name, val in knobs:
        old = ctx.tune_get(name)
        try:
            ctx.tune_set(name, val)
            _say(f"knob {name}={val}")
            res = ctx.join(col.chars, col.offsets, K, r, z, m, seed=5, L=L)
            _assert_join_equal(res, ref)
        finally:
            ctx.tune_set(name, old)
    with pytest.raises(ej.EmbedJoinError):
        ctx.tune_set("radix_bits", 3)
    with pytest.raises(ej.EmbedJoinError):
        ctx.tune_set("verify_split", 3)
    with pytest.raises(ej.EmbedJoinError):
        ctx.tune_set("no_such_knob", 1)


def test_autotune_keeps_results(ej, ctx, oracle_lib):
    """The autotuner picks launch knobs on the caller's workload; the join
    at the chosen setting still equals the oracle's."""
    col = sd.clusters(31, 30, lambda rr, b: 4, lambda rr: rr.integers(200, 700),
                      lambda rr, LL: rr.poisson(15))
    K, r, z, m, L = 60, 4, 6, 4, 48
    ref = _oracle_join(oracle_lib, col, K, r, z, m, 8, L)
    chars, offs = to_device(col)
    before = ctx.knobs()
    try:
        _say("autotune")
        best, knobs = ctx.autotune(chars, offs, K, r, z, m, seed=8, L=L, reps=1)
        assert best > 0
        assert knobs["verify_mode"] in (0, 1, 2, 3) and 4 <= knobs["radix_bits"] <= 11
        res = ctx.join(chars, offs, K, r, z, m, seed=8, L=L)
        _assert_join_equal(res, ref)
    finally:
        for k, v in before.items():
            ctx.tune_set(k, v)


def test_autotune_survives_settings_that_cannot_run(ej, ctx, oracle_lib):
    """Strings of 350,000 letters: their whole-pattern match masks do not fit
    in LDS, so the mask-layout knob 0 cannot run them.  A join at that
    setting fails cleanly and leaves the context usable (graph mode and
    timers reset); the autotuner scores such a trial as infinitely slow and
    still returns a working setting."""
    col = sd.clusters(41, 2, lambda rr, b: 3, lambda rr: rr.integers(350000, 352000),
                      lambda rr, LL: rr.poisson(25))
    K, r, z, m, L = 60, 2, 2, 4, 64
    ref = _oracle_join(oracle_lib, col, K, r, z, m, 4, L)
    chars, offs = to_device(col)
    before = ctx.knobs()
    try:
        for mode in (0, 1):
            ctx.tune_set("verify_mode", mode)
            ctx.tune_set("verify_ring", 0)
            _say(f"whole-pattern masks of 350k-letter strings, mode {mode}")
            with pytest.raises(ej.EmbedJoinError) as e:
                ctx.join(chars, offs, K, r, z, m, seed=4, L=L, flags=ej.FLAG_GRAPH)
            assert e.value.status == ej.EJ_EUNSUPPORTED
            ctx.tune_set("verify_ring", 1)
            _assert_join_equal(ctx.join(chars, offs, K, r, z, m, seed=4, L=L), ref)
        for k, v in before.items():
            ctx.tune_set(k, v)
        _say("autotune over long strings")
        ctx.autotune(chars, offs, K, r, z, m, seed=4, L=L, reps=1)
        knobs = ctx.knobs()
        flags = ej.FLAG_GRAPH if knobs["verify_mode"] >= 1 else 0
        _assert_join_equal(ctx.join(chars, offs, K, r, z, m, seed=4, L=L, flags=flags), ref)
    finally:
        for k, v in before.items():
            ctx.tune_set(k, v)


def test_result_left_on_the_device(ej, ctx, oracle_lib):
    """FLAG_DEVICE_OUT: the same pairs and distances, handed over in device
    memory (torch tensors); a later join does not change them; an empty
    result works too."""
    col = sd.clusters(17, 30, lambda rr, b: 4, lambda rr: rr.integers(200, 600),
                      lambda rr, LL: rr.poisson(10))
    K, r, z, m, L = 40, 4, 6, 4, 48
    ref = _oracle_join(oracle_lib, col, K, r, z, m, 3, L)
    chars, offs = to_device(col)
    for mode in _each_verify_mode(ctx):
        _say(f"device-resident result, mode {mode}")
        res = ctx.join(chars, offs, K, r, z, m, seed=3, L=L,
                       flags=ej.FLAG_DEVICE_OUT | ej.FLAG_TIMING)
        assert res.pairs_device.is_cuda and res.count == len(ref.out)
        other = ctx.join(chars, offs, 0, r, z, m, seed=3, L=L, flags=ej.FLAG_DEVICE_OUT)
        _assert_join_equal(res, ref)
        assert other.count <= res.count
        plus = ctx.join_plus(chars, offs, K, r, z, m, delta=20, T=2, seed=3, L=L,
                             flags=ej.FLAG_DEVICE_OUT)
        pref = oracle_lib.join_plus(col.chars, col.offsets, K, r, z, m, delta=20, T=2, seed=3,
                                    L=L)
        assert pairs_to_codes(plus.pairs).tolist() == pref.out.tolist()
    none = ctx.join(chars, offs, 0, r, z, m, seed=3, L=L, flags=ej.FLAG_DEVICE_OUT)
    assert none.count == len(_oracle_join(oracle_lib, col, 0, r, z, m, 3, L).out)
    assert none.pairs.shape == (none.count, 2)


@pytest.mark.parametrize("letters,K", [("protein", 0), ("protein", 31), ("protein", 100),
                                       ("protein", 254), ("protein", 300), ("wide", 63),
                                       ("wide", 160)])
def test_lane_form_wide_alphabets(ej, ctx, oracle_lib, letters, K):
    """The lane form (one pair per lane, band in registers) over 25 and 32
    letters, band widths of 1 to 8 words (and beyond: the other forms take
    over), equals the oracle's threshold distances."""
    import torch
    alpha = sd.PROTEIN25 if letters == "protein" else bytes(range(65, 97))
    probs = sd.zipf_probs(25, 1.1) if letters == "protein" else None
    col = sd.clusters(300 + K, 20, lambda rr, b: 5, lambda rr: rr.integers(0, 2 * K + 200),
                      lambda rr, LL: rr.poisson(max(1, K // 3)), letters=alpha, probs=probs)
    rng = np.random.default_rng(K + 1)
    a = rng.integers(0, col.n, size=500)
    b = rng.integers(0, col.n, size=500)
    codes = (a.astype(np.uint64) << np.uint64(32)) | b.astype(np.uint64)
    want = oracle_lib.verify_pairs(col.chars, col.offsets, codes, K)
    chars, offs = to_device(col)
    old = ctx.knobs()
    try:
        ctx.tune_set("verify_mode", 2)
        ctx.tune_set("verify_split", 0)
        _say(f"lane form {letters} K={K}")
        got = ctx.verify(chars, offs, torch.from_numpy(codes.astype(np.int64)).cuda(), K)
        assert got.cpu().numpy().astype(np.uint32).tolist() == want.tolist()
        res = ctx.join(chars, offs, K, 3, 5, 4, seed=2, L=64, flags=ej.FLAG_TIMING)
        _assert_join_equal(res, _oracle_join(oracle_lib, col, K, 3, 5, 4, 2, 64))
        if K <= 254 and res.n_candidates:
            assert res.verify_form == 2
        # grouped by pattern (bands up to 16 words)
        ctx.tune_set("verify_mode", 3)
        _say(f"grouped form {letters} K={K}")
        got = ctx.verify(chars, offs, torch.from_numpy(codes.astype(np.int64)).cuda(), K)
        assert got.cpu().numpy().astype(np.uint32).tolist() == want.tolist()
        res = ctx.join(chars, offs, K, 3, 5, 4, seed=2, L=64, flags=ej.FLAG_TIMING)
        _assert_join_equal(res, _oracle_join(oracle_lib, col, K, 3, 5, 4, 2, 64))
        if K <= 510 and res.n_candidates:
            assert res.verify_form == 4
    finally:
        for k, v in old.items():
            ctx.tune_set(k, v)


def test_graph_replays_match_eager(ej, ctx, oracle_lib):
    """Persistent verification (both forms) captured into a HIP graph: the
    first join captures, later joins of the same shape replay it, with eager
    joins and synchronisations in between; every replay equals the oracle."""
    import torch
    col = sd.clusters(41, 40, lambda rr, b: 4, lambda rr: rr.integers(150, 600),
                      lambda rr, LL: rr.poisson(10))
    K, r, z, m, L = 50, 4, 6, 4, 48
    ref = _oracle_join(oracle_lib, col, K, r, z, m, 4, L)
    chars, offs = to_device(col)
    col2 = sd.clusters(42, 20, lambda rr, b: 3, lambda rr: rr.integers(100, 300),
                       lambda rr, LL: rr.poisson(5))
    ref2 = _oracle_join(oracle_lib, col2, 20, r, z, m, 4, L)
    old = ctx.tune_get("verify_mode")
    try:
        for mode in (0, 1, 2, 3):
            ctx.tune_set("verify_mode", mode)
            ran = []
            for i in range(4):
                _say(f"graph replay mode={mode} {i}")
                res = ctx.join(chars, offs, K, r, z, m, seed=4, L=L, flags=ej.FLAG_GRAPH)
                _assert_join_equal(res, ref)
                ran.append(res.graph)
                eager = ctx.join(chars, offs, K, r, z, m, seed=4, L=L)
                _assert_join_equal(eager, ref)
                assert eager.graph == 0
                torch.cuda.synchronize()
            # host-sized, then device-sized uncaptured, then graph replays
            assert ran[0] == 0 and ran[-1] == 2, ran
            # de-duplication by a sort, host-sized and replayed
            ctx.tune_set("dedup_sort", 1)
            for i in range(4):
                res = ctx.join(chars, offs, K, r, z, m, seed=4, L=L, flags=ej.FLAG_GRAPH)
                _assert_join_equal(res, ref)
                _assert_join_equal(ctx.join(chars, offs, K, r, z, m, seed=4, L=L), ref)
            assert res.graph == 2
            ctx.tune_set("dedup_sort", 0)
            # a different shape in between, then the first shape again
            _assert_join_equal(ctx.join(col2.chars, col2.offsets, 20, r, z, m, seed=4, L=L,
                                         flags=ej.FLAG_GRAPH), ref2)
            _assert_join_equal(ctx.join(chars, offs, K, r, z, m, seed=4, L=L,
                                        flags=ej.FLAG_GRAPH), ref)
    finally:
        ctx.tune_set("verify_mode", old)


def test_whole_join_graph_capacity_overflow(ej, ctx, oracle_lib):
    """The whole join replayed from a graph, then new contents in the same
    device buffers (same lengths, so the same shape) with many more
    candidates than the capacities taken from the first contents: that join
    is redone host-sized, the capacities grow, later joins replay again; every
    result equals the oracle, in host and device output."""
    import torch
    rng = np.random.default_rng(5)
    DNA = np.frombuffer(b"ACGT", np.uint8)
    lens = rng.integers(80, 200, size=600)
    # few candidates: unrelated random strings
    sparse = sd.from_strings([bytes(DNA[rng.integers(0, 4, size=int(x))]) for x in lens])
    # many candidates: 4 groups of prefixes of one string each, same lengths
    bases = [DNA[rng.integers(0, 4, size=220)] for _ in range(4)]
    dense = sd.from_strings([bytes(bases[i % 4][:int(x)]) for i, x in enumerate(lens)])
    assert np.array_equal(sparse.offsets, dense.offsets)
    K, r, z, m, L = 30, 3, 4, 8, 40
    ref_s = _oracle_join(oracle_lib, sparse, K, r, z, m, 9, L)
    ref_d = _oracle_join(oracle_lib, dense, K, r, z, m, 9, L)
    assert len(ref_d.cand) > 4 * len(ref_s.cand) + 10000 and ref_d.n_raw > 100 * ref_s.n_raw
    chars, offs = to_device(sparse)
    dchars = torch.from_numpy(dense.chars.copy()).cuda()
    for mode, dsort in ((1, 0), (2, 0), (0, 1), (3, 0)):
        ctx.tune_set("verify_mode", mode)
        ctx.tune_set("dedup_sort", dsort)
        chars.copy_(torch.from_numpy(sparse.chars.copy()).cuda())
        for i in range(3):
            res = ctx.join(chars, offs, K, r, z, m, seed=9, L=L, flags=ej.FLAG_GRAPH)
            _assert_join_equal(res, ref_s)
        assert res.graph == 2
        chars.copy_(dchars)
        torch.cuda.synchronize()
        _say(f"overflow mode={mode}")
        res = ctx.join(chars, offs, K, r, z, m, seed=9, L=L, flags=ej.FLAG_GRAPH)
        _assert_join_equal(res, ref_d)
        assert res.graph == 0
        for i in range(3):
            res = ctx.join(chars, offs, K, r, z, m, seed=9, L=L,
                           flags=ej.FLAG_GRAPH | ej.FLAG_DEVICE_OUT)
            _assert_join_equal(res, ref_d)
        assert res.graph == 2
    ctx.tune_set("verify_mode", 0)
    ctx.tune_set("dedup_sort", 0)


def test_grouped_form_many_partners_per_pattern(ej, ctx, oracle_lib):
    """Grouped by pattern: runs of one pattern longer than a chunk (64 pairs),
    patterns of very different lengths in one launch, pairs whose lengths
    differ by more than K, empty texts, per-pair thresholds and a device
    count (through the whole-join graph)."""
    import torch
    rng = np.random.default_rng(12)
    DNA = np.frombuffer(b"ACGT", np.uint8)
    # patterns on both sides of 1,024 letters (the two launches of the form)
    base = DNA[rng.integers(0, 4, size=1500)]
    strings = [bytes(sd.mutate(rng, base[:int(rng.integers(600, 1500))], int(rng.poisson(20)),
                               DNA)) for _ in range(150)]
    strings += [bytes(DNA[rng.integers(0, 4, size=int(x))]) for x in rng.integers(0, 120, 60)]
    strings += [b"", b"A", b""]
    col = sd.from_strings(strings)
    n = col.n
    a = np.repeat(np.arange(5), 200)            # five patterns with 200 partners each
    # pairs of empty strings (an empty pattern) among them
    b = rng.integers(0, n, size=a.size)
    a2 = rng.integers(0, n, size=800)
    b2 = rng.integers(0, n, size=800)
    aa = np.concatenate([a, a2, [n - 3, n - 1, n - 3]])
    bb = np.concatenate([b, b2, [n - 1, n - 3, n - 2]])
    codes = (aa.astype(np.uint64) << np.uint64(32)) | bb.astype(np.uint64)
    chars, offs = to_device(col)
    d_codes = torch.from_numpy(codes.astype(np.int64)).cuda()
    old = ctx.knobs()
    try:
        ctx.tune_set("verify_mode", 3)
        for K in (0, 40, 200, 510):
            want = oracle_lib.verify_pairs(col.chars, col.offsets, codes, K)
            _say(f"grouped many partners K={K}")
            got = ctx.verify(chars, offs, d_codes, K).cpu().numpy()
            assert got.astype(np.uint32).tolist() == want.tolist()
        Kq = rng.integers(0, 300, size=codes.size).astype(np.int32)
        want = np.array([oracle_lib.verify_pairs(col.chars, col.offsets, codes[i:i + 1], int(k))[0]
                         for i, k in enumerate(Kq)])
        got = ctx.verify(chars, offs, d_codes, 0, d_Kq=torch.from_numpy(Kq).cuda()).cpu().numpy()
        assert got.astype(np.uint32).tolist() == want.tolist()
        K, r, z, m, L = 60, 3, 5, 6, 64
        ref = _oracle_join(oracle_lib, col, K, r, z, m, 6, L)
        for i in range(4):
            res = ctx.join(chars, offs, K, r, z, m, seed=6, L=L, flags=ej.FLAG_GRAPH)
            _assert_join_equal(res, ref)
        assert res.graph == 2
    finally:
        for k, v in old.items():
            ctx.tune_set(k, v)


def test_grouped_form_short_and_long_patterns(ej, ctx, oracle_lib):
    """Grouped by pattern over 25 letters with strings of 0..3,000 letters at
    32 waves per CU asked for: rows sized for the longest string leave room
    for fewer waves than that, so the chunks of patterns up to a length limit
    run with shorter rows and the longer ones in a second launch.  Clusters
    of each length (pairs inside them near, random pairs far), per-pair
    thresholds, and the whole-join graph (device count) in both launches."""
    import torch
    rng = np.random.default_rng(21)
    LET = np.frombuffer(b"ACDEFGHIKLMNPQRSTVWYBZXJO", np.uint8)
    strings = []
    for size in (2500, 1800, 1200, 700, 300, 90):
        bse = LET[rng.integers(0, 25, size=size)]
        strings += [bytes(sd.mutate(rng, bse, int(rng.poisson(size * 0.02)), LET))
                    for _ in range(16)]
    strings += [bytes(LET[rng.integers(0, 25, size=int(x))]) for x in rng.integers(0, 3000, 40)]
    col = sd.from_strings(strings)
    n = col.n
    ia, ib = np.triu_indices(16, 1)
    a = np.concatenate([16 * c + ia for c in range(6)] + [rng.integers(0, n, 500)])
    b = np.concatenate([16 * c + ib for c in range(6)] + [rng.integers(0, n, 500)])
    codes = (a.astype(np.uint64) << np.uint64(32)) | b.astype(np.uint64)
    chars, offs = to_device(col)
    d_codes = torch.from_numpy(codes.astype(np.int64)).cuda()
    old = ctx.knobs()
    try:
        ctx.tune_set("verify_mode", 3)
        ctx.tune_set("verify_blocks_per_cu", 32)
        for K in (0, 100, 300):
            want = oracle_lib.verify_pairs(col.chars, col.offsets, codes, K)
            _say(f"grouped short and long patterns K={K}")
            got = ctx.verify(chars, offs, d_codes, K).cpu().numpy()
            assert got.astype(np.uint32).tolist() == want.tolist()
        Kq = rng.integers(0, 200, size=codes.size).astype(np.int32)
        want = np.array([oracle_lib.verify_pairs(col.chars, col.offsets, codes[i:i + 1], int(k))[0]
                         for i, k in enumerate(Kq)])
        got = ctx.verify(chars, offs, d_codes, 0, d_Kq=torch.from_numpy(Kq).cuda()).cpu().numpy()
        assert got.astype(np.uint32).tolist() == want.tolist()
        K, r, z, m, L = 100, 3, 4, 6, 64
        ref = _oracle_join(oracle_lib, col, K, r, z, m, 8, L)
        assert len(ref.cand) > 200
        for i in range(4):
            res = ctx.join(chars, offs, K, r, z, m, seed=8, L=L, flags=ej.FLAG_GRAPH)
            _assert_join_equal(res, ref)
        assert res.graph == 2
    finally:
        for k, v in old.items():
            ctx.tune_set(k, v)


def test_candidates_in_passes(ej, ctx, oracle_lib):
    """More raw pairs than one sort may hold (the raw_limit knob lowers the
    2^32 - 2 limit): the candidate stage runs in passes over ranges of the
    pairs' smaller index, halved while a range has too many, down to single
    indexes.  The join equals the oracle's (and the one-pass join) in the
    two-pass form and in the persistent form with the multiplicity order;
    with the graph flag it stays host-sized."""
    col = sd.clusters(23, 60, lambda rr, b: rr.integers(2, 9), lambda rr: rr.integers(80, 400),
                      lambda rr, LL: rr.poisson(6))
    K, r, z, m, L = 40, 6, 8, 3, 48
    ref = _oracle_join(oracle_lib, col, K, r, z, m, 4, L)
    chars, offs = to_device(col)
    one = ctx.join(chars, offs, K, r, z, m, seed=4, L=L)
    _assert_join_equal(one, ref)
    assert one.n_raw > 2000, one.n_raw
    old = ctx.knobs()
    try:
        for limit in (500, 37, 1):
            ctx.tune_set("raw_limit", limit)
            for mode in (0, 1):
                ctx.tune_set("verify_mode", mode)
                _say(f"candidates in passes raw_limit={limit} verify_mode={mode}")
                res = ctx.join(chars, offs, K, r, z, m, seed=4, L=L)
                _assert_join_equal(res, ref)
                assert res.n_raw == one.n_raw
        for i in range(3):
            res = ctx.join(chars, offs, K, r, z, m, seed=4, L=L, flags=ej.FLAG_GRAPH)
            _assert_join_equal(res, ref)
            assert res.graph == 0
    finally:
        for k, v in old.items():
            ctx.tune_set(k, v)


def test_verified_columns_counter(ej, ctx, oracle_lib):
    """EJ_FLAG_TIMING's count of verified text columns (summed per wave, one
    atomic each): the same over repeated joins, positive, at most the total
    text length of the candidates rounded up to 32-column blocks, and at
    least the text length of every output pair (those run to their end).
    Each pair counts up to the 32-column block where it is decided, not where
    its wave stops: the two-pass form at every width counts exactly what the
    persistent form, which retires each pair at its decision, counts."""
    col = sd.clusters(51, 30, lambda rr, b: 4, lambda rr: rr.integers(100, 700),
                      lambda rr, LL: rr.poisson(8))
    K, r, z, m, L = 40, 4, 6, 4, 48
    ref = _oracle_join(oracle_lib, col, K, r, z, m, 5, L)
    lens = col.lengths().astype(np.int64)
    ca = (ref.cand >> np.uint64(32)).astype(np.int64)
    cb = (ref.cand & np.uint64(0xFFFFFFFF)).astype(np.int64)
    text = np.minimum(lens[ca], lens[cb])
    oa = (ref.out >> np.uint64(32)).astype(np.int64)
    ob = (ref.out & np.uint64(0xFFFFFFFF)).astype(np.int64)
    chars, offs = to_device(col)
    counts = {}
    for mode in _each_verify_mode(ctx):
        a = ctx.join(chars, offs, K, r, z, m, seed=5, L=L, flags=ej.FLAG_TIMING)
        b = ctx.join(chars, offs, K, r, z, m, seed=5, L=L, flags=ej.FLAG_TIMING)
        _assert_join_equal(a, ref)
        _say(f"verified columns mode={mode}: {a.verify_columns}")
        assert a.verify_columns == b.verify_columns > 0
        assert a.verify_columns <= int((((text + 31) // 32) * 32).sum())
        assert a.verify_columns >= int(np.minimum(lens[oa], lens[ob]).sum())
        counts[mode] = a.verify_columns
    assert counts[0] == counts["0w2"] == counts["0w4"] == counts[1]
    # a first pass of 64 columns: pairs resumed in pass 2 count once
    old = (ctx.tune_get("verify_mode"), ctx.tune_get("verify_pass1_cols"))
    try:
        ctx.tune_set("verify_mode", 0)
        ctx.tune_set("verify_pass1_cols", 64)
        a = ctx.join(chars, offs, K, r, z, m, seed=5, L=L, flags=ej.FLAG_TIMING)
        _assert_join_equal(a, ref)
        _say(f"verified columns two passes of 64 + rest: {a.verify_columns}")
        assert a.verify_columns == counts[1]
    finally:
        ctx.tune_set("verify_mode", old[0])
        ctx.tune_set("verify_pass1_cols", old[1])
