"""Distortion diagnostics and automated calibration on the GPU:
ej_embed_hamming against the oracle's embedding Hamming distances (bit for
bit: whole strings and minimum over suffix pairs, alphabets on both sides of
32 letters), and ej_calibrate's predictions against the closed form written
out here from the oracle's distances, and against the recall a join at the
chosen point then measures."""
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


def _sample_pairs(col, rng, n_planted, n_random):
    planted = sd.planted_pairs(col)
    pick = planted[rng.choice(len(planted), size=min(n_planted, len(planted)), replace=False)]
    rand = rng.integers(0, col.n, size=(n_random, 2))
    rand = rand[rand[:, 0] != rand[:, 1]]
    allp = np.concatenate([pick, np.sort(rand, axis=1)])
    return pairs_to_codes(allp)


LETTERS40 = bytes(range(48, 88))


@pytest.mark.parametrize("alphabet,delta,L", [("dna", 0, 0), ("dna", 15, 96), ("protein", 0, 64),
                                              ("wide", 0, 0), ("wide", 20, 128)])
def test_embed_hamming_matches_oracle(ej, ctx, oracle_lib, alphabet, delta, L):
    import torch
    letters = {"dna": sd.DNA, "protein": sd.PROTEIN25, "wide": LETTERS40}[alphabet]
    col = sd.clusters(5, 30, lambda rr, b: 4, lambda rr: rr.integers(20, 300),
                      lambda rr, LL: rr.poisson(4), letters=letters)
    rng = np.random.default_rng(8)
    codes = _sample_pairs(col, rng, 80, 80)
    codes = np.concatenate([codes, np.array([0, (3 << 32) | 3], dtype=np.uint64)])
    K, r, seed = 45, 5, 17
    want = oracle_lib.embed_hamming(col.chars, col.offsets, codes, r, L=L, seed=seed, K=K,
                                    delta=delta)
    chars, offs = to_device(col)
    _say(f"embed_hamming {alphabet} delta={delta} L={L}")
    got = ctx.embed_hamming(chars, offs, torch.from_numpy(codes.astype(np.int64)).cuda(), r, L=L,
                            seed=seed, K=K, delta=delta).cpu().numpy()
    assert got.astype(np.uint32).tolist() == want.tolist()


def _closed_form(ham, L, r, z, m, T=1):
    """P[candidate] per pair from its per-seed Hamming distances: the number
    of agreeing tables is a sum of Binomial(z, (1 - H_l/L)^m) over seeds."""
    from math import comb
    q = (1.0 - ham[:, :r] / L) ** m
    if T == 1:
        return 1.0 - np.prod((1.0 - q) ** z, axis=1)
    out = []
    for row in q:
        dist = np.zeros(T + 1)
        dist[0] = 1.0
        for p in row:
            b = np.array([comb(z, k) * p ** k * (1 - p) ** (z - k) for k in range(z + 1)])
            nx = np.zeros(T + 1)
            for c in range(T + 1):
                for k in range(z + 1):
                    nx[min(T, c + k)] += dist[c] * b[k]
            dist = nx
        out.append(dist[T])
    return np.array(out)


def test_calibration_predictions_and_chosen_point(ej, ctx, oracle_lib):
    """The tiny DNA workload (2,000 strings, K=50): the table of predicted
    recall and false rate equals the closed form evaluated from the oracle's
    Hamming distances; the chosen point reaches the target; a join there
    measures a recall close to the prediction."""
    import torch
    col, prm = sd.tiny_dna(0)
    K = prm["K"]
    rng = np.random.default_rng(3)
    codes = _sample_pairs(col, rng, 400, 400)
    chars, offs = to_device(col)
    dp = torch.from_numpy(codes.astype(np.int64)).cuda()
    zl, ml, Ll = [4, 8, 16], [8, 12, 16, 24], [64, 128, 0]
    r_max, seed = 12, 0
    _say("calibrate tiny workload")
    cal = ctx.calibrate(chars, offs, dp, K, r_max, zl, ml, Ll, target_recall=0.99, seed=seed,
                        want_table=True)
    d = oracle_lib.verify_pairs(col.chars, col.offsets, codes, K)
    sim = d <= K
    assert cal["n_similar"] == int(sim.sum()) and cal["n_dissimilar"] == int((~sim).sum())
    tab = cal["table"]
    for li, Lr in enumerate(Ll):
        L = oracle_lib.effective_L(col.offsets, Lr)
        ham = oracle_lib.embed_hamming(col.chars, col.offsets, codes, r_max, L=L,
                                       seed=seed).astype(np.float64)
        for r in (1, 5, r_max):
            for zi, z in enumerate(zl):
                for mi, m in enumerate(ml):
                    pc = _closed_form(ham, L, r, z, m)
                    assert abs(tab[li, r - 1, zi, mi, 0] - pc[sim].mean()) < 1e-9
                    assert abs(tab[li, r - 1, zi, mi, 1] - pc[~sim].mean()) < 1e-9
    assert cal["r"] > 0 and cal["recall"] >= 0.99
    assert cal["recall"] == tab[Ll.index(cal["L"]) if cal["L"] in Ll else 2,
                                cal["r"] - 1, zl.index(cal["z"]), ml.index(cal["m"]), 0]
    # the chosen point has the least predicted work among those reaching 0.99
    ok = tab[..., 0] >= 0.99
    assert abs(cal["work"] - tab[..., 2][ok].min()) < 1e-6 * cal["work"]
    # measured recall of a join at the chosen point (planted pairs within K)
    res = ctx.join(chars, offs, K, cal["r"], cal["z"], cal["m"], seed=seed, L=cal["L"])
    planted = sd.planted_pairs(col)
    pcodes = pairs_to_codes(planted)
    within = pcodes[oracle_lib.verify_pairs(col.chars, col.offsets, pcodes, K) <= K]
    found = np.isin(within, res.codes).mean()
    _say(f"chosen {cal['r'], cal['z'], cal['m'], cal['L']} predicted {cal['recall']:.4f} "
         f"measured {found:.4f}")
    assert found >= 0.97 and abs(found - cal["recall"]) < 0.03


def test_calibration_plus_lower_bound(ej, ctx, oracle_lib):
    """EmbedJoin+ (T=2, three suffixes): the predicted recall evaluates the
    closest suffix pair only, so it never exceeds the recall a join at that
    point measures (beyond sampling noise), and it equals the closed form
    over the oracle's minimum-over-suffixes distances."""
    import torch
    col, _ = sd.shifted_reads(2, n_bases=60, copies=5, base_len=(300, 500), shift=40,
                              edit_rate=0.01)
    K, delta, T = 60, 20, 2
    rng = np.random.default_rng(4)
    codes = _sample_pairs(col, rng, 400, 200)
    chars, offs = to_device(col)
    dp = torch.from_numpy(codes.astype(np.int64)).cuda()
    zl, ml, Ll = [6, 12], [6, 10], [96]
    _say("calibrate EmbedJoin+")
    cal = ctx.calibrate(chars, offs, dp, K, 6, zl, ml, Ll, target_recall=0.9, seed=1,
                        delta=delta, T=T, want_table=True)
    d = oracle_lib.verify_pairs(col.chars, col.offsets, codes, K)
    sim = d <= K
    ham = oracle_lib.embed_hamming(col.chars, col.offsets, codes, 6, L=96, seed=1, K=K,
                                   delta=delta).astype(np.float64)
    tab = cal["table"]
    for r in (1, 6):
        pc = _closed_form(ham, 96, r, zl[1], ml[0], T=T)
        assert abs(tab[0, r - 1, 1, 0, 0] - pc[sim].mean()) < 1e-9
    pick = (6, zl[1], ml[0])
    res = ctx.join_plus(chars, offs, K, *pick, delta=delta, T=T, seed=1, L=96)
    pcodes = codes[sim]
    found = np.isin(pcodes, res.codes).mean()
    _say(f"plus predicted {tab[0, 5, 1, 0, 0]:.4f} measured on the sample {found:.4f}")
    assert found >= tab[0, 5, 1, 0, 0] - 0.05


def test_calibration_with_short_pass(ej, ctx, oracle_lib):
    """exact_len: sample pairs whose strings are both no longer than it count
    as candidates with certainty; the others keep the closed form."""
    import torch
    col = sd.clusters(9, 30, lambda rr, b: 3, lambda rr: rr.integers(30, 400),
                      lambda rr, LL: rr.poisson(0.05 * LL))
    rng = np.random.default_rng(9)
    codes = _sample_pairs(col, rng, 150, 250)
    chars, offs = to_device(col)
    dp = torch.from_numpy(codes.astype(np.int64)).cuda()
    K, S, zl, ml, Ll = 60, 150, [4, 8], [6, 12], [64]
    cal = ctx.calibrate(chars, offs, dp, K, 4, zl, ml, Ll, target_recall=0.9, seed=2,
                        want_table=True, exact_len=S)
    d = oracle_lib.verify_pairs(col.chars, col.offsets, codes, K)
    sim = d <= K
    lens = col.lengths()
    a = (codes >> np.uint64(32)).astype(np.int64)
    b = (codes & np.uint64(0xFFFFFFFF)).astype(np.int64)
    short = (lens[a] <= S) & (lens[b] <= S)
    assert short.any() and (~short).any()
    ham = oracle_lib.embed_hamming(col.chars, col.offsets, codes, 4, L=64,
                                   seed=2).astype(np.float64)
    for r in (1, 4):
        for zi, z in enumerate(zl):
            for mi, m in enumerate(ml):
                pc = np.where(short, 1.0, _closed_form(ham, 64, r, z, m))
                assert abs(cal["table"][0, r - 1, zi, mi, 0] - pc[sim].mean()) < 1e-9
                assert abs(cal["table"][0, r - 1, zi, mi, 1] - pc[~sim].mean()) < 1e-9
