"""Benchmark of the EmbedJoin hot path on one MI355X.

A step is one complete self-join (A0-A6: preparation, CGK walk + keys,
bucketing, candidate pairs, verification, output) of a device-resident
synthetic string collection.  Prints one JSON line: the headline workload
(20,000 DNA strings, K=500, at its recall-calibrated point) in the batched
form, beside the plain per-stage form, and the other workloads as keys of
their own (tiny, uneven, protein, plus, serving) plus the oracle's CPU
baseline.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--legs tiny,uneven,...]
"""
import argparse
import json
import multiprocessing
import os
import platform
import shutil
import sys
import tempfile
import time
from concurrent.futures import ProcessPoolExecutor, ThreadPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("end-to-end join sec & verified candidate pairs/s at recall≥0.99; "
          "query p99 ms")
# Integer VALU peak from the unit counts and clock: 256 CUs x 4 SIMDs x 32
# lanes per cycle x 2.4 GHz = 78.6 T lane-ops/s, the rate of the fp32 vector
# figure (157.3 TFLOP/s counts an FMA as 2).  The probe kernel measures it for
# the full-rate integer instructions (v_add_u32, v_xor_b32, v_bitop3_b32 with
# register operands: a wave64 instruction every 2 cycles per SIMD); a second
# class (v_alignbit_b32, the carry adds, compares, DPP moves, v_bcnt, v_add3)
# issues at half that rate (4 cycles), 39.3 T.
MI355X_INT32_LANE_OPS = 256 * 4 * 32 * 2.4e9
MI355X_INT32_LANE_OPS_HALF = 256 * 4 * 16 * 2.4e9

# Work units of verification, in 32-bit integer lane operations per 32-cell
# word of the K+1 band (diagonals a threshold-K distance needs):
#  - the recurrence unit: Myers' step is 10 gfx950 instructions (the match
#    word, Xv, Eq&Pv, the add, Xh/Ph/Mh as 3-input logic, the one-bit shift,
#    Pv, Mv) -- the method's own work;
#  - the unit of the work estimate the build started from: about 20 per word,
#    which also counts the cross-word carry and band shift of a band split
#    over lanes.
OPS_PER_WORD_STEP = 10
SURVEY_OPS_PER_WORD = 20
OPS_PER_WALK_STEP = 3    # walk: read the symbol, select its pi bit, advance
VERIFY_KERNEL = {0: "k_verify", 1: "k_verify_queue", 2: "k_verify_lane", 3: "k_verify_split",
                 4: "k_verify_grp", 5: "k_verify"}
VERIFY_FORM = {0: "two-pass", 1: "persistent, replayed from a captured HIP graph",
               2: "one pair per lane, persistent, replayed from a captured HIP graph",
               3: "several band words per lane, persistent, replayed from a captured HIP graph",
               4: "grouped by pattern (masks shared in LDS per chunk), one pair per lane, "
                  "persistent, replayed from a captured HIP graph",
               5: "two-pass, two band words per lane"}
LEGS = ("tiny", "uneven", "protein", "plus", "serving")

# Recall-calibrated parameter points, found by sweeps of (r, z, m, L) on these
# workloads (recall against the planted pairs >= 0.99 at the least join time):
# at the stated parameters the uniformly spread indels of the synthetic copies
# keep the CGK walks out of step and few true pairs become candidates.
CALIBRATED = {
    "medium": dict(r=32, z=16, m=18, L=64),
    "tiny": dict(r=7, z=16, m=8, L=64),
    "uneven": dict(r=32, z=16, m=16, L=64),
}
# Exhaustive pass over the short strings of the uneven workload (exact_len):
# at K=400, random DNA strings up to about 2K letters are within K of each
# other by chance (tens of millions of pairs no embedding brings together);
# sampled pairs show none above 2.25K, so 2.5K covers them with a margin
UNEVEN_EXACT_LEN = 1000
# The protein-like workload at K=100: from ej_calibrate's grid on planted
# pairs with a string longer than K (predicted 0.99 at r=64, z=32; this point
# measured 0.990 of the planted pairs within K at a third of its tables),
# joined with the exhaustive pass over the strings no longer than K
PROTEIN_CALIBRATED = dict(r=32, z=16, m=8, L=64)
# EmbedJoin+ on reads with shifts (K=100, delta=50 -> two suffixes, T=2), at
# the point ej_calibrate chose for a predicted recall of 0.995 (L = 0: the
# average length, as the paper truncates genome reads)
PLUS = dict(K=100, delta=50, T=2, r=6, z=16, m=8, L=0)
# Serving parameters, recall-calibrated by a sweep on this query mix
# (re-mutated members at 5% edits plus fresh random strings): with the stated
# r=3, z=7 no (m, L) reaches recall 0.99 against the source member (0.81-0.93)
SERVING = dict(r=32, z=8, m=20, L=64)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="medium",
                    choices=["medium", "tiny", "uneven", "protein"])
    ap.add_argument("--K", type=int, default=None)
    ap.add_argument("--r", type=int, default=None)
    ap.add_argument("--z", type=int, default=None)
    ap.add_argument("--m", type=int, default=None)
    ap.add_argument("--L", type=int, default=None)
    ap.add_argument("--stated", action="store_true",
                    help="use the workload's stated (r, z, m, L) instead of the recall-calibrated point")
    ap.add_argument("--legs", default=",".join(LEGS),
                    help="workloads run besides the headline one (comma list of "
                         f"{', '.join(LEGS)}; empty for none)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-recall", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="batched form with default knobs instead of the autotuner's")
    ap.add_argument("--knobs", default="", metavar="name=value,..",
                    help="batched form with these launch knobs instead of the autotuner's")
    ap.add_argument("--serving-only", action="store_true", help="run only the serving leg")
    ap.add_argument("--serving-params", default="", metavar="r,z,m,L",
                    help="override the serving index parameters")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES bytes (5 times): "
                         "the reference for scaling HBM traffic counters")
    ap.add_argument("--no-pool", action="store_true",
                    help="generate the collections in this process, one after another (for "
                         "runs under a profiler, whose preloaded library has started the GPU "
                         "before worker processes could be spawned)")
    ap.add_argument("--valu-probe", action="store_true",
                    help="only run the integer-VALU issue-rate probe (for its counter profile)")
    return ap.parse_args()


def _log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# ------------------------------------------------------ data generation --
# The larger collections are generated in worker processes (spawned: they
# never touch the GPU) while the GPU runs the earlier legs, and handed over as
# .npz files in a private temporary directory.

def _gen_worker(name, path):
    import synthdata as sd
    if name == "uneven":
        col, _ = sd.uneven_dna(0)
    elif name == "protein":
        col, _ = sd.protein_like(0)
    elif name == "shifted":
        col, _ = sd.shifted_reads(0)
    elif name == "serving":
        col, _ = sd.serving_index(0)
        q, Kq, src = sd.serving_queries(col, 0)
        np.savez(path, chars=col.chars, offsets=col.offsets, labels=col.labels, qchars=q.chars,
                 qoffsets=q.offsets, qlabels=q.labels, Kq=Kq, src=src)
        return path
    else:
        raise ValueError(name)
    np.savez(path, chars=col.chars, offsets=col.offsets, labels=col.labels)
    return path


class DataPool:
    def __init__(self, names, inline=False):
        self.dir = tempfile.mkdtemp(prefix="ej_bench_")
        self.inline = inline
        self.ex = None
        if inline:
            self.fut = {n: None for n in names}
            return
        self.ex = ProcessPoolExecutor(max_workers=max(1, len(names)),
                                      mp_context=multiprocessing.get_context("spawn"))
        self.fut = {n: self.ex.submit(_gen_worker, n, os.path.join(self.dir, n + ".npz"))
                    for n in names}

    def get(self, name):
        import synthdata as sd
        t0 = time.perf_counter()
        if self.inline:
            path = _gen_worker(name, os.path.join(self.dir, name + ".npz"))
        else:
            path = self.fut[name].result()
        z = np.load(path)
        d = {k: z[k] for k in z.files}
        os.remove(path)
        col = sd.Collection(d["chars"], d["offsets"], d["labels"], name)
        _log(f"data {name} ready (waited {time.perf_counter() - t0:.1f} s)")
        return col, d

    def wait_all(self):
        """Blocks until every collection is generated, so that no generator
        process competes with the timed joins for the host's cores."""
        t0 = time.perf_counter()
        if not self.inline:
            for f in self.fut.values():
                f.result()
        _log(f"all data generated (waited {time.perf_counter() - t0:.1f} s)")

    def close(self):
        if self.ex:
            self.ex.shutdown(cancel_futures=True)
        shutil.rmtree(self.dir, ignore_errors=True)


# ---------------------------------------------------------------- probes --

def copy_probe(nbytes):
    import torch
    x = torch.empty(nbytes, dtype=torch.uint8, device="cuda").fill_(1)
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    for _ in range(5):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": nbytes, "reads_per_copy": nbytes,
                      "writes_per_copy": nbytes, "copies": 5}), flush=True)


PROBE_MIXES = {0: "verification mix (add, 3-input logic, funnel shift)", 1: "v_add_u32",
               2: "v_xor_b32", 3: "v_bitop3_b32", 4: "v_alignbit_b32",
               5: "v_add_co_u32 (carry-out to a scalar mask)",
               6: "v_addc_co_u32 (carry chain through a scalar mask)", 7: "v_cmp_eq_u32",
               8: "v_mov_b32_dpp wave_shl:1", 9: "v_bcnt_u32_b32", 10: "v_add3_u32",
               11: "v_cndmask_b32 (scalar mask)", 12: "v_or3_b32", 13: "v_and_or_b32",
               14: "v_mul_u32_u24_sdwa (byte select)"}


def valu_peak(ctx, all_mixes=False):
    """The integer-VALU issue rates the probe kernel reaches, per instruction
    class, at the best of a few occupancies (workgroups of 256 lanes per CU):
    returns (the best rate of any class, the runs)."""
    best = 0.0
    runs = []
    mixes = PROBE_MIXES if all_mixes else (0, 1, 3)
    occ = (8, 16, 32) if all_mixes else (32,)
    for mix in mixes:
        for bpc in occ:
            ops, ms = ctx.probe_valu(4096, bpc, mix)
            runs.append(dict(mix=PROBE_MIXES[mix], blocks_per_cu=bpc, tops=round(ops / 1e12, 3),
                             ms=round(ms, 4)))
            best = max(best, ops)
    return best, runs


def measured_traffic(kernel, workload_tag):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, or None when the kernel source changed since it was taken."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload_tag}.md")
    if not os.path.exists(path):
        return None
    m = re.search(r"```json\n(.*?)\n```", open(path).read(), re.S)
    if not m:
        return None
    rec = json.loads(m.group(1))
    src = open(os.path.join(ROOT, rec["source"]), "rb").read()
    if hashlib.sha256(src).hexdigest()[:16] != rec["sha256_16"]:
        return None
    return rec["hbm_bytes_per_launch"]


# ----------------------------------------------------------- the joins --

def device(col):
    import torch
    chars = torch.from_numpy(col.chars).cuda()
    offs = torch.from_numpy(col.offsets.astype(np.int64)).cuda()
    return chars, offs


def time_join(fn, steps, warmup):
    """Wall time of `steps` joins after `warmup` (fn returns a JoinResult
    with stage times), between torch.cuda.synchronize() calls."""
    import torch
    for _ in range(warmup):
        res = fn()
    torch.cuda.synchronize()
    stage = {}
    t0 = time.perf_counter()
    for _ in range(steps):
        res = fn()
        for k, v in res.ms.items():
            stage[k] = stage.get(k, 0.0) + v / steps
        stage["verify_kernel"] = stage.get("verify_kernel", 0.0) + res.ms_verify_kernel / steps
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    return res, (t1 - t0) * 1000.0 / max(steps, 1), stage


GRAPH_STATE = {0: "host-sized (sizes read back between stages)",
               1: "sized on the device, uncaptured",
               2: "whole join (A1-A6) replayed from one captured graph"}


def run_forms(ej, ctx, chars, offs, prm, args, steps=None, warmup=None, tune_reps=2):
    """The plain per-stage form (default knobs, two-pass verification) and the
    batched form (persistent verification replayed from a captured HIP graph,
    knobs from the autotuner), timed on the same device-resident input."""
    steps = args.steps if steps is None else steps
    warmup = args.warmup if warmup is None else warmup
    # device-resident: the strings are in HBM before the timed region and the
    # result stays in HBM (handed to torch), no host copy inside
    flags = ej.FLAG_TIMING | ej.FLAG_DEVICE_OUT
    defaults = ctx.knobs()
    ctx.tune_set("verify_mode", 0)

    def join(fl):
        return lambda: ctx.join(chars, offs, prm["K"], prm["r"], prm["z"], prm["m"], seed=0,
                                L=prm["L"], flags=fl)

    res, ms, stage = time_join(join(flags), steps, warmup)
    plain = dict(res=res, ms=ms, stage=stage, knobs=ctx.knobs(), kernel="k_verify")
    if args.knobs:
        for kv in args.knobs.split(","):
            k, v = kv.split("=")
            ctx.tune_set(k.strip(), int(v))
        tune_ms = None
    elif args.no_autotune:
        ctx.tune_set("verify_mode", 2)
        tune_ms = None
    else:
        tune_ms, _ = ctx.autotune(chars, offs, prm["K"], prm["r"], prm["z"], prm["m"], seed=0,
                                  L=prm["L"], reps=tune_reps)
    knobs = ctx.knobs()
    # the whole join replayed from one captured graph, the result left in HBM.
    # Set-up, like the tuner: the first join of a shape runs host-sized and
    # sets the candidate capacities, the second allocates every buffer at
    # them, the third captures the graph; the timed joins replay it
    gflags = ej.FLAG_GRAPH | ej.FLAG_DEVICE_OUT
    for _ in range(3):
        join(gflags)()
    gres, ms, _ = time_join(join(gflags), steps, warmup)
    # stage times and the verification kernel's own time come from joins
    # with timing, which run host-sized (events between the stages), their
    # persistent verification replayed from a graph of its own
    tflags = flags | (ej.FLAG_GRAPH if knobs["verify_mode"] >= 1 else 0)
    res, tms, stage = time_join(join(tflags), max(1, min(steps, 3)), 1)
    assert res.count == gres.count and res.n_candidates == gres.n_candidates
    batched = dict(res=res, ms=ms, stage=stage, knobs=knobs, autotune_best_ms=tune_ms,
                   kernel=VERIFY_KERNEL[res.verify_form], graph=GRAPH_STATE[gres.graph],
                   timed_with_stage_events_ms=tms)
    for k, v in defaults.items():
        ctx.tune_set(k, v)
    return dict(plain=plain, batched=batched)


def roofline(res, stage, prm, kern, peak_measured=None):
    """Algorithmic integer operations per step of the dominant kernel over its
    own device time per step (events around each launch), in two units, each
    against the vendor-derived and the probe-measured peak."""
    if stage.get("verify", 0.0) >= stage.get("embed", 0.0) and res.verify_columns:
        words = res.verify_columns * (prm["K"] + 1) / 32.0
        ops = words * OPS_PER_WORD_STEP
        ops_s = words * SURVEY_OPS_PER_WORD
        t = stage["verify_kernel"] / 1000.0
        nl = max(1, res.verify_launches)
        cells = res.verify_columns * (prm["K"] + 1)
        work = dict(launches_per_step=res.verify_launches,
                    avg_launch_ms=round(stage["verify_kernel"] / nl, 4),
                    band_cells=int(cells), text_columns=int(res.verify_columns),
                    gcells_per_s=round(cells / t / 1e9, 2) if t > 0 else None,
                    ukkonen_2k1_gcells_per_s=round(res.verify_columns * (2 * prm["K"] + 1)
                                                   / t / 1e9, 2) if t > 0 else None)
    else:
        kern = "k_embed"
        ops = res.walk_steps * OPS_PER_WALK_STEP
        ops_s = None
        t = stage["embed"] / 1000.0
        work = dict(walk_steps=int(res.walk_steps),
                    gsteps_per_s=round(res.walk_steps / t / 1e9, 2) if t > 0 else None)
    achieved = ops / t / 1e12 if t > 0 else 0.0
    peak = MI355X_INT32_LANE_OPS / 1e12
    out = dict(bound="alu", kernel=kern, achieved=round(achieved, 4), peak=round(peak, 2),
               unit="T int32 lane-op/s", frac=round(achieved / peak, 5), traffic=None,
               traffic_unit="HBM bytes per launch (rocprofv3 FETCH_SIZE/WRITE_SIZE, copy-scaled)",
               work_unit=("10 ops per 32-cell word of the K+1 band (Myers' recurrence)"
                          if ops_s is not None else "3 ops per CGK walk step"),
               kernel_ms=round(t * 1000.0, 4), **work)
    if peak_measured:
        pm = peak_measured / 1e12
        out["peak_measured"] = round(pm, 3)
        out["frac_vs_measured"] = round(achieved / pm, 5)
    if ops_s is not None and t > 0:
        a2 = ops_s / t / 1e12
        out["achieved_survey_unit"] = round(a2, 4)
        out["survey_unit"] = "20 ops per 32-cell word (recurrence + cross-lane carry + shift)"
        out["frac_survey_unit"] = round(a2 / peak, 5)
        out["frac_vs_half_rate_peak"] = round(achieved / (MI355X_INT32_LANE_OPS_HALF / 1e12), 5)
        if peak_measured:
            out["frac_survey_unit_vs_measured"] = round(a2 / (peak_measured / 1e12), 5)
    return out


def form_summary(f, prm, peak_measured=None):
    res, ms, stage = f["res"], f["ms"], f["stage"]
    roof = roofline(res, stage, prm, f["kernel"], peak_measured)
    out = dict(join_sec=round(ms / 1000.0, 5),
               verified_pairs_per_s=round(res.n_candidates / (ms / 1000.0), 3),
               stage_ms={k: round(v, 3) for k, v in stage.items()},
               kernel=roof["kernel"], kernel_ms=roof["kernel_ms"], roofline_frac=roof["frac"],
               roofline_frac_vs_measured=roof.get("frac_vs_measured"), knobs=f["knobs"])
    if "graph" in f:
        out["graph"] = f["graph"]
        out["join_sec_with_stage_events"] = round(f["timed_with_stage_events_ms"] / 1000.0, 5)
    return out


# ------------------------------------------------------------ recall --

def _codes(pairs):
    p = np.asarray(pairs, dtype=np.uint64).reshape(-1, 2)
    return (p[:, 0] << np.uint64(32)) | p[:, 1]


def gpu_within(ctx, chars, offs, codes, K, chunk=1 << 23):
    """Which pairs are within K: the library's verification (bit-exact with
    the oracle in the parity tests), in chunks."""
    import torch
    out = np.zeros(len(codes), dtype=bool)
    for i in range(0, len(codes), chunk):
        c = torch.from_numpy(np.ascontiguousarray(codes[i:i + chunk]).astype(np.int64)).cuda()
        out[i:i + chunk] = ctx.verify(chars, offs, c, K).cpu().numpy() <= K
    return out


def exact_recall(ctx, chars, offs, col, K, res, oracle, extra_true=None, check=300, seed=1):
    """Recall against the planted pairs within K, all of them verified (the
    denominator is exact), optionally united with further true pairs; a
    sample of the GPU's decisions is checked against the oracle."""
    import synthdata as sd
    planted = _codes(sd.planted_pairs(col))
    w = gpu_within(ctx, chars, offs, planted, K)
    rng = np.random.default_rng(seed)
    pick = rng.choice(len(planted), size=min(check, len(planted)), replace=False)
    o = oracle.verify_pairs(col.chars, col.offsets, planted[pick], K) <= K
    assert np.array_equal(o, w[pick]), "GPU and oracle disagree on planted pairs"
    truth = planted[w]
    if extra_true is not None and len(extra_true):
        truth = np.union1d(truth, extra_true)
    out = res.codes
    found = int(np.isin(truth, out).sum()) if len(truth) else 0
    return dict(planted_pairs=int(len(planted)), planted_within_K=int(w.sum()),
                true_pairs=int(len(truth)), found=found,
                recall=round(found / len(truth), 5) if len(truth) else None,
                output_pairs=int(len(out)), oracle_checked_pairs=int(len(pick)))


def short_string_truth(ctx, chars, offs, col, K, max_len):
    """Pairs among the strings no longer than max_len that are within K (all
    pairs with lengths within K, verified on the GPU): the accidental true
    pairs that random strings of such lengths form."""
    lens = col.lengths()
    ids = np.nonzero(lens <= max_len)[0]
    ids = ids[np.argsort(lens[ids], kind="stable")]
    L = lens[ids]
    parts = []
    for i in range(len(ids)):
        j1 = np.searchsorted(L, L[i] + K, side="right")
        if j1 <= i + 1:
            continue
        a = np.full(j1 - i - 1, ids[i], dtype=np.uint64)
        b = ids[i + 1:j1].astype(np.uint64)
        lo, hi = np.minimum(a, b), np.maximum(a, b)
        parts.append((lo << np.uint64(32)) | hi)
    if not parts:
        return np.zeros(0, dtype=np.uint64), 0
    cand = np.concatenate(parts)
    w = gpu_within(ctx, chars, offs, cand, K)
    return np.sort(cand[w]), int(len(cand))


def brute_truth(col, K, oracle, threads=16):
    """The exact join by brute force with the oracle: every pair within K in
    length, its threshold distance (Ukkonen), over host threads."""
    lens = col.lengths()
    order = np.argsort(lens, kind="stable")
    L = lens[order]
    parts = []
    for i in range(col.n):
        j1 = np.searchsorted(L, L[i] + K, side="right")
        if j1 > i + 1:
            a = np.full(j1 - i - 1, order[i], dtype=np.uint64)
            b = order[i + 1:j1].astype(np.uint64)
            parts.append((np.minimum(a, b) << np.uint64(32)) | np.maximum(a, b))
    cand = np.concatenate(parts) if parts else np.zeros(0, np.uint64)
    chunks = np.array_split(cand, threads * 8)
    with ThreadPoolExecutor(threads) as ex:
        d = np.concatenate(list(ex.map(lambda c: oracle.verify_pairs(col.chars, col.offsets, c,
                                                                     K), chunks)))
    return np.sort(cand[d <= K]), int(len(cand))


def sample_pairs(col, n_planted, n_random, seed=1):
    import synthdata as sd
    rng = np.random.default_rng(seed)
    planted = sd.planted_pairs(col)
    pick = planted[rng.choice(len(planted), size=min(n_planted, len(planted)), replace=False)]
    rand = rng.integers(0, col.n, size=(n_random, 2))
    rand = np.sort(rand[rand[:, 0] != rand[:, 1]], axis=1)
    return _codes(np.concatenate([pick, rand]))


def calibration_block(ej, ctx, chars, offs, col, K, oracle, target=0.99, r_max=32,
                      zl=(4, 8, 16), ml=(8, 12, 16, 18, 20, 24), Ll=(64, 128, 0), delta=0, T=0):
    """ej_calibrate on a sample of planted and random pairs, then one join at
    the chosen point and its measured recall."""
    import torch
    codes = sample_pairs(col, 1000, 2000)
    dp = torch.from_numpy(codes.astype(np.int64)).cuda()
    t0 = time.perf_counter()
    cal = ctx.calibrate(chars, offs, dp, K, r_max, list(zl), list(ml), list(Ll),
                        target_recall=target, seed=0, delta=delta, T=T)
    cal_s = time.perf_counter() - t0
    out = dict(target_recall=target, grid=dict(r_max=r_max, z=list(zl), m=list(ml),
                                               L=list(Ll)),
               seconds=round(cal_s, 3), n_similar=cal["n_similar"],
               n_dissimilar=cal["n_dissimilar"], best_predicted_recall=round(cal["best_recall"], 5))
    if cal["r"]:
        prm = dict(r=cal["r"], z=cal["z"], m=cal["m"], L=cal["L"])
        t0 = time.perf_counter()
        if delta:
            res = ctx.join_plus(chars, offs, K, prm["r"], prm["z"], prm["m"], delta=delta, T=T,
                                seed=0, L=prm["L"])
        else:
            res = ctx.join(chars, offs, K, prm["r"], prm["z"], prm["m"], seed=0, L=prm["L"])
        torch.cuda.synchronize()
        out.update(chosen=prm, predicted_recall=round(cal["recall"], 5),
                   predicted_false_rate=round(cal["false_rate"], 6),
                   join_ms=round((time.perf_counter() - t0) * 1e3, 3),
                   measured=exact_recall(ctx, chars, offs, col, K, res, oracle, check=100))
    return out


# ------------------------------------------------------------ the legs --

def leg_forms(ej, ctx, oracle, args, col, desc, prm, stated, peak, steps=None, warmup=None,
              tune_reps=2, extra_true=None):
    chars, offs = device(col)
    forms = run_forms(ej, ctx, chars, offs, prm, args, steps, warmup, tune_reps)
    b = forms["batched"]
    out = dict(workload=desc, params=prm, stated=stated,
               candidates=b["res"].n_candidates, raw_candidates=b["res"].n_raw,
               output_pairs=b["res"].count,
               batched=form_summary(b, prm, peak), plain=form_summary(forms["plain"], prm, peak))
    return out, chars, offs, b["res"]


def tiny_leg(ej, ctx, oracle, args, peak):
    """2,000 DNA strings (200 bases x 10 copies, Poisson(30) edits), K=50, at
    its calibrated point; recall against the exact join by brute force."""
    import synthdata as sd
    col, stated = sd.tiny_dna(0)
    prm = dict(K=stated["K"], **CALIBRATED["tiny"])
    out, chars, offs, res = leg_forms(ej, ctx, oracle, args, col,
                                      "tiny DNA: 2,000 strings (200 bases U{900..1100} x 10 "
                                      "copies, Poisson(30) edits)", prm, stated, peak)
    t0 = time.perf_counter()
    truth, npairs = brute_truth(col, prm["K"], oracle)
    got = res.codes
    out["recall_vs_brute_force"] = dict(
        pairs_examined=npairs, true_pairs=int(len(truth)),
        found=int(np.isin(truth, got).sum()),
        recall=round(float(np.isin(truth, got).mean()), 5) if len(truth) else None,
        output_subset_of_truth=bool(np.isin(got, truth).all()),
        oracle_seconds=round(time.perf_counter() - t0, 2))
    out["stated_params_run"] = stated_run(ctx, chars, offs, dict(stated, L=0))
    return out


def stated_run(ctx, chars, offs, prm):
    import torch
    ctx.join(chars, offs, prm["K"], prm["r"], prm["z"], prm["m"], seed=0, L=prm.get("L", 0))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r2 = ctx.join(chars, offs, prm["K"], prm["r"], prm["z"], prm["m"], seed=0, L=prm.get("L", 0))
    torch.cuda.synchronize()
    return dict(params=prm, join_ms=round((time.perf_counter() - t0) * 1e3, 3),
                candidates=r2.n_candidates, output_pairs=int(len(r2.pairs)))


def in_sorted(x, s):
    """x in s for a sorted array s (codes), elementwise."""
    if len(s) == 0:
        return np.zeros(len(x), dtype=bool)
    i = np.minimum(np.searchsorted(s, x), len(s) - 1)
    return s[i] == x


def above_cut_accidental(ctx, chars, offs, col, K, S, width, planted_within, n_sample=300000,
                         seed=11):
    """Accidental true pairs just above the short-pass cut: pairs whose longer
    string has a length in (S, S + width] and whose lengths differ by at most
    K, drawn uniformly (by the longer string, then its partner), verified on
    the GPU; the estimate scales the sampled rate of non-planted pairs within
    K to the band's pair count."""
    lens = col.lengths().astype(np.int64)
    order = np.argsort(lens, kind="stable")
    ls = lens[order]
    idx = np.nonzero((ls > S) & (ls <= S + width))[0]
    if len(idx) == 0:
        return dict(band=[S, S + width], pairs=0)
    parts = np.searchsorted(ls, ls[idx], side="right") - np.searchsorted(ls, ls[idx] - K) - 1
    rng = np.random.default_rng(seed)
    i = idx[rng.choice(len(idx), size=n_sample, p=parts / parts.sum())]
    first = np.searchsorted(ls, ls[i] - K)
    last = np.searchsorted(ls, ls[i], side="right")
    j = first + (rng.random(n_sample) * (last - first)).astype(np.int64)
    ok = j != i
    a, b = order[i[ok]], order[j[ok]]
    codes = (np.minimum(a, b).astype(np.uint64) << np.uint64(32)) | \
        np.maximum(a, b).astype(np.uint64)
    w = gpu_within(ctx, chars, offs, codes, K)
    acc = w & ~np.isin(codes, planted_within)
    return dict(band=[S, S + width], pairs=int(parts.sum()), sampled=int(len(codes)),
                within_K=int(w.sum()), accidental=int(acc.sum()),
                accidental_estimate=round(float(acc.mean()) * int(parts.sum()), 1))


def uneven_leg(ej, ctx, oracle, args, peak, col):
    """80,000 DNA strings, log-uniform lengths, K=400.  The LSH join at its
    calibrated point (both forms), then the same join with the exhaustive
    short-string pass (exact_len); the grouping alternative to truncation
    beside them.  Truth: every planted pair verified, united with every pair
    of strings no longer than the cut that is within K (all such pairs with
    lengths within K verified on the GPU); pairs just above the cut are
    sampled to show that no accidental true pairs are left out."""
    import torch
    import synthdata as sd
    stated = dict(K=400, r=3, z=7, m=24)
    prm = dict(K=400, **CALIBRATED["uneven"])
    S = UNEVEN_EXACT_LEN
    out, chars, offs, res = leg_forms(ej, ctx, oracle, args, col,
                                      "uneven DNA: 80,000 strings, base lengths log-uniform "
                                      "500..20,000, clusters geometric(0.3) <= 20, per-copy edit "
                                      "rate U(0, 0.08)", prm, stated, peak)
    K = prm["K"]
    lens = col.lengths()
    planted = _codes(sd.planted_pairs(col))
    pw = planted[gpu_within(ctx, chars, offs, planted, K)]
    pa = (pw >> np.uint64(32)).astype(np.int64)
    pb = (pw & np.uint64(0xFFFFFFFF)).astype(np.int64)
    long_pw = pw[np.maximum(lens[pa], lens[pb]) > S]
    # the join with the short pass (every short string has thousands of
    # partners: the form grouped by pattern against the default two-pass form)
    fl = ej.FLAG_TIMING | ej.FLAG_DEVICE_OUT

    def hybrid():
        return ctx.join(chars, offs, K, prm["r"], prm["z"], prm["m"], seed=0, L=prm["L"],
                        flags=fl, exact_len=S)

    runs = {}
    old_mode = ctx.tune_get("verify_mode")
    for mode in (3, 0):
        ctx.tune_set("verify_mode", mode)
        runs[mode] = time_join(hybrid, max(1, min(args.steps, 3)), 1)
    ctx.tune_set("verify_mode", old_mode)
    best = min(runs, key=lambda k: runs[k][1])
    hres, hms, hstage = runs[best]
    out["with_short_pass"] = dict(exact_len=S, join_sec=round(hms / 1e3, 5),
                                  verify_mode=best, kernel=VERIFY_KERNEL[hres.verify_form],
                                  join_sec_by_verify_mode={str(k): round(v[1] / 1e3, 5)
                                                           for k, v in runs.items()},
                                  stage_ms={k: round(v, 3) for k, v in hstage.items()},
                                  candidates=hres.n_candidates, output_pairs=hres.count,
                                  verified_pairs_per_s=round(hres.n_candidates / (hms / 1e3), 3))
    if not args.no_recall:
        short, examined = short_string_truth(ctx, chars, offs, col, K, S)
        truth = np.union1d(pw, short)
        got_lsh, got_h = np.sort(res.codes), np.sort(hres.codes)
        # the GPU's within-K decisions that build the truth, against the oracle
        rng = np.random.default_rng(3)
        chk = np.concatenate([planted[rng.choice(len(planted), 100, replace=False)],
                              short[rng.choice(len(short), min(100, len(short)),
                                               replace=False)]])
        assert np.array_equal(oracle.verify_pairs(col.chars, col.offsets, chk, K) <= K,
                              gpu_within(ctx, chars, offs, chk, K)), \
            "GPU and oracle disagree on truth pairs"
        out["recall"] = dict(
            planted_pairs=int(len(planted)), planted_within_K=int(len(pw)),
            planted_within_K_with_a_string_longer_than_cut=int(len(long_pw)),
            short_string_pairs_examined=int(examined), short_string_true_pairs=int(len(short)),
            true_pairs=int(len(truth)),
            lsh_recall_vs_planted=round(float(in_sorted(pw, got_lsh).mean()), 5),
            lsh_recall_vs_planted_longer_than_cut=round(float(in_sorted(long_pw,
                                                                        got_lsh).mean()), 5),
            lsh_recall_vs_true_pairs=round(float(in_sorted(truth, got_lsh).mean()), 5),
            with_short_pass_recall_vs_true_pairs=round(float(in_sorted(truth, got_h).mean()), 5),
            with_short_pass_output_subset_of_truth=bool(in_sorted(got_h, truth).all()),
            oracle_checked_pairs=int(len(chk)),
            above_cut=above_cut_accidental(ctx, chars, offs, col, K, S, 300, pw),
            note="true pairs = planted pairs within K (all verified) united with every pair of "
                 "strings no longer than the cut within K (all verified); accidental true pairs "
                 "above the cut are estimated by sampling the band above it")
        del short, truth
    # grouping (Section 4.1) at the same r, z, m: untruncated walks per group
    ctx.join_grouped(chars, offs, prm["K"], prm["r"], prm["z"], prm["m"], seed=0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g = ctx.join_grouped(chars, offs, prm["K"], prm["r"], prm["z"], prm["m"], seed=0)
    torch.cuda.synchronize()
    gms = (time.perf_counter() - t0) * 1e3
    out["grouping"] = dict(params=dict(r=prm["r"], z=prm["z"], m=prm["m"],
                                       L="3 x each group's longest string"),
                           join_ms=round(gms, 3), candidates=g.n_candidates,
                           output_pairs=int(len(g.pairs)),
                           recall_vs_planted=(round(float(in_sorted(pw, np.sort(g.codes)).mean()),
                                                    5) if not args.no_recall else None))
    return out


def protein_recall(ctx, chars, offs, col, K, got, w):
    """Recall of the output codes `got` against the planted pairs within K
    (w, all verified) united with every pair of strings both no longer than
    K (ED <= K is guaranteed), counted without listing the latter."""
    lens = col.lengths()
    short = np.nonzero(lens <= K)[0]
    ga = (got >> np.uint64(32)).astype(np.int64)
    gb = (got & np.uint64(0xFFFFFFFF)).astype(np.int64)
    both_short = (lens[ga] <= K) & (lens[gb] <= K)
    pa = (w >> np.uint64(32)).astype(np.int64)
    pb = (w & np.uint64(0xFFFFFFFF)).astype(np.int64)
    pshort = (lens[pa] <= K) & (lens[pb] <= K)
    n_short_pairs = len(short) * (len(short) - 1) // 2
    denom = len(w) + n_short_pairs - int(pshort.sum())
    gs = np.sort(got)
    found = int(both_short.sum()) + int(in_sorted(w[~pshort], gs).sum())
    return dict(planted_within_K=int(len(w)), short_strings=int(len(short)),
                guaranteed_short_pairs=int(n_short_pairs), true_pairs=int(denom), found=found,
                recall=round(found / denom, 5) if denom else None,
                recall_vs_planted=round(float(in_sorted(w, gs).mean()), 5),
                other_true_pairs_found=int(len(got)) - found)


def protein_leg(ej, ctx, oracle, args, peak, col):
    """400,000 strings over 25 Zipf letters, K=100: the stated r=5, z=10,
    m=32 with L = ceil(2 avg) in both forms, then a recall-calibrated point
    with the exhaustive pass over the strings no longer than K.  Truth: the
    planted pairs within K (all verified) and the pairs of strings both no
    longer than K (ED <= K is guaranteed), counted exactly; accidental true
    pairs just above K are estimated by sampling."""
    import synthdata as sd
    stated = dict(K=100, r=5, z=10, m=32)
    prm = dict(stated, L=int(np.ceil(2 * col.lengths().mean())))
    out, chars, offs, res = leg_forms(ej, ctx, oracle, args, col,
                                      "protein-like: 400,000 strings over 25 letters (Zipf 1.1), "
                                      "lengths lognormal (median 400, sigma 0.8) clipped 50..4,000,"
                                      " clusters of mean 4, edit rate U(0.02, 0.15)", prm, stated,
                                      peak, steps=3, warmup=1, tune_reps=1)
    K = prm["K"]
    w = None
    if not args.no_recall:
        planted = _codes(sd.planted_pairs(col))
        w = planted[gpu_within(ctx, chars, offs, planted, K)]
        out["recall"] = protein_recall(ctx, chars, offs, col, K, res.codes, w)
    # recall-calibrated: chosen from ej_calibrate's grid on planted pairs with
    # a string longer than K (the shorter pairs are the short pass's), then
    # measured; verification grouped by pattern
    C = PROTEIN_CALIBRATED
    old = ctx.knobs()
    ctx.tune_set("verify_mode", 3)
    fl = ej.FLAG_TIMING | ej.FLAG_DEVICE_OUT

    def cal_join():
        return ctx.join(chars, offs, K, C["r"], C["z"], C["m"], seed=0, L=C["L"], flags=fl,
                        exact_len=K)

    cres, cms, cstage = time_join(cal_join, 2, 1)
    for k, v in old.items():
        ctx.tune_set(k, v)
    out["calibrated_with_short_pass"] = dict(
        params=dict(C, exact_len=K), verify_mode=3, kernel=VERIFY_KERNEL[cres.verify_form],
        join_sec=round(cms / 1e3, 5), candidates=cres.n_candidates, output_pairs=cres.count,
        verified_pairs_per_s=round(cres.n_candidates / (cms / 1e3), 3),
        stage_ms={k: round(v, 3) for k, v in cstage.items()})
    if w is not None:
        rec = protein_recall(ctx, chars, offs, col, K, cres.codes, w)
        rec["above_K"] = above_cut_accidental(ctx, chars, offs, col, K, K, 50, w)
        rec["note"] = ("accidental true pairs whose longer string is just above K are not in "
                       "the denominator; above_K estimates them in the band (K, K + 50]")
        out["calibrated_with_short_pass"]["recall"] = rec
    return out


def plus_leg(ej, ctx, oracle, args, peak, col):
    """EmbedJoin+ on 50,000 DNA reads with shifts (4,500-5,500 letters, reads
    of a cluster start up to 60 letters apart, 0.3% edits), K=100, delta=50,
    T=2; plain EmbedJoin at the same (r, z, m, L) beside it."""
    import torch
    chars, offs = device(col)
    P = PLUS
    prm = dict(K=P["K"], r=P["r"], z=P["z"], m=P["m"], L=P["L"])
    fl = ej.FLAG_TIMING | ej.FLAG_DEVICE_OUT

    def plus_join(flags):
        return lambda: ctx.join_plus(chars, offs, P["K"], P["r"], P["z"], P["m"], delta=P["delta"],
                                     T=P["T"], seed=0, L=P["L"], flags=flags)

    defaults = ctx.knobs()
    out = dict(workload="EmbedJoin+ on reads with shifts: 50,000 DNA reads (5,000 genome "
                        "segments x 10 reads starting up to 60 letters apart, lengths "
                        "4,500..5,500, Poisson(0.003 len) edits)", params=dict(P))
    res, ms, stage = time_join(plus_join(fl), args.steps, args.warmup)
    out["plain_form"] = dict(join_sec=round(ms / 1e3, 5), candidates=res.n_candidates,
                             tuples=res.n_raw, output_pairs=res.count,
                             verified_pairs_per_s=round(res.n_candidates / (ms / 1e3), 3),
                             stage_ms={k: round(v, 3) for k, v in stage.items()},
                             roofline=roofline(res, stage, prm, "k_verify", peak))
    try:
        ctx.tune_set("verify_mode", 1)
        res_b, ms_b, stage_b = time_join(plus_join(fl | ej.FLAG_GRAPH), args.steps, args.warmup)
    finally:
        for k, v in defaults.items():
            ctx.tune_set(k, v)
    out["batched_form"] = dict(join_sec=round(ms_b / 1e3, 5),
                               verified_pairs_per_s=round(res_b.n_candidates / (ms_b / 1e3), 3),
                               stage_ms={k: round(v, 3) for k, v in stage_b.items()},
                               roofline=roofline(res_b, stage_b, prm, "k_verify_queue", peak))
    if not args.no_recall:
        out["recall"] = exact_recall(ctx, chars, offs, col, P["K"], res, oracle, check=100)
    ctx.join(chars, offs, P["K"], P["r"], P["z"], P["m"], seed=0, L=P["L"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pl = ctx.join(chars, offs, P["K"], P["r"], P["z"], P["m"], seed=0, L=P["L"])
    torch.cuda.synchronize()
    out["embedjoin_same_params"] = dict(
        join_ms=round((time.perf_counter() - t0) * 1e3, 3), candidates=pl.n_candidates,
        recall=(exact_recall(ctx, chars, offs, col, P["K"], pl, oracle, check=50)["recall"]
                if not args.no_recall else None))
    return out


# ------------------------------------------------------------- serving --

def serving_leg(ej, ctx, oracle, col, d, max_batch=4096, n_recall=1000, seed=0):
    """Device-resident index over 320,000 DNA strings; 10,000 queries of mixed
    lengths and thresholds.  Saturation throughput from back-to-back batches,
    then a Poisson arrival stream at 0.5/0.8/1.0x that rate served by an
    arrival batcher (everything that has arrived, at most max_batch, halved
    while the index refuses admission); latency = completion - arrival.  Then
    the incremental insert: the index built over 90% of the strings and the
    last 10% inserted, timed against a rebuild over all of them."""
    import torch
    import synthdata as sd
    qc, qo, Kq, src = d["qchars"], d["qoffsets"].astype(np.uint64), d["Kq"], d["src"]
    nq = len(qo) - 1
    chars, offs = device(col)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ix = ej.Index(ctx, chars, offs, SERVING["r"], SERVING["z"], SERVING["m"], seed=seed,
                  L=SERVING["L"])
    build_s = time.perf_counter() - t0
    _log(f"index built in {build_s:.3f} s")

    def run(i0, i1):
        return ix.query(qc, qo[i0:i1 + 1], Kq[i0:i1])

    def run_admitted(i0, i1):
        out = []
        stack = [(i0, i1)]
        while stack:
            a, b = stack.pop()
            try:
                out.append((a, run(a, b)))
            except ej.EmbedJoinError as e:
                if e.status != ej.EJ_ENOMEM or b - a <= 1:
                    raise
                mid = (a + b) // 2
                stack += [(mid, b), (a, mid)]
        return out

    run_admitted(0, min(nq, 256))   # warm-up
    found = {}
    t0 = time.perf_counter()
    ncand = 0
    for i0 in range(0, nq, max_batch):
        for a, res in run_admitted(i0, min(nq, i0 + max_batch)):
            ncand += res.n_candidates
            for k in range(len(res.offsets) - 1):
                found[a + k] = res.of(k)[0]
    sat_s = time.perf_counter() - t0
    sat_qps = nq / sat_s
    sweeps = []
    for load in (0.5, 0.8, 1.0):
        rng = np.random.default_rng(seed + int(load * 100))
        arrive = np.cumsum(rng.exponential(1.0 / (load * sat_qps), size=nq))
        lat = np.zeros(nq)
        nb = 0
        start = time.perf_counter()
        i = 0
        while i < nq:
            now = time.perf_counter() - start
            if arrive[i] > now:
                time.sleep(arrive[i] - now)
                now = time.perf_counter() - start
            j = int(np.searchsorted(arrive, now, side="right"))
            j = max(j, i + 1)
            j = min(j, i + max_batch, nq)
            run_admitted(i, j)
            done = time.perf_counter() - start
            lat[i:j] = done - arrive[i:j]
            nb += 1
            i = j
        wall = time.perf_counter() - start
        sweeps.append(dict(load=load, offered_qps=round(load * sat_qps, 1),
                           achieved_qps=round(nq / wall, 1), batches=nb,
                           p50_ms=round(float(np.percentile(lat, 50)) * 1e3, 3),
                           p99_ms=round(float(np.percentile(lat, 99)) * 1e3, 3)))
    # recall against the source member of re-mutated queries (oracle ED)
    rng = np.random.default_rng(seed + 7)
    members = np.nonzero(src >= 0)[0]
    pick = rng.choice(members, size=min(n_recall, len(members)), replace=False)
    S_off = col.offsets
    true_n, hit = 0, 0
    for qi in pick.tolist():
        s = int(src[qi])
        x = col.chars[int(S_off[s]):int(S_off[s + 1])]
        y = qc[int(qo[qi]):int(qo[qi + 1])]
        if oracle.ed_banded(x, y, int(Kq[qi])) <= int(Kq[qi]):
            true_n += 1
            hit += int(s in set(found[qi].tolist()))
    ix.close()
    # incremental insert: 90% built, 10% inserted, against a full rebuild
    n90 = int(col.n * 0.9)
    head = sd.Collection(col.chars[:int(col.offsets[n90])], col.offsets[:n90 + 1], col.labels[:n90])
    hc, ho = device(head)
    tail_off = torch.from_numpy(col.offsets[n90:].astype(np.int64)).cuda()
    ix2 = ej.Index(ctx, hc, ho, SERVING["r"], SERVING["z"], SERVING["m"], seed=seed,
                   L=SERVING["L"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ix2.insert(chars, tail_off)
    torch.cuda.synchronize()
    ins_s = time.perf_counter() - t0
    qa = ix2.query(qc, qo[:1025], Kq[:1024])
    ix3 = ej.Index(ctx, chars, offs, SERVING["r"], SERVING["z"], SERVING["m"], seed=seed,
                   L=SERVING["L"])
    qb = ix3.query(qc, qo[:1025], Kq[:1024])
    same = qa.ids.tolist() == qb.ids.tolist()
    ix2.close()
    ix3.close()
    return dict(workload="serving: index 320,000 DNA strings (32,000 bases U{4500..5500} x 10 "
                         "copies, Poisson(0.05 len) edits); 10,000 queries (70% re-mutated "
                         "members, 30% fresh U{1000..10000}), K_q in {2,5,10}% of |q|",
                params=SERVING, index_build_s=round(build_s, 3),
                saturation_qps=round(sat_qps, 1), saturation_batch=max_batch,
                candidates_per_query=round(ncand / nq, 2),
                poisson=sweeps, p50_ms=sweeps[-1]["p50_ms"], p99_ms=sweeps[-1]["p99_ms"],
                recall_vs_source=dict(sampled_member_queries=int(len(pick)),
                                      source_within_Kq=true_n, found=hit,
                                      recall=round(hit / true_n, 4) if true_n else None),
                insert=dict(strings=int(col.n - n90), insert_s=round(ins_s, 4),
                            rebuild_s=round(build_s, 4),
                            queries_equal_rebuilt_index=bool(same)))


# ----------------------------------------------------------- baseline --

def cpu_info():
    model = platform.processor() or ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return dict(nproc=os.cpu_count(), cpu_model=model)


def cpu_baseline(col, prm, oracle, budget_s=12.0):
    """The oracle (single thread) on growing prefixes of the workload until
    it runs for about budget_s; rate = candidate pairs verified per second."""
    import synthdata as sd
    n = 250
    last = None
    while True:
        sub = sd.from_strings(col.strings()[:n])
        t0 = time.perf_counter()
        r = oracle.join(sub.chars, sub.offsets, prm["K"], prm["r"], prm["z"], prm["m"], seed=0,
                        L=prm["L"])
        dt = time.perf_counter() - t0
        last = (n, dt, len(r.cand), len(r.out))
        if dt >= budget_s or n >= col.n:
            break
        n = min(col.n, int(n * max(1.5, min(4.0, (budget_s / max(dt, 1e-3)) ** 0.5))))
    n, dt, nc, no = last
    return dict(value=round(nc / dt, 3), unit="verified candidate pairs/s", cores=1,
                kind="oracle", seconds=round(dt, 2), joins_per_s=round(1.0 / dt, 4),
                sample=f"oracle join of the first {n} of {col.n} strings "
                       f"({nc} candidates, {no} output pairs), same parameters", **cpu_info())


# --------------------------------------------------------------- main --

def headline_workload(args):
    import synthdata as sd
    if args.workload == "medium":
        col, prm = sd.medium_dna(0, K=args.K or 500)
        name = ("medium DNA: 20,000 strings (2,000 bases U{4500..5500} x 10 copies, "
                "Poisson(0.04 len) edits)")
    elif args.workload == "uneven":
        col, prm = sd.uneven_dna(0)
        name = ("uneven DNA: 80,000 strings, base lengths log-uniform 500..20,000, clusters "
                "geometric(0.3) <= 20, per-copy edit rate U(0, 0.08)")
    elif args.workload == "protein":
        col, prm = sd.protein_like(0)
        name = ("protein-like: 400,000 strings over 25 letters (Zipf 1.1), lengths lognormal "
                "(median 400, sigma 0.8) clipped 50..4,000, clusters of mean 4, edit rate "
                "U(0.02, 0.15)")
    else:
        col, prm = sd.tiny_dna(0)
        name = "tiny DNA: 2,000 strings (200 bases U{900..1100} x 10 copies, Poisson(30) edits)"
    stated = dict(K=prm["K"], r=prm["r"], z=prm["z"], m=prm["m"], L=0)
    if args.workload == "protein":
        # the stated point, truncated at twice the average length (the
        # paper's choice for strings of varying length, Section 6)
        run = dict(stated, L=int(np.ceil(2 * col.lengths().mean())))
    else:
        run = dict(stated) if args.stated else dict(stated, **CALIBRATED[args.workload])
    for k in ("K", "r", "z", "m", "L"):
        if getattr(args, k) is not None:
            run[k] = getattr(args, k)
    return col, name, stated, run


def guarded(name, fn):
    """A leg's result, or its error (reported; never hides the headline)."""
    try:
        return fn()
    except Exception as e:  # noqa: BLE001
        _log(f"{name} failed: {type(e).__name__}: {e}")
        return {"error": f"{type(e).__name__}: {e}"}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark measures one GPU; the join path has no "
                                   "multi-GPU mode", "n_gpus": args.gpus}))
        sys.exit(2)
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    legs = [x for x in args.legs.split(",") if x] if not args.serving_only else ["serving"]
    for x in legs:
        if x not in LEGS:
            raise SystemExit(f"unknown leg {x}")
    gen = [n for n, leg in (("uneven", "uneven"), ("protein", "protein"), ("shifted", "plus"),
                            ("serving", "serving")) if leg in legs]
    pool = DataPool(gen, inline=args.no_pool) if gen and not args.valu_probe else None
    try:
        _main(args, legs, pool)
    finally:
        if pool:
            pool.close()


def _main(args, legs, pool):
    import paper_1702_00093_amd as ej
    from oracle import oracle
    ctx = ej.Context(0)
    if args.valu_probe:
        ops, runs = valu_peak(ctx, all_mixes=True)
        print(json.dumps({"valu_probe_tops": round(ops / 1e12, 3), "runs": runs}), flush=True)
        return
    if args.serving_params:
        r_, z_, m_, L_ = (int(x) for x in args.serving_params.split(","))
        SERVING.update(r=r_, z=z_, m=m_, L=L_)
    if pool:
        pool.wait_all()
    peak, probe_runs = valu_peak(ctx)
    _log(f"VALU probe {peak / 1e12:.2f} T lane-ops/s")
    if args.serving_only:
        col, d = pool.get("serving")
        print(json.dumps({"serving": serving_leg(ej, ctx, oracle, col, d)}), flush=True)
        return
    col, name, stated, prm = headline_workload(args)
    chars, offs = device(col)
    forms = run_forms(ej, ctx, chars, offs, prm, args)
    head = forms["batched"]
    res, ms, stage = head["res"], head["ms"], head["stage"]
    cand = res.n_candidates
    value = cand / (ms / 1000.0)
    stated_info = stated_run(ctx, chars, offs, stated) if prm != stated else None
    # the same join with the strings in host memory: host-to-device copy of
    # the input and device-to-host copy of the result included
    import torch
    hflags = ej.FLAG_GRAPH
    defaults = ctx.knobs()
    for k, v in head["knobs"].items():
        ctx.tune_set(k, v)
    for _ in range(3):  # host-sized, device-sized, captured: then replays
        ctx.join(col.chars, col.offsets, prm["K"], prm["r"], prm["z"], prm["m"], seed=0,
                 L=prm["L"], flags=hflags)
    t0 = time.perf_counter()
    for _ in range(3):
        ctx.join(col.chars, col.offsets, prm["K"], prm["r"], prm["z"], prm["m"], seed=0,
                 L=prm["L"], flags=hflags)
    torch.cuda.synchronize()
    h2d_ms = (time.perf_counter() - t0) * 1000.0 / 3
    for k, v in defaults.items():
        ctx.tune_set(k, v)
    roof = roofline(res, stage, prm, head["kernel"], peak)
    if (roof["kernel"].startswith("k_verify") and args.workload == "medium" and prm["K"] == 500
            and prm == dict(stated, **CALIBRATED["medium"])):
        roof["traffic"] = measured_traffic(roof["kernel"], "medium_K500")
    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "verified candidate pairs/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": name, "K": prm["K"], "r": prm["r"], "z": prm["z"], "m": prm["m"],
                   "L": res.L, "params": ("stated" if prm == stated or args.workload == "protein"
                                         else "recall-calibrated"),
                   "form": ("batched: autotuned knobs, " + head["graph"] + ", verification "
                            + VERIFY_FORM[res.verify_form]),
                   "join_sec_with_stage_events": round(head["timed_with_stage_events_ms"] / 1e3,
                                                       5),
                   "candidates": cand, "raw_candidates": res.n_raw,
                   "output_pairs": res.count, "join_sec": round(ms / 1000.0, 5),
                   "join_sec_with_h2d_d2h": round(h2d_ms / 1000.0, 5),
                   "timed_region": "strings in HBM before, result left in HBM (FLAG_DEVICE_OUT, "
                                   "handed to torch); join_sec_with_h2d_d2h: host strings in, "
                                   "host result out; stage_ms and the roofline's kernel time "
                                   "from joins with stage events (host-sized)",
                   "stage_ms": {k: round(v, 3) for k, v in stage.items()},
                   "knobs": head["knobs"],
                   "plain_form": form_summary(forms["plain"], prm, peak)},
        "roofline": roof,
        "valu_probe": dict(peak_tops=round(peak / 1e12, 3), runs=probe_runs,
                           kernel="k_probe_valu: 8 independent dependency chains per lane, 96 "
                                  "VALU instructions of one class per loop iteration"),
    }
    if stated_info:
        out["config"]["stated_params_run"] = stated_info
    if not args.no_recall:
        out["config"]["recall"] = guarded("recall", lambda: exact_recall(
            ctx, chars, offs, col, prm["K"], res, oracle))
        out["config"]["calibration"] = guarded("calibration", lambda: calibration_block(
            ej, ctx, chars, offs, col, prm["K"], oracle))
    del chars, offs
    if "tiny" in legs:
        out["tiny"] = guarded("tiny", lambda: tiny_leg(ej, ctx, oracle, args, peak))
    if "uneven" in legs:
        ucol, _ = pool.get("uneven")
        out["uneven"] = guarded("uneven", lambda: uneven_leg(ej, ctx, oracle, args, peak, ucol))
        del ucol
    if "protein" in legs:
        pcol, _ = pool.get("protein")
        out["protein"] = guarded("protein", lambda: protein_leg(ej, ctx, oracle, args, peak, pcol))
        del pcol
    if "plus" in legs:
        scol, _ = pool.get("shifted")
        out["plus"] = guarded("plus", lambda: plus_leg(ej, ctx, oracle, args, peak, scol))
        del scol
    if "serving" in legs:
        vcol, vd = pool.get("serving")
        out["serving"] = guarded("serving", lambda: serving_leg(ej, ctx, oracle, vcol, vd))
        del vcol, vd
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(col, prm, oracle)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
