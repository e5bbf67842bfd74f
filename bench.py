"""Benchmark of the EmbedJoin hot path on one MI355X.

A step is one complete self-join (A0-A6: preparation, CGK walk + keys,
bucketing, candidate pairs, verification, output) of a device-resident
synthetic string collection.  Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload medium|tiny]
                  [--K ..] [--r ..] [--z ..] [--m ..] [--L ..] [--stated]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("end-to-end join sec & verified candidate pairs/s at recall≥0.99; "
          "query p99 ms")
MI355X_INT32_LANE_OPS = 256 * 4 * 16 * 2.4e9    # CUs x SIMDs x lanes x clock
MI355X_HBM = 8.0e12

# Work the method itself must do, in 32-bit integer lane operations:
#  - verification: Myers' bit-parallel step over one 32-cell word of the band
#    is 10 gfx950 instructions (the match word, Xv, Eq&Pv, the add, Xh/Ph/Mh
#    in three 3-input logic operations, the one-bit shift, Pv and Mv), i.e.
#    10/32 operations per DP cell; with 2-input logic alone it would be 15.
#    The band a threshold-K verification needs is K+1 diagonals wide (a path
#    through diagonal d costs at least |d| + |d - d*|);
#  - walk: 3 operations per CGK step (read the symbol, select its pi bit,
#    advance the pointer).
OPS_PER_WORD_STEP = 10
# the verification kernel of each form (JoinResult.verify_form)
VERIFY_KERNEL = {0: "k_verify", 1: "k_verify_queue", 2: "k_verify_lane", 3: "k_verify_split"}
VERIFY_FORM = {0: "two-pass", 1: "persistent, replayed from a captured HIP graph",
               2: "one pair per lane, persistent, replayed from a captured HIP graph",
               3: "several band words per lane, persistent, replayed from a captured HIP graph"}
OPS_PER_WALK_STEP = 3


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="medium", choices=["medium", "tiny", "uneven"])
    ap.add_argument("--K", type=int, default=None)
    ap.add_argument("--r", type=int, default=None)
    ap.add_argument("--z", type=int, default=None)
    ap.add_argument("--m", type=int, default=None)
    ap.add_argument("--L", type=int, default=None)
    ap.add_argument("--stated", action="store_true",
                    help="use the workload's stated (r, z, m, L) instead of the recall-calibrated point")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-recall", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="batched form with default knobs instead of the autotuner's")
    ap.add_argument("--knobs", default="", metavar="name=value,..",
                    help="batched form with these launch knobs instead of the autotuner's")
    ap.add_argument("--no-uneven", action="store_true",
                    help="skip the uneven-length join (80,000 strings, K=400)")
    ap.add_argument("--with-protein", action="store_true",
                    help="also run the protein-like join (400,000 strings, K=100; ~1 min of "
                         "data generation)")
    ap.add_argument("--no-serving", action="store_true",
                    help="skip the serving leg (index of 320,000 strings, 10,000 queries)")
    ap.add_argument("--serving-only", action="store_true",
                    help="run only the serving leg")
    ap.add_argument("--serving-params", default="", metavar="r,z,m,L",
                    help="override the serving index parameters")
    ap.add_argument("--serving-sweep", default="", metavar="r,z,m,L;r,z,m,L;..",
                    help="with --serving-only: one serving run per parameter point, same data")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES bytes (5 times): "
                         "the reference for scaling HBM traffic counters")
    return ap.parse_args()


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


# Recall-calibrated parameter points, found by a sweep of (r, z, m, L) on these
# workloads (recall against the planted pairs >= 0.99 at the least join time):
# at the stated parameters the uniformly spread indels of the synthetic copies
# keep the CGK walks out of step and no true pair becomes a candidate.
CALIBRATED = {
    "medium": dict(r=32, z=16, m=18, L=64),
    "tiny": dict(r=7, z=16, m=8, L=64),
    "uneven": dict(r=32, z=16, m=18, L=64),
}


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


def workload(args):
    import synthdata as sd
    if args.workload == "medium":
        col, prm = sd.medium_dna(0, K=args.K or 500)
        name = "medium DNA: 20,000 strings (2,000 bases U{4500..5500} x 10 copies, Poisson(0.04 len) edits)"
    elif args.workload == "uneven":
        col, prm = sd.uneven_dna(0)
        name = ("uneven DNA: 80,000 strings, base lengths log-uniform 500..20,000, clusters "
                "geometric(0.3) <= 20, per-copy edit rate U(0, 0.08)")
    else:
        col, prm = sd.tiny_dna(0)
        name = "tiny DNA: 2,000 strings (200 bases U{900..1100} x 10 copies, Poisson(30) edits)"
    stated = dict(K=prm["K"], r=prm["r"], z=prm["z"], m=prm["m"], L=0)
    run = dict(stated) if args.stated else dict(stated, **CALIBRATED[args.workload])
    for k in ("K", "r", "z", "m", "L"):
        if getattr(args, k) is not None:
            run[k] = getattr(args, k)
    return col, name, stated, run


def time_join(ctx, chars, offs, prm, steps, warmup, flags):
    import torch
    for _ in range(warmup):
        res = ctx.join(chars, offs, prm["K"], prm["r"], prm["z"], prm["m"], seed=0, L=prm["L"],
                       flags=flags)
    torch.cuda.synchronize()
    stage = {}
    t0 = time.perf_counter()
    for _ in range(steps):
        res = ctx.join(chars, offs, prm["K"], prm["r"], prm["z"], prm["m"], seed=0, L=prm["L"],
                       flags=flags)
        for k, v in res.ms.items():
            stage[k] = stage.get(k, 0.0) + v / steps
        stage["verify_kernel"] = stage.get("verify_kernel", 0.0) + res.ms_verify_kernel / steps
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    return res, (t1 - t0) * 1000.0 / max(steps, 1), stage


def recall_estimate(col, res, K, oracle, n_sample=200, seed=1):
    """Recall against the planted pairs: the fraction of planted pairs within
    K is estimated with the oracle on a sample; every reported pair is exact."""
    import synthdata as sd
    planted = sd.planted_pairs(col)
    if len(planted) == 0:
        return None
    rng = np.random.default_rng(seed)
    idx = rng.choice(len(planted), size=min(n_sample, len(planted)), replace=False)
    codes = (planted[idx, 0].astype(np.uint64) << np.uint64(32)) | planted[idx, 1].astype(np.uint64)
    d = oracle.verify_pairs(col.chars, col.offsets, codes, K)
    frac_true = float((d <= K).mean())
    lab = col.labels
    out = res.pairs
    found_planted = int(((lab[out[:, 0]] == lab[out[:, 1]]) & (lab[out[:, 0]] >= 0)).sum())
    denom = frac_true * len(planted)
    return dict(planted_pairs=int(len(planted)), planted_within_K_frac=round(frac_true, 4),
                planted_within_K_sample=int(len(idx)), found_planted=found_planted,
                recall_vs_planted=(round(found_planted / denom, 4) if denom > 0 else None),
                output_pairs=int(len(out)))


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
                       f"({nc} candidates, {no} output pairs), same parameters")


# Serving parameters, recall-calibrated by a sweep on this query mix
# (re-mutated members at 5% edits plus fresh random strings): with the
# stated r=3, z=7 no (m, L) reaches recall 0.99 against the source member
# (0.81-0.93), because an edit near the start of a string desynchronises the
# walks of all seeds at once; 32 seeds x 8 functions with m=20, L=64 reach
# 0.993 at 26 candidates per query.
SERVING = dict(r=32, z=8, m=20, L=64)


_SERVING_DATA = {}


def _log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def serving_bench(ej, ctx, oracle, max_batch=4096, n_recall=1000, seed=0):
    """Device-resident index over 320,000 DNA strings; 10,000 queries of mixed
    lengths and thresholds.  Saturation throughput from back-to-back batches,
    then a Poisson arrival stream at 0.5/0.8/1.0x that rate served by an
    arrival batcher (everything that has arrived, at most max_batch, halved
    while the index refuses admission); latency = completion - arrival."""
    import torch
    import synthdata as sd
    t0 = time.perf_counter()
    if seed not in _SERVING_DATA:
        col, _ = sd.serving_index(seed)
        _SERVING_DATA[seed] = (col,) + tuple(sd.serving_queries(col, seed))
    col, q, Kq, src = _SERVING_DATA[seed]
    gen_s = time.perf_counter() - t0
    _log(f"serving data ready ({gen_s:.1f} s), params {SERVING}")
    chars = torch.from_numpy(col.chars).cuda()
    offs = torch.from_numpy(col.offsets.astype(np.int64)).cuda()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ix = ej.Index(ctx, chars, offs, SERVING["r"], SERVING["z"], SERVING["m"], seed=seed,
                  L=SERVING["L"])
    build_s = time.perf_counter() - t0
    del chars, offs
    _log(f"index built in {build_s:.3f} s")
    qc, qo = q.chars, q.offsets.astype(np.uint64)
    nq = q.n

    def run(i0, i1):
        # queries i0..i1-1: their offsets index into the whole query buffer
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
    # saturation
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
    _log(f"saturation {sat_qps:.0f} queries/s, {ncand / nq:.1f} candidates per query")
    # Poisson arrivals
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
        _log(f"poisson load {load}: {nb} batches")
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
    return dict(workload="serving: index 320,000 DNA strings (32,000 bases U{4500..5500} x 10 "
                         "copies, Poisson(0.05 len) edits); 10,000 queries (70% re-mutated "
                         "members, 30% fresh U{1000..10000}), K_q in {2,5,10}% of |q|",
                params=SERVING, gen_s=round(gen_s, 1), index_build_s=round(build_s, 3),
                saturation_qps=round(sat_qps, 1), saturation_batch=max_batch,
                candidates_per_query=round(ncand / nq, 2),
                poisson=sweeps, p50_ms=sweeps[-1]["p50_ms"], p99_ms=sweeps[-1]["p99_ms"],
                recall_vs_source=dict(sampled_member_queries=int(len(pick)),
                                      source_within_Kq=true_n, found=hit,
                                      recall=round(hit / true_n, 4) if true_n else None))


def run_forms(ej, ctx, chars, offs, prm, args):
    """The plain per-stage form (default knobs, two-pass verification) and the
    batched form (persistent verification replayed from a captured HIP graph,
    knobs from the autotuner), timed on the same device-resident input."""
    flags = ej.FLAG_TIMING
    defaults = ctx.knobs()
    ctx.tune_set("verify_mode", 0)
    res, ms, stage = time_join(ctx, chars, offs, prm, args.steps, args.warmup, flags)
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
                                  L=prm["L"], reps=2)
    knobs = ctx.knobs()
    gflags = flags | (ej.FLAG_GRAPH if knobs["verify_mode"] >= 1 else 0)
    res, ms, stage = time_join(ctx, chars, offs, prm, args.steps, args.warmup, gflags)
    batched = dict(res=res, ms=ms, stage=stage, knobs=knobs, autotune_best_ms=tune_ms,
                   kernel=VERIFY_KERNEL[res.verify_form])
    for k, v in defaults.items():
        ctx.tune_set(k, v)
    return dict(plain=plain, batched=batched)


def roofline(res, stage, prm, kern):
    """Algorithmic integer operations per step of the dominant kernel over
    its own device time per step (events around each launch)."""
    if stage.get("verify", 0.0) >= stage.get("embed", 0.0) and res.verify_columns:
        cells = res.verify_columns * (prm["K"] + 1)
        ops = cells / 32.0 * OPS_PER_WORD_STEP
        t = stage["verify_kernel"] / 1000.0
        nl = max(1, res.verify_launches)
        work = dict(launches_per_step=res.verify_launches,
                    avg_launch_ms=round(stage["verify_kernel"] / nl, 4),
                    band_cells=int(cells), text_columns=int(res.verify_columns),
                    gcells_per_s=round(cells / t / 1e9, 2) if t > 0 else None,
                    ukkonen_2k1_gcells_per_s=round(res.verify_columns * (2 * prm["K"] + 1)
                                                   / t / 1e9, 2) if t > 0 else None)
    else:
        kern = "k_embed"
        ops = res.walk_steps * OPS_PER_WALK_STEP
        t = stage["embed"] / 1000.0
        work = dict(walk_steps=int(res.walk_steps),
                    gsteps_per_s=round(res.walk_steps / t / 1e9, 2) if t > 0 else None)
    achieved = ops / t / 1e12 if t > 0 else 0.0
    peak = MI355X_INT32_LANE_OPS / 1e12
    return dict(bound="alu", kernel=kern, achieved=round(achieved, 4), peak=round(peak, 2),
                unit="T int32 lane-op/s", frac=round(achieved / peak, 5), traffic=None,
                traffic_unit="HBM bytes per launch (rocprofv3 FETCH_SIZE/WRITE_SIZE, "
                             "copy-scaled)",
                kernel_ms=round(t * 1000.0, 4), **work)


def form_summary(f, prm):
    res, ms, stage = f["res"], f["ms"], f["stage"]
    roof = roofline(res, stage, prm, f["kernel"])
    return dict(join_sec=round(ms / 1000.0, 5),
                verified_pairs_per_s=round(res.n_candidates / (ms / 1000.0), 3),
                stage_ms={k: round(v, 3) for k, v in stage.items()},
                kernel=roof["kernel"], kernel_ms=roof["kernel_ms"], roofline_frac=roof["frac"],
                knobs=f["knobs"])


def leg_bench(ej, ctx, oracle, args, col, desc, prm, stated):
    """One more workload in both forms (plain, batched) at parameters prm."""
    import torch
    _log(f"leg: {desc}")
    chars = torch.from_numpy(col.chars).cuda()
    offs = torch.from_numpy(col.offsets.astype(np.int64)).cuda()
    forms = run_forms(ej, ctx, chars, offs, prm, args)
    b = forms["batched"]
    out = dict(workload=desc, params=prm, stated=stated,
               candidates=b["res"].n_candidates, output_pairs=int(len(b["res"].pairs)),
               batched=form_summary(b, prm), plain=form_summary(forms["plain"], prm))
    if not args.no_recall:
        out["recall"] = recall_estimate(col, b["res"], prm["K"], oracle)
    return out


def uneven_bench(ej, ctx, oracle, args):
    """The batched uneven-length join (80,000 DNA strings, log-uniform
    lengths, K=400) in both forms at its recall-calibrated point."""
    import synthdata as sd
    col, stated = sd.uneven_dna(0)
    prm = dict(K=stated["K"], **CALIBRATED["uneven"])
    return leg_bench(ej, ctx, oracle, args, col,
                     "uneven DNA: 80,000 strings, base lengths log-uniform 500..20,000, clusters "
                     "geometric(0.3) <= 20, per-copy edit rate U(0, 0.08)", prm, stated)


def protein_bench(ej, ctx, oracle, args):
    """The protein-like join (400,000 strings over 25 Zipf letters, K=100)
    at its stated parameters with L = ceil(2 avg)."""
    import synthdata as sd
    col, stated = sd.protein_like(0)
    prm = dict(stated, L=int(np.ceil(2 * col.lengths().mean())))
    return leg_bench(ej, ctx, oracle, args, col,
                     "protein-like: 400,000 strings over 25 letters (Zipf 1.1), lengths lognormal "
                     "(median 400, sigma 0.8) clipped 50..4,000, clusters of mean 4, edit rate "
                     "U(0.02, 0.15)", prm, stated)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark measures one GPU; the join path has no "
                                   "multi-GPU mode", "n_gpus": args.gpus}))
        sys.exit(2)
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    import torch
    import paper_1702_00093_amd as ej
    from oracle import oracle
    if args.serving_params:
        r_, z_, m_, L_ = (int(x) for x in args.serving_params.split(","))
        SERVING.update(r=r_, z=z_, m=m_, L=L_)
    if args.serving_only:
        sctx = ej.Context(0)
        points = [tuple(int(x) for x in pt.split(",")) for pt in args.serving_sweep.split(";")] \
            if args.serving_sweep else [(SERVING["r"], SERVING["z"], SERVING["m"], SERVING["L"])]
        for r_, z_, m_, L_ in points:
            SERVING.update(r=r_, z=z_, m=m_, L=L_)
            print(json.dumps({"serving": serving_bench(ej, sctx, oracle)}), flush=True)
        return
    col, name, stated, prm = workload(args)
    chars = torch.from_numpy(col.chars.copy()).cuda()
    offs = torch.from_numpy(col.offsets.astype(np.int64)).cuda()
    ctx = ej.Context(0)
    forms = run_forms(ej, ctx, chars, offs, prm, args)
    head = forms["batched"]
    res, ms, stage = head["res"], head["ms"], head["stage"]
    cand = res.n_candidates
    value = cand / (ms / 1000.0)
    # context run at the stated parameters (one join, not the headline)
    stated_info = None
    if prm != stated:
        r2, ms2, st2 = time_join(ctx, chars, offs, stated, 2, 1, ej.FLAG_TIMING)
        stated_info = dict(params=stated, join_ms=round(ms2, 3), candidates=r2.n_candidates,
                           output_pairs=int(len(r2.pairs)),
                           stage_ms={k: round(v, 3) for k, v in st2.items()})
    roof = roofline(res, stage, prm, head["kernel"])
    if (roof["kernel"].startswith("k_verify") and args.workload == "medium" and prm["K"] == 500
            and prm == dict(stated, **CALIBRATED["medium"])):
        roof["traffic"] = measured_traffic(roof["kernel"], "medium_K500")
    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "verified candidate pairs/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": name, "K": prm["K"], "r": prm["r"], "z": prm["z"], "m": prm["m"],
                   "L": res.L, "params": "stated" if prm == stated else "recall-calibrated",
                   "form": ("batched: autotuned knobs, verification "
                            + VERIFY_FORM[res.verify_form]),
                   "candidates": cand, "raw_candidates": res.n_raw,
                   "output_pairs": int(len(res.pairs)), "join_sec": round(ms / 1000.0, 5),
                   "stage_ms": {k: round(v, 3) for k, v in stage.items()},
                   "knobs": head["knobs"],
                   "plain_form": form_summary(forms["plain"], prm)},
        "roofline": roof,
    }
    if stated_info:
        out["config"]["stated_params_run"] = stated_info
    if not args.no_recall:
        out["config"]["recall"] = recall_estimate(col, res, prm["K"], oracle)
    if not args.no_uneven:
        try:
            out["uneven"] = uneven_bench(ej, ctx, oracle, args)
        except Exception as e:  # reported, never hides the join line
            out["uneven"] = {"error": f"{type(e).__name__}: {e}"}
    if args.with_protein:
        try:
            out["protein"] = protein_bench(ej, ctx, oracle, args)
        except Exception as e:  # reported, never hides the join line
            out["protein"] = {"error": f"{type(e).__name__}: {e}"}
    if not args.no_serving:
        try:
            out["serving"] = serving_bench(ej, ctx, oracle)
        except Exception as e:  # reported, never hides the join line
            out["serving"] = {"error": f"{type(e).__name__}: {e}"}
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(col, prm, oracle)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
