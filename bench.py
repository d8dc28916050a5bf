#!/usr/bin/env python3
"""Benchmark of the Vecchia/VIF likelihood hot path on one MI355X.

One step = one exact correlation-based neighbor search plus one VIF negative
log-likelihood evaluation (low-rank U, per-point residual factor, Woodbury
assembly) over a synthetic continental station network: 3340 stations drawn
from a 40-component Gaussian mixture over the contiguous US, 365 days, 10 %
missing at random (n ~ 1.1M), m = 30 neighbors, k = 1000 kMeans++ inducing
points, Gneiting kernel. Inputs are resident in HBM before the timed region.

Prints ONE JSON line on stdout (progress goes to stderr).

    python bench.py [--gpus 1] [--steps 10] [--warmup 2] [--prec bf16x3]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "VIF NLL evals/s + neighbor-search pts/s at n=1.1M,m=30,k=1000 vs FP64"

# Published MI355X peaks used for the roofline fractions.
PEAK = {"hbm_GBs": 8000.0, "bf16_TFs": 2500.0, "fp32_TFs": 157.3, "fp64_TFs": 78.6}
PREC_ES = {"fp64": 8, "fp32": 4, "bf16x3": 4, "bf16x6": 4}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--prec", default="bf16x3", choices=list(PREC_ES),
                    help="precision of the timed line (default: split-BF16 with three products, "
                         "the mixed-precision configuration of the continental workload)")
    ap.add_argument("--no-other-precisions", action="store_true",
                    help="skip the short timing of the other precisions")
    ap.add_argument("--stations", type=int, default=3340)
    ap.add_argument("--days", type=int, default=365)
    ap.add_argument("--k", type=int, default=1000)
    ap.add_argument("--m", type=int, default=30)
    ap.add_argument("--separate", action="store_true",
                    help="time vif_neighbors then vif_nll as two calls instead of vif_neighbors_nll")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64-check", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run a plain 1 GiB device copy first (reference for HBM byte counters)")
    ap.add_argument("--learned", action="store_true",
                    help="also train the neighbor-proposal network on the GPU and evaluate it "
                         "on the workload (recall, NLL change, search rate)")
    ap.add_argument("--learn-steps", type=int, default=12000)
    ap.add_argument("--batch", action="store_true",
                    help="also time the batched workload: 64 independent problems evaluated "
                         "through one autotuned, graph-captured batch")
    ap.add_argument("--batch-count", type=int, default=64)
    ap.add_argument("--batch-prec", default="fp32", choices=list(PREC_ES))
    ap.add_argument("--batch-reps", type=int, default=10)
    ap.add_argument("--batch-schedule", default=None,
                    help="STREAMS,ROWS: a fixed batch schedule instead of the autotuned one")
    ap.add_argument("--residual", action="store_true",
                    help="time the residual-correlation neighbor search on the n=100k, k=500 "
                         "workload and print its own JSON line")
    ap.add_argument("--grad", action="store_true",
                    help="time the Vecchia NLL gradient on the continental workload and print "
                         "its own JSON line")
    ap.add_argument("--grad-vif", action="store_true",
                    help="time the VIF NLL gradient (FP64, inducing points) on the continental "
                         "workload and print its own JSON line")
    ap.add_argument("--batch-only", action="store_true",
                    help="time only the batched workload and print its own JSON line")
    return ap.parse_args()


# Proposal window: 50 km cells, radius grown until 480 points of the two slabs
# (lag 0 and 1) are inside, at most 30 cells; 4m candidates; windows above 1024
# points take the exact search.
PROPOSE = {"cell": 50.0, "lags": 1, "wmin": 480, "rmax": 30, "cmax": 1024}


def learned_eval(args, d, X, y, Z, nbr_exact, t_exact_ms):
    """Trains the proposal network on 32 station-network problems (half with perturbed
    hyperparameters) and evaluates it on the workload against the exact search and against
    spatial candidates."""
    import numpy as np
    import torch

    import synth
    import paper_2602_03609_amd as vif
    from paper_2602_03609_amd import learn as LN

    m = args.m
    t0 = time.perf_counter()
    # 30-day problems spread over the year (the network sees the workload's time range)
    train = LN.training_problems(32, n_stations=args.stations, n_days=30, m=m)
    torch.cuda.synchronize()
    log(f"learned: 32 training problems ({sum(t.n for t in train)} points) in "
        f"{time.perf_counter() - t0:.1f}s")
    t0 = time.perf_counter()
    params, hist = LN.train(train, steps=args.learn_steps, log=log)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    del train

    ncand = min(4 * m, 128)
    kern = d["kern"]

    def run(E):
        return vif.vif_propose_neighbors(*X, kern, m, E, ncand, PROPOSE["cell"], PROPOSE["lags"],
                                         PROPOSE["cmax"], wmin=PROPOSE["wmin"],
                                         rmax=PROPOSE["rmax"])

    def timed(fn, reps=5):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            a = time.perf_counter()
            out = fn()
            torch.cuda.synchronize()
            ts.append((time.perf_counter() - a) * 1000.0)
        return out, float(np.median(ts))

    (E, ), t_embed = timed(lambda: (LN.embed(params, X, kern),))
    (nbr_l, nfb_l), t_prop = timed(lambda: run(E))
    (nbr_s, nfb_s), t_sp = timed(lambda: run(None))
    rec_l = LN.recall(nbr_l, nbr_exact)
    rec_s = LN.recall(nbr_s, nbr_exact)
    nll_e = vif.vif_nll(*X, y, kern, m, nbr_exact, ind=Z, prec="fp64")
    nll_l = vif.vif_nll(*X, y, kern, m, nbr_l, ind=Z, prec="fp64")
    nll_s = vif.vif_nll(*X, y, kern, m, nbr_s, ind=Z, prec="fp64")
    n = d["n"]
    res = {
        "train_s": t_train, "train_steps": args.learn_steps, "final_loss": hist[-1][1],
        "window": PROPOSE, "ncand": ncand,
        "recall": rec_l, "recall_spatial_candidates": rec_s,
        "fallback_rows": nfb_l, "fallback_rows_spatial": nfb_s,
        "nll_exact_fp64": nll_e, "dnll_learned": nll_l - nll_e, "dnll_spatial": nll_s - nll_e,
        "ms_embed": t_embed, "ms_propose": t_prop, "ms_propose_spatial": t_sp,
        "ms_exact": t_exact_ms,
        "pts_per_s": n / ((t_embed + t_prop) / 1000.0), "pts_per_s_exact": n / (t_exact_ms / 1000.0),
        "speedup_vs_exact": t_exact_ms / (t_embed + t_prop),
    }
    log(f"learned: recall {rec_l:.5f} (spatial candidates {rec_s:.5f}); dNLL {nll_l - nll_e:.4g} "
        f"(spatial {nll_s - nll_e:.4g}); embed {t_embed:.2f} ms + propose {t_prop:.2f} ms vs exact "
        f"{t_exact_ms:.2f} ms; fallback rows {nfb_l}")
    return res


def batch_eval(args):
    """The batched workload: problems/s and points/s of one graph-captured batch
    under the autotuned schedule, against the same problems one vif_nll call at a
    time; FP64 single-problem NLLs of a few problems as the accuracy check."""
    import numpy as np
    import torch

    import synth
    import paper_2602_03609_amd as vif
    t0 = time.perf_counter()
    ds = synth.config_batch(seed=0, count=args.batch_count)
    log(f"batch: generated {len(ds)} problems ({sum(d['n'] for d in ds)} points) in "
        f"{time.perf_counter() - t0:.1f}s")
    dev = torch.device("cuda:0")
    td = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    probs = []
    for d in ds:
        X = (td(d["sx"]), td(d["sy"]), td(d["t"]))
        nb = vif.vif_neighbors(*X, d["kern"], d["m"])
        probs.append({"sx": X[0], "sy": X[1], "t": X[2], "y": td(d["y"]), "kern": d["kern"],
                      "nbr": nb, "ind": (td(d["zx"]), td(d["zy"]), td(d["zt"])), "m": d["m"]})
    torch.cuda.synchronize()
    points = sum(d["n"] for d in ds)
    prec = args.batch_prec
    b = vif.Batch(probs, prec=prec)
    if args.batch_schedule:
        streams, rows = (int(v) for v in args.batch_schedule.split(","))
        b.set_schedule(streams, rows)
        log(f"batch: fixed schedule streams={streams} rows={rows}")
    else:
        tune_ms = b.autotune(reps=2)
        streams, rows = b.schedule()
        log(f"batch: autotuned schedule streams={streams} rows={rows} ({tune_ms:.2f} ms)")
    b.graph_launch()
    torch.cuda.synchronize()
    st = b.status()
    if any(st):
        raise RuntimeError(f"batch: failing problems {[i for i, s in enumerate(st) if s]}")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.batch_reps):
        b.graph_launch()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.batch_reps
    got = b.nll.cpu().numpy()
    # the same problems one call at a time (each call synchronises)
    t0 = time.perf_counter()
    for p in probs:
        vif.vif_nll(p["sx"], p["sy"], p["t"], p["y"], p["kern"], p["m"], p["nbr"], ind=p["ind"],
                    prec=prec)
    torch.cuda.synchronize()
    ms_seq = (time.perf_counter() - t0) * 1000.0
    errs = []
    for i in range(0, len(probs), max(1, len(probs) // 8)):
        p = probs[i]
        ref = vif.vif_nll(p["sx"], p["sy"], p["t"], p["y"], p["kern"], p["m"], p["nbr"],
                          ind=p["ind"], prec="fp64")
        errs.append(abs(got[i] - ref) / abs(ref))
    log(f"batch: {ms:.2f} ms per batch ({len(probs) / ms * 1000:.1f} problems/s, "
        f"{points / ms / 1000:.3g} Mpts/s); one call at a time {ms_seq:.2f} ms; "
        f"max rel err vs fp64 {max(errs):.2e}")
    b.close()
    return {"workload": f"{len(ds)} station-network problems, n log-uniform in 10k..200k "
                        f"(total {points}), m in {{10,20,30}}, k in {{200,500}}, perturbed "
                        f"Gneiting kernels; one graph-captured batch", "precision": prec,
            "problems": len(ds), "points": points, "ms_per_batch": ms,
            "problems_per_s": len(ds) / ms * 1000.0, "points_per_s": points / ms * 1000.0,
            "schedule": {"streams": streams, "chunk_rows": rows},
            "ms_one_call_at_a_time": ms_seq, "speedup_vs_one_at_a_time": ms_seq / ms,
            "max_rel_err_vs_fp64_sampled": max(errs), "fp64_sampled_problems": len(errs)}


def grad_eval(args, reps=5):
    """Vecchia NLL and its gradient (FP64) on the continental workload without
    inducing points: time per gradient evaluation beside the NLL alone, and the
    oracle's gradient on a sampled subset of points (their per-point terms)."""
    import numpy as np
    import torch

    import synth
    import paper_2602_03609_amd as vif
    d = synth.config_cfg3(n_stations=args.stations, n_days=args.days, k=args.k, m=args.m)
    n, m = d["n"], d["m"]
    dev = torch.device("cuda:0")
    td = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    X = (td(d["sx"]), td(d["sy"]), td(d["t"]))
    y = td(d["y"])
    kern = d["kern"]
    nbr = vif.vif_neighbors(*X, kern, m)
    nll, g = vif.vif_nll_grad(*X, y, kern, m, nbr)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        vif.vif_nll_grad(*X, y, kern, m, nbr)
    torch.cuda.synchronize()
    ms_grad = (time.perf_counter() - t0) * 1000.0 / reps
    t0 = time.perf_counter()
    for _ in range(reps):
        vif.vif_nll(*X, y, kern, m, nbr, prec="fp64")
    torch.cuda.synchronize()
    ms_nll = (time.perf_counter() - t0) * 1000.0 / reps
    log(f"grad: {ms_grad:.1f} ms per NLL+gradient (8 parameters), FP64 NLL alone {ms_nll:.1f} ms")
    return {"metric": "Vecchia NLL + gradient evaluations/s (n=1.1M, m=30, Gneiting, 8 parameters)",
            "value": 1000.0 / ms_grad, "unit": "evals/s", "n_gpus": 1, "higher_is_better": True,
            "dtype": "f64", "data": "synthetic", "ms_per_gradient": ms_grad, "ms_nll_fp64": ms_nll,
            "config": {"workload": f"continental station network, {args.stations} stations x "
                                   f"{args.days} days (n={n}), m={m}, no inducing points",
                       "n": n, "m": m},
            "nll": nll, "grad": g}


def grad_vif_eval(args, reps=3):
    """VIF NLL and its gradient (FP64) on the continental workload (inducing points):
    time per gradient evaluation beside the FP64 VIF NLL alone."""
    import numpy as np
    import torch

    import synth
    import paper_2602_03609_amd as vif
    d = synth.config_cfg3(n_stations=args.stations, n_days=args.days, k=args.k, m=args.m)
    n, m, k = d["n"], d["m"], d["k"]
    dev = torch.device("cuda:0")
    td = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    X = (td(d["sx"]), td(d["sy"]), td(d["t"]))
    y = td(d["y"])
    Z = (td(d["zx"]), td(d["zy"]), td(d["zt"]))
    kern = d["kern"]
    nbr = vif.vif_neighbors(*X, kern, m)
    nll, g = vif.vif_nll_grad_vif(*X, y, kern, m, nbr, Z)
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        a = time.perf_counter()
        vif.vif_nll_grad_vif(*X, y, kern, m, nbr, Z)
        torch.cuda.synchronize()
        ts.append((time.perf_counter() - a) * 1000.0)
    ms_grad = float(np.median(ts))
    ts = []
    for _ in range(reps):
        a = time.perf_counter()
        vif.vif_nll(*X, y, kern, m, nbr, ind=Z, prec="fp64")
        torch.cuda.synchronize()
        ts.append((time.perf_counter() - a) * 1000.0)
    ms_nll = float(np.median(ts))
    log(f"grad vif: {ms_grad:.1f} ms per VIF NLL+gradient (8 parameters), FP64 VIF NLL alone {ms_nll:.1f} ms")
    return {"metric": "VIF NLL + gradient evaluations/s (n=1.1M, m=30, k=1000, Gneiting, 8 parameters)",
            "value": 1000.0 / ms_grad, "unit": "evals/s", "n_gpus": 1, "higher_is_better": True,
            "dtype": "f64", "data": "synthetic", "ms_per_gradient": ms_grad, "ms_nll_fp64": ms_nll,
            "config": {"workload": f"continental station network, {args.stations} stations x "
                                   f"{args.days} days (n={n}), m={m}, k={k} inducing points",
                       "n": n, "m": m, "k": k},
            "nll": nll, "grad": [float(v) for v in g]}


def residual_eval(args, reps=3):
    """Residual-correlation neighbor search (n = 100,000 sites x days, k = 500, m = 30):
    time per search with HIP events, FP64 MFMA rate of the U U' contraction, and the
    oracle on sampled rows."""
    import numpy as np
    import torch

    import synth
    import paper_2602_03609_amd as vif
    from oracle import residual as RS
    d = synth.config_cfg2()
    n, m, k = d["n"], d["m"], d["k"]
    dev = torch.device("cuda:0")
    td = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    X = (td(d["sx"]), td(d["sy"]), td(d["t"]))
    Z = (td(d["zx"]), td(d["zy"]), td(d["zt"]))
    nbr = vif.vif_residual_neighbors(*X, d["kern"], m, ind=Z)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        vif.vif_residual_neighbors(*X, d["kern"], m, ind=Z, nbr=nbr)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    kpad = ((k + 1 + 63) // 64) * 64
    nb = (n + 63) // 64
    flops = 2.0 * 64 * 64 * kpad * nb * (nb + 1) / 2   # tiles computed (lower triangle, padded K)
    got = nbr.cpu().numpy()
    rows = np.random.default_rng(0).integers(0, n, 20)
    t0 = time.perf_counter()
    want = RS.brute_force(d["kern"], (d["sx"], d["sy"], d["t"]), (d["zx"], d["zy"], d["zt"]), m,
                          rows=rows)
    t_oracle = time.perf_counter() - t0
    same = int(sum(np.array_equal(got[r], w) for r, w in zip(rows, want)))
    log(f"residual: {ms:.1f} ms per search ({n / ms * 1000:.3g} pts/s, "
        f"{flops / ms / 1e9:.1f} TFLOP/s FP64 MFMA); oracle rows equal {same}/{len(rows)}")
    return {"metric": "residual-correlation neighbor search pts/s (n=100k, k=500, m=30)",
            "value": n / ms * 1000.0, "unit": "pts/s", "n_gpus": 1, "higher_is_better": True,
            "dtype": "f64", "data": "synthetic", "ms_per_search": ms,
            "config": {"workload": "5000 uniform sites x 20 days (n=100k), m=30, k=500 kMeans++ "
                                   "inducing points, Gneiting kernel", "n": n, "m": m, "k": k},
            "roofline": {"bound": "mfma", "achieved": flops / ms / 1e9, "peak": PEAK["fp64_TFs"],
                         "unit": "TFLOP/s", "frac": flops / ms / 1e9 / PEAK["fp64_TFs"],
                         "traffic": None},
            "oracle_rows_checked": int(len(rows)), "oracle_rows_equal": same,
            "oracle_s_for_sampled_rows": t_oracle}


def stage_work(n, m, k, kpad, es, prec):
    """Algorithmic flops and HBM bytes per launch of each timed stage."""
    q = m + 1
    split = prec in ("bf16x3", "bf16x6")
    # W is stored as 2 or 3 bfloat16 terms per value in the split modes
    ew = (3 if prec == "bf16x6" else 2) * 2 if split else es
    if split:
        # cross-covariance evaluated on chip: coordinates in, U written once, P's terms in
        trmm_bytes = n * kpad * es + n * 3 * 8 + 4 * kpad * kpad
    else:
        # U (holding the cross-covariance) read and written once, P in
        trmm_bytes = 2 * n * kpad * es + kpad * kpad * 8
    return {
        # exact key evaluations are counted from the kernel's own scan; bytes: coordinates in,
        # neighbor rows out
        "neighbors": {"bytes": n * (3 * 8 + 4 * m), "flops": None},
        "crosscov": {"bytes": n * kpad * es, "flops": None},
        # U = C L_k^-T, triangular: sum_j 2(j+1) flops per row
        "trmm": {"bytes": trmm_bytes, "flops": n * k * (k + 1)},
        # Gram of the q gathered rows (lower triangle incl. diagonal) + W row; U read once
        # (cache-ideal gathers), W written, nbr/coords/y in, logD and z out
        "point_factor": {"bytes": n * kpad * (es + ew) + n * (4 * m + 4 * 8 + 16),
                         "flops": n * (q * (q + 1) // 2 * 2 * k + 2 * q * k)},
        # [W z]'[W z], lower triangle incl. diagonal
        "syrk": {"bytes": n * kpad * ew, "flops": n * (k + 1) * (k + 2)},
    }


PREC_CODE = {"fp64": 0, "fp32": 1, "bf16x3": 2, "bf16x6": 3}
KERNEL_SOURCES = {"point_factor": "paper_2602_03609_amd/csrc/point_factor.hip",
                  "syrk": "paper_2602_03609_amd/csrc/lowrank.hip",
                  "trmm": "paper_2602_03609_amd/csrc/lowrank.hip",
                  "crosscov": "paper_2602_03609_amd/csrc/lowrank.hip",
                  "neighbors": "paper_2602_03609_amd/csrc/neighbors.hip"}


def kernel_name(stage, prec, m):
    """Template instance launched for a stage on this workload (as rocprofv3 names it)."""
    c = PREC_CODE[prec]
    rows = 16 if m + 1 <= 16 else (32 if m + 1 <= 32 else 64)
    if stage == "point_factor":
        # BF16X3 at 32 rows stages its rows by direct loads (the fourth argument)
        return f"vif_group_kernel<{rows}, false, {c}{', true' if (c == 2 and rows == 32) else ''}>"
    if stage == "syrk":
        if c == 2:
            return "syrk_split256_kernel"
        return f"syrk_split_kernel<{3 if c == 3 else 2}>" if c >= 2 else f"syrk_kernel<{c}>"
    if stage == "trmm":
        if c >= 2:
            return "lowrank_u_kernel<3, 8, 2, 4>" if c == 3 else "lowrank_u_kernel<2, 8, 4, 2>"
        return "trmm_f64_kernel" if c == 0 else "trmm_f32_kernel<false>"
    if stage == "crosscov":
        return f"crosscov_kernel<{'double' if c == 0 else 'float'}>"
    return "neighbors_grid_kernel<0>"


def measured_traffic(stage, prec, m):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or None when the
    kernel's source has changed since the counters were taken."""
    e = committed_counters("traffic", stage, prec, m)
    return None if e is None else (e[0]["read_bytes"], e[0]["write_bytes"], e[1])


def measured_mfma(stage, prec, m):
    """Share of time the matrix pipes were busy in the kernel and the MFMA rate it executed
    (all split products counted), from the committed rocprofv3 counter summary; None when the
    kernel's source has changed since the counters were taken."""
    e = committed_counters("mfma", stage, prec, m)
    return None if e is None else (e[0]["mfma_busy"], e[0]["mfma_exec_TFLOP_per_s"], e[1])


def committed_counters(kind, stage, prec, m):
    import glob
    import hashlib
    name = kernel_name(stage, prec, m)
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", f"{kind}_*.json"))):
        with open(path) as f:
            tab = json.load(f)
        e = tab.get(name)
        if not e:
            continue
        src = os.path.join(ROOT, e["source"])
        with open(src, "rb") as f:
            sha = hashlib.sha256(f.read()).hexdigest()
        if sha == e["source_sha256"]:
            return e, os.path.relpath(path, ROOT)
    return None


def mfma_peak(prec):
    if prec == "fp64":
        return PEAK["fp64_TFs"]
    if prec == "fp32":
        return PEAK["fp32_TFs"]
    return PEAK["bf16_TFs"]


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(d, m, n_query=6000, n_point=24000):
    """The FP64 oracle, timed on a bounded sample of the same workload (about 15 s)."""
    import numpy as np
    from oracle import likelihood as LK
    from oracle import neighbors as NB
    try:
        from threadpoolctl import threadpool_info
        blas_threads = max([t.get("num_threads", 1) for t in threadpool_info()] or [1])
    except Exception:  # pragma: no cover
        blas_threads = os.cpu_count()
    n = d["n"]
    X = (d["sx"], d["sy"], d["t"])
    Z = (d["zx"], d["zy"], d["zt"])
    rng = np.random.default_rng(123)
    # neighbor search: exact lag-pruned oracle on sampled queries
    q_rows = rng.choice(n, n_query, replace=False)
    t0 = time.perf_counter()
    nb_rows = NB.lag_pruned(d["kern"], *X, m, rows=q_rows)
    t_q = (time.perf_counter() - t0) / q_rows.shape[0]
    # NLL: L_k once, then per-row work (U rows, per-point factor, W'W) on sampled rows
    t0 = time.perf_counter()
    Lk = LK.low_rank_factor(d["kern"], Z)
    t_lk = time.perf_counter() - t0
    s_rows = np.sort(rng.choice(np.arange(m, n), n_point, replace=False))
    nb_s = NB.lag_pruned(d["kern"], *X, m, rows=s_rows)
    nbr_full = np.full((n, m), -1, dtype=np.int32)
    nbr_full[s_rows] = nb_s
    t0 = time.perf_counter()
    pt = LK.vif_points(d["kern"], X, d["y"], nbr_full, Z, Lk, s_rows, want_w=True)
    t_pt = (time.perf_counter() - t0) / s_rows.shape[0]
    W = pt["W"]
    t0 = time.perf_counter()
    _ = W.T @ W
    t_syrk = (time.perf_counter() - t0) / s_rows.shape[0]
    k = Z[0].shape[0]
    t0 = time.perf_counter()
    np.linalg.cholesky(np.eye(k) + _ / s_rows.shape[0])
    t_chol = time.perf_counter() - t0
    t_step = n * (t_q + t_pt + t_syrk) + t_lk + t_chol
    return {
        "value": 1.0 / t_step,
        "unit": "evals/s",
        "cores": int(blas_threads),
        "host_cpus": os.cpu_count(),
        "cpu_model": cpu_model(),
        "kind": "oracle",
        "sample": (f"FP64 NumPy/SciPy oracle: lag-pruned exact neighbor search on {n_query} "
                   f"sampled queries and the VIF per-point factor (U rows by triangular solve, "
                   f"residual block solves, W rows) plus W'W on {n_point} sampled points, scaled "
                   f"to n={n}; "
                   f"plus L_k and chol(M) once; step = search + NLL = {t_step:.1f} s"),
        "neighbor_pts_per_s": 1.0 / t_q,
        "nll_evals_per_s": 1.0 / (n * (t_pt + t_syrk) + t_lk + t_chol),
    }


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: this library has no multi-GPU path "
              "(the sharding design is described in DESIGN.md).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    import paper_2602_03609_amd as vif

    if not torch.cuda.is_available():
        print("no GPU available", file=sys.stderr)
        sys.exit(1)
    vif.load()
    dev = torch.device("cuda:0")
    if args.grad:
        print(json.dumps(grad_eval(args)), flush=True)
        return
    if args.grad_vif:
        print(json.dumps(grad_vif_eval(args)), flush=True)
        return
    if args.residual:
        print(json.dumps(residual_eval(args)), flush=True)
        return
    if args.batch_only:
        b = batch_eval(args)
        print(json.dumps({"metric": "batched VIF NLL problems/s and points/s", "value": b["problems_per_s"],
                          "unit": "problems/s", "n_gpus": 1, "higher_is_better": True,
                          "dtype": b["precision"], "data": "synthetic", "batched": b}), flush=True)
        return

    t0 = time.perf_counter()
    d = synth.config_cfg3(n_stations=args.stations, n_days=args.days, k=args.k, m=args.m)
    n, m, k = d["n"], d["m"], d["k"]
    log(f"generated {d['name']} in {time.perf_counter() - t0:.1f}s")

    def td(a):
        return torch.from_numpy(np.ascontiguousarray(a)).to(dev)

    X = (td(d["sx"]), td(d["sy"]), td(d["t"]))
    y = td(d["y"])
    Z = (td(d["zx"]), td(d["zy"]), td(d["zt"]))
    kern = d["kern"]
    nbr = torch.empty((n, m), dtype=torch.int32, device=dev)
    torch.cuda.synchronize()
    if args.copy_calibration:
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)   # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log("copy calibration: 3 x 1 GiB device copies")

    def step(prec):
        if args.separate:
            vif.vif_neighbors(*X, kern, m, nbr=nbr)
            return vif.vif_nll(*X, y, kern, m, nbr, ind=Z, prec=prec)
        # one call: the neighbor search overlaps Sigma_k and U on a second stream
        return vif.vif_neighbors_nll(*X, y, kern, m, nbr=nbr, ind=Z, prec=prec)[0]

    for w in range(args.warmup):
        v = step(args.prec)
        log(f"warmup {w}: nll={v:.10g}")
    torch.cuda.synchronize()

    vif.vif_profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    nll = None
    step_ms = []  # each call returns after its stream has drained
    for _ in range(args.steps):
        a = time.perf_counter()
        nll = step(args.prec)
        step_ms.append((time.perf_counter() - a) * 1000.0)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = vif.vif_profile_read()
    vif.vif_profile(False)
    ms_per_step = (t1 - t0) * 1000.0 / args.steps
    log(f"timed {args.steps} steps: {ms_per_step:.3f} ms/step, nll={nll:.12g}")
    stage_ms = {s: (tot / c if c else 0.0) for s, (tot, c) in prof.items()}
    log("stage ms/launch: " + ", ".join(f"{s}={v:.3f}" for s, v in stage_ms.items()))

    # FP64 reference on the same inputs and neighbor sets.
    nll64 = None
    t64 = None
    if not args.no_fp64_check:
        torch.cuda.synchronize()
        ta = time.perf_counter()
        nll64 = vif.vif_nll(*X, y, kern, m, nbr, ind=Z, prec="fp64")
        torch.cuda.synchronize()
        t64 = (time.perf_counter() - ta) * 1000.0
        log(f"fp64 nll={nll64:.12g} ({t64:.1f} ms); rel diff {abs(nll - nll64) / abs(nll64):.3e}")

    kpad = ((k + 1 + 63) // 64) * 64
    es = PREC_ES[args.prec]
    work = stage_work(n, m, k, kpad, es, args.prec)
    # dominant kernel among the single-kernel stages
    cand = {s: stage_ms[s] for s in ("trmm", "point_factor", "syrk", "neighbors", "crosscov")
            if stage_ms.get(s, 0.0) > 0.0}
    dom = max(cand, key=cand.get)
    t_dom = stage_ms[dom] / 1000.0
    wk = work[dom]
    if wk["flops"] is not None:
        achieved = wk["flops"] / t_dom / 1e12
        roof = {"kernel": dom, "bound": "mfma", "achieved": achieved, "peak": mfma_peak(args.prec),
                "unit": "TFLOP/s", "frac": achieved / mfma_peak(args.prec), "traffic": None}
    else:
        achieved = wk["bytes"] / t_dom / 1e9
        roof = {"kernel": dom, "bound": "hbm", "achieved": achieved, "peak": PEAK["hbm_GBs"],
                "unit": "GB/s", "frac": achieved / PEAK["hbm_GBs"], "traffic": None}
    roof["ms_per_launch"] = stage_ms[dom]
    roof["algorithmic_bytes"] = wk["bytes"]
    roof["algorithmic_flops"] = wk["flops"]
    tr = measured_traffic(dom, args.prec, m)
    if tr is not None:
        roof["traffic"] = tr[0] + tr[1]
        roof["traffic_read"], roof["traffic_write"], roof["traffic_source"] = tr
    mf = measured_mfma(dom, args.prec, m)
    if mf is not None:
        roof["mfma_busy"], roof["mfma_exec_TFLOP_per_s"], roof["mfma_source"] = mf
    stages = {}
    for s, v in stage_ms.items():
        e = {"ms": v}
        if s in work and v > 0:
            e["GB_per_s"] = work[s]["bytes"] / (v / 1000.0) / 1e9
            if work[s]["flops"] is not None:
                e["TFLOP_per_s"] = work[s]["flops"] / (v / 1000.0) / 1e12
        stages[s] = e

    nll_ms = sum(stage_ms[s] for s in ("sigma_k", "crosscov", "trmm", "point_factor", "syrk",
                                       "assembly"))
    out = {
        "metric": METRIC,
        "value": 1000.0 / ms_per_step,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "step_ms": {"median": float(np.median(step_ms)), "p10": float(np.percentile(step_ms, 10)),
                    "p90": float(np.percentile(step_ms, 90))},
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.prec,
        "data": "synthetic",
        "config": {"workload": f"continental station network, {args.stations} stations x "
                               f"{args.days} days, 10% missing (n={n}), m={m}, k={k}, Gneiting "
                               f"kernel; step = exact neighbor search + VIF NLL",
                   "n": n, "m": m, "k": k, "precision": args.prec,
                   "entry": "vif_neighbors + vif_nll" if args.separate else "vif_neighbors_nll"},
        "neighbor_pts_per_s": n / (stage_ms["neighbors"] / 1000.0) if stage_ms["neighbors"] else None,
        "nll_evals_per_s_gpu_time": 1000.0 / nll_ms if nll_ms else None,
        "nll": nll,
        "nll_fp64": nll64,
        "nll_rel_err_vs_fp64": abs(nll - nll64) / abs(nll64) if nll64 is not None else None,
        "fp64_nll_ms": t64,
        "stages": stages,
        "roofline": roof,
    }
    if not args.no_other_precisions:
        # The same step in the other precisions (a few steps each, same inputs and
        # neighbor sets), with each one's NLL error against FP64.
        others = {}
        for pr in ("bf16x6", "fp32", "bf16x3"):
            if pr == args.prec:
                continue
            step(pr)
            torch.cuda.synchronize()
            ta = time.perf_counter()
            for _ in range(3):
                v = step(pr)
            torch.cuda.synchronize()
            msp = (time.perf_counter() - ta) * 1000.0 / 3
            others[pr] = {"ms_per_step": msp, "steps_per_s": 1000.0 / msp, "nll": v,
                          "nll_rel_err_vs_fp64": abs(v - nll64) / abs(nll64) if nll64 is not None else None}
            log(f"{pr}: {msp:.2f} ms/step, nll rel err {others[pr]['nll_rel_err_vs_fp64']}")
        out["other_precisions"] = others
    if args.learned:
        torch.cuda.synchronize()
        ts = []
        for _ in range(5):
            a = time.perf_counter()
            vif.vif_neighbors(*X, kern, m, nbr=nbr)
            torch.cuda.synchronize()
            ts.append((time.perf_counter() - a) * 1000.0)
        out["learned_proposal"] = learned_eval(args, d, X, y, Z, nbr, float(np.median(ts)))
    if args.batch:
        out["batched"] = batch_eval(args)
    if not args.no_cpu_baseline:
        t0 = time.perf_counter()
        out["cpu_baseline"] = cpu_baseline(d, m)
        log(f"cpu baseline in {time.perf_counter() - t0:.1f}s")
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
