#!/usr/bin/env python3
"""Throughput of the mini-batch landmark kernel k-means hot path on one MI355X.

One step = the whole path on one synthetic dataset, inputs already in HBM:
  kkm_fit    -- seed only: the library draws the landmarks and the k-means++ uniforms on the host
                inside the step; then per mini-batch the landmark block and loop, the batch-wide
                distance pass with FP64 re-decisions, member counts, batch medoids (Eq. 10) and the
                merge (Eq. 11-13);
  kkm_assign -- every sample of the dataset against the fitted medoids (Eq. 2).

Default workload: the 64-d precision workload -- N = 10^6 samples, a 100-component anisotropic
Gaussian mixture (means uniform in [-10, 10]^64, per-dimension std uniform in [0.5, 2], float32),
RBF sigma = 8, C = 100, B = 50 mini-batches, s = 0.02 (400 landmarks per batch), T = 20 -- timed in
the plain FP32 form and in the bfloat16 forms (BF16x3: split products; BF16: one product gating the
FP64 re-decisions), each for --steps steps after --warmup.

Metric: algorithmic kernel evaluations per second (Eq. 18's n|L| per batch plus the n x C medoid
blocks, plus N x C for the assign pass) and samples assigned per second, FP32 against the bfloat16
forms, with the assign latency at a fixed request size.  Printed as one JSON line with a roofline
entry for the dominant kernel (HIP events on the library's stream inside the timed steps) and the
FP64 oracle timed on the host on a bounded prefix of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

WORKLOADS = {
    # name: (config index, description)
    "mixture16": (1, "gaussian-mixture N=100000 d=16 K=20 rbf(sigma=4) C=20 B=10 s=0.1 T=20"),
    "mixture64": (3, "gaussian-mixture N=1000000 d=64 K=100 aniso rbf(sigma=8) C=100 B=50 s=0.02 T=20"),
    "rings": (0, "two-rings N=2000 d=2 float64 rbf(sigma=1) C=2 B=1 s=1 T=30 random-init"),
    "md": (2, "md-frames N=200000 A=50 templates=10 rmsd(sigma=1.5) C=50 B=20 s=0.05 T=20"),
}

PEAK_FP32_VECTOR = 157.3e12   # published MI355X FP32 FLOP/s (vector and matrix cores)
PEAK_FP64_VECTOR = 78.6e12    # published MI355X FP64 FLOP/s
PEAK_BF16_MATRIX = 2.5e15     # published MI355X dense BF16 matrix-core FLOP/s

# HBM bytes per launch from rocprofv3 FETCH_SIZE / WRITE_SIZE passes (scaled by the copy-kernel
# calibration: FETCH_SIZE x 2.0, WRITE_SIZE x 1.0), keyed by (kernel, workload), with the source file
# and its SHA-1 prefix at measurement time: a changed kernel source reports null.
TRAFFIC_MEASURED = {
    ("mfma_dist_kernel", "mixture64"): (16.42e6, "k_mfma.hip", "233890992b32"),
    ("landmark_phase_kernel", "mixture64"): (3.63e6, "k_landmark.hip", "15eb76f94bb8"),
    ("mfma_assign1_kernel", "mixture64"): (260.34e6, "k_mfma.hip", "233890992b32"),
    ("rmsd_pairs_kernel+mfma_dist_kernel", "md"): (102.45e6, "k_mfma.hip", "233890992b32"),
    ("rmsd_pairs_kernel+mfma_assign1_kernel", "md"): (231.14e6, "k_mfma.hip", "233890992b32"),
}


def _traffic():
    import hashlib
    out = {}
    for key, (nbytes, src, sha) in TRAFFIC_MEASURED.items():
        path = os.path.join(ROOT, "paper_1710_03013_amd", "csrc", src)
        try:
            now = hashlib.sha1(open(path, "rb").read()).hexdigest()[:12]
        except OSError:
            continue
        if now == sha:
            out[key] = nbytes
    return out


TRAFFIC = _traffic()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def dist_flops_per_eval(kind: str, d: int) -> float:
    """Algorithmic FP work of one kernel evaluation in the batch-wide pass:
    dot product 2d, squared distance 3, scaling + exponential 2, coefficient FMA 2."""
    if kind == "linear":
        return 2 * d + 2
    if kind == "rbf":
        return 2 * d + 7
    # RMSD: 9 correlation sums over A atoms (18 A) and the key-matrix solve
    A = d // 3
    return 18 * A + KEY_SOLVE_FLOPS


# FP64 flops of one key-matrix solve as the library's code performs it: coefficients with their
# rounding terms ~142 (det N over 2x2 minors 72, the key matrix 20, ||R||^2 18, det R and its
# absolute terms 16, the rest 16), ~37 per Laguerre step at the 4.7 steps a pair of MD frames takes
# on average from (Ga + Gb) / 2, the acceptance test 17 and r^2 3.
KEY_SOLVE_FLOPS = 142 + 37 * 4.7 + 17 + 3


def landmark_flops_per_launch(ell: int, updates: int, C: int) -> float:
    """Algorithmic FP64 work of one landmark-loop launch: every assignment evaluated on the
    landmarks costs l^2 adds for S = K_LL Z, l adds for g^ and 3 l C for Eq. 15; the loop
    evaluates (landmark updates + 1) assignments.  (K_LL itself is built by another kernel.)"""
    return (updates + 1) * (ell * ell + ell + 3 * ell * C)


def cpu_baseline(X, cfg, seed, max_batches):
    """The FP64 oracle, as it stands, on a bounded sample of the same workload: the fit of the first
    `max_batches` stride batches (a prefix of the step's fit, same per-batch sizes and draws) and an
    assign pass of one batch's rows against the resulting medoids."""
    import kkm_inputs as ki
    from oracle import kkm as okkm
    from oracle.kernels import Kernel
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        threads = 1
    N, B = X.shape[0], cfg["B"]
    k = min(B, max_batches)
    n = (N + B - 1) // B
    idx = np.asarray([i + B * j for j in range(n) for i in range(k) if i + B * j < N])
    Xp = X[idx]
    L = ki.draw_all_landmarks(seed, N, B, cfg["s"])[:k]
    kern = Kernel(cfg["kernel"], cfg.get("sigma", 1.0), cfg.get("n_atoms", 0))
    uniforms = ki.draw_kmpp_uniforms(seed, cfg["C"]) if cfg["init"] == "kmeans++" else None
    init_labels = (ki.draw_init_labels(seed, len(ki.batch_index_sets(N, B)[0]), cfg["C"])
                   if cfg["init"] == "random" else None)
    t0 = time.perf_counter()
    ref = okkm.fit(Xp, cfg["C"], kern, k, cfg["T"], L, init=cfg["init"], kmpp_uniforms=uniforms,
                   init_labels=init_labels)
    t1 = time.perf_counter()
    rows = Xp[: len(idx) // k]
    okkm.assign(kern, rows, okkm.medoid_model(ref))
    t2 = time.perf_counter()
    evals = ref.evals + rows.shape[0] * cfg["C"]
    return {"value": evals / (t2 - t0), "unit": "kernel evals/s", "cores": int(threads), "kind": "oracle",
            "sample": f"fit of the first {k} of {B} stride batches ({len(idx)} samples, {t1 - t0:.1f} s) and an "
                      f"assign pass of {rows.shape[0]} samples ({t2 - t1:.1f} s); BLAS threads={threads}, numpy "
                      f"elementwise single-threaded"}


SERVING_DESC = ("resident models of md-frames (rmsd, C=50) and mixture64 (rbf, C=100); assign sizes log-uniform "
                "[1,65536]; 5% fit jobs N log-uniform [1e4,5e5] (md capped at 2e5), C in {10,50,100}, B=10, s=0.05")


def _serving_plan(rng, rate, seconds, data, prec, burst=None):
    """Poisson arrivals at `rate` for `seconds` (or `burst` requests all at t = 0) of the serving mix."""
    import kkm_inputs as ki
    c4, c3 = ki.datasets.CONFIGS[3], ki.datasets.CONFIGS[2]
    if burst:
        arrivals = np.zeros(burst)
    else:
        n_req = max(1, int(rate * seconds))
        arrivals = np.cumsum(rng.exponential(1.0 / rate, size=n_req))
    plan = []
    for a in arrivals:
        fam = "mix64" if rng.random() < 0.5 else "md"
        if rng.random() < 0.05:
            N = min(int(round(np.exp(rng.uniform(np.log(1e4), np.log(5e5))))), data[fam].shape[0])
            C = int(rng.choice([10, 50, 100]))
            o = int(rng.integers(0, data[fam].shape[0] - N + 1))
            kw = dict(kernel="rbf", sigma=c4["sigma"]) if fam == "mix64" else \
                dict(kernel="rmsd", sigma=c3["sigma"], n_atoms=c3["n_atoms"])
            kw.update(C=C, B=10, s=0.05, max_iter=20, seed=int(rng.integers(1 << 30)), precision=prec)
            plan.append(("fit", float(a), fam, (o, N), kw))
        else:
            n = int(round(np.exp(rng.uniform(0.0, np.log(65536)))))
            o = int(rng.integers(0, data[fam].shape[0] - n + 1))
            plan.append(("assign", float(a), fam, (o, n), None))
    return plan


def _serve(models, data, plan, prec, budget_bytes, seconds):
    """Run one arrival plan through the serving loop; returns its summary."""
    from paper_1710_03013_amd.serve import KkmBackend, Server
    be = KkmBackend(n_streams=4, precision=prec)
    if budget_bytes is None:
        # the tight budget: just above the largest single request of the plan, so that every request
        # is admissible alone but big ones cannot run beside each other
        need = [be.fit_bytes(data[fam][o:o + n], kw) if kind == "fit"
                else be.assign_bytes(models[fam], n, False) for kind, _, fam, (o, n), kw in plan]
        budget_bytes = int(1.1 * max(need))
    srv = Server(be, budget_bytes=int(budget_bytes), assign_slots=4, fit_workers=2)
    for k_, m in models.items():
        srv.add_model(k_, m)
    reqs = []
    t0 = time.perf_counter()
    i = 0
    while i < len(plan) or not srv.idle:
        now = time.perf_counter() - t0
        while i < len(plan) and plan[i][1] <= now:
            kind, a, fam, (o, n), kw = plan[i]
            X = data[fam][o:o + n]
            reqs.append(srv.submit_fit(X, arrival=t0 + a, **kw) if kind == "fit"
                        else srv.submit_assign(fam, X, arrival=t0 + a))
            i += 1
        srv.poll()
        if time.perf_counter() - t0 > seconds * 20 + 60:
            raise TimeoutError("serving run did not drain")
    wall = time.perf_counter() - t0
    lat_a = np.array([r.latency for r in reqs if r.kind == "assign" and r.error is None]) * 1e3
    lat_f = np.array([r.latency for r in reqs if r.kind == "fit" and r.error is None]) * 1e3
    samples = sum(r.n for r in reqs if r.kind == "assign" and r.error is None)
    pct = lambda v, q: float(np.percentile(v, q)) if v.size else None
    return {"requests": len(reqs), "assign_requests": int(lat_a.size), "fit_jobs": int(lat_f.size),
            "errors": sum(1 for r in reqs if r.error is not None), "wall_s": wall,
            "assign_p50_ms": pct(lat_a, 50), "assign_p99_ms": pct(lat_a, 99),
            "fit_p50_ms": pct(lat_f, 50), "fit_p99_ms": pct(lat_f, 99),
            "samples_assigned_per_s": samples / wall, "requests_per_s": len(reqs) / wall,
            "launches": srv.launches, "peak_hbm_gb_admitted": srv.peak_in_use / 1e9,
            "budget_waits": srv.budget_waits, "budget_gb": budget_bytes / 1e9}


def serving_at_load(models, data, prec, seconds, budget_bytes, small_budget_bytes=None, burst=300, seed=7):
    """Saturation first (a burst of the mix, all arriving at t = 0: requests per second while it drains),
    then Poisson arrivals at 25 / 50 / 80 % of it under the stated budget, and the 80 % load once more
    under a budget small enough to hold requests back (by default 1.1x the largest request of that
    run)."""
    rng = np.random.default_rng(seed)
    sat = _serve(models, data, _serving_plan(rng, 0, 0, data, prec, burst=burst), prec, budget_bytes, seconds)
    lam = sat["requests_per_s"]
    log(f"[serve] saturation: {lam:.1f} requests/s, {sat['samples_assigned_per_s']:.3g} samples/s")
    runs = []
    for frac in (0.25, 0.5, 0.8):
        res = _serve(models, data, _serving_plan(rng, frac * lam, seconds, data, prec), prec, budget_bytes, seconds)
        res.update(load=frac, rate_per_s=frac * lam)
        log(f"[serve] {int(frac * 100)}% load ({frac * lam:.1f}/s): assign p50 {res['assign_p50_ms']:.3f} ms, "
            f"p99 {res['assign_p99_ms']:.3f} ms")
        runs.append(res)
    tight = _serve(models, data, _serving_plan(rng, 0.8 * lam, seconds, data, prec), prec, small_budget_bytes, seconds)
    tight.update(load=0.8, rate_per_s=0.8 * lam)
    log(f"[serve] 80% load, {tight['budget_gb']:.2f} GB budget: {tight['budget_waits']} budget waits, "
        f"assign p99 {tight['assign_p99_ms']:.3f} ms")
    return {"saturation": sat, "at_load": runs, "tight_budget": tight}


def serving_models(prec):
    import torch
    import kkm_inputs as ki
    import paper_1710_03013_amd as kk
    dev = torch.device("cuda:0")
    X4, _ = ki.datasets.config_data(3)
    X3, _ = ki.datasets.config_data(2)
    data = {"mix64": torch.from_numpy(X4).to(dev), "md": torch.from_numpy(X3).to(dev)}
    c4, c3 = ki.datasets.CONFIGS[3], ki.datasets.CONFIGS[2]
    fit_prec = prec if prec != "bf16" else "bf16x3"
    models = {"mix64": kk.kkm_fit(data["mix64"], "rbf", sigma=c4["sigma"], C=c4["C"], B=c4["B"], s=c4["s"],
                                  max_iter=c4["T"], precision=fit_prec, seed=2003)[0],
              "md": kk.kkm_fit(data["md"], "rmsd", sigma=c3["sigma"], n_atoms=c3["n_atoms"], C=c3["C"], B=c3["B"],
                               s=c3["s"], max_iter=c3["T"], precision=fit_prec, seed=2002)[0]}
    torch.cuda.synchronize()
    return models, data


def serving_bench(args) -> int:
    """Serving form: fitted models of the MD-frame and 64-d mixture workloads resident in HBM, Poisson
    streams of assign requests (sizes log-uniform in [1, 65536]) with fit jobs on ~5% of the arrivals,
    admitted by an HBM budget, at 25 / 50 / 80 % of the measured saturation rate.  Inputs are resident
    before their arrival stamp.  Reports p50/p99 latency from the arrival stamp to the host seeing
    completion, and assigned samples/s, per load."""
    prec = args.precision or "fp32"
    log("[serve] generating the 64-d mixture and the MD frames, fitting the resident models")
    models, data = serving_models(prec)
    res = serving_at_load(models, data, prec, args.serving_seconds, args.serving_budget_gb * 1e9,
                          None if args.serving_small_budget_gb is None else args.serving_small_budget_gb * 1e9)
    out = {"metric": "serving: assign latency p50/p99 and samples assigned/s under a Poisson request stream",
           "value": res["at_load"][-1]["samples_assigned_per_s"], "unit": "samples/s", "n_gpus": 1,
           "higher_is_better": True, "dtype": {"fp32": "f32", "bf16x3": "bf16x3+f32", "bf16": "bf16+f32",
                                               "fp64": "f64"}[prec],
           "data": "synthetic",
           "config": {"workload": "serving: " + SERVING_DESC, "precision": prec,
                      "seconds_per_load": args.serving_seconds, "budget_gb": args.serving_budget_gb},
           "serving": res}
    print(json.dumps(out), flush=True)
    return 0


def restarts_bench(args) -> int:
    """Best of R k-means++ restarts of the workload (seeds 2000 + config .. + R - 1): R fits and R FP64
    cost passes over all of X per step, timed over --steps steps after --warmup."""
    import torch
    import kkm_inputs as ki
    from paper_1710_03013_amd.restarts import fit_best_of
    k_idx, desc = WORKLOADS[args.workload]
    cfg = dict(ki.datasets.CONFIGS[k_idx])
    prec = args.precision or ("fp64" if cfg["dtype"] == "f64" else "fp32")
    X, _ = ki.datasets.config_data(k_idx)
    Xd = torch.from_numpy(X).to("cuda:0")
    kw = dict(kernel=cfg["kernel"], sigma=cfg.get("sigma", 1.0), n_atoms=cfg.get("n_atoms", 0), C=cfg["C"],
              B=cfg["B"], s=cfg["s"], max_iter=cfg["T"], init="kmeans++", precision=prec)
    R = args.restarts
    for _ in range(args.warmup):
        fit_best_of(Xd, restarts=R, seed=2000 + k_idx, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, _, info = fit_best_of(Xd, restarts=R, seed=2000 + k_idx, **kw)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    out = {"metric": f"best of {R} k-means++ restarts: fits per second (fit + FP64 cost each)",
           "value": R * args.steps / elapsed, "unit": "fits/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": elapsed / args.steps * 1e3, "higher_is_better": True,
           "dtype": prec, "data": "synthetic",
           "config": {"workload": desc, "restarts": R, "precision": prec},
           "restart_costs": [float(c) for c in info["restart_costs"]], "chosen_restart": int(info["restart"])}
    print(json.dumps(out), flush=True)
    return 0


def sweep_bench(args) -> int:
    """Accuracy and time against (B, s) on the 16-d mixture (the experiment of Sec. 4.2 / Fig. 5 on this
    workload): one seed-only fit per pair, its majority-vote accuracy and NMI against the generating
    components, its wall time and FP32 cost; then the (B, s) procedure of Sec. 4.2 for a time budget
    and a memory budget, with its check on one mini-batch against the reference (B_min, 1)."""
    import torch
    import kkm_inputs as ki
    import paper_1710_03013_amd as kk
    from paper_1710_03013_amd import tuning
    cfg = dict(ki.datasets.CONFIGS[1])
    X, y = ki.datasets.config_data(1)
    Xd = torch.from_numpy(X).to("cuda:0")
    N, d = X.shape
    kspec = kk._kernel("rbf", cfg["sigma"])
    common = dict(kernel="rbf", sigma=cfg["sigma"], C=cfg["C"], max_iter=cfg["T"], seed=2001, precision="fp32")
    rows = []
    for B in [int(b) for b in args.sweep_b.split(",")]:
        for sv in [float(x) for x in args.sweep_s.split(",")]:
            need = kk.kkm_fit_workspace_bytes(N, d, kk.KKM_F32, kspec, C=cfg["C"], B=B, s=sv, max_iter=cfg["T"],
                                              sampling="stride", init="kmeans++", precision="fp32", seed=2001,
                                              landmarks=None, kmpp_uniforms=None, init_labels=None, init_medoids=None)
            if need == 0:
                rows.append({"B": B, "s": sv, "supported": False, "reason": kk.lib().kkm_last_error().decode()})
                continue
            kk.kkm_fit(Xd, B=B, s=sv, **common)            # warm-up (kernel loading, workspace)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            model, labels, info = kk.kkm_fit(Xd, B=B, s=sv, **common)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            lab = labels.cpu().numpy()
            rows.append({"B": B, "s": sv, "supported": True, "seconds": wall,
                         "accuracy": tuning.majority_accuracy(y, lab), "nmi": tuning.nmi(y, lab),
                         "cost": kk.kkm_cost(model, Xd), "landmarks_per_batch": kk.kkm_landmark_count(N // B, sv),
                         "workspace_bytes": need})
            log(f"[sweep] B={B} s={sv}: {rows[-1]['seconds'] * 1e3:.2f} ms, accuracy {rows[-1]['accuracy']:.4f}")
    mem = int(args.sweep_memory_gb * 1e9)
    ch = tuning.choose_batches_and_fraction(Xd, args.sweep_time_budget, mem, kernel="rbf", sigma=cfg["sigma"],
                                            C=cfg["C"], max_iter=cfg["T"], seed=2001)
    # the check of Sec. 4.2 on one mini-batch: the chosen s against s = 1 on the first batch of the chosen B
    rows0 = Xd[0::ch.B]
    _, lab_ref, _ = kk.kkm_fit(rows0, B=1, s=1.0, **common)
    _, lab_ch, _ = kk.kkm_fit(rows0, B=1, s=ch.s, **common)
    check = {"rows": int(rows0.shape[0]), "nmi_vs_full_support": tuning.nmi(lab_ref.cpu().numpy(), lab_ch.cpu().numpy())}
    out = {"metric": "clustering accuracy and fit time against (B, s) on the 16-d mixture (Sec. 4.2, Fig. 5)",
           "value": max(r["accuracy"] for r in rows if r["supported"]), "unit": "majority-vote accuracy",
           "n_gpus": 1, "higher_is_better": True, "dtype": "f32", "data": "synthetic",
           "config": {"workload": WORKLOADS["mixture16"][1]}, "sweep": rows,
           "procedure": {"time_budget_s": args.sweep_time_budget, "memory_budget_bytes": mem, "B_min": ch.B_min,
                         "B": ch.B, "s": ch.s, "expected_s": ch.expected_s, "met": ch.met, "trials": ch.trials,
                         "check_on_one_batch": check}}
    print(json.dumps(out), flush=True)
    return 0


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="mixture64", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default=None, choices=["fp32", "fp64", "bf16x3", "bf16"],
                    help="one form only (default: FP32 and the bfloat16 forms where they apply)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--latency-requests", type=int, default=200)
    ap.add_argument("--latency-size", type=int, default=4096)
    ap.add_argument("--no-phase-timing", action="store_true",
                    help="do not record HIP events around the fit phases (no roofline entry)")
    ap.add_argument("--serving", action="store_true", help="run the serving benchmark instead")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run ten device-to-device copies of MIB MiB (the reference kernel for scaling "
                         "rocprofv3 FETCH_SIZE / WRITE_SIZE counts to bytes) and exit")
    ap.add_argument("--restarts", type=int, default=0, metavar="R",
                    help="instead: time the best of R k-means++ restarts of the workload (fits and FP64 costs)")
    ap.add_argument("--sweep", action="store_true",
                    help="instead: accuracy and time against (B, s) on the 16-d mixture, and the (B, s) procedure")
    ap.add_argument("--sweep-b", default="2,4,8,16")
    ap.add_argument("--sweep-s", default="0.025,0.05,0.1,0.2,0.4,0.7,1.0")
    ap.add_argument("--sweep-time-budget", type=float, default=0.01, help="seconds, for the (B, s) procedure")
    ap.add_argument("--sweep-memory-gb", type=float, default=0.5, help="workspace budget of the (B, s) procedure")
    ap.add_argument("--serving-seconds", type=float, default=3.0, help="arrival window per load")
    ap.add_argument("--serving-budget-gb", type=float, default=200.0, help="HBM admission budget")
    ap.add_argument("--serving-small-budget-gb", type=float, default=None,
                    help="budget of the extra 80%% load run that makes admission wait "
                         "(default: 1.1x that run's largest request)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); this build has no multi-GPU path",
              file=sys.stderr)
        return 2

    import torch
    import kkm_inputs as ki
    import paper_1710_03013_amd as kk

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 2
    if args.serving:
        return serving_bench(args)
    if args.restarts > 0:
        return restarts_bench(args)
    if args.sweep:
        return sweep_bench(args)
    if args.calibrate_copy > 0:
        nbytes = args.calibrate_copy << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(10):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "copies": 10}), flush=True)
        del src, dst
        return 0
    return step_bench(args)


# bounded oracle sample per workload: stride batches of the fit (about 10-30 s of host work)
CPU_BASELINE_BATCHES = {"mixture64": 2, "mixture16": 10, "md": 1, "rings": 1}


def step_bench(args) -> int:
    import torch
    import kkm_inputs as ki
    import paper_1710_03013_amd as kk

    k_idx, desc = WORKLOADS[args.workload]
    cfg = dict(ki.datasets.CONFIGS[k_idx])
    if args.precision:
        precs = [args.precision]
    elif cfg["dtype"] == "f64":
        precs = ["fp64"]
    elif cfg["kernel"] == "rmsd":
        precs = ["fp32"]            # the bfloat16 forms are matrix-core forms of linear / RBF kernels
    else:
        precs = ["fp32", "bf16x3", "bf16"]
    seed = 2000 + k_idx
    log(f"[bench] generating {desc}")
    X, _ = ki.datasets.config_data(k_idx)
    N, d = X.shape
    C, B, s, T = cfg["C"], cfg["B"], cfg["s"], cfg["T"]
    dev = torch.device("cuda:0")
    props = torch.cuda.get_device_properties(dev)
    log(f"[bench] device {props.name} CUs={props.multi_processor_count}")
    Xd = torch.from_numpy(X).to(dev)
    batch_n = [len(ix) for ix in ki.batch_index_sets(N, B)]
    ells = [ki.landmark_count(n, s) for n in batch_n]
    results, lab_by_prec, models = {}, {}, {}
    for prec in precs:
        # seed-only fits: the library draws the landmarks and k-means++ uniforms inside every step
        fit_kw = dict(kernel=cfg["kernel"], sigma=cfg.get("sigma", 1.0), n_atoms=cfg.get("n_atoms", 0), C=C, B=B,
                      s=s, max_iter=T, init=cfg["init"], precision=prec, seed=seed)
        model = kk.kkm_model_create(cfg["kernel"], d=d, C=C, dtype=cfg["dtype"], sigma=cfg.get("sigma", 1.0),
                                    n_atoms=cfg.get("n_atoms", 0))
        wbytes = kk.kkm_fit(Xd, model=model, **fit_kw)[2]["workspace_bytes"]
        ws = torch.empty(wbytes, dtype=torch.uint8, device=dev)
        labels = torch.empty(N, dtype=torch.int32, device=dev)
        aws = torch.empty(max(256, kk.kkm_assign_workspace_bytes(model, N, prec)), dtype=torch.uint8, device=dev)
        ev_a = []

        def step(time_phases=0):
            _, _, info = kk.kkm_fit(Xd, model=model, workspace=ws, want_labels=True, time_phases=time_phases,
                                    **fit_kw)
            if time_phases:   # events around the assign pass, on the stream it runs on (the current one)
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
            kk.kkm_assign(model, Xd, precision=prec, workspace=aws, labels=labels)
            if time_phases:
                e1.record()
                ev_a.append((e0, e1))
            return info

        for w in range(args.warmup):
            step()
        torch.cuda.synchronize()
        log(f"[bench] {prec}: {args.warmup} warmup steps done")
        ev_a.clear()
        infos = []
        t0 = time.perf_counter()
        for _ in range(args.steps):
            # events only around the landmark loop and the batch-wide distance kernel (three per batch)
            # and around the assign pass
            infos.append(step(time_phases=0 if args.no_phase_timing else 2))
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        elapsed = t1 - t0
        log(f"[bench] {prec}: {args.steps} timed steps in {elapsed:.3f} s")
        assign_ms = float(np.mean([a.elapsed_time(b) for a, b in ev_a])) if ev_a else None
        # the breakdown over all phases from one more (untimed) step with events around every phase
        phase_info = step(time_phases=1) if not args.no_phase_timing else None
        torch.cuda.synchronize()
        info = infos[-1]
        evals_step = info["evals_algorithmic"] + N * C
        assigned_step = int(np.dot(batch_n, info["updates_per_batch"])) + N
        ms = ({k_: float(np.mean([i["ms"][k_] for i in infos])) for k_ in infos[0]["ms"]}
              if not args.no_phase_timing else None)
        # assign latency at a fixed request size
        lat = []
        q = Xd[: min(args.latency_size, N)]
        qlab = torch.empty(q.shape[0], dtype=torch.int32, device=dev)
        qws = torch.empty(max(256, kk.kkm_assign_workspace_bytes(model, q.shape[0], prec)), dtype=torch.uint8,
                          device=dev)
        for _ in range(args.latency_requests):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            kk.kkm_assign(model, q, precision=prec, workspace=qws, labels=qlab)
            e1.record()
            e1.synchronize()
            lat.append(e0.elapsed_time(e1))
        lat = np.asarray(lat) if lat else np.zeros(1)
        lab_by_prec[prec] = labels.clone()
        models[prec] = model
        results[prec] = {
            "kernel_evals_per_s": evals_step * args.steps / elapsed,
            "samples_assigned_per_s": assigned_step * args.steps / elapsed,
            "ms_per_step": elapsed / args.steps * 1e3,
            "assign_pass_ms": assign_ms,
            "assign_samples_per_s": N / (assign_ms * 1e-3) if assign_ms else None,
            "kernel_ms_per_step": ({"landmark_loop": ms["landmark_loop"], "dist": ms["dist"],
                                    "assign_pass": assign_ms} if ms else None),
            "phase_ms_per_step": {k_: float(v) for k_, v in phase_info["ms"].items()} if phase_info else None,
            "rows_refined_per_step": int(info["rows_refined"]),
            "medoid_candidates_per_step": int(info["medoid_candidates"]),
            "assign_latency_ms": {"request_size": int(q.shape[0]), "p50": float(np.percentile(lat, 50)),
                                  "p99": float(np.percentile(lat, 99))},
            "_infos": infos, "_ms": ms,
        }
        del ws, aws, qws, qlab, q

    # label agreement of every form's assign pass with the FP64 assign of the same fitted model, over
    # the rows whose FP64 relative margin exceeds 1e-6 (the others are ties for the label rule: rows far
    # from every medoid, whose kernel values all underflow, and exact ties)
    for prec in precs:
        if prec == "fp64":
            results[prec]["label_agreement_vs_fp64"] = 1.0
            continue
        ref, gap = kk.kkm_assign(models[prec], Xd, precision="fp64", want_gap=True)
        decisive = gap > 1e-6
        same = (ref == lab_by_prec[prec]) | ~decisive
        results[prec]["label_agreement_vs_fp64"] = float(same.float().mean().item())
        results[prec]["rows_within_1e-6_margin"] = int((~decisive).sum().item())

    # roofline entries of the primary form (the first precision), HIP events inside its timed steps
    prim = precs[0]
    r = results[prim]
    rooflines, roofline = {}, None
    if r["_ms"] is not None:
        info, ms = r["_infos"][-1], r["_ms"]
        upd = [int(u) - 1 for u in info["updates_per_batch"]]   # landmark-only updates
        lm_flops = float(np.mean([landmark_flops_per_launch(ells[i], upd[i], C) for i in range(B)]))
        dist_flops = float(np.mean([batch_n[i] * ells[i] for i in range(B)])) * dist_flops_per_eval(cfg["kernel"], d)
        peak = {"fp64": PEAK_FP64_VECTOR, "fp32": PEAK_FP32_VECTOR, "bf16x3": PEAK_BF16_MATRIX,
                "bf16": PEAK_BF16_MATRIX}[prim]
        # RMSD frames of an even atom count up to 64 in float run on the matrix cores as well
        mfma = prim != "fp64" and (cfg["kernel"] != "rmsd" or
                                   (cfg["n_atoms"] % 2 == 0 and cfg["n_atoms"] <= 64 and Xd.dtype == torch.float32))
        dist_name = "mfma_dist_kernel" if mfma else "dist_kernel"
        assign_name = "mfma_assign1_kernel" if mfma else "dist_kernel"
        cands = {
            "landmark_phase_kernel": (ms["landmark_loop"], B, lm_flops, PEAK_FP64_VECTOR, "alu"),
            dist_name: (ms["dist"], B, dist_flops, peak, "mfma" if mfma else "alu"),
        }
        if cfg["kernel"] == "rmsd" and mfma:
            # the RMSD distance pass is the pair pass (FP32 cross-covariance on the matrix cores, then the
            # FP64 key-matrix solve on the VALU, which bounds it) and the segment reduction: priced as
            # FP64 ALU work on the solve's flops
            pairs = float(np.mean([batch_n[i] * ells[i] for i in range(B)]))
            cands = {"landmark_phase_kernel": cands["landmark_phase_kernel"],
                     "rmsd_pairs_kernel+mfma_dist_kernel": (ms["dist"], B, pairs * KEY_SOLVE_FLOPS,
                                                            PEAK_FP64_VECTOR, "alu")}
        if r["assign_pass_ms"] and cfg["kernel"] != "rmsd":
            # the assign pass's contraction: N x C dot products of length d
            cands[assign_name + " (assign pass)"] = (r["assign_pass_ms"], 1, 2.0 * N * C * d, peak,
                                                     "mfma" if mfma else "alu")
        elif r["assign_pass_ms"]:
            cands["rmsd_pairs_kernel+mfma_assign1_kernel (assign pass)"] = (r["assign_pass_ms"], 1,
                                                                          float(N) * C * KEY_SOLVE_FLOPS,
                                                                          PEAK_FP64_VECTOR, "alu")
        for name, (tot_ms, launches, flops, pk, bound) in cands.items():
            dur = tot_ms / launches * 1e-3
            achieved = flops / dur if dur > 0 else 0.0
            rooflines[name] = {"bound": bound, "achieved": achieved / 1e12, "peak": pk / 1e12, "unit": "TFLOP/s",
                               "frac": achieved / pk, "traffic": TRAFFIC.get((name.split()[0], args.workload)),
                               "kernel": name, "avg_launch_us": dur * 1e6, "flop_per_launch": flops,
                               "ms_per_step": tot_ms}
        dom = max(cands, key=lambda k_: cands[k_][0])
        roofline = dict(rooflines[dom])
        roofline["kernel_ms_per_step"] = r["kernel_ms_per_step"]
        roofline["phase_ms_per_step"] = r["phase_ms_per_step"]
    for prec in precs:
        results[prec].pop("_infos")
        results[prec].pop("_ms")
    ratios = {}
    for prec in precs[1:]:
        ratios[prec] = {"step_speedup": r["ms_per_step"] / results[prec]["ms_per_step"],
                        "assign_pass_speedup": (r["assign_pass_ms"] / results[prec]["assign_pass_ms"]
                                                if r["assign_pass_ms"] and results[prec]["assign_pass_ms"] else None)}
    out = {
        "metric": "kernel evals/s + samples assigned/s (BF16 vs FP32); p50/p99 assign latency",
        "value": r["kernel_evals_per_s"],
        "unit": "kernel evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "f32", "fp64": "f64", "bf16x3": "bf16x3+f32", "bf16": "bf16+f32"}[prim]
                 + " (landmark loop, medoids, merge: f64)",
        "data": "synthetic",
        "config": {"workload": desc, "N": N, "d": d, "C": C, "B": B, "s": s, "T": T, "precision": prim,
                   "draws": "seed only (landmarks and k-means++ uniforms drawn by the library inside each step)"},
        "samples_assigned_per_s": r["samples_assigned_per_s"],
        "assign_latency_ms": r["assign_latency_ms"],
        "precisions": results,
        "vs_fp32": ratios,
        "roofline": roofline,
        "rooflines": rooflines,
    }
    if not args.no_cpu_baseline:
        nb = CPU_BASELINE_BATCHES.get(args.workload, 1)
        log(f"[bench] timing the FP64 oracle on the host ({nb} batches + an assign pass)")
        out["cpu_baseline"] = cpu_baseline(X, cfg, seed, nb)
        log("[bench] oracle done")
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    _rc = main()
    if _rc:
        sys.exit(_rc)
