#!/usr/bin/env python3
"""Throughput of the mini-batch landmark kernel k-means hot path on one MI355X.

One step = the whole path on one synthetic dataset, inputs already in HBM:
  kkm_fit   -- per mini-batch: landmark block + landmark loop (one kernel with
               grid barriers), the batch-wide distance pass with FP64 re-decisions,
               member counts, batch medoids (Eq. 10) and the merge (Eq. 11-13);
  kkm_assign -- every sample of the dataset against the fitted medoids (Eq. 2).

Default workload: N = 100 000 samples, d = 16, a 20-component isotropic Gaussian
mixture (means uniform in [-10, 10]^16, std 1, float32), RBF sigma = 4,
C = 20, B = 10 mini-batches, s = 0.1 (1000 landmarks per batch), T = 20.

Metric: algorithmic kernel evaluations per second (Eq. 18's n|L| per batch plus
the n x C medoid blocks, plus N x C for the assign pass).  Printed as one JSON
line with a roofline entry for the dominant kernel (timed with HIP events on the
library's stream inside the timed steps) and the FP64 oracle timed on the host.
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

# kernel names as rocprofv3 reports them, per (kernel function, precision)
DIST_KERNEL_NAME = {("rbf", "fp32"): "mfma_dist_kernel", ("linear", "fp32"): "mfma_dist_kernel",
                    ("rbf", "bf16x3"): "mfma_dist_kernel", ("linear", "bf16x3"): "mfma_dist_kernel"}

# HBM bytes per launch from rocprofv3 FETCH_SIZE / WRITE_SIZE passes (scaled by the copy-kernel
# calibration: FETCH_SIZE x 2.0, WRITE_SIZE x 1.0), keyed by (kernel, workload), with the source file
# and its SHA-1 prefix at measurement time: a changed kernel source reports null.
TRAFFIC_MEASURED = {
    ("landmark_phase_kernel", "mixture16"): (10.579e6, "k_landmark.hip", "12c51db228ac"),
    ("mfma_dist_kernel", "mixture16"): (2.890e6, "k_mfma.hip", "8f0dd5a930b6"),
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
    # RMSD: 9 correlation sums over A atoms (18 A), key-matrix polynomial and Newton (~150)
    A = d // 3
    return 18 * A + 150


def landmark_flops_per_launch(ell: int, updates: int, C: int) -> float:
    """Algorithmic FP64 work of one landmark-loop launch: every assignment evaluated on the
    landmarks costs l^2 adds for S = K_LL Z, l adds for g^ and 3 l C for Eq. 15; the loop
    evaluates (landmark updates + 1) assignments.  (K_LL itself is built by another kernel.)"""
    return (updates + 1) * (ell * ell + ell + 3 * ell * C)


def cpu_baseline(X, cfg, landmarks, uniforms, init_labels):
    """The FP64 oracle, as it stands, on the same workload (one whole fit + one assign pass)."""
    from oracle import kkm as okkm
    from oracle.kernels import Kernel
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        threads = 1
    kern = Kernel(cfg["kernel"], cfg.get("sigma", 1.0), cfg.get("n_atoms", 0))
    t0 = time.perf_counter()
    ref = okkm.fit(X, cfg["C"], kern, cfg["B"], cfg["T"], landmarks, init=cfg["init"],
                   kmpp_uniforms=uniforms, init_labels=init_labels)
    t1 = time.perf_counter()
    okkm.assign(kern, X, okkm.medoid_model(ref))
    t2 = time.perf_counter()
    evals = ref.evals + X.shape[0] * cfg["C"]
    return {"value": evals / (t2 - t0), "unit": "kernel evals/s", "cores": int(threads), "kind": "oracle",
            "sample": f"one full fit ({t1 - t0:.1f} s) and one assign pass ({t2 - t1:.1f} s) of the same workload; "
                      f"BLAS threads={threads}, numpy elementwise single-threaded"}


def serving_bench(args) -> int:
    """Serving form: fitted models of the MD-frame and 64-d mixture workloads resident in HBM, a
    Poisson stream of assign requests (sizes log-uniform in [1, 65536]) with fit jobs on ~5% of the
    arrivals (N log-uniform in [1e4, 5e5], C in {10, 50, 100}, B = 10, s = 0.05), admitted by a
    200 GB budget.  Inputs are resident before their arrival stamp.  Reports p50/p99 latency from
    the arrival stamp to the host seeing completion, and assigned samples/s, per request rate."""
    import torch
    import kkm_inputs as ki
    import paper_1710_03013_amd as kk
    from paper_1710_03013_amd.serve import KkmBackend, Server

    prec = args.precision or "fp32"
    dev = torch.device("cuda:0")
    log("[serve] generating the 64-d mixture and the MD frames")
    X4, _ = ki.datasets.config_data(3)
    X3, _ = ki.datasets.config_data(2)
    data = {"mix64": torch.from_numpy(X4).to(dev), "md": torch.from_numpy(X3).to(dev)}
    c4, c3 = ki.datasets.CONFIGS[3], ki.datasets.CONFIGS[2]
    models = {}
    log("[serve] fitting the resident models")
    models["mix64"] = kk.kkm_fit(data["mix64"], "rbf", sigma=c4["sigma"], C=c4["C"], B=c4["B"], s=c4["s"],
                                 max_iter=c4["T"], precision=prec, seed=2003)[0]
    models["md"] = kk.kkm_fit(data["md"], "rmsd", sigma=c3["sigma"], n_atoms=c3["n_atoms"], C=c3["C"], B=c3["B"],
                              s=c3["s"], max_iter=c3["T"], precision=prec, seed=2002)[0]
    torch.cuda.synchronize()
    rates = [float(r) for r in args.serving_rates.split(",")]
    results = []
    for rate in rates:
        rng = np.random.default_rng(int(rate) + 7)
        n_req = max(1, int(rate * args.serving_seconds))
        gaps = rng.exponential(1.0 / rate, size=n_req)
        arrivals = np.cumsum(gaps)
        plan = []
        for a in arrivals:
            fam = "mix64" if rng.random() < 0.5 else "md"
            if rng.random() < 0.05:
                N = int(round(np.exp(rng.uniform(np.log(1e4), np.log(5e5)))))
                N = min(N, data[fam].shape[0])   # the MD set holds 2e5 frames
                C = int(rng.choice([10, 50, 100]))
                o = int(rng.integers(0, data[fam].shape[0] - N + 1))
                kw = dict(kernel="rbf", sigma=c4["sigma"]) if fam == "mix64" else \
                    dict(kernel="rmsd", sigma=c3["sigma"], n_atoms=c3["n_atoms"])
                kw.update(C=C, B=10, s=0.05, max_iter=20, seed=int(rng.integers(1 << 30)), precision=prec)
                plan.append(("fit", a, fam, (o, N), kw))
            else:
                n = int(round(np.exp(rng.uniform(0.0, np.log(65536)))))
                o = int(rng.integers(0, data[fam].shape[0] - n + 1))
                plan.append(("assign", a, fam, (o, n), None))
        srv = Server(KkmBackend(n_streams=4, precision=prec), budget_bytes=200 << 30, assign_slots=4, fit_workers=2)
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
                r = (srv.submit_fit(X, arrival=t0 + a, **kw) if kind == "fit"
                     else srv.submit_assign(fam, X, arrival=t0 + a))
                reqs.append(r)
                i += 1
            srv.poll()
            if time.perf_counter() - t0 > args.serving_seconds * 20 + 60:
                raise TimeoutError("serving run did not drain")
        wall = time.perf_counter() - t0
        lat_a = np.array([r.latency for r in reqs if r.kind == "assign" and r.error is None]) * 1e3
        lat_f = np.array([r.latency for r in reqs if r.kind == "fit" and r.error is None]) * 1e3
        errors = sum(1 for r in reqs if r.error is not None)
        samples = sum(r.n for r in reqs if r.kind == "assign" and r.error is None)
        res = {"rate_per_s": rate, "requests": len(reqs), "assign_requests": int(lat_a.size),
               "fit_jobs": int(lat_f.size), "errors": errors, "wall_s": wall,
               "assign_p50_ms": float(np.percentile(lat_a, 50)) if lat_a.size else None,
               "assign_p99_ms": float(np.percentile(lat_a, 99)) if lat_a.size else None,
               "fit_p50_ms": float(np.percentile(lat_f, 50)) if lat_f.size else None,
               "fit_p99_ms": float(np.percentile(lat_f, 99)) if lat_f.size else None,
               "samples_assigned_per_s": samples / wall, "launches": srv.launches,
               "peak_hbm_gb_admitted": srv.peak_in_use / 1e9}
        log(f"[serve] rate {rate}/s: {res}")
        results.append(res)
    out = {"metric": "serving: assign latency p50/p99 and samples assigned/s under a Poisson request stream",
           "value": results[-1]["samples_assigned_per_s"], "unit": "samples/s", "n_gpus": 1,
           "higher_is_better": True, "dtype": {"fp32": "f32", "bf16x3": "bf16x3+f32", "fp64": "f64"}[prec],
           "data": "synthetic",
           "config": {"workload": "serving: resident models of md-frames (rmsd, C=50) and mixture64 (rbf, C=100); "
                                  "assign sizes log-uniform [1,65536]; 5% fit jobs N in [1e4,5e5], C in {10,50,100}, "
                                  "B=10, s=0.05; HBM budget 200 GB", "precision": prec,
                      "seconds_per_rate": args.serving_seconds},
           "serving": results}
    print(json.dumps(out), flush=True)
    del srv, models, data
    import gc
    gc.collect()
    torch.cuda.synchronize()
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


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="mixture16", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default=None, choices=["fp32", "fp64", "bf16x3"])
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
    ap.add_argument("--serving-rates", default="100,400,1600", help="request rates (per second) to sweep")
    ap.add_argument("--serving-seconds", type=float, default=3.0, help="arrival window per rate")
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
    k_idx, desc = WORKLOADS[args.workload]
    cfg = dict(ki.datasets.CONFIGS[k_idx])
    prec = args.precision or ("fp64" if cfg["dtype"] == "f64" else "fp32")
    seed = 2000 + k_idx
    log(f"[bench] generating {desc}")
    X, _ = ki.datasets.config_data(k_idx)
    N, d = X.shape
    C, B, s, T = cfg["C"], cfg["B"], cfg["s"], cfg["T"]
    landmarks = ki.draw_all_landmarks(seed, N, B, s)
    uniforms = ki.draw_kmpp_uniforms(seed, C) if cfg["init"] == "kmeans++" else None
    n0 = len(ki.batch_index_sets(N, B)[0])
    init_labels = ki.draw_init_labels(seed, n0, C) if cfg["init"] == "random" else None
    dev = torch.device("cuda:0")
    props = torch.cuda.get_device_properties(dev)
    log(f"[bench] device {props.name} CUs={props.multi_processor_count} "
        f"lds/block={getattr(props, 'shared_memory_per_block', '?')}")
    Xd = torch.from_numpy(X).to(dev)
    fit_kw = dict(kernel=cfg["kernel"], sigma=cfg.get("sigma", 1.0), n_atoms=cfg.get("n_atoms", 0), C=C, B=B, s=s,
                  max_iter=T, init=cfg["init"], precision=prec, seed=seed, landmarks=landmarks,
                  kmpp_uniforms=uniforms, init_labels=init_labels)
    model = kk.kkm_model_create(cfg["kernel"], d=d, C=C, dtype=cfg["dtype"], sigma=cfg.get("sigma", 1.0),
                                n_atoms=cfg.get("n_atoms", 0))
    wbytes = kk.kkm_fit(Xd, model=model, **fit_kw)[2]["workspace_bytes"]
    ws = torch.empty(wbytes, dtype=torch.uint8, device=dev)
    labels = torch.empty(N, dtype=torch.int32, device=dev)
    aws = torch.empty(max(256, kk.kkm_assign_workspace_bytes(model, N, prec)), dtype=torch.uint8, device=dev)

    def step(time_phases=False):
        _, _, info = kk.kkm_fit(Xd, model=model, workspace=ws, want_labels=True, time_phases=time_phases,
                                **fit_kw)
        kk.kkm_assign(model, Xd, precision=prec, workspace=aws, labels=labels)
        return info

    for w in range(args.warmup):
        step()
        log(f"[bench] warmup {w + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    infos = []
    t0 = time.perf_counter()
    for k in range(args.steps):
        # events only around the two candidate dominant kernels (three per batch)
        infos.append(step(time_phases=0 if args.no_phase_timing else 2))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    log(f"[bench] {args.steps} timed steps in {t1 - t0:.3f} s")
    # the breakdown over all phases from one more (untimed) step with events around every phase
    phase_info = step(time_phases=True) if not args.no_phase_timing else None
    torch.cuda.synchronize()
    elapsed = t1 - t0
    info = infos[-1]
    evals_step = info["evals_algorithmic"] + N * C
    value = evals_step * args.steps / elapsed
    batch_n = [len(ix) for ix in ki.batch_index_sets(N, B)]
    assigned_step = int(np.dot(batch_n, info["updates_per_batch"])) + N
    ms = ({k_: float(np.mean([i["ms"][k_] for i in infos])) for k_ in infos[0]["ms"]}
          if not args.no_phase_timing else None)

    # dominant kernel: the isolated kernel with the largest time per step (HIP events around exactly
    # that kernel's launches on the library's stream, inside the timed steps)
    ells = [len(l) for l in landmarks]
    roofline = None
    rooflines = {}
    if ms is not None:
        upd = [int(u) - 1 for u in info["updates_per_batch"]]   # landmark-only updates
        lm_flops = float(np.mean([landmark_flops_per_launch(ells[i], upd[i], C) for i in range(B)]))
        dist_flops = float(np.mean([batch_n[i] * ells[i] for i in range(B)])) * dist_flops_per_eval(cfg["kernel"], d)
        dist_peak = {"fp64": PEAK_FP64_VECTOR, "fp32": PEAK_FP32_VECTOR, "bf16x3": PEAK_BF16_MATRIX}[prec]
        cands = {
            "landmark_phase_kernel": (ms["landmark_loop"], lm_flops, PEAK_FP64_VECTOR, "alu"),
            DIST_KERNEL_NAME.get((cfg["kernel"], prec), "dist_kernel"):
                (ms["dist"], dist_flops, dist_peak, "mfma" if (cfg["kernel"] != "rmsd" and prec != "fp64") else "alu"),
        }
        for name, (tot_ms, flops, peak, bound) in cands.items():
            dur = tot_ms / B * 1e-3
            achieved = flops / dur if dur > 0 else 0.0
            rooflines[name] = {"bound": bound, "achieved": achieved / 1e12, "peak": peak / 1e12, "unit": "TFLOP/s",
                               "frac": achieved / peak, "traffic": TRAFFIC.get((name, args.workload)),
                               "kernel": name, "avg_launch_us": dur * 1e6, "flop_per_launch": flops}
        dom = max(cands, key=lambda k_: cands[k_][0])
        roofline = dict(rooflines[dom])
        roofline["kernel_ms_per_step"] = {"landmark_loop": ms["landmark_loop"], "dist": ms["dist"]}
        roofline["phase_ms_per_step"] = {k_: float(v) for k_, v in phase_info["ms"].items()}

    # assign latency at a fixed request size
    lat = []
    q = Xd[: min(args.latency_size, N)]
    qlab = torch.empty(q.shape[0], dtype=torch.int32, device=dev)
    qws = torch.empty(max(256, kk.kkm_assign_workspace_bytes(model, q.shape[0], prec)), dtype=torch.uint8, device=dev)
    for r in range(args.latency_requests):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        kk.kkm_assign(model, q, precision=prec, workspace=qws, labels=qlab)
        e1.record()
        e1.synchronize()
        lat.append(e0.elapsed_time(e1))
    lat = np.asarray(lat) if lat else np.zeros(1)

    out = {
        "metric": "kernel evals/s (fit + assign, algorithmic count)",
        "value": value,
        "unit": "kernel evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "f32", "fp64": "f64", "bf16x3": "bf16x3+f32"}[prec] + " (landmark loop, medoids, merge: f64)",
        "data": "synthetic",
        "config": {"workload": desc, "N": N, "d": d, "C": C, "B": B, "s": s, "T": T, "precision": prec},
        "samples_assigned_per_s": assigned_step * args.steps / elapsed,
        "assign_latency_ms": {"request_size": int(q.shape[0]), "p50": float(np.percentile(lat, 50)),
                              "p99": float(np.percentile(lat, 99))},
        "refined_rows_per_step": int(info["rows_refined"]),
        "medoid_candidates_per_step": int(info["medoid_candidates"]),
        "roofline": roofline,
        "rooflines": rooflines,
    }
    if not args.no_cpu_baseline:
        log("[bench] timing the FP64 oracle on the host (one fit + one assign pass)")
        out["cpu_baseline"] = cpu_baseline(X, cfg, landmarks, uniforms, init_labels)
        log("[bench] oracle done")
    print(json.dumps(out), flush=True)
    # release device objects before the interpreter exits (profilers finalise after this point)
    del model, ws, labels, aws, qws, qlab, q, Xd
    import gc
    gc.collect()
    torch.cuda.synchronize()
    return 0


if __name__ == "__main__":
    _rc = main()
    if _rc:
        sys.exit(_rc)
