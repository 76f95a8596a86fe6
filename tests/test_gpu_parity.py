"""Parity of the HIP library (through the C ABI) with the FP64 oracle.

Labels must match the oracle exactly wherever the oracle's relative margin
(d2 - d1) / max(|d1|, |d2|, |K(x,x)|) exceeds 1e-6; costs within 1e-9 (FP64) or
1e-5 (FP32) relative.  Inputs are seeded synthetic sets shaped like the
workloads, at sizes the oracle finishes in seconds, spanning several 64-row
tiles with a ragged tail."""
import os
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import kkm_inputs as ki  # noqa: E402
from oracle import kkm as okkm  # noqa: E402
from oracle.kernels import Kernel  # noqa: E402

GAP = 1e-6
# relative cost tolerances per precision (the bfloat16 forms share the BF16 bar)
COST_TOL = {"fp64": 1e-9, "fp32": 1e-5, "bf16x3": 1e-3, "bf16": 1e-3}


def _kk():
    import paper_1710_03013_amd as kk
    return kk


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _labels_match(got, want, gaps, what):
    bad = (got != want) & (gaps > GAP)
    assert not bad.any(), f"{what}: {int(bad.sum())} labels differ with margin > {GAP} (first at {np.flatnonzero(bad)[:5]})"


def _medoid_model_from_rows(kk, kern, rows, dtype):
    C, d = rows.shape
    m = kk.kkm_model_create(kern.kind, d=d, C=C, dtype=dtype, sigma=kern.sigma, n_atoms=kern.n_atoms)
    kk.kkm_model_load(m, rows, np.arange(C + 1), np.ones(C))
    return m


# ------------------------------------------------------------------------------------------ assign
@pytest.mark.parametrize("kind,sigma,d,C,n,prec,dtype", [
    ("rbf", 4.0, 16, 20, 1000 + 17, "fp32", "f32"),
    ("rbf", 8.0, 64, 100, 4096 + 63, "fp32", "f32"),
    ("rbf", 1.0, 2, 2, 2000, "fp64", "f64"),
    ("linear", 1.0, 16, 7, 777, "fp32", "f32"),
    ("linear", 1.0, 5, 3, 65, "fp64", "f64"),
    ("rbf", 2.0, 3, 5, 1, "fp32", "f32"),
    ("rbf", 3.0, 33, 9, 130, "fp32", "f64"),
    ("rbf", 8.0, 64, 100, 4096 + 63, "bf16x3", "f32"),
    ("rbf", 4.0, 16, 20, 1000 + 17, "bf16x3", "f32"),
    ("linear", 1.0, 16, 7, 777, "bf16x3", "f32"),
    ("rbf", 2.0, 128, 33, 300, "bf16x3", "f32"),
    ("rbf", 2.0, 128, 33, 300, "fp32", "f32"),
    ("rbf", 8.0, 64, 100, 4096 + 63, "bf16", "f32"),
    ("rbf", 4.0, 16, 20, 1000 + 17, "bf16", "f32"),
    ("linear", 1.0, 16, 7, 777, "bf16", "f32"),
    ("rbf", 2.0, 128, 33, 300, "bf16", "f32"),
    ("rbf", 3.0, 33, 9, 130, "bf16", "f64"),
])
def test_assign_medoid_model(kind, sigma, d, C, n, prec, dtype):
    kk = _kk()
    _say(f"assign {kind} d={d} C={C} n={n} {prec} {dtype}")
    npdt = np.float64 if dtype == "f64" else np.float32
    X, _ = ki.datasets.gaussian_mixture(n + C, d, max(C, 2), seed=100 + d, sigma=1.0, dtype=npdt)
    rows, Y = X[:C], X[C:] if n > 0 else X[:0]
    kern = Kernel(kind, sigma)
    m = _medoid_model_from_rows(kk, kern, rows, dtype)
    Yd = torch.from_numpy(np.ascontiguousarray(Y)).cuda()
    lab, gap = kk.kkm_assign(m, Yd, precision=prec, want_gap=True)
    torch.cuda.synchronize()
    model = okkm.SparseModel(rows.astype(np.float64), np.arange(C + 1), np.ones(C))
    rl, rg, rd = okkm.assign(kern, Y, model)
    _labels_match(lab.cpu().numpy(), rl, rg, "assign")
    g = gap.cpu().numpy()
    fin = np.isfinite(rg) & (rg > 1e-3)
    # (a row re-decided in FP64 carries the FP64 margin; the others the margin of the pass's own sums,
    # which for plain BF16 is only as good as its wide bound: its labels and cost are checked instead)
    if prec != "bf16":
        gtol = {"fp32": (1e-3, 2e-4), "bf16x3": (1e-2, 5e-3), "fp64": (2e-7, 1e-12)}[prec]
        np.testing.assert_allclose(g[fin], rg[fin], rtol=gtol[0], atol=gtol[1])
    cost = kk.kkm_cost(m, Yd, precision=prec)
    want = okkm.cost(kern, Y, model)
    assert abs(cost - want) <= COST_TOL[prec] * max(1.0, abs(want))


def test_assign_bf16_cascade_near_duplicate_medoids():
    """Plain BF16 against medoids in near-duplicate pairs: the one-product pass cannot tell a pair apart,
    so it marks most rows (every group, the last one ragged) and the compensated products decide them
    again; the labels must still be the oracle's wherever its margin exceeds the tie bar."""
    kk = _kk()
    _say("assign bf16 cascade near-duplicate medoids")
    d, P, n = 64, 20, 3000 + 13
    X, _ = ki.datasets.gaussian_mixture(n + P, d, P, seed=321, sigma=1.0, dtype=np.float32)
    base, Y = X[:P].astype(np.float64), X[P:]
    rng = np.random.default_rng(7)
    twin = base + 0.02 * rng.standard_normal(base.shape)
    rows = np.empty((2 * P, d), dtype=np.float32)
    rows[0::2], rows[1::2] = base, twin
    kern = Kernel("rbf", 8.0)
    m = _medoid_model_from_rows(kk, kern, rows, "f32")
    Yd = torch.from_numpy(np.ascontiguousarray(Y)).cuda()
    model = okkm.SparseModel(rows.astype(np.float64), np.arange(2 * P + 1), np.ones(2 * P))
    rl, rg, _ = okkm.assign(kern, Y, model)
    # (the oracle's margins: most rows sit between the two medoids of a pair, far inside the BF16 bound)
    assert np.median(rg) < 1e-2, np.median(rg)
    for prec in ("bf16", "bf16x3", "fp32"):
        lab = kk.kkm_assign(m, Yd, precision=prec)
        torch.cuda.synchronize()
        _labels_match(lab.cpu().numpy(), rl, rg, f"assign {prec}")
    cost = kk.kkm_cost(m, Yd, precision="bf16")
    want = okkm.cost(kern, Y, model)
    assert abs(cost - want) <= COST_TOL["bf16"] * max(1.0, abs(want))


def test_assign_sparse_centroids():
    """General sparse centroids: several support rows per cluster, unequal coefficients, an empty cluster."""
    kk = _kk()
    _say("assign sparse centroids")
    X, _ = ki.datasets.gaussian_mixture(3000, 16, 6, seed=5, sigma=1.5, box=5.0)
    rng = np.random.default_rng(0)
    S = X[:40]
    offsets = np.array([0, 10, 10, 17, 30, 31, 40])
    coef = rng.uniform(0.2, 1.0, size=40)
    for j in range(6):
        a, b = offsets[j], offsets[j + 1]
        if b > a:
            coef[a:b] /= coef[a:b].sum()
    kern = Kernel("rbf", 3.0)
    m = kk.kkm_model_create("rbf", d=16, C=6, max_support=40, dtype="f32", sigma=3.0)
    kk.kkm_model_load(m, S, offsets, coef)
    exp = kk.kkm_model_export(m)
    model = okkm.SparseModel(S.astype(np.float64), offsets, coef)
    K_ss = kern(S, S)
    for j in range(6):
        a, b = offsets[j], offsets[j + 1]
        if b > a:
            w = coef[a:b]
            assert abs(exp["self"][j] - w @ K_ss[a:b, a:b] @ w) < 1e-12
        else:
            assert np.isinf(exp["self"][j])
    Y = X[40:]
    for prec in ("fp32", "bf16", "bf16x3", "fp64"):
        lab, gap = kk.kkm_assign(m, torch.from_numpy(Y).cuda(), precision=prec, want_gap=True)
        rl, rg, _ = okkm.assign(kern, Y, model)
        got = lab.cpu().numpy()
        _labels_match(got, rl, rg, f"sparse {prec}")
        assert not np.any(got == 1)


@pytest.mark.parametrize("kind,d,dtype", [("rbf", 40, "f32"), ("rbf", 16, "f64"), ("linear", 40, "f32")])
def test_assign_near_ties_decided_in_fp64(kind, d, dtype):
    """Cluster 2 repeats cluster 0's rows with coefficients scaled by 1 + 1e-4, so the two are
    1e-7 to 1e-5 apart (relative) on every row: below the FP32 error bound, so the FP32 pass lists those
    rows and the FP64 re-decision (a whole workgroup per row, the support being over 256 rows)
    decides them.  Labels must follow the oracle wherever its margin exceeds 1e-6."""
    kk = _kk()
    _say(f"assign near ties {kind} d={d} {dtype}")
    X, _ = ki.datasets.gaussian_mixture(2300, d, 4, seed=11, sigma=1.0, box=4.0)
    if kind == "linear":
        X = X / np.sqrt(d)
    rng = np.random.default_rng(3)
    A, Bs, D = X[:200], X[200:300], X[300:400]
    S = np.concatenate([A, Bs, A, D])
    offsets = np.array([0, 200, 300, 500, 600])
    cA = rng.uniform(0.2, 1.0, 200)
    cA /= cA.sum()
    cD = rng.uniform(0.2, 1.0, 100)
    cD /= cD.sum()
    coef = np.concatenate([cA, np.full(100, 0.01), cA * (1.0 + 1e-4), cD])
    sigma = 1.5 * np.sqrt(d)
    kern = Kernel(kind, sigma)
    m = kk.kkm_model_create(kind, d=d, C=4, max_support=600, dtype=dtype, sigma=sigma)
    kk.kkm_model_load(m, S, offsets, coef)
    Y = np.ascontiguousarray(X[400:], dtype=np.float32 if dtype == "f32" else np.float64)
    rl, rg, _ = okkm.assign(kern, Y.astype(np.float64), okkm.SparseModel(S.astype(np.float64), offsets, coef))
    near = (rl == 0) | (rl == 2)
    assert (near & (rg > GAP)).sum() > 50
    for prec in ("fp32", "bf16x3", "bf16", "fp64") if dtype == "f32" else ("fp32", "fp64"):
        lab, _ = kk.kkm_assign(m, torch.from_numpy(Y).cuda(), precision=prec, want_gap=True)
        _labels_match(lab.cpu().numpy(), rl, rg, f"near ties {kind} d={d} {prec}")


# ------------------------------------------------------------------------------------------ fit
def _fit_both(kk, X, kern, C, B, s, T, init, seed, prec, sampling="stride", dtype=None, **kw):
    N = X.shape[0]
    L = ki.draw_all_landmarks(seed, N, B, s, sampling)
    u = ki.draw_kmpp_uniforms(seed, C) if init == "kmeans++" else None
    n0 = len(ki.batch_index_sets(N, B, sampling)[0])
    lab0 = ki.draw_init_labels(seed, n0, C) if init == "random" else None
    med0 = kw.get("init_medoids")
    Xd = torch.from_numpy(np.ascontiguousarray(X)).cuda()
    model, labels, info = kk.kkm_fit(Xd, kern.kind, sigma=kern.sigma, n_atoms=kern.n_atoms, C=C, B=B, s=s,
                                     max_iter=T, sampling=sampling, init=init, precision=prec, seed=seed,
                                     landmarks=L, kmpp_uniforms=u, init_labels=lab0, init_medoids=med0,
                                     cost_trace=True, global_cost=kw.get("global_cost", False))
    torch.cuda.synchronize()
    _say(f"  device fit done ({info['updates_per_batch'].tolist()} updates); oracle fit")
    ref = okkm.fit(X, C, kern, B, T, L, sampling=sampling, init=init, kmpp_uniforms=u, init_labels=lab0,
                   init_medoids=med0)
    ref.parts = okkm.batches(N, B, sampling)
    return model, labels.cpu().numpy(), info, ref


def _device_updates(ref, T):
    """Label updates the device makes per batch: landmark-only updates until the landmark labels
    first repeat (at most T-1), plus the one batch-wide pass.  Read off the oracle's trajectory of
    landmark labels, which the landmark-only loop follows step for step."""
    out = []
    for lp in ref.loops:
        tr = lp.trajectory
        k = T - 1
        for t in range(1, min(len(tr), T)):
            if np.array_equal(tr[t], tr[t - 1]):
                k = t
                break
        out.append(k + 1)
    return np.asarray(out)


def _check_fit(kk, model, labels, info, ref, kern, X, T, expect="strict"):
    """Trajectory parity with the oracle, batch by batch.

    Medoid choices (Eq. 10, 12) are compared exactly, except where the oracle's minimum is tied
    (several positions within 1e-12 relative, ref.medoid_ties / ref.merge_ties): any member of the tie
    is a correct choice, rounding decides which, and the two trajectories may split from there on;
    the comparison then stops after that batch.
    expect="strict": the test's inputs are chosen so that the oracle's smallest relative label margin
    exceeds 1e-6 (asserted); labels, batch counts and update counts must be equal in every compared batch.
    expect="trajectory": the oracle takes some label decision with margin <= 1e-6, which licenses the
    device to diverge there: the first batch whose labels, counts or update counts differ must be one
    whose loop took such a decision, and the comparison stops there.
    The branch taken is printed and returned."""
    B = len(ref.updates)
    C = ref.batch_counts.shape[1]
    upd = _device_updates(ref, T)
    parts = ref.parts
    if expect == "strict":
        assert ref.min_gap > GAP, f"strict parity needs oracle margins > {GAP}; smallest is {ref.min_gap:.3g}"
    for i in range(B):
        p = parts[i]
        same = (np.array_equal(labels[p], ref.labels[p]) and np.array_equal(info["batch_counts"][i], ref.batch_counts[i])
                and info["updates_per_batch"][i] == upd[i])
        if not same:
            assert expect == "trajectory", f"batch {i}: labels, counts or update counts differ"
            assert ref.loops[i].min_gap <= GAP, f"batch {i} diverged although its oracle margins exceed {GAP}"
            _labels_match(labels[p], ref.labels[p], ref.label_gaps[p], f"fit labels, batch {i}")
            _say(f"  trajectory diverged at batch {i} of {B} (its oracle min margin {ref.loops[i].min_gap:.3g})")
            return f"diverged at batch {i}"
        split = False
        for j in range(C):
            got, want = info["batch_medoids"][i][j], ref.batch_medoids[i][j]
            if got != want:
                assert got in ref.medoid_ties[i][j], f"batch {i} cluster {j}: batch medoid {got} vs {want}, not tied"
                split = True
        for j in range(C):
            got, want = info["global_medoids"][i][j], ref.global_medoids[i][j]
            if got != want:
                assert split or got in ref.merge_ties[i][j], f"batch {i} cluster {j}: medoid {got} vs {want}, not tied"
                split = True
        if split:
            _say(f"  batches 0..{i - 1} equal; batch {i} labels equal and a tied medoid chosen otherwise "
                 f"(oracle min margin {ref.min_gap:.3g})")
            return f"tie at batch {i}"
    exp = kk.kkm_model_export(model)
    np.testing.assert_array_equal(exp["medoid_index"], ref.medoid_index)
    np.testing.assert_array_equal(exp["counts"], ref.counts)
    _say(f"  every batch equal (oracle min margin {ref.min_gap:.3g})")
    return "identical"


def test_fit_two_rings_fp64():
    """Two-ring workload at full size: exact kernel k-means (B = 1, s = 1), FP64, random labels."""
    kk = _kk()
    _say("fit rings fp64")
    X, y = ki.datasets.config_data(0)
    kern = Kernel("rbf", 1.0)
    T = 30
    model, labels, info, ref = _fit_both(kk, X, kern, 2, 1, 1.0, T, "random", 2000, "fp64")
    _check_fit(kk, model, labels, info, ref, kern, X, T)


@pytest.mark.parametrize("N,prec", [(20_000, "fp32"), (20_000, "fp64"), (100_000, "fp32"), (20_000, "bf16x3")])
def test_fit_gaussian_mixture(N, prec):
    """Mini-batch landmark form on the 16-d, 20-component mixture (B = 10, s = 0.1, T = 20)."""
    kk = _kk()
    _say(f"fit mixture N={N} {prec}")
    X, y = ki.datasets.gaussian_mixture(N, 16, 20, seed=1001, sigma=1.0)
    kern = Kernel("rbf", 4.0)
    T = 20
    model, labels, info, ref = _fit_both(kk, X, kern, 20, 10, 0.1, T, "kmeans++", 2001, prec)
    _check_fit(kk, model, labels, info, ref, kern, X, T)
    assert info["evals_algorithmic"] == ref.evals
    if ref.min_gap > GAP:
        _check_displacement(info, ref, kern, X, 20, 10, 2001)
    # partial cost of every batch (Sec. 4.1), to the cost tolerance of the precision
    np.testing.assert_allclose(info["partial_cost"], okkm.partial_costs(ref), rtol=COST_TOL[prec])


def test_fit_listed_candidates_with_small_merge_grid():
    """Selection forms by grid size: 5120 rows per batch and 150 clusters give a candidate scan of
    20 row chunks x 150 clusters (beyond the form that evaluates its candidates in place, so they are
    listed and evaluated by their own pass) but a merge of 80 x 10 tiles (small enough for every tile
    to settle its clusters itself, without the separate settle pass)."""
    kk = _kk()
    _say("fit C=150, 5120 rows per batch")
    X, _ = ki.datasets.gaussian_mixture(15360, 16, 150, seed=1501, sigma=1.0)
    kern = Kernel("rbf", 4.0)
    T = 20
    model, labels, info, ref = _fit_both(kk, X, kern, 150, 3, 0.05, T, "kmeans++", 1502, "fp32")
    _check_fit(kk, model, labels, info, ref, kern, X, T)   # oracle margins all above 1e-6 (5e-5 at least)
    np.testing.assert_allclose(info["partial_cost"], okkm.partial_costs(ref), rtol=COST_TOL["fp32"])


def test_fit_initial_labels_over_two_wide_tiles():
    """Eq. 8 for 80 clusters in 3 dimensions: rows of 4 padded dimensions take 64-wide tiles in the
    landmark block kernel, so the medoid columns span two tiles, whose per-row minima the loop kernel
    combines (the 16-d and 64-d fits cover 32-wide tiles)."""
    kk = _kk()
    _say("fit d=3, C=80")
    X, _ = ki.datasets.gaussian_mixture(8000, 3, 80, seed=4003, sigma=0.3)
    kern = Kernel("rbf", 1.0)
    T = 20
    model, labels, info, ref = _fit_both(kk, X, kern, 80, 2, 0.1, T, "kmeans++", 4004, "fp32")
    _check_fit(kk, model, labels, info, ref, kern, X, T)   # oracle margins all above 1e-6 (3.4e-5 at least)


def _check_displacement(info, ref, kern, X, C, B, seed):
    """Medoid displacement per batch (Sec. 4.1 observable) against the oracle's definition, the
    medoids before batch 0 being the k-means++ picks of the same draws."""
    idx0 = okkm.batches(X.shape[0], B)[0]
    before = idx0[okkm.kmeanspp(kern, np.asarray(X[idx0], dtype=np.float64), C, ki.draw_kmpp_uniforms(seed, C))]
    got = info["medoid_displacement"]
    for i in range(B):
        want = okkm.medoid_displacement(kern, X, before, ref.global_medoids[i])
        np.testing.assert_array_equal(np.isnan(got[i]), np.isnan(want))
        ok = ~np.isnan(want)
        np.testing.assert_allclose(got[i][ok], want[ok], rtol=1e-9, atol=1e-12)
        before = ref.global_medoids[i]


def test_fit_linear_block_ragged_explicit_medoids():
    """Linear kernel, block sampling, N not a multiple of B, explicit initial medoids."""
    kk = _kk()
    _say("fit linear block ragged")
    X, _ = ki.datasets.gaussian_mixture(5003, 8, 6, seed=3, sigma=1.0, box=6.0)
    kern = Kernel("linear")
    T = 15
    model, labels, info, ref = _fit_both(kk, X, kern, 6, 7, 0.3, T, "medoids", 9, "fp32", sampling="block",
                                         init_medoids=np.array([0, 100, 200, 300, 400, 500]))
    _check_fit(kk, model, labels, info, ref, kern, X, T)


@pytest.mark.parametrize("C,B,s,T", [(1, 3, 0.5, 5), (4, 2, 0.001, 3), (3, 5, 1.0, 1), (5, 4, 0.25, 2)])
def test_fit_edge_cases(C, B, s, T):
    """One cluster, a single landmark per batch, one update, tiny batches."""
    kk = _kk()
    _say(f"fit edge C={C} B={B} s={s} T={T}")
    X, _ = ki.datasets.gaussian_mixture(641, 4, 4, seed=C * 10 + B, sigma=1.0, box=3.0)
    kern = Kernel("rbf", 2.0)
    model, labels, info, ref = _fit_both(kk, X, kern, C, B, s, T, "kmeans++", 5, "fp32")
    _check_fit(kk, model, labels, info, ref, kern, X, T)


def test_fit_anisotropic_mixture_64d_bf16x3():
    """The 64-d, 100-component anisotropic workload at reduced N, split-bf16 products on the matrix cores."""
    kk = _kk()
    _say("fit aniso 64d bf16x3")
    X, _ = ki.datasets.gaussian_mixture(60_000, 64, 100, seed=1003, sigma=None)
    kern = Kernel("rbf", 8.0)
    T = 20
    model, labels, info, ref = _fit_both(kk, X, kern, 100, 3, 0.02, T, "kmeans++", 2003, "bf16x3")
    # the oracle meets near ties here (min margin about 2e-8): trajectory parity, branch reported
    _check_fit(kk, model, labels, info, ref, kern, X, T, expect="trajectory")
    _sampled_assign_parity(kk, model, kern, X, 5000, 79, "bf16x3", COST_TOL["bf16x3"])


def test_fit_is_deterministic():
    kk = _kk()
    _say("fit determinism")
    X, _ = ki.datasets.gaussian_mixture(30_000, 16, 20, seed=4, sigma=1.0)
    Xd = torch.from_numpy(X).cuda()
    outs = []
    for _ in range(2):
        m, lab, info = kk.kkm_fit(Xd, "rbf", sigma=4.0, C=20, B=10, s=0.1, max_iter=20, seed=77)
        outs.append((lab.cpu().numpy(), kk.kkm_model_export(m)["support"], info["global_medoids"]))
    np.testing.assert_array_equal(outs[0][0], outs[1][0])
    np.testing.assert_array_equal(outs[0][1], outs[1][1])
    np.testing.assert_array_equal(outs[0][2], outs[1][2])


def test_fit_best_of_restarts():
    """Best of four k-means++ restarts (seeds 51..54): every restart's FP64 cost and the chosen seed
    against the oracle's four fits with the same draws; the winner (not the first seed here) must
    be the oracle's best fit, batch by batch."""
    kk = _kk()
    from paper_1710_03013_amd.restarts import fit_best_of
    _say("fit best of restarts")
    X, _ = ki.datasets.gaussian_mixture(6000, 8, 6, seed=41, sigma=1.0, box=4.0)
    kern = Kernel("rbf", 2.0)
    C, B, s, T, R, seed0 = 6, 2, 0.2, 10, 4, 51
    N = X.shape[0]
    refs, costs = [], []
    for r in range(R):
        L = ki.draw_all_landmarks(seed0 + r, N, B, s, "stride")
        u = ki.draw_kmpp_uniforms(seed0 + r, C)
        ref = okkm.fit(X, C, kern, B, T, L, kmpp_uniforms=u)
        ref.parts = okkm.batches(N, B)
        assert ref.min_gap > GAP
        refs.append(ref)
        costs.append(okkm.cost(kern, X, okkm.medoid_model(ref)))
    Xd = torch.from_numpy(X).cuda()
    model, labels, info = fit_best_of(Xd, restarts=R, seed=seed0, kernel="rbf", sigma=2.0, C=C, B=B, s=s,
                                      max_iter=T)
    np.testing.assert_allclose(info["restart_costs"], costs, rtol=1e-9)
    want = int(np.argmin(costs))
    assert want != 0 and info["restart"] == want
    _check_fit(kk, model, labels.cpu().numpy(), info, refs[want], kern, X, T)


def test_fit_landmark_block_in_hbm():
    """One batch of 3500 landmarks: a workgroup's rows of K_LL exceed its LDS at every grid size, so
    the loop kernel reads them from HBM (its other variant)."""
    kk = _kk()
    _say("fit landmark block in HBM")
    X, _ = ki.datasets.gaussian_mixture(3500, 8, 5, seed=11, sigma=1.0, box=4.0)
    kern = Kernel("rbf", 2.0)
    T = 10
    model, labels, info, ref = _fit_both(kk, X, kern, 5, 1, 1.0, T, "kmeans++", 31, "fp32")
    _check_fit(kk, model, labels, info, ref, kern, X, T)


def test_fit_cooperative_launch_matches_plain():
    """The cooperative-launch flag changes how the grid-synchronised kernels are launched, not what
    they compute: both fits agree bit for bit."""
    kk = _kk()
    _say("fit cooperative vs plain")
    X, _ = ki.datasets.gaussian_mixture(20_000, 16, 20, seed=6, sigma=1.0)
    Xd = torch.from_numpy(X).cuda()
    outs = []
    for coop in (False, True):
        m, lab, info = kk.kkm_fit(Xd, "rbf", sigma=4.0, C=20, B=10, s=0.1, max_iter=20, seed=78, cooperative=coop)
        outs.append((lab.cpu().numpy(), kk.kkm_model_export(m)["support"], info["global_medoids"],
                     info["updates_per_batch"]))
    for a, b in zip(*outs):
        np.testing.assert_array_equal(a, b)


def test_fit_rejects_nonfinite_input():
    kk = _kk()
    X, _ = ki.datasets.gaussian_mixture(500, 4, 3, seed=1, sigma=1.0)
    X[123, 2] = np.nan
    with pytest.raises(kk.KkmError) as e:
        kk.kkm_fit(torch.from_numpy(X).cuda(), "rbf", sigma=1.0, C=3, B=2, s=0.5, max_iter=5, seed=1)
    assert e.value.status == -4


# ------------------------------------------------------------------------------------------ RMSD
def test_rmsd_assign_and_fit_small():
    kk = _kk()
    _say("rmsd small")
    X, y = ki.datasets.md_frames(600, A=12, n_templates=4, seed=8)
    kern = Kernel("rmsd", 1.5, 12)
    T = 10
    model, labels, info, ref = _fit_both(kk, X, kern, 4, 3, 0.2, T, "kmeans++", 3, "fp32")
    _check_fit(kk, model, labels, info, ref, kern, X, T)
    Y, _ = ki.datasets.md_frames(257, A=12, n_templates=4, seed=9)
    lab = kk.kkm_assign(model, torch.from_numpy(Y).cuda()).cpu().numpy()
    rl, rg, _ = okkm.assign(kern, Y, okkm.medoid_model(ref))
    _labels_match(lab, rl, rg, "rmsd assign")


def test_rmsd_assign_large_request():
    """An RMSD assign large enough (n >= 32768) for one lane per sample, where the sample tile is
    staged in LDS as float: sampled rows against the oracle."""
    kk = _kk()
    _say("rmsd large assign")
    A, C = 50, 50
    kern = Kernel("rmsd", 1.5, A)
    X, _ = ki.datasets.md_frames(40000 + C, A=A, n_templates=10, seed=21)   # one set of templates
    M = X[:C].reshape(C, A, 3)
    M = (M - M.mean(axis=1, keepdims=True)).reshape(C, 3 * A).astype(np.float32)
    m = kk.kkm_model_create("rmsd", d=3 * A, C=C, dtype="f32", sigma=1.5, n_atoms=A)
    kk.kkm_model_load(m, M, np.arange(C + 1), np.ones(C))
    Y = np.ascontiguousarray(X[C:])
    got = kk.kkm_assign(m, torch.from_numpy(Y).cuda()).cpu().numpy()
    rows = np.sort(np.random.default_rng(5).choice(Y.shape[0], size=1500, replace=False))
    want, gaps, _ = okkm.assign(kern, Y[rows].astype(np.float64), okkm.SparseModel(M.astype(np.float64), np.arange(C + 1), np.ones(C)))
    _labels_match(got[rows], want, gaps, "rmsd large assign")


# ------------------------------------------------------------------------------------------ full sizes
def _stride_prefix(X, B, k):
    """Rows of the first k stride batches of X (B batches), laid out so that k stride batches of the
    result are exactly those batches: row k*j + i of the result is row i + B*j of X."""
    N = X.shape[0]
    n = (N + B - 1) // B
    idx = [i + B * j for j in range(n) for i in range(k) if i + B * j < N]
    return X[np.asarray(idx)]


def _sampled_assign_parity(kk, model, kern, X, n_sample, seed, prec, cost_tol):
    rng = np.random.default_rng(seed)
    rows = np.sort(rng.choice(X.shape[0], size=n_sample, replace=False))
    Y = np.ascontiguousarray(X[rows])
    exp = kk.kkm_model_export(model)
    omodel = okkm.SparseModel(exp["support"].astype(np.float64), exp["offsets"], exp["coef"])
    want, gaps, _ = okkm.assign(kern, Y, omodel)
    Yd = torch.from_numpy(Y).cuda()
    got = kk.kkm_assign(model, Yd, precision=prec).cpu().numpy()
    _labels_match(got, want, gaps, f"sampled assign {prec}")
    c_got = kk.kkm_cost(model, Yd, precision=prec)
    c_want = okkm.cost(kern, Y, omodel)
    assert abs(c_got - c_want) <= cost_tol * abs(c_want), (c_got, c_want)


@pytest.mark.parametrize("prec,cost_tol", [("fp32", 1e-5), ("bf16x3", 1e-3), ("bf16", 1e-3)])
def test_full_size_mixture64(prec, cost_tol):
    """The 64-d workload at full size (N = 1e6, C = 100, B = 50, s = 0.02) in the benchmark's launch
    configuration: the fitted model checked on a seeded 20 000-sample subsample (assign and cost
    against the oracle), and the first three mini-batches teacher-forced against the oracle."""
    kk = _kk()
    _say(f"full mixture64 {prec}")
    cfg = ki.datasets.CONFIGS[3]
    X, _ = ki.datasets.config_data(3)
    kern = Kernel("rbf", cfg["sigma"])
    seed = 2003
    L = ki.draw_all_landmarks(seed, X.shape[0], cfg["B"], cfg["s"])
    u = ki.draw_kmpp_uniforms(seed, cfg["C"])
    Xd = torch.from_numpy(X).cuda()
    model, _, info = kk.kkm_fit(Xd, "rbf", sigma=cfg["sigma"], C=cfg["C"], B=cfg["B"], s=cfg["s"],
                                max_iter=cfg["T"], precision=prec, seed=seed, landmarks=L, kmpp_uniforms=u)
    torch.cuda.synchronize()
    assert info["global_medoids"].shape == (cfg["B"], cfg["C"])
    _sampled_assign_parity(kk, model, kern, X, 20_000, 77, prec, cost_tol)
    # first three batches: the same landmarks and k-means++ draws, teacher-forced through the oracle
    Xp = _stride_prefix(X, cfg["B"], 3)
    model3, labels3, info3, ref3 = _fit_both(kk, Xp, kern, cfg["C"], 3, cfg["s"], cfg["T"], "kmeans++", seed, prec)
    _check_fit(kk, model3, labels3, info3, ref3, kern, Xp, cfg["T"])


def test_full_size_md_frames():
    """The MD-frame workload at full size (N = 2e5 frames of 50 atoms, C = 50, B = 20, s = 0.05):
    the fitted model checked on a seeded 4000-frame subsample against the oracle's RMSD kernel."""
    kk = _kk()
    _say("full md frames")
    cfg = ki.datasets.CONFIGS[2]
    X, _ = ki.datasets.config_data(2)
    kern = Kernel("rmsd", cfg["sigma"], cfg["n_atoms"])
    Xd = torch.from_numpy(X).cuda()
    model, _, info = kk.kkm_fit(Xd, "rmsd", sigma=cfg["sigma"], n_atoms=cfg["n_atoms"], C=cfg["C"], B=cfg["B"],
                                s=cfg["s"], max_iter=cfg["T"], seed=2002)
    torch.cuda.synchronize()
    _sampled_assign_parity(kk, model, kern, X, 4000, 78, "fp32", 1e-5)


# ------------------------------------------------------------------------------------------ large assign
_LARGE = {}


def _large_assign_case():
    """150 017 rows of the 64-d anisotropic mixture against 100 medoids: more 32-row groups than the
    matrix-core pass launches workgroups (8 per CU), so every workgroup walks its grid-stride loop."""
    if not _LARGE:
        X, _ = ki.datasets.gaussian_mixture(150_017 + 100, 64, 100, seed=1013, sigma=None)
        rows, Y = X[:100], np.ascontiguousarray(X[100:])
        kern = Kernel("rbf", 8.0)
        model = okkm.SparseModel(rows.astype(np.float64), np.arange(101), np.ones(100))
        _LARGE.update(rows=rows, Y=Y, kern=kern, ref=okkm.assign(kern, Y, model), cost=okkm.cost(kern, Y, model))
    return _LARGE


@pytest.mark.parametrize("prec", ["fp32", "bf16x3", "bf16"])
def test_assign_grid_stride_every_row(prec):
    kk = _kk()
    c = _large_assign_case()
    _say(f"large assign n={c['Y'].shape[0]} {prec}")
    m = _medoid_model_from_rows(kk, c["kern"], c["rows"], "f32")
    Yd = torch.from_numpy(c["Y"]).cuda()
    lab = kk.kkm_assign(m, Yd, precision=prec).cpu().numpy()
    rl, rg, _ = c["ref"]
    _labels_match(lab, rl, rg, f"large assign {prec}")
    cost = kk.kkm_cost(m, Yd, precision=prec)
    assert abs(cost - c["cost"]) <= COST_TOL[prec] * abs(c["cost"]), (cost, c["cost"])


# ------------------------------------------------------------------------------------------ kernel block
def _rigid(rng, F):
    R = ki.datasets.random_rotations(rng, 1)[0]
    return F @ R.T + rng.uniform(-20, 20, size=3)


def test_kernel_block_rmsd_against_eigh_on_degenerate_frames():
    """FP64 RMSD kernel values against the oracle's eigh of the key matrix (1e-9 relative), on pairs
    whose largest eigenvalue is multiple or nearly so -- identical (rotated, translated) copies,
    mirror images, collinear chains, planar frames -- and on ordinary frames of the MD workload."""
    kk = _kk()
    _say("kernel block rmsd degenerate")
    rng = np.random.default_rng(44)
    A, sigma = 50, 1.5
    base, _ = ki.datasets.md_frames(6, A=A, n_templates=3, seed=45)
    frames = [f.reshape(A, 3).astype(np.float64) for f in base]
    line = np.outer(np.linspace(-20, 20, A) + rng.normal(scale=0.5, size=A), [0.3, -0.5, 0.81])
    plane = np.stack([rng.normal(scale=8, size=A), rng.normal(scale=5, size=A), np.zeros(A)], axis=1)
    xs, ys = [], []
    for F in frames[:3] + [line, plane]:
        xs += [F, F, F, F]
        ys += [_rigid(rng, F), F * np.array([1.0, 1.0, -1.0]), _rigid(rng, F + rng.normal(scale=0.05, size=F.shape)),
               F]
    xs += frames[3:]
    ys += frames[:3]
    X = np.stack([x.reshape(-1) for x in xs])
    Y = np.stack([y.reshape(-1) for y in ys])
    kern = Kernel("rmsd", sigma, A)
    c = 1.0 / (2 * sigma * sigma)
    for dt, u in ((np.float64, 2.0 ** -53), (np.float32, 2.0 ** -24)):
        Xt, Yt = X.astype(dt), Y.astype(dt)
        got = kk.kkm_kernel_block(torch.from_numpy(Xt).cuda(), torch.from_numpy(Yt).cuda(), "rmsd", sigma=sigma,
                                  n_atoms=A).cpu().numpy()
        ref = kern(Xt, Yt)
        # G_x + G_y - 2 lambda cancels: a few units of 2^-53 of (G_x + G_y) / A in the squared RMSD, and
        # the device keeps a Newton root only when its a-posteriori error is within 1e-13 (G_x + G_y) / 2
        # (else Jacobi); for float rows the device also rounds each centred coordinate to float (its
        # frames are centred in the row type), which moves the squared RMSD by at most about
        # 8 u (G_x + G_y) / A
        F = lambda Z: Z.reshape(len(Z), A, 3).astype(np.float64)
        G = (np.sum((F(Xt) - F(Xt).mean(1, keepdims=True)) ** 2, axis=(1, 2))[:, None]
             + np.sum((F(Yt) - F(Yt).mean(1, keepdims=True)) ** 2, axis=(1, 2))[None])
        cent = 0.0 if dt == np.float64 else 8 * u * G / A
        tol = 1e-9 * ref + ((64 * 2.0 ** -53 + 1e-13) * G / A + cent) * c * ref
        err = np.abs(got - ref)
        assert np.all(err <= tol + 1e-300), (dt.__name__, float(np.max(err / np.maximum(tol, 1e-300))))
        _say(f"  {dt.__name__}: max error / tolerance {float(np.max(err / np.maximum(tol, 1e-300))):.3g}")
    # the identical copies come out as 1 and the mirror images strictly below
    assert np.all(np.abs(np.diag(got)[0:20:4] - 1.0) < 1e-9)


@pytest.mark.parametrize("kind,dtype", [("rbf", np.float32), ("linear", np.float64), ("rbf", np.float64)])
def test_kernel_block_linear_rbf(kind, dtype):
    kk = _kk()
    _say(f"kernel block {kind}")
    X, _ = ki.datasets.gaussian_mixture(333, 20, 4, seed=46, sigma=1.0, dtype=dtype)
    Y, _ = ki.datasets.gaussian_mixture(65, 20, 4, seed=47, sigma=1.0, dtype=dtype)
    kern = Kernel(kind, 3.0)
    got = kk.kkm_kernel_block(torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda(), kind, sigma=3.0).cpu().numpy()
    np.testing.assert_allclose(got, kern(X, Y), rtol=1e-12, atol=1e-12)


# ------------------------------------------------------------------------------------------ RMSD fits
def test_rmsd_fit_iterates_with_many_clusters():
    """An RMSD fit whose landmark loop iterates (at least two updates in some batch) with more
    clusters than one 32-column tile, so Eq. 8 runs in the separate RMSD initial-label kernel."""
    kk = _kk()
    _say("rmsd fit C=40")
    X, _ = ki.datasets.md_frames(3000, A=16, n_templates=6, seed=48, noise=0.8)
    kern = Kernel("rmsd", 2.0, 16)
    T = 20
    model, labels, info, ref = _fit_both(kk, X, kern, 40, 3, 0.3, T, "kmeans++", 49, "fp32")
    assert max(ref.updates) >= 3, ref.updates       # the oracle loop takes >= 2 updates before it repeats
    _check_fit(kk, model, labels, info, ref, kern, X, T)   # oracle margins all above 1e-6 (1.07e-6 at least)
    assert max(info["updates_per_batch"]) >= 3


@pytest.mark.timeout(900)   # the oracle's 1.5e7 FP64 key-matrix eigensolves take a minute or two
def test_full_size_md_prefix():
    """The MD-frame workload at full batch shape (A = 50, C = 50, n = 10 000, l = 500): the first
    three stride batches of the 2e5-frame set, fitted on the device and by the oracle with the same
    draws, compared batch by batch."""
    kk = _kk()
    _say("full md prefix (3 batches)")
    cfg = ki.datasets.CONFIGS[2]
    X, _ = ki.datasets.config_data(2)
    Xp = _stride_prefix(X, cfg["B"], 3)
    kern = Kernel("rmsd", cfg["sigma"], cfg["n_atoms"])
    model, labels, info, ref = _fit_both(kk, Xp, kern, cfg["C"], 3, cfg["s"], cfg["T"], "kmeans++", 2002, "fp32")
    assert max(ref.updates) >= 3, ref.updates
    _check_fit(kk, model, labels, info, ref, kern, Xp, cfg["T"], expect="trajectory")
    _sampled_assign_parity(kk, model, kern, Xp, 2000, 81, "fp32", COST_TOL["fp32"])


def test_rmsd_assign_near_ties_on_the_matrix_cores():
    """RMSD frames on the matrix-core path with two medoids that nearly superpose (a rotated copy
    moved by 0.01 A per coordinate): for frames near them the two squared RMSDs differ by less than
    the FP32 cross-covariance bound, so those rows are decided again in FP64; labels must follow the
    oracle wherever its margin exceeds 1e-6, in FP32 and in the cost."""
    kk = _kk()
    _say("rmsd near ties (matrix cores)")
    A, sigma = 50, 1.5
    X, _ = ki.datasets.md_frames(4000, A=A, n_templates=4, seed=52)
    rng = np.random.default_rng(53)
    F0 = X[0].reshape(A, 3).astype(np.float64)
    F1 = F0 @ ki.datasets.random_rotations(rng, 1)[0].T + rng.normal(scale=0.01, size=F0.shape)
    M = np.concatenate([X[:1], F1.reshape(1, -1).astype(np.float32), X[1:9]])
    kern = Kernel("rmsd", sigma, A)
    m = kk.kkm_model_create("rmsd", d=3 * A, C=10, dtype="f32", sigma=sigma, n_atoms=A)
    kk.kkm_model_load(m, M, np.arange(11), np.ones(10))
    Y = np.ascontiguousarray(X[10:])
    model = okkm.SparseModel(M.astype(np.float64), np.arange(11), np.ones(10))
    rl, rg, _ = okkm.assign(kern, Y, model)
    near = (rl == 0) | (rl == 1)
    assert near.sum() > 100
    Yd = torch.from_numpy(Y).cuda()
    want = okkm.cost(kern, Y, model)
    # float frames are centred by the device into float (one rounding per coordinate, |dx| <= 2^-24 |x|),
    # which moves each squared RMSD by at most 6 2^-24 (G_x + G_m) / A and so each row's distance
    # 2 - 2K by at most 2 K c 6 2^-24 (G_x + G_m) / A (c = 1 / (2 sigma^2)); the FP64 form is exact for
    # the centred float frames, so its cost bar adds this to the 1e-9 of FP64 arithmetic
    G = lambda Z: np.sum((Z.reshape(len(Z), A, 3) - Z.reshape(len(Z), A, 3).mean(1, keepdims=True)) ** 2, axis=(1, 2))
    Gy, Gm = G(Y.astype(np.float64)), G(M.astype(np.float64))
    _, _, dist = okkm.assign(kern, Y, model)
    K = 1.0 - dist[np.arange(len(Y)), rl] / 2.0
    centring = float(np.sum(2.0 * K / (2 * sigma * sigma) * 6 * 2.0 ** -24 * (Gy + Gm[rl]) / A))
    for prec in ("fp32", "fp64"):
        lab = kk.kkm_assign(m, Yd, precision=prec).cpu().numpy()
        _labels_match(lab, rl, rg, f"rmsd near ties {prec}")
        cost = kk.kkm_cost(m, Yd, precision=prec)
        assert abs(cost - want) <= COST_TOL[prec] * abs(want) + centring, (prec, cost, want, centring)
        _say(f"  {prec}: cost error {abs(cost - want):.3g} (centring bound {centring:.3g})")


@pytest.mark.parametrize("prec", ["fp32", "fp64", "bf16x3"])
def test_fit_global_cost_trace(prec):
    """Global cost Omega(W) after every batch (Sec. 4.1, Fig. 4): the device's value of each batch
    against the oracle's Eq. 1 over all N samples with the global medoids of that moment."""
    kk = _kk()
    _say(f"global cost trace {prec}")
    X, _ = ki.datasets.gaussian_mixture(20_000, 16, 20, seed=1001, sigma=1.0)
    kern = Kernel("rbf", 4.0)
    T = 20
    model, labels, info, ref = _fit_both(kk, X, kern, 20, 10, 0.1, T, "kmeans++", 2001, prec, global_cost=True)
    _check_fit(kk, model, labels, info, ref, kern, X, T)
    want = okkm.global_costs(kern, X, ref)
    np.testing.assert_allclose(info["global_cost"], want, rtol=COST_TOL[prec])
    # the cost after the last batch is the final model's cost
    assert abs(info["global_cost"][-1] - kk.kkm_cost(model, torch.from_numpy(X).cuda(), precision=prec)) <= \
        COST_TOL[prec] * want[-1]
