"""Pins of the FP64 oracle against facts the paper and the mathematics fix.

Each test checks the oracle against something other than itself: a textbook
routine written independently (Lloyd with explicit means, exact kernel k-means
on the full matrix), brute force over all partitions of a tiny set, closed
forms, invariances, or a property the paper states (Sec. 2 linear case, the
B = 1 single-batch mode, Eq. 13's exactness under correct labels, the
empty-cluster rule, the evaluation count of Eq. 18)."""
import itertools

import numpy as np
import pytest

import kkm_inputs as ki
from oracle import kkm, reference, metrics
from oracle.kernels import Kernel, rbf, sqdist, rmsd2_horn, rmsd2_kabsch, horn_matrix


def _blobs(n, d, k, seed, spread=6.0):
    rng = np.random.default_rng(seed)
    c = rng.uniform(-spread, spread, size=(k, d))
    lab = rng.integers(0, k, size=n)
    return c[lab] + rng.normal(size=(n, d)), lab


# ---------------------------------------------------------------- kernels
def test_rbf_factorises_over_dimensions():
    rng = np.random.default_rng(1)
    X, Y = rng.normal(size=(7, 5)), rng.normal(size=(4, 5))
    prod = np.ones((7, 4))
    for k in range(5):
        prod *= rbf(X[:, k:k + 1], Y[:, k:k + 1], 1.7)
    np.testing.assert_allclose(rbf(X, Y, 1.7), prod, rtol=1e-13)


def test_rbf_scale_invariance_unit_diagonal_and_psd():
    rng = np.random.default_rng(2)
    X = rng.normal(size=(30, 3))
    np.testing.assert_allclose(rbf(X, X, 0.8), rbf(3.0 * X, 3.0 * X, 2.4), rtol=1e-13)
    K = rbf(X, X, 0.8)
    np.testing.assert_array_equal(np.diag(K), 1.0)
    np.testing.assert_allclose(K, K.T, rtol=0, atol=0)
    assert np.linalg.eigvalsh(K).min() > -1e-12


def test_sqdist_matches_norm_expansion_on_exact_integers():
    rng = np.random.default_rng(3)
    X = rng.integers(-50, 50, size=(9, 4)).astype(float)
    Y = rng.integers(-50, 50, size=(6, 4)).astype(float)
    expand = (X * X).sum(1)[:, None] + (Y * Y).sum(1)[None, :] - 2 * X @ Y.T
    np.testing.assert_array_equal(sqdist(X, Y), expand)


def test_point_distances_linear_equal_explicit_squared_distance():
    rng = np.random.default_rng(4)
    X, P = rng.normal(size=(11, 3)), rng.normal(size=(5, 3))
    d = kkm.point_distances(Kernel("linear"), X, P)
    np.testing.assert_allclose(d, ((X[:, None, :] - P[None]) ** 2).sum(-1), atol=1e-12)


# ---------------------------------------------------------------- RMSD
def _rot(rng):
    return ki.datasets.random_rotations(rng, 1)[0]


def test_rmsd_rigid_copy_is_zero_and_symmetric():
    rng = np.random.default_rng(5)
    a = rng.normal(scale=5.0, size=(12, 3))
    b = a @ _rot(rng).T + rng.uniform(-20, 20, size=3)
    c = rng.normal(scale=5.0, size=(12, 3))
    d2 = rmsd2_horn(np.stack([a, c]), np.stack([b, a]))
    # zero up to the rounding of G_x + G_y - 2 lambda (relative 1e-14 of the scale)
    scale = (np.sum((a - a.mean(0)) ** 2) * 2) / 12
    assert d2[0, 0] <= 1e-14 * scale
    assert abs(d2[1, 1] - rmsd2_horn(a[None], c[None])[0, 0]) < 1e-10  # symmetry
    assert d2[1, 0] > 0.1


def test_rmsd_two_atom_closed_form():
    rng = np.random.default_rng(6)
    for _ in range(5):
        a, b = rng.normal(size=3), rng.normal(size=3)
        fx = np.stack([np.zeros(3), a])
        fy = np.stack([np.ones(3), np.ones(3) + b])
        want = (np.linalg.norm(a) - np.linalg.norm(b)) ** 2 / 4.0
        assert abs(rmsd2_horn(fx[None], fy[None])[0, 0] - want) < 1e-12


def test_rmsd_mirror_image_is_not_superposable():
    rng = np.random.default_rng(7)
    a = rng.normal(scale=3.0, size=(8, 3))
    mirror = a * np.array([1.0, 1.0, -1.0])
    assert rmsd2_horn(a[None], mirror[None])[0, 0] > 1e-2
    # a reflection would superpose it: the proper-rotation SVD route agrees
    assert abs(rmsd2_kabsch(a, mirror) - rmsd2_horn(a[None], mirror[None])[0, 0]) < 1e-9


def test_rmsd_horn_matches_kabsch():
    X, _ = ki.datasets.md_frames(12, A=50, n_templates=3, seed=9)
    F = X.reshape(12, 50, 3).astype(np.float64)
    H = rmsd2_horn(F, F)
    for i, j in itertools.product(range(12), range(12)):
        k = rmsd2_kabsch(F[i], F[j])
        assert abs(H[i, j] - k) <= 1e-9 * max(1.0, k)


def test_horn_matrix_is_traceless_symmetric():
    R = np.random.default_rng(8).normal(size=(3, 3))
    N = horn_matrix(R)
    assert abs(np.trace(N)) < 1e-14
    np.testing.assert_array_equal(N, N.T)


# ---------------------------------------------------------------- Sec. 2 reductions
def _full_batch_fit(X, C, kern, U0, T):
    L = [np.arange(X.shape[0])]
    return kkm.fit(X, C, kern, 1, T, L, init="random", init_labels=U0)


def test_linear_kernel_full_batch_is_lloyd():
    """Sec. 2: with the linear kernel the update is Lloyd's k-means."""
    for seed in range(4):
        X, _ = _blobs(60, 3, 4, seed)
        U0 = np.random.default_rng(seed).integers(0, 4, size=60)
        res = _full_batch_fit(X, 4, Kernel("linear"), U0, 30)
        hist, _ = reference.lloyd(X, U0, 4, 30)
        traj = res.loops[0].trajectory[1:]
        assert len(traj) == len(hist)
        for a, b in zip(traj, hist):
            np.testing.assert_array_equal(a, b)
        if np.array_equal(hist[-1], hist[-2] if len(hist) > 1 else U0):
            d = res.loops[0].dist
            J = d[np.arange(60), res.labels].sum()
            assert abs(J - reference.explicit_cost(X, res.labels, 4)) < 1e-9 * max(1, J)


def test_single_batch_full_support_is_exact_kernel_kmeans():
    """B = 1, s = 1 is the single-batch mode: plain kernel k-means (Eq. 4-6)."""
    X, _ = ki.datasets.two_rings(300, seed=11)
    kern = Kernel("rbf", 1.0)
    U0 = ki.draw_init_labels(5, 300, 3)
    res = _full_batch_fit(X, 3, kern, U0, 25)
    hist, d = reference.exact_kkm(kern(X, X), U0, 3, 25)
    traj = res.loops[0].trajectory[1:]
    assert len(traj) == len(hist)
    for a, b in zip(traj, hist):
        np.testing.assert_array_equal(a, b)
    np.testing.assert_allclose(res.loops[0].dist, d, rtol=1e-11, atol=1e-12)


def test_cost_never_increases_on_full_batch_updates():
    """Eq. 1 is non-increasing along full-batch updates for PSD kernels."""
    for seed, kern in [(0, Kernel("rbf", 1.5)), (1, Kernel("linear")), (2, Kernel("rbf", 0.7))]:
        X, _ = _blobs(80, 2, 5, seed, spread=3.0)
        U0 = np.random.default_rng(seed).integers(0, 5, size=80)
        res = _full_batch_fit(X, 5, kern, U0, 40)
        K = kern(X, X)
        Js = [reference.partition_cost(K, u, 5) for u in res.loops[0].trajectory]
        for a, b in zip(Js, Js[1:]):
            assert b <= a * (1 + 1e-12) + 1e-12


# ---------------------------------------------------------------- brute force
def test_partition_cost_linear_equals_explicit_for_every_labelling():
    X, _ = _blobs(7, 2, 2, 3)
    K = X @ X.T
    for u in itertools.product(range(3), repeat=7):
        u = np.asarray(u)
        assert abs(reference.partition_cost(K, u, 3) - reference.explicit_cost(X, u, 3)) < 1e-9


def test_brute_force_optimum_is_a_fixed_point_and_reached_by_restarts():
    X, _ = _blobs(9, 2, 3, 21, spread=8.0)
    kern = Kernel("rbf", 2.0)
    K = kern(X, X)
    Jstar, ustar, _ = reference.brute_force(K, 3)
    # one update from the optimum keeps the partition
    res = kkm.inner_loop(K, np.ones(9), np.arange(9), ustar, 3, 1)
    assert reference.partition_cost(K, res.labels, 3) <= Jstar + 1e-12
    np.testing.assert_array_equal(res.labels, ustar)
    # the best of seeded restarts reaches the optimum on well-separated data
    best = np.inf
    for seed in range(50):
        U0 = np.random.default_rng(seed).integers(0, 3, size=9)
        r = _full_batch_fit(X, 3, kern, U0, 50)
        best = min(best, reference.partition_cost(K, r.labels, 3))
    assert abs(best - Jstar) < 1e-12


# ---------------------------------------------------------------- Sec. 3.1
def test_batches_partition_the_data():
    for N, B in [(10, 3), (11, 4), (7, 7), (100, 1)]:
        for s in ("stride", "block"):
            parts = kkm.batches(N, B, s)
            np.testing.assert_array_equal(np.sort(np.concatenate(parts)), np.arange(N))
            sizes = [len(p) for p in parts]
            assert max(sizes) - min(sizes) <= 1
        for i, p in enumerate(kkm.batches(N, B, "stride")):
            np.testing.assert_array_equal(p % B, i)


def test_eq13_merge_recovers_full_mean_under_correct_labels():
    """Eq. 13: alpha = |w^1|/(|w^1|+|w^0|) combines two batch means into the full mean;
    Eq. 12 then picks the sample nearest to it (linear kernel)."""
    rng = np.random.default_rng(12)
    X0 = rng.normal(size=(6, 3)) + 2.0
    X1 = rng.normal(size=(9, 3)) - 1.0
    X1 = np.vstack([X1, X1.mean(axis=0)])        # batch-1 mean is itself a sample
    mu0 = X0.mean(axis=0)
    full = np.vstack([X0, X1]).mean(axis=0)
    kern = Kernel("linear")
    M, valid, w, chosen = kkm.merge(kern, X1, mu0[None], np.array([True]), np.array([6]),
                                    np.array([9]), np.array([10]))
    alpha = 10 / 16
    np.testing.assert_allclose((1 - alpha) * mu0 + alpha * X1[9], full, atol=1e-12)
    nearest = np.argmin(((X1 - full) ** 2).sum(1))
    assert chosen[0] == nearest and w[0] == 16
    np.testing.assert_array_equal(M[0], X1[nearest])


def test_empty_cluster_keeps_its_global_medoid():
    """Empty-cluster remark (Sec. 3.1): |w_j^i| = 0 gives alpha = 0, no update."""
    rng = np.random.default_rng(13)
    Xb = rng.normal(size=(10, 2))
    M0 = rng.normal(size=(2, 2))
    M, valid, w, chosen = kkm.merge(Kernel("rbf", 1.0), Xb, M0, np.array([True, True]),
                                    np.array([5, 7]), np.array([3, -1]), np.array([10, 0]))
    np.testing.assert_array_equal(M[1], M0[1])
    assert chosen[1] == -1 and w[1] == 7 and w[0] == 15


def test_merge_first_batch_takes_the_batch_medoid():
    rng = np.random.default_rng(14)
    Xb = rng.normal(size=(12, 3))
    M, valid, w, chosen = kkm.merge(Kernel("rbf", 1.0), Xb, np.zeros((1, 3)), np.array([False]),
                                    np.array([0]), np.array([7]), np.array([4]))
    assert chosen[0] == 7 and valid[0]


# ---------------------------------------------------------------- Sec. 3.2
def test_full_support_reduces_sparse_form_to_minibatch_form():
    """s = 1: every batch runs exact kernel k-means on its own kernel matrix (Sec. 3.1)."""
    X, _ = _blobs(90, 2, 3, 15, spread=4.0)
    kern = Kernel("rbf", 1.2)
    B, C = 3, 3
    parts = kkm.batches(90, B, "stride")
    L = [np.arange(len(p)) for p in parts]
    u = ki.draw_kmpp_uniforms(3, C)
    res = kkm.fit(X, C, kern, B, 30, L, kmpp_uniforms=u)
    for i, p in enumerate(parts):
        Xb = X[p]
        U0 = res.loops[i].trajectory[0]
        hist, _ = reference.exact_kkm(kern(Xb, Xb), U0, C, 30)
        np.testing.assert_array_equal(hist[-1], res.loops[i].labels)
        assert len(hist) == res.loops[i].updates


def test_landmark_labels_evolve_on_their_own():
    """Eq. 16-17 depend only on landmark labels, so a loop over the landmarks alone
    has the same landmark trajectory, and one pass from its final centroids gives
    the full loop's final labels (T caps the number of updates)."""
    X, _ = ki.datasets.gaussian_mixture(600, 4, 6, seed=16, sigma=1.5, box=4.0)
    kern = Kernel("rbf", 2.0)
    for seed, T in itertools.product(range(3), (1, 2, 3, 5, 50)):
        L = ki.draw_landmarks(seed, 0, 600, 0.1)
        U0 = np.random.default_rng(seed).integers(0, 6, size=600)
        K = kern(X, X[L])
        full = kkm.inner_loop(K, np.ones(600), L, U0, 6, T)
        # landmark-only loop: stop at the first repeat or after T-1 updates
        traj = [U0[L]]
        for _ in range(T - 1):
            r = kkm.inner_loop(K[L], np.ones(len(L)), np.arange(len(L)), traj[-1], 6, 1)
            if np.array_equal(r.labels, traj[-1]):
                break
            traj.append(r.labels)
        last = kkm.inner_loop(K, np.ones(600), L, _embed(traj[-1], L, 600), 6, 1)
        np.testing.assert_array_equal(last.labels, full.labels)
        for a, b in zip(full.trajectory, traj):
            np.testing.assert_array_equal(a, b)


def _embed(lab_l, L, n):
    U = np.zeros(n, dtype=np.int64)
    U[L] = lab_l
    return U


def test_evaluation_count_eq18():
    """Kernel evaluations of the landmark block: N|L| = s N^2 / B (Eq. 18), plus n C per batch
    for the medoid blocks."""
    N, B, s, C = 1000, 4, 0.2, 5
    X, _ = _blobs(N, 2, C, 17)
    L = ki.draw_all_landmarks(7, N, B, s)
    assert all(len(l) == 50 for l in L)
    res = kkm.fit(X, C, Kernel("rbf", 2.0), B, 10, L, kmpp_uniforms=ki.draw_kmpp_uniforms(7, C))
    n = N // B
    merge_terms = sum(int(np.count_nonzero(res.batch_counts[i])) * n for i in range(B))
    assert res.evals == int(s * N * N / B) + n * C * B + merge_terms


# ---------------------------------------------------------------- k-means++
def test_kmeanspp_follows_d2_sampling_intervals():
    X = np.array([[0.0], [1.0], [3.0], [6.0]])
    kern = Kernel("linear")
    # first medoid: floor(u0 * n) = 0 -> D2 = [0, 1, 9, 36], total 46
    edges = np.cumsum([0, 1, 9, 36]) / 46.0
    for k, (lo, hi) in enumerate(zip(np.r_[0.0, edges[:-1]], edges)):
        if hi <= lo:
            continue
        for u in (lo + 1e-9, (lo + hi) / 2, hi - 1e-9):
            got = kkm.kmeanspp(kern, X, 2, np.array([0.1, u]))
            assert got[0] == 0 and got[1] == k


def test_kmeanspp_picks_distinct_points_until_exhausted():
    X, _ = _blobs(12, 2, 3, 18)
    u = ki.draw_kmpp_uniforms(9, 12)
    m = kkm.kmeanspp(Kernel("rbf", 1.0), X, 12, u)
    assert len(set(m.tolist())) == 12


# ---------------------------------------------------------------- model use
def test_assign_and_cost_of_a_medoid_model():
    X, _ = _blobs(40, 2, 3, 19)
    kern = Kernel("linear")
    model = kkm.SparseModel(X[[0, 5, 9]], np.array([0, 1, 2, 3]), np.ones(3))
    lab, gap, d = kkm.assign(kern, X, model)
    want = ((X[:, None, :] - X[[0, 5, 9]][None]) ** 2).sum(-1)
    np.testing.assert_allclose(d, want, atol=1e-10)
    np.testing.assert_array_equal(lab, np.argmin(want, axis=1))
    assert abs(kkm.cost(kern, X, model) - want.min(1).sum()) < 1e-9


def test_sparse_model_mean_centroid_linear():
    rng = np.random.default_rng(20)
    S = rng.normal(size=(7, 3))
    Y = rng.normal(size=(5, 3))
    model = kkm.SparseModel(S, np.array([0, 3, 3, 7]), np.r_[np.full(3, 1 / 3), np.full(4, 0.25)])
    d = kkm.centroid_distances(Kernel("linear"), Y, model)
    mu0, mu2 = S[:3].mean(0), S[3:].mean(0)
    np.testing.assert_allclose(d[:, 0], ((Y - mu0) ** 2).sum(1), atol=1e-12)
    np.testing.assert_allclose(d[:, 2], ((Y - mu2) ** 2).sum(1), atol=1e-12)
    assert np.all(np.isinf(d[:, 1]))


def test_gap_rel():
    d = np.array([[1.0, 1.5, 3.0], [2.0, 2.0, 0.5], [0.2, np.inf, np.inf]])
    g = kkm.gap_rel(d, np.array([1.0, 1.0, 1.0]))
    np.testing.assert_allclose(g[:2], [0.5 / 1.5, 1.5 / 2.0])
    assert np.isinf(g[2])


# ---------------------------------------------------------------- metrics
def test_accuracy_and_nmi_closed_cases():
    y = np.array([0, 0, 1, 1, 2, 2])
    assert metrics.accuracy(y, np.array([2, 2, 0, 0, 1, 1])) == 1.0
    assert abs(metrics.nmi(y, np.array([5, 5, 3, 3, 4, 4])) - 1.0) < 1e-12
    assert abs(metrics.nmi(np.array([0, 0, 1, 1]), np.array([0, 1, 0, 1]))) < 1e-12
    assert metrics.accuracy(np.array([0, 0, 1, 1]), np.array([0, 0, 0, 0])) == 0.5
    # two clusters of 2+2 vs classes split 3+1: I = H(u) - H(u|y)
    y = np.array([0, 0, 0, 1]); u = np.array([0, 0, 1, 1])
    Hu = np.log(2.0)
    Hy = -(0.75 * np.log(0.75) + 0.25 * np.log(0.25))
    I = Hu - 0.75 * (-(2 / 3) * np.log(2 / 3) - (1 / 3) * np.log(1 / 3))
    assert abs(metrics.nmi(y, u) - I / np.sqrt(Hu * Hy)) < 1e-12


def test_medoid_displacement_closed_forms():
    """Sec. 4.1 observable: for the linear kernel the feature-space displacement is the Euclidean
    distance between the two medoids; for RBF it is sqrt(2 - 2 exp(-|a-b|^2 / 2 sigma^2)); a kept
    medoid moves 0 and an unset one gives NaN."""
    rng = np.random.default_rng(12)
    X = rng.normal(size=(30, 5))
    before = np.array([3, 7, -1, 11, 4])
    after = np.array([9, 7, 2, 20, 28])
    lin = kkm.medoid_displacement(Kernel("linear", 1.0), X, before, after)
    for j in (0, 3, 4):
        assert abs(lin[j] - np.linalg.norm(X[after[j]] - X[before[j]])) < 1e-12
    assert lin[1] == 0.0 and np.isnan(lin[2])
    sig = 1.7
    rbf = kkm.medoid_displacement(Kernel("rbf", sig), X, before, after)
    for j in (0, 3, 4):
        r2 = float(np.sum((X[after[j]] - X[before[j]]) ** 2))
        assert abs(rbf[j] - np.sqrt(2.0 - 2.0 * np.exp(-r2 / (2 * sig * sig)))) < 1e-12


def test_partial_cost_of_a_converged_full_batch_is_the_partition_cost():
    """Sec. 4.1 partial cost: once the labels of a full batch (B = 1, s = 1) no longer change, the
    centroids are the means of the final partition, so the partial cost equals the explicit
    partition cost of the final labels (linear: the Euclidean k-means cost)."""
    for seed in range(3):
        X, _ = _blobs(40, 2, 3, seed)
        U0 = np.random.default_rng(seed).integers(0, 3, size=40)
        res = _full_batch_fit(X, 3, Kernel("linear"), U0, 50)
        tr = res.loops[0].trajectory
        assert np.array_equal(tr[-1], tr[-2])   # converged
        pc = kkm.partial_costs(res)[0]
        assert abs(pc - reference.explicit_cost(X, res.labels, 3)) < 1e-9 * max(1.0, pc)


# ---------------------------------------------------------------- Eq. 8, Eq. 10 and the RMSD kernel
def test_eq8_initial_labels_are_nearest_euclidean_medoid_for_linear_kernel():
    """Eq. 8 with the full feature-space distance K(x,x) - 2K(x,m) + K(m,m): for the linear kernel
    the initial labels of batch i >= 1 are the labels of the nearest global medoid in plain
    Euclidean distance.  The data make the printed form (K(m,m) dropped) pick other labels, so a
    dropped term fails here."""
    rng = np.random.default_rng(31)
    # medoids of very different norms: dropping ||m||^2 favours the long one
    M = np.array([[0.5, 0.0], [6.0, 0.0], [0.0, -4.0]])
    X = rng.normal(scale=2.0, size=(200, 2))
    want = np.argmin(((X[:, None, :] - M[None]) ** 2).sum(-1), axis=1)
    got = kkm.nearest_medoid_labels(Kernel("linear"), X, M, np.ones(3, dtype=bool))
    np.testing.assert_array_equal(got, want)
    dropped = np.argmin(-2.0 * X @ M.T, axis=1)
    assert (dropped != want).sum() > 20          # the pin discriminates the misprint
    # a skipped (unset) medoid never wins
    got2 = kkm.nearest_medoid_labels(Kernel("linear"), X, M, np.array([True, False, True]))
    want2 = np.argmin(np.where([True, False, True], ((X[:, None, :] - M[None]) ** 2).sum(-1), np.inf), axis=1)
    np.testing.assert_array_equal(got2, want2)


def test_eq8_through_the_fit_on_the_second_batch():
    """The same pin through fit(): linear kernel, B = 2, s = 1 (every sample a landmark), so the
    loop's starting labels on batch 1 are visible as the first entry of its trajectory; they must
    be the nearest-Euclidean-medoid labels for the global medoids left by batch 0."""
    rng = np.random.default_rng(32)
    C = 4
    cen = np.array([[0.0, 0.0], [8.0, 0.0], [0.0, 8.0], [8.0, 8.0]]) + 3.0
    X = cen[rng.integers(0, C, size=400)] + rng.normal(scale=1.5, size=(400, 2))
    L = [np.arange(200), np.arange(200)]
    res = kkm.fit(X, C, Kernel("linear"), 2, 20, L, kmpp_uniforms=ki.draw_kmpp_uniforms(4, C))
    Mg = X[res.global_medoids[0]]
    X1 = X[kkm.batches(400, 2)[1]]
    want = np.argmin(((X1[:, None, :] - Mg[None]) ** 2).sum(-1), axis=1)
    np.testing.assert_array_equal(res.loops[1].trajectory[0], want)
    assert (np.argmin(-2.0 * X1 @ Mg.T, axis=1) != want).any()


def test_eq10_batch_medoid_minimises_over_the_whole_batch():
    """Eq. 10: m_j^i = argmin over all of X^i (not only the members of cluster j) of the distance to
    w_j.  Linear kernel, s = 1, a converged batch: w_j is the explicit mean of cluster j.  Cluster 0
    is two far groups whose mean lies near a member of cluster 1, so its medoid is that non-member;
    restricting the argmin to members would pick a point of the far groups."""
    X = np.array([[-10.0, 0.0], [10.0, 0.0], [0.0, 0.5], [0.0, 1.0], [-9.0, 0.0], [9.0, 0.0]])
    U0 = np.array([0, 0, 1, 1, 0, 0])
    res = kkm.fit(X, 2, Kernel("linear"), 1, 20, [np.arange(6)], init="random", init_labels=U0)
    np.testing.assert_array_equal(res.labels, U0)            # converged with the given partition
    mu0 = X[U0 == 0].mean(axis=0)
    nearest = int(np.argmin(((X - mu0) ** 2).sum(1)))
    assert U0[nearest] != 0                                  # the nearest sample is not a member
    assert res.batch_medoids[0, 0] == nearest
    mu1 = X[U0 == 1].mean(axis=0)
    assert res.batch_medoids[0, 1] == int(np.argmin(((X - mu1) ** 2).sum(1)))
    # the same through the function on the loop's distances
    Mi, members = kkm.batch_medoids(res.loops[0].dist, res.labels, 2)
    assert Mi[0] == nearest and members.tolist() == [4, 2]


def test_rmsd_kernel_on_atom_major_rows():
    """K(x, y) = exp(-RMSD^2 / (2 sigma^2)) on rows laid out atom by atom (x0 y0 z0 x1 y1 z1 ...):
    a rigid copy gives exactly 1 (to rounding), and two-atom frames follow the closed form
    RMSD^2 = (|a| - |b|)^2 / 4 for bonds a and b.  A sigma^2 / 2 sigma^2 slip or a coordinate-major
    reshape of the rows fails one of these."""
    rng = np.random.default_rng(33)
    sigma = 1.3
    kern = Kernel("rmsd", sigma, 2)
    for _ in range(6):
        p0, a = rng.normal(size=3), rng.normal(scale=2.0, size=3)
        q0, b = rng.normal(size=3), rng.normal(scale=2.0, size=3)
        x = np.concatenate([p0, p0 + a])[None]
        y = np.concatenate([q0, q0 + b])[None]
        r2 = (np.linalg.norm(a) - np.linalg.norm(b)) ** 2 / 4.0
        assert abs(kern(x, y)[0, 0] - np.exp(-r2 / (2 * sigma * sigma))) < 1e-12
    A = 9
    kern9 = Kernel("rmsd", sigma, A)
    F = rng.normal(scale=4.0, size=(A, 3))
    R = ki.datasets.random_rotations(rng, 1)[0]
    G = F @ R.T + rng.uniform(-20, 20, size=3)
    assert abs(kern9(F.reshape(1, -1), G.reshape(1, -1))[0, 0] - 1.0) < 1e-12
    # a known perturbation: the Kabsch route (pinned above) gives the value
    H = F + rng.normal(scale=0.3, size=F.shape)
    want = np.exp(-rmsd2_kabsch(F, H) / (2 * sigma * sigma))
    assert abs(kern9(F.reshape(1, -1), H.reshape(1, -1))[0, 0] - want) < 1e-12
    assert kern9.diag(F.reshape(1, -1))[0] == 1.0


def test_global_cost_after_every_batch_closed_form():
    """Sec. 4.1 global cost: after batch i, Eq. 1 over all N samples with the global medoids of that
    moment.  Linear kernel: the explicit sum over samples of the squared Euclidean distance to the
    nearest medoid; the last batch's value is the cost of the final medoid model."""
    rng = np.random.default_rng(34)
    X, _ = _blobs(300, 3, 4, 34)
    L = ki.draw_all_landmarks(8, 300, 3, 0.5)
    res = kkm.fit(X, 4, Kernel("linear"), 3, 10, L, kmpp_uniforms=ki.draw_kmpp_uniforms(8, 4))
    gc = kkm.global_costs(Kernel("linear"), X, res)
    assert len(gc) == 3
    for i in range(3):
        M = X[res.global_medoids[i]]
        want = float(np.min(((X[:, None, :] - M[None]) ** 2).sum(-1), axis=1).sum())
        assert abs(gc[i] - want) <= 1e-9 * want
    assert abs(gc[-1] - kkm.cost(Kernel("linear"), X, kkm.medoid_model(res))) <= 1e-12 * gc[-1]
