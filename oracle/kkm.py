"""Approximate mini-batch kernel k-means, written out step by step in float64.

Oracle -- test infrastructure only.  It follows the paper's order:

Sec. 3.1  mini-batch fetching (stride or block sampling), batch
          initialisation (kernel k-means++ for the first batch, Eq. 8 from the
          global medoids afterwards), the inner gradient-descent loop on the
          batch (Eq. 9 with the updates of Eq. 2-6), the batch medoids (Eq. 10)
          and the merge into the global medoids (Eq. 11-13, empty-cluster rule).
Sec. 3.2  centroids restricted to a-priori landmarks (Eq. 14), with the
          approximate compactness g^ (Eq. 16), similarity f^ (Eq. 17) and
          label update (Eq. 15).

Readings taken where the paper is silent or garbled (each is also listed with
the design notes of the repository):

* |w_j| in Eq. 14, 16, 17 is the number of landmarks labelled j, so that w_j
  is the mean of those landmarks in feature space.
* Eq. 8 is applied with the full distance K(x,x) - 2K(x,m) + K(m,m); the
  printed form drops K(m,m), which is only constant for normalised kernels.
* Every argmin takes the lowest index on ties (cluster index for labels,
  batch position for medoids).
* A cluster with no landmarks has distance +inf inside the loop.
* The loop stops when no label of the batch changes, or after T label
  updates; the final labels and distances are those of the last update.
* alpha = |w_j^i| / (|w_j^i| + |w_j|) with |w_j| the running sum of earlier
  batch member counts, and alpha = 0 when both are zero.
* Batches are numbered 0..B-1.

Random draws (landmark sets, k-means++ uniforms, random labels) are inputs.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .kernels import Kernel

INF = np.inf


# --------------------------------------------------------------------------
# Mini-batch fetching (Sec. 3.1)
# --------------------------------------------------------------------------
def batches(N: int, B: int, sampling: str = "stride") -> list[np.ndarray]:
    """Global indices of mini-batch i.

    stride: X^i = {x_(i + jB)};  block: X^i = a contiguous run, run lengths
    differing by at most one when B does not divide N (longer runs first)."""
    if sampling == "stride":
        return [np.arange(i, N, B) for i in range(B)]
    if sampling == "block":
        sizes = [N // B + (1 if i < N % B else 0) for i in range(B)]
        starts = np.concatenate([[0], np.cumsum(sizes)])
        return [np.arange(starts[i], starts[i + 1]) for i in range(B)]
    raise ValueError(sampling)


# --------------------------------------------------------------------------
# Distances in feature space
# --------------------------------------------------------------------------
def argmin_lowest(d: np.ndarray, axis: int) -> np.ndarray:
    """Index of the minimum; numpy returns the first occurrence, i.e. the lowest index."""
    return np.argmin(d, axis=axis)


def point_distances(kern: Kernel, X: np.ndarray, P: np.ndarray) -> np.ndarray:
    """||phi(x) - phi(p)||^2 = K(x,x) - 2K(x,p) + K(p,p) for every row x and point p (Eq. 2, 8)."""
    return kern.diag(X)[:, None] - 2.0 * kern(X, P) + kern.diag(P)[None, :]


def gap_rel(d: np.ndarray, kxx: np.ndarray) -> np.ndarray:
    """Relative margin between best and second-best distance of each row.

    (d2 - d1) / max(|d1|, |d2|, |K(x,x)|); +inf when fewer than two finite distances."""
    if d.shape[1] < 2:
        return np.full(d.shape[0], INF)
    part = np.sort(d, axis=1)[:, :2]
    d1, d2 = part[:, 0], part[:, 1]
    with np.errstate(invalid="ignore"):
        scale = np.maximum(np.maximum(np.abs(d1), np.abs(d2)), np.abs(kxx))
        g = (d2 - d1) / np.where(scale > 0, scale, 1.0)
    g[~np.isfinite(d2)] = INF
    return g


# --------------------------------------------------------------------------
# Initialisation (Sec. 3.1): kernel k-means++ and Eq. 8
# --------------------------------------------------------------------------
def kmeanspp(kern: Kernel, Xb: np.ndarray, C: int, uniforms: np.ndarray) -> np.ndarray:
    """Kernel k-means++ seeding on one batch (Arthur & Vassilvitskii's D^2 sampling
    carried out in feature space).

    uniforms[0] picks the first medoid uniformly; for k >= 1 the next medoid is
    the lowest index whose running sum of D^2 (in index order) exceeds
    uniforms[k] times the total, D^2 being the squared feature-space distance to
    the nearest medoid chosen so far.  If every D^2 is zero the uniform picks an
    index directly."""
    n = Xb.shape[0]
    chosen = [min(int(np.floor(uniforms[0] * n)), n - 1)]
    D2 = np.maximum(0.0, point_distances(kern, Xb, Xb[chosen[-1:]])[:, 0])
    for k in range(1, C):
        cs = np.cumsum(D2)
        total = cs[-1]
        if total > 0.0:
            nxt = int(np.searchsorted(cs, uniforms[k] * total, side="right"))
            nxt = min(nxt, n - 1)
        else:
            nxt = min(int(np.floor(uniforms[k] * n)), n - 1)
        chosen.append(nxt)
        D2 = np.minimum(D2, np.maximum(0.0, point_distances(kern, Xb, Xb[[nxt]])[:, 0]))
    return np.asarray(chosen, dtype=np.int64)


def nearest_medoid_labels(kern: Kernel, Xb: np.ndarray, M: np.ndarray, valid: np.ndarray) -> np.ndarray:
    """Eq. 8: u = argmin_j K(x,x) - 2K(x, m_j) + K(m_j, m_j); clusters without a medoid are skipped."""
    d = point_distances(kern, Xb, M)
    d[:, ~valid] = INF
    return argmin_lowest(d, axis=1).astype(np.int64)


# --------------------------------------------------------------------------
# Inner loop on one batch (Eq. 9, 14-17)
# --------------------------------------------------------------------------
@dataclass
class LoopResult:
    labels: np.ndarray            # U_last, n labels
    dist: np.ndarray              # d_last[x, j] = K(x,x) - 2 f^(x,j) + g^(j) under the last centroids
    ghat: np.ndarray              # g^ of the last centroids
    landmark_counts: np.ndarray   # c_j of the last centroids
    updates: int                  # number of label updates performed (<= T)
    trajectory: list = field(default_factory=list)   # landmark labels at every step
    min_gap: float = INF          # smallest relative margin over every label decision


def inner_loop(K_xl: np.ndarray, kxx: np.ndarray, landmarks: np.ndarray, U0: np.ndarray,
               C: int, T: int) -> LoopResult:
    """Self-consistent label updates with centroids spanned by the landmarks.

    K_xl[x, m] = K(x, l_m) for every batch sample x and landmark l_m.  Centroid j
    is the mean of the landmarks labelled j (Eq. 14); then
      g^_j   = 1/c_j^2 sum_{m,n in L_j} K(l_m, l_n)            (Eq. 16)
      f^_xj  = 1/c_j   sum_{m in L_j}   K(x, l_m)              (Eq. 17)
      u_x    = argmin_j K(x,x) - 2 f^_xj + g^_j                (Eq. 15)
    repeated until no label of the batch changes or T updates were made."""
    n = K_xl.shape[0]
    K_ll = K_xl[landmarks, :]
    U = np.asarray(U0, dtype=np.int64).copy()
    traj = [U[landmarks].copy()]
    min_gap = INF
    updates = 0
    d = None
    ghat = np.zeros(C)
    c = np.zeros(C, dtype=np.int64)
    for _ in range(T):
        W = U[landmarks]
        c = np.bincount(W, minlength=C)
        fhat = np.zeros((n, C))
        ghat = np.zeros(C)
        for j in range(C):
            if c[j] == 0:
                continue
            mem = np.flatnonzero(W == j)
            fhat[:, j] = K_xl[:, mem].sum(axis=1) / c[j]
            ghat[j] = K_ll[np.ix_(mem, mem)].sum() / (c[j] * c[j])
        d = kxx[:, None] - 2.0 * fhat + ghat[None, :]
        d[:, c == 0] = INF
        U_new = argmin_lowest(d, axis=1).astype(np.int64)
        min_gap = min(min_gap, float(np.min(gap_rel(d, kxx))))
        updates += 1
        traj.append(U_new[landmarks].copy())
        if np.array_equal(U_new, U):
            U = U_new
            break
        U = U_new
    return LoopResult(U, d, ghat, c, updates, traj, min_gap)


# --------------------------------------------------------------------------
# Batch medoids (Eq. 10) and merge (Eq. 11-13)
# --------------------------------------------------------------------------
# Relative width within which two argmin candidates count as tied.  Diagnostic only: the argmins
# themselves take the lowest index; the tie sets let a comparison accept any member of a set that
# rounding (not the method) decides.
TIE_REL = 1e-12


def _near_minimum(v: np.ndarray, k: int) -> np.ndarray:
    """Positions whose value is within TIE_REL (relative) of the minimum v[k]."""
    return np.flatnonzero(np.abs(v - v[k]) <= TIE_REL * max(abs(float(v[k])), 1.0))


def batch_medoids(dist: np.ndarray, labels: np.ndarray, C: int, ties: list | None = None):
    """m_j^i = argmin over the batch of d_last[x, j], for clusters with members (Eq. 10).

    ties (optional out): per cluster, the positions within TIE_REL of the minimum."""
    members = np.bincount(labels, minlength=C)
    Mi = np.full(C, -1, dtype=np.int64)
    for j in range(C):
        if members[j] > 0:
            Mi[j] = int(argmin_lowest(dist[:, j], axis=0))
            if ties is not None:
                ties.append(_near_minimum(dist[:, j], Mi[j]))
        elif ties is not None:
            ties.append(np.zeros(0, dtype=np.int64))
    return Mi, members


def merge(kern: Kernel, Xb: np.ndarray, M: np.ndarray, M_valid: np.ndarray, wcount: np.ndarray,
          Mi: np.ndarray, members: np.ndarray, ties: list | None = None):
    """Convex merge of batch medoids into the global medoids (Eq. 11-13).

    alpha_j = |w_j^i| / (|w_j^i| + |w_j|)  (0 when both are 0: empty clusters are not updated);
    m_j <- argmin_x ||phi(x) - (1-alpha) phi(m_j) - alpha phi(m_j^i)||^2 over the batch
         = argmin_x K(x,x) - 2(1-alpha) K(x, m_j) - 2 alpha K(x, m_j^i) (+ a constant in x);
    |w_j| += |w_j^i|.
    Returns the new (M, valid, wcount) and the chosen batch positions (-1 = not updated); ties
    (optional out) receives per cluster the positions within TIE_REL of the minimum score."""
    C = len(wcount)
    M = M.copy()
    M_valid = M_valid.copy()
    wcount = wcount.copy()
    chosen = np.full(C, -1, dtype=np.int64)
    kxx = kern.diag(Xb)
    for j in range(C):
        denom = members[j] + wcount[j]
        alpha = members[j] / denom if denom > 0 else 0.0
        if alpha > 0.0:
            score = kxx - 2.0 * alpha * kern(Xb, Xb[[Mi[j]]])[:, 0]
            if alpha < 1.0:
                assert M_valid[j]
                score = score - 2.0 * (1.0 - alpha) * kern(Xb, M[[j]])[:, 0]
            x = int(argmin_lowest(score, axis=0))
            chosen[j] = x
            M[j] = Xb[x]
            M_valid[j] = True
            if ties is not None:
                ties.append(_near_minimum(score, x))
        elif ties is not None:
            ties.append(np.zeros(0, dtype=np.int64))
        wcount[j] += members[j]
    return M, M_valid, wcount, chosen


# --------------------------------------------------------------------------
# Whole fit (Alg. 1 structure, one process)
# --------------------------------------------------------------------------
@dataclass
class FitResult:
    medoids: np.ndarray          # (C, d) coordinates of the global medoids
    medoid_index: np.ndarray     # (C,) global sample index of each medoid, -1 if never set
    valid: np.ndarray            # (C,) medoid defined
    counts: np.ndarray           # (C,) |w_j| after the last batch
    labels: np.ndarray           # (N,) each sample's label U_last from its own batch
    updates: list                # per batch: number of label updates
    batch_medoids: np.ndarray    # (B, C) global index of m_j^i (-1 if empty in that batch)
    batch_counts: np.ndarray     # (B, C) |w_j^i|
    global_medoids: np.ndarray   # (B, C) global index of m_j after merging batch i
    min_gap: float               # smallest relative margin over every label decision
    label_gaps: np.ndarray       # (N,) relative margin of each final label
    evals: int                   # algorithmic kernel evaluations: n|L| + n C (init) + n C (merge)
    loops: list                  # LoopResult per batch
    medoid_ties: list = field(default_factory=list)   # [B][C] global indices tied for Eq. 10's minimum
    merge_ties: list = field(default_factory=list)    # [B][C] global indices tied for Eq. 12's minimum


def fit(X: np.ndarray, C: int, kern: Kernel, B: int, T: int, landmarks: list,
        sampling: str = "stride", init: str = "kmeans++", kmpp_uniforms=None,
        init_labels=None, init_medoids=None) -> FitResult:
    """Mini-batch kernel k-means with a-priori landmark centroids (Sec. 3.1-3.2).

    landmarks[i]: sorted batch-positions of the landmarks of batch i (drawn
    uniformly without replacement; s = |L| B / N, Eq. 18).
    init: 'kmeans++' (needs kmpp_uniforms, C values), 'random' (init_labels for
    every sample of batch 0) or 'medoids' (init_medoids, C batch-0 positions)."""
    X = np.asarray(X)
    N, dim = X.shape
    parts = batches(N, B, sampling)
    M = np.zeros((C, dim))
    M_idx = np.full(C, -1, dtype=np.int64)
    valid = np.zeros(C, dtype=bool)
    wcount = np.zeros(C, dtype=np.int64)
    labels = np.zeros(N, dtype=np.int64)
    gaps = np.zeros(N)
    bmed = np.full((B, C), -1, dtype=np.int64)
    bcnt = np.zeros((B, C), dtype=np.int64)
    gmed = np.full((B, C), -1, dtype=np.int64)
    updates, loops = [], []
    med_ties, mrg_ties = [], []
    min_gap = INF
    evals = 0
    for i, idx in enumerate(parts):
        Xb = np.asarray(X[idx], dtype=np.float64)
        n = Xb.shape[0]
        L = np.asarray(landmarks[i], dtype=np.int64)
        kxx = kern.diag(Xb)
        K_xl = kern(Xb, Xb[L])                       # the n x |L| kernel block
        evals += n * len(L)
        if i == 0:
            if init == "random":
                U0 = np.asarray(init_labels, dtype=np.int64)
            else:
                if init == "kmeans++":
                    m0 = kmeanspp(kern, Xb, C, np.asarray(kmpp_uniforms))
                    evals += n * C
                elif init == "medoids":
                    m0 = np.asarray(init_medoids, dtype=np.int64)
                else:
                    raise ValueError(init)
                M = Xb[m0].copy()
                M_idx = idx[m0].copy()
                valid = np.ones(C, dtype=bool)
                U0 = nearest_medoid_labels(kern, Xb, M, valid)
        else:
            U0 = nearest_medoid_labels(kern, Xb, M, valid)   # Eq. 8 (auxiliary n x C block)
            evals += n * C
        res = inner_loop(K_xl, kxx, L, U0, C, T)
        loops.append(res)
        updates.append(res.updates)
        min_gap = min(min_gap, res.min_gap)
        mt, gt = [], []
        Mi, members = batch_medoids(res.dist, res.labels, C, ties=mt)
        evals += n * int(np.count_nonzero(members))
        M, valid, wcount, chosen = merge(kern, Xb, M, valid, wcount, Mi, members, ties=gt)
        med_ties.append([idx[t] for t in mt])
        mrg_ties.append([idx[t] for t in gt])
        for j in range(C):
            if chosen[j] >= 0:
                M_idx[j] = idx[chosen[j]]
            if Mi[j] >= 0:
                bmed[i, j] = idx[Mi[j]]
        bcnt[i] = members
        gmed[i] = M_idx
        labels[idx] = res.labels
        gaps[idx] = gap_rel(res.dist, kxx)
    return FitResult(M, M_idx, valid, wcount, labels, updates, bmed, bcnt, gmed, min_gap,
                     gaps, evals, loops, med_ties, mrg_ties)


# --------------------------------------------------------------------------
# Using a model: Eq. 1-2 on new data
# --------------------------------------------------------------------------
@dataclass
class SparseModel:
    """Centroids w_j = sum_{l in segment j} coef_l phi(support_l).

    A medoid model has one support row per cluster with coefficient 1; a
    landmark centroid has the landmarks labelled j with coefficient 1/c_j."""
    support: np.ndarray
    offsets: np.ndarray
    coef: np.ndarray

    @property
    def C(self) -> int:
        return len(self.offsets) - 1


def medoid_model(fitres: FitResult) -> SparseModel:
    rows = fitres.medoids[fitres.valid]
    offs = np.concatenate([[0], np.cumsum(fitres.valid.astype(np.int64))])
    return SparseModel(rows, offs, np.ones(rows.shape[0]))


def centroid_distances(kern: Kernel, Y: np.ndarray, model: SparseModel) -> np.ndarray:
    """d[y, j] = K(y,y) - 2 sum_l a_l K(y, s_l) + sum_{l,l'} a_l a_l' K(s_l, s_l'); +inf for empty j."""
    Y = np.asarray(Y, dtype=np.float64)
    S = np.asarray(model.support, dtype=np.float64)
    K_ys = kern(Y, S) if S.shape[0] else np.zeros((Y.shape[0], 0))
    K_ss = kern(S, S) if S.shape[0] else np.zeros((0, 0))
    d = np.full((Y.shape[0], model.C), INF)
    kyy = kern.diag(Y)
    for j in range(model.C):
        a, b = int(model.offsets[j]), int(model.offsets[j + 1])
        if b <= a:
            continue
        w = np.asarray(model.coef[a:b], dtype=np.float64)
        f = K_ys[:, a:b] @ w
        g = w @ K_ss[a:b, a:b] @ w
        d[:, j] = kyy - 2.0 * f + g
    return d


def assign(kern: Kernel, Y: np.ndarray, model: SparseModel):
    """Labels by Eq. 2 (lowest j on ties) and their relative margins."""
    d = centroid_distances(kern, Y, model)
    return argmin_lowest(d, axis=1).astype(np.int64), gap_rel(d, kern.diag(Y)), d


def cost(kern: Kernel, Y: np.ndarray, model: SparseModel) -> float:
    """Eq. 1 with labels from Eq. 2: sum over samples of the distance to the nearest centroid."""
    d = centroid_distances(kern, Y, model)
    return float(np.sum(np.min(d, axis=1)))


# --------------------------------------------------------------------------
# Sampling-quality observable (Sec. 4.1, Fig. 4)
# --------------------------------------------------------------------------
def medoid_displacement(kern: Kernel, X: np.ndarray, before: np.ndarray, after: np.ndarray) -> np.ndarray:
    """Feature-space displacement of every cluster centre across one outer iteration:
    ||phi(x_after) - phi(x_before)|| = sqrt(K(a,a) - 2 K(a,b) + K(b,b)) for the global medoid
    indices before and after the merge of a batch; 0 when the medoid is kept and NaN when it was
    unset before (index -1)."""
    out = np.full(len(after), np.nan)
    for j, (b, a) in enumerate(zip(np.asarray(before), np.asarray(after))):
        if b < 0:
            continue
        if a == b:
            out[j] = 0.0
            continue
        xa = np.asarray(X[a:a + 1], dtype=np.float64)
        xb = np.asarray(X[b:b + 1], dtype=np.float64)
        v = kern.diag(xa)[0] - 2.0 * kern(xa, xb)[0, 0] + kern.diag(xb)[0]
        out[j] = np.sqrt(max(v, 0.0))
    return out


def global_costs(kern: Kernel, X: np.ndarray, fitres: FitResult) -> list:
    """Global cost Omega(W) after every batch (Sec. 4.1, Fig. 4): Eq. 1 over ALL N samples with the
    global medoids as they stand after the merge of batch i (clusters without a medoid yet are
    skipped)."""
    out = []
    for i in range(fitres.global_medoids.shape[0]):
        idx = fitres.global_medoids[i]
        rows = np.asarray(X[idx[idx >= 0]], dtype=np.float64)
        model = SparseModel(rows, np.arange(rows.shape[0] + 1), np.ones(rows.shape[0]))
        out.append(cost(kern, X, model))
    return out


def partial_costs(fitres: FitResult) -> list:
    """Partial cost Omega(W^i) of every batch (Sec. 4.1, Fig. 4): Eq. 1 over the batch's rows with
    the batch's landmark centroids after its loop, i.e. the sum of each row's distance to its
    nearest centroid under those centroids."""
    return [float(np.sum(np.min(lp.dist, axis=1))) for lp in fitres.loops]
