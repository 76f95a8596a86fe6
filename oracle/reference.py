"""Textbook routines the method must reduce to (oracle; test infrastructure only).

* ``exact_kkm``  -- kernel k-means on the full kernel matrix (Sec. 2, Eq. 4-6),
                    the B = 1, s = 1 limit of the method;
* ``lloyd``      -- k-means with explicit means (the linear-kernel case of Sec. 2);
* ``partition_cost`` / ``brute_force`` -- the cost of Eq. 1 with centroids set
                    to the cluster means (Eq. 3), and its exhaustive minimum
                    over every labelling of a tiny set.
"""
from __future__ import annotations

import itertools

import numpy as np

INF = np.inf


def exact_kkm(K: np.ndarray, U0: np.ndarray, C: int, T: int):
    """Eq. 4 iterated on the full N x N kernel matrix.

    u_i <- argmin_j g_j - 2 f_ij (+ K_ii, constant per row), with
    g_j = 1/|w_j|^2 sum_{m,n} K_mn d(u_m,j) d(u_n,j) (Eq. 5) and
    f_ij = 1/|w_j| sum_m K_im d(u_m,j) (Eq. 6), written as matrix products with the
    membership matrix Z (N x C).  Stops when no label changes or after T updates.
    Returns (labels after every update, final distance matrix)."""
    K = np.asarray(K, dtype=np.float64)
    U = np.asarray(U0, dtype=np.int64).copy()
    N = K.shape[0]
    history = []
    d = None
    for _ in range(T):
        Z = np.zeros((N, C))
        Z[np.arange(N), U] = 1.0
        card = Z.sum(axis=0)
        nz = card > 0
        F = np.zeros((N, C))
        F[:, nz] = (K @ Z[:, nz]) / card[nz]
        G = np.full(C, INF)
        G[nz] = np.einsum("mj,mn,nj->j", Z[:, nz], K, Z[:, nz]) / card[nz] ** 2
        d = np.diag(K)[:, None] - 2.0 * F + G[None, :]
        d[:, ~nz] = INF
        U_new = np.argmin(d, axis=1)
        history.append(U_new.copy())
        if np.array_equal(U_new, U):
            break
        U = U_new
    return history, d


def lloyd(X: np.ndarray, U0: np.ndarray, C: int, T: int):
    """Lloyd's k-means with explicit centroid coordinates, same stopping rule.

    Returns (labels after every update, final squared distances)."""
    X = np.asarray(X, dtype=np.float64)
    U = np.asarray(U0, dtype=np.int64).copy()
    history = []
    d = None
    for _ in range(T):
        d = np.full((X.shape[0], C), INF)
        for j in range(C):
            mem = U == j
            if mem.any():
                mu = X[mem].mean(axis=0)
                diff = X - mu
                d[:, j] = np.einsum("ij,ij->i", diff, diff)
        U_new = np.argmin(d, axis=1)
        history.append(U_new.copy())
        if np.array_equal(U_new, U):
            break
        U = U_new
    return history, d


def partition_cost(K: np.ndarray, U: np.ndarray, C: int) -> float:
    """Eq. 1 with w_j the feature-space mean of cluster j (Eq. 3):

    sum_j [ sum_{x in j} K_xx - 1/|j| sum_{x,y in j} K_xy ]."""
    K = np.asarray(K, dtype=np.float64)
    U = np.asarray(U)
    J = 0.0
    for j in range(C):
        mem = np.flatnonzero(U == j)
        if len(mem) == 0:
            continue
        J += np.trace(K[np.ix_(mem, mem)]) - K[np.ix_(mem, mem)].sum() / len(mem)
    return float(J)


def explicit_cost(X: np.ndarray, U: np.ndarray, C: int) -> float:
    """Sum of squared distances to explicit cluster means (linear kernel)."""
    X = np.asarray(X, dtype=np.float64)
    J = 0.0
    for j in range(C):
        mem = np.asarray(U) == j
        if mem.any():
            J += float(((X[mem] - X[mem].mean(axis=0)) ** 2).sum())
    return J


def brute_force(K: np.ndarray, C: int):
    """Minimum of partition_cost over all C^N labellings (tiny N only).

    Returns (best cost, one optimal labelling, costs of every labelling in
    lexicographic order of the label tuple)."""
    N = K.shape[0]
    costs = []
    best, best_u = INF, None
    for u in itertools.product(range(C), repeat=N):
        u = np.asarray(u)
        J = partition_cost(K, u, C)
        costs.append(J)
        if J < best:
            best, best_u = J, u
    return best, best_u, np.asarray(costs)
