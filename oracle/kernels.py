"""Kernel functions in float64 (oracle; test infrastructure only).

The paper leaves the Mercer kernel generic (Sec. 2: K(x_m, x_n) replaces the
feature-space inner product).  Three kernels are used by the workloads:

* linear   K(x, y) = x . y  -- the case in which kernel k-means is Lloyd's
  k-means (Sec. 2, closing remark on the linear case);
* Gaussian K(x, y) = exp(-||x - y||^2 / (2 sigma^2)), with the squared
  distance formed from explicit coordinate differences (no norm expansion);
* RMSD     K(x, y) = exp(-RMSD(x, y)^2 / (2 sigma^2)) for frames of A atoms,
  RMSD after optimal superposition by a proper rotation and a translation,
  equal atom weights (the roto-translation invariance demanded in Sec. 1 and
  Sec. 4.5).  The optimum comes from the largest eigenvalue of Horn's 4x4
  quaternion key matrix, found with a dense symmetric eigensolver (LAPACK via
  numpy.linalg.eigh).  ``rmsd2_kabsch`` is an independent SVD route used to
  pin it.
"""
from __future__ import annotations

import numpy as np


def linear(X: np.ndarray, Y: np.ndarray) -> np.ndarray:
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    return X @ Y.T


def sqdist(X: np.ndarray, Y: np.ndarray, chunk: int = 256) -> np.ndarray:
    """Squared Euclidean distances from explicit differences."""
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    out = np.empty((X.shape[0], Y.shape[0]), dtype=np.float64)
    for a in range(0, X.shape[0], chunk):
        diff = X[a:a + chunk, None, :] - Y[None, :, :]
        out[a:a + chunk] = np.einsum("ijk,ijk->ij", diff, diff)
    return out


def rbf(X: np.ndarray, Y: np.ndarray, sigma: float) -> np.ndarray:
    return np.exp(-sqdist(X, Y) / (2.0 * sigma * sigma))


def as_frames(X: np.ndarray, n_atoms: int) -> np.ndarray:
    X = np.asarray(X, dtype=np.float64)
    return X.reshape(X.shape[0], n_atoms, 3)


def centred(F: np.ndarray) -> np.ndarray:
    return F - F.mean(axis=1, keepdims=True)


def horn_matrix(R: np.ndarray) -> np.ndarray:
    """Horn's symmetric 4x4 key matrix from the 3x3 correlation R[p,q] = sum_a x_ap y_aq.

    Its largest eigenvalue is max over unit quaternions q of sum_a (rot(q) x_a) . y_a."""
    Sxx, Sxy, Sxz = R[..., 0, 0], R[..., 0, 1], R[..., 0, 2]
    Syx, Syy, Syz = R[..., 1, 0], R[..., 1, 1], R[..., 1, 2]
    Szx, Szy, Szz = R[..., 2, 0], R[..., 2, 1], R[..., 2, 2]
    N = np.empty(R.shape[:-2] + (4, 4), dtype=np.float64)
    N[..., 0, 0] = Sxx + Syy + Szz
    N[..., 0, 1] = Syz - Szy
    N[..., 0, 2] = Szx - Sxz
    N[..., 0, 3] = Sxy - Syx
    N[..., 1, 1] = Sxx - Syy - Szz
    N[..., 1, 2] = Sxy + Syx
    N[..., 1, 3] = Szx + Sxz
    N[..., 2, 2] = -Sxx + Syy - Szz
    N[..., 2, 3] = Syz + Szy
    N[..., 3, 3] = -Sxx - Syy + Szz
    for i in range(4):
        for j in range(i):
            N[..., i, j] = N[..., j, i]
    return N


def rmsd2_horn(Fx: np.ndarray, Fy: np.ndarray, chunk: int = 64) -> np.ndarray:
    """Squared minimal RMSD between every frame of Fx (n,A,3) and of Fy (m,A,3)."""
    Fx = centred(np.asarray(Fx, dtype=np.float64))
    Fy = centred(np.asarray(Fy, dtype=np.float64))
    A = Fx.shape[1]
    Gx = np.einsum("nai,nai->n", Fx, Fx)
    Gy = np.einsum("nai,nai->n", Fy, Fy)
    out = np.empty((Fx.shape[0], Fy.shape[0]), dtype=np.float64)
    for a in range(0, Fx.shape[0], chunk):
        R = np.einsum("nap,maq->nmpq", Fx[a:a + chunk], Fy)
        lam = np.linalg.eigh(horn_matrix(R))[0][..., -1]
        out[a:a + chunk] = np.maximum(0.0, (Gx[a:a + chunk, None] + Gy[None, :] - 2.0 * lam) / A)
    return out


def rmsd2_kabsch(fx: np.ndarray, fy: np.ndarray) -> float:
    """Independent route for one pair: SVD of the correlation matrix with the
    reflection fix (W. Kabsch, Acta Cryst. A32, 1976; A34, 1978)."""
    x = centred(np.asarray(fx, dtype=np.float64)[None])[0]
    y = centred(np.asarray(fy, dtype=np.float64)[None])[0]
    R = x.T @ y
    U, S, Vt = np.linalg.svd(R)
    sgn = np.sign(np.linalg.det(U @ Vt))
    if sgn == 0:
        sgn = 1.0
    e = S[0] + S[1] + sgn * S[2]
    A = x.shape[0]
    return max(0.0, (np.sum(x * x) + np.sum(y * y) - 2.0 * e) / A)


def rmsd(X: np.ndarray, Y: np.ndarray, sigma: float, n_atoms: int) -> np.ndarray:
    d2 = rmsd2_horn(as_frames(X, n_atoms), as_frames(Y, n_atoms))
    return np.exp(-d2 / (2.0 * sigma * sigma))


class Kernel:
    """A kernel function by name: 'linear', 'rbf' (needs sigma) or 'rmsd' (sigma, n_atoms)."""

    def __init__(self, kind: str, sigma: float = 1.0, n_atoms: int = 0):
        if kind not in ("linear", "rbf", "rmsd"):
            raise ValueError(kind)
        self.kind, self.sigma, self.n_atoms = kind, float(sigma), int(n_atoms)

    def __call__(self, X: np.ndarray, Y: np.ndarray) -> np.ndarray:
        if self.kind == "linear":
            return linear(X, Y)
        if self.kind == "rbf":
            return rbf(X, Y, self.sigma)
        return rmsd(X, Y, self.sigma, self.n_atoms)

    def diag(self, X: np.ndarray) -> np.ndarray:
        """K(x, x) for every row."""
        X = np.asarray(X, dtype=np.float64)
        if self.kind == "linear":
            return np.einsum("ij,ij->i", X, X)
        return np.ones(X.shape[0], dtype=np.float64)
