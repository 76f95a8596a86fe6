"""Seeded synthetic datasets with the shapes and structure of the paper's workloads.

None of the paper's own datasets (MNIST, RCV1, noisy MNIST, the PNP/DADMe-immH
trajectory) is available, so every workload is a stand-in drawn from a seed:

* ``two_rings``       -- two concentric noisy rings (the classic non-linearly
                         separable case that motivates the kernel form, Sec. 1);
* ``gaussian_mixture`` -- isotropic or anisotropic Gaussian mixtures (the
                         feature-vector workloads of Sec. 4.4);
* ``md_frames``       -- molecular-dynamics-shaped frames: rigid-body moved,
                         noisy copies of a few chain templates, where only a
                         roto-translation-invariant similarity sees the
                         clusters (Sec. 4.5).

Each returns ``(X, y)``: the samples (row-major) and the generating component
of each sample (for accuracy / NMI only).
"""
from __future__ import annotations

import numpy as np


def two_rings(N: int = 2000, radii=(1.0, 3.0), noise: float = 0.1, seed: int = 1000,
              dtype=np.float64):
    """N points split evenly over concentric rings (ring 0 first), uniform angle,
    isotropic Gaussian noise of std `noise`."""
    rng = np.random.default_rng(seed)
    k = len(radii)
    sizes = [N // k + (1 if i < N % k else 0) for i in range(k)]
    xs, ys = [], []
    for i, (r, m) in enumerate(zip(radii, sizes)):
        t = rng.uniform(0.0, 2.0 * np.pi, size=m)
        p = np.stack([r * np.cos(t), r * np.sin(t)], axis=1)
        p = p + rng.normal(0.0, noise, size=p.shape)
        xs.append(p)
        ys.append(np.full(m, i, dtype=np.int32))
    return np.concatenate(xs).astype(dtype), np.concatenate(ys)


def gaussian_mixture(N: int, d: int, K: int, seed: int, box: float = 10.0,
                     sigma: float | None = 1.0, sigma_range=(0.5, 2.0), dtype=np.float32,
                     chunk: int = 1 << 18):
    """Equal-weight mixture of K Gaussians with means uniform in [-box, box]^d.

    sigma given: isotropic std `sigma`; sigma None: each component draws a
    per-dimension std uniform in `sigma_range` (anisotropic).  Component of each
    point is drawn i.i.d. uniform."""
    rng = np.random.default_rng(seed)
    means = rng.uniform(-box, box, size=(K, d))
    if sigma is None:
        stds = rng.uniform(sigma_range[0], sigma_range[1], size=(K, d))
    else:
        stds = np.full((K, d), float(sigma))
    y = rng.integers(0, K, size=N).astype(np.int32)
    X = np.empty((N, d), dtype=dtype)
    for a in range(0, N, chunk):
        b = min(N, a + chunk)
        z = rng.standard_normal(size=(b - a, d))
        X[a:b] = (means[y[a:b]] + z * stds[y[a:b]]).astype(dtype)
    return X, y


def random_rotations(rng: np.random.Generator, n: int) -> np.ndarray:
    """n Haar-uniform proper rotations (QR of a Gaussian matrix with sign fix)."""
    g = rng.standard_normal(size=(n, 3, 3))
    q, r = np.linalg.qr(g)
    s = np.sign(np.diagonal(r, axis1=1, axis2=2))
    s[s == 0] = 1.0
    q = q * s[:, None, :]
    det = np.linalg.det(q)
    q[det < 0, :, 0] *= -1.0
    return q


def chain_templates(rng: np.random.Generator, T: int, A: int, bond: float = 3.8) -> np.ndarray:
    """T random-walk chains of A atoms with fixed bond length, directions uniform on the sphere."""
    v = rng.standard_normal(size=(T, A - 1, 3))
    v /= np.linalg.norm(v, axis=2, keepdims=True)
    chain = np.concatenate([np.zeros((T, 1, 3)), np.cumsum(bond * v, axis=1)], axis=1)
    return chain - chain.mean(axis=1, keepdims=True)


def md_frames(N: int, A: int = 50, n_templates: int = 10, seed: int = 1002, noise: float = 0.5,
              shift: float = 20.0, bond: float = 3.8, dtype=np.float32, chunk: int = 1 << 15):
    """N frames of A atoms x 3 coordinates, returned as an (N, 3A) row-major array
    (atom-major: x0 y0 z0 x1 y1 z1 ...).

    Each frame: a template chosen uniformly, plus per-coordinate Gaussian noise,
    then a Haar-uniform rotation about the origin and a translation uniform in
    [-shift, shift]^3."""
    rng = np.random.default_rng(seed)
    tpl = chain_templates(rng, n_templates, A, bond)
    y = rng.integers(0, n_templates, size=N).astype(np.int32)
    X = np.empty((N, 3 * A), dtype=dtype)
    for a in range(0, N, chunk):
        b = min(N, a + chunk)
        m = b - a
        f = tpl[y[a:b]] + rng.normal(0.0, noise, size=(m, A, 3))
        R = random_rotations(rng, m)
        f = np.einsum("nij,naj->nai", R, f)
        f = f + rng.uniform(-shift, shift, size=(m, 1, 3))
        X[a:b] = f.reshape(m, 3 * A).astype(dtype)
    return X, y


def config_data(k: int, scale: float = 1.0):
    """Synthetic dataset of workload k (0..3) with data seed 1000+k.

    scale < 1 shrinks N (for tests) keeping every other parameter."""
    if k == 0:
        return two_rings(N=max(4, int(round(2000 * scale))), seed=1000)
    if k == 1:
        return gaussian_mixture(max(20, int(round(100_000 * scale))), 16, 20, seed=1001, sigma=1.0)
    if k == 2:
        return md_frames(max(20, int(round(200_000 * scale))), A=50, n_templates=10, seed=1002)
    if k == 3:
        return gaussian_mixture(max(100, int(round(1_000_000 * scale))), 64, 100, seed=1003, sigma=None)
    raise ValueError(k)


# Model hyper-parameters of each workload (kernel, C, B, s, T).
CONFIGS = {
    0: dict(kernel="rbf", sigma=1.0, C=2, B=1, s=1.0, T=30, init="random", dtype="f64"),
    1: dict(kernel="rbf", sigma=4.0, C=20, B=10, s=0.1, T=20, init="kmeans++", dtype="f32"),
    2: dict(kernel="rmsd", sigma=1.5, C=50, B=20, s=0.05, T=20, init="kmeans++", dtype="f32", n_atoms=50),
    3: dict(kernel="rbf", sigma=8.0, C=100, B=50, s=0.02, T=20, init="kmeans++", dtype="f32"),
}
