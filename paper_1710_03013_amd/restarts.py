"""Best of several kernel k-means++ restarts (the paper keeps the lowest-cost run of five, Sec. 4.5).

The restarts are independent fits with seeds ``seed, seed + 1, ...`` (each seed fixes the
landmarks, the k-means++ draws and everything else the RNG specification derives from it).  The
library's ``kkm_fit_restarts`` runs them back to back on one stream out of one workspace, takes each
fitted model's FP64 cost (Eq. 1) over all of X, and keeps the lowest (the lowest seed on equal
costs); this module is the Python face of that entry point.
"""
from __future__ import annotations

from . import kkm_fit_restarts

__all__ = ["fit_best_of"]


def fit_best_of(X, restarts: int = 5, seed: int = 0, stream=None, **fit_kwargs):
    """Fit ``restarts`` times (seeds seed .. seed + restarts - 1) and keep the lowest-cost model.

    Returns (model, labels, info) of the winner, as ``kkm_fit`` does; ``info`` also holds
    ``restart`` (the winner's index, its seed being seed + restart) and ``restart_costs``."""
    if restarts < 1:
        raise ValueError("restarts must be >= 1")
    for k in ("landmarks", "kmpp_uniforms", "init_labels"):   # (they follow from each restart's seed)
        if k in fit_kwargs:
            raise ValueError(f"fit_best_of sets {k} itself")
    return kkm_fit_restarts(X, restarts=restarts, seed=seed, stream=stream, **fit_kwargs)
