"""Best of several kernel k-means++ restarts (the paper keeps the lowest-cost run of five).

The restarts are independent fits with seeds ``seed, seed + 1, ...`` (each seed fixes the
landmarks, the k-means++ draws and everything else the RNG specification derives from it), run one
after another on the caller's stream.  Each fitted model's cost (Eq. 1) over all of X is taken on
the GPU in FP64 by ``kkm_cost``, and the lowest cost wins (the lowest seed on equal costs).  All
device work runs in the library's kernels; this module only sequences the calls.
"""
from __future__ import annotations

from . import kkm_cost, kkm_fit

__all__ = ["fit_best_of"]


def fit_best_of(X, restarts: int = 5, seed: int = 0, cost_precision: str = "fp64", stream=None, **fit_kwargs):
    """Fit ``restarts`` times (seeds seed .. seed + restarts - 1) and keep the lowest-cost model.

    Returns (model, labels, info) of the winner, as ``kkm_fit`` does; ``info`` also holds
    ``restart`` (the winner's index, its seed being seed + restart) and ``restart_costs``."""
    if restarts < 1:
        raise ValueError("restarts must be >= 1")
    for k in ("landmarks", "kmpp_uniforms", "init_labels"):   # (they follow from each restart's seed)
        if k in fit_kwargs:
            raise ValueError(f"fit_best_of sets {k} itself")
    best, costs = None, []
    for r in range(restarts):
        model, labels, info = kkm_fit(X, seed=seed + r, stream=stream, **fit_kwargs)
        cost = kkm_cost(model, X, precision=cost_precision, stream=stream)
        costs.append(cost)
        if best is None or cost < best[3]:   # strict: the lowest seed wins on equal costs
            best = (model, labels, info, cost, r)
        del model, labels, info                 # a losing model is released here
    model, labels, info, _, r = best
    return model, labels, dict(info, restart=r, restart_costs=costs)
