"""Choosing the two trade-off parameters: the number of mini-batches B and the landmark fraction s.

Sec. 4.2 of the paper suggests fixing a target execution time: take the smallest B the memory allows
(Eq. 19; here ``kkm_fit_min_batches``, which searches this library's own footprint, any s included)
and s = 1; estimate the time of the whole fit as B times the time of a fit on a single mini-batch; if
that is too long, first lower s step by step, and only when s would fall below about 0.2 raise B.  The
approximation can then be checked on one mini-batch against the reference parameters (B_min, 1).

Every fit runs in the library; this module only sequences the calls, times them on the host and
compares clusterings (normalised mutual information, written out below).
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field
from typing import Callable, List, Optional

import numpy as np

__all__ = ["Choice", "choose_batches_and_fraction", "nmi", "majority_accuracy"]


@dataclass
class Choice:
    B: int                      # mini-batches
    s: float                    # landmark fraction
    expected_s: float           # B x the single-batch time of the last trial
    met: bool                   # the expected time is within the budget
    B_min: int                  # smallest B the memory budget allows
    trials: List[dict] = field(default_factory=list)   # (B, s, single-batch seconds, expected) in order


def _entropy(counts: np.ndarray) -> float:
    p = counts[counts > 0] / counts.sum()
    return float(-(p * np.log(p)).sum())


def nmi(a: np.ndarray, b: np.ndarray) -> float:
    """I(a; b) / sqrt(H(a) H(b)) from the joint histogram of two labellings (1 when both are constant)."""
    a = np.unique(np.asarray(a), return_inverse=True)[1]
    b = np.unique(np.asarray(b), return_inverse=True)[1]
    joint = np.zeros((a.max() + 1, b.max() + 1))
    np.add.at(joint, (a, b), 1.0)
    ha, hb = _entropy(joint.sum(1)), _entropy(joint.sum(0))
    if ha == 0.0 or hb == 0.0:
        return 1.0 if ha == hb else 0.0
    return (ha + hb - _entropy(joint.ravel())) / np.sqrt(ha * hb)


def majority_accuracy(truth: np.ndarray, labels: np.ndarray) -> float:
    """Fraction of samples whose cluster's most frequent true class is their own class."""
    truth = np.asarray(truth)
    labels = np.asarray(labels)
    hit = 0
    for u in np.unique(labels):
        cls = truth[labels == u]
        hit += np.bincount(np.unique(cls, return_inverse=True)[1]).max()
    return hit / truth.size


def choose_batches_and_fraction(X, time_budget_s: float, memory_budget_bytes: int, kernel: str = "rbf",
                                sigma: float = 1.0, n_atoms: int = 0, C: int = 2, max_iter: int = 20,
                                precision: str = "fp32", seed: int = 0, s_floor: float = 0.2, s_factor: float = 0.7,
                                B_max: Optional[int] = None, single_batch_time: Optional[Callable] = None) -> Choice:
    """The procedure of Sec. 4.2.  single_batch_time(B, s) -> seconds defaults to timing kkm_fit of the
    first stride mini-batch (B = 1 on those rows, the same s); it may be replaced (tests, other
    estimates).  s is multiplied by s_factor while it stays >= s_floor, then B is doubled (s kept)."""
    from . import kkm_fit, kkm_fit_min_batches, _kernel, _dtype_code
    N, d = X.shape
    kspec = _kernel(kernel, sigma, n_atoms)
    common = dict(C=C, max_iter=max_iter, precision=precision, seed=seed)
    B_min = kkm_fit_min_batches(N, d, _dtype_code(X), kspec, int(memory_budget_bytes), s=1.0, sampling="stride",
                                init="kmeans++", landmarks=None, kmpp_uniforms=None, init_labels=None,
                                init_medoids=None, **common)
    B_max = B_max or max(1, N // max(1, C))

    if single_batch_time is None:
        def single_batch_time(B, s):
            import torch
            rows = X[0::B]
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            kkm_fit(rows, kernel, sigma=sigma, n_atoms=n_atoms, B=1, s=s, want_labels=False, **common)
            return time.perf_counter() - t0

    B, s = B_min, 1.0
    trials = []
    while True:
        t1 = float(single_batch_time(B, s))
        expected = B * t1
        trials.append(dict(B=B, s=s, single_batch_s=t1, expected_s=expected))
        if expected <= time_budget_s:
            return Choice(B, s, expected, True, B_min, trials)
        if s * s_factor >= s_floor:
            s = s * s_factor
        elif 2 * B <= B_max:
            B = 2 * B
        else:
            return Choice(B, s, expected, False, B_min, trials)
