"""Clustering quality measures of Sec. 4 (oracle; test infrastructure only).

* accuracy: fraction of samples whose cluster, mapped to a class by majority
  vote over its members, equals the true class;
* NMI: I(y; u) / sqrt(H(y) H(u)).  The printed NMI formula is garbled in the
  available text (product of entropies, no square root); the standard
  normalisation by the geometric mean of the entropies is used.
"""
from __future__ import annotations

import numpy as np


def accuracy(y: np.ndarray, u: np.ndarray) -> float:
    y = np.asarray(y)
    u = np.asarray(u)
    correct = 0
    for c in np.unique(u):
        mem = y[u == c]
        correct += np.bincount(mem).max()
    return correct / len(y)


def nmi(y: np.ndarray, u: np.ndarray) -> float:
    y = np.asarray(y)
    u = np.asarray(u)
    N = len(y)
    ys, yi = np.unique(y, return_inverse=True)
    us, ui = np.unique(u, return_inverse=True)
    o = np.zeros((len(us), len(ys)))
    np.add.at(o, (ui, yi), 1.0)
    n = o.sum(axis=1)
    m = o.sum(axis=0)
    nzo = o > 0
    I = np.sum(o[nzo] / N * np.log(N * o[nzo] / np.outer(n, m)[nzo]))
    Hu = -np.sum(n / N * np.log(n / N))
    Hy = -np.sum(m / N * np.log(m / N))
    if Hu == 0 or Hy == 0:
        return 1.0 if Hu == Hy else 0.0
    return float(I / np.sqrt(Hu * Hy))
