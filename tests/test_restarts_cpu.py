"""The restarts entry point without a GPU: its workspace holds one fit (plus its medoid model and
labels) per restart and one assign pass, it refuses draws that each restart must make itself, and the
Python face refuses them before calling the library."""
import numpy as np
import pytest

import paper_1710_03013_amd as kk
import paper_1710_03013_amd.restarts as rs


def _args(**kw):
    a = dict(C=20, B=10, s=0.1, max_iter=20, sampling="stride", init="kmeans++", precision="fp32", seed=7,
             landmarks=None, kmpp_uniforms=None, init_labels=None, init_medoids=None)
    a.update(kw)
    return a


def _ws(R, **kw):
    k = kk._kernel("rbf", 4.0)
    keep = []
    p = kk._params(**_args(**kw), keep=keep)
    return int(kk.lib().kkm_fit_restarts_workspace_bytes(100_000, 16, kk.KKM_F32, kk.ct.byref(k), kk.ct.byref(p), R))


def test_workspace_grows_by_one_fit_per_restart():
    one = kk.kkm_fit_workspace_bytes(100_000, 16, kk.KKM_F32, kk._kernel("rbf", 4.0), **_args())
    w1, w2, w5 = _ws(1), _ws(2), _ws(5)
    assert w1 > one
    per = w2 - w1
    assert per >= one + 4 * 100_000          # a fit, its medoid model and its labels
    assert w5 == w1 + 4 * per


def test_restart_draws_are_refused():
    assert _ws(3, landmarks=[np.arange(1000)] * 10) == 0
    assert _ws(3, kmpp_uniforms=np.full(20, 0.5)) == 0
    assert _ws(0) == 0 and _ws(2000) == 0


def test_python_face_refuses_draws():
    for key in ("landmarks", "kmpp_uniforms", "init_labels"):
        with pytest.raises(ValueError):
            rs.fit_best_of(None, restarts=2, **{key: np.zeros(3)})
    with pytest.raises(ValueError):
        rs.fit_best_of(None, restarts=0)
