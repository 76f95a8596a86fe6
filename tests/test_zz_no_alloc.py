"""kkm_assign_noalloc: the assign pass with the library's fixed device scratch (no allocation).

Its labels and margins must equal kkm_assign's on the same rows, on two calls in a row (the second
with fewer rows, so the scratch holds the first call's contents), for a linear / RBF medoid model in
each precision, general sparse centroids and RMSD frames; sizes beyond the scratch are refused."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import kkm_inputs as ki  # noqa: E402


def _kk():
    import paper_1710_03013_amd as kk
    return kk


def _both(kk, m, Y, prec):
    Yd = torch.from_numpy(np.ascontiguousarray(Y)).cuda()
    want_l, want_g = kk.kkm_assign(m, Yd, precision=prec, want_gap=True)
    lab = torch.full((Yd.shape[0],), -7, dtype=torch.int32, device="cuda")
    gap = torch.full((Yd.shape[0],), -7.0, dtype=torch.float32, device="cuda")
    kk.kkm_assign_noalloc(m, Yd, lab, gap, precision=prec)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(lab.cpu().numpy(), want_l.cpu().numpy())
    np.testing.assert_array_equal(gap.cpu().numpy(), want_g.cpu().numpy())


@pytest.mark.parametrize("prec", ["fp32", "bf16x3", "bf16", "fp64"])
def test_noalloc_assign_equals_assign_medoid_model(prec):
    kk = _kk()
    print(f"noalloc medoid model {prec}", flush=True)
    X, _ = ki.datasets.gaussian_mixture(70_000 + 100, 64, 100, seed=1014, sigma=None)
    m = kk.kkm_model_create("rbf", d=64, C=100, dtype="f32", sigma=8.0)
    kk.kkm_model_load(m, X[:100], np.arange(101), np.ones(100))
    _both(kk, m, X[100:], prec)           # 70 000 rows
    _both(kk, m, X[100:1337], prec)       # then fewer: the scratch still holds the first call's data


def test_noalloc_assign_sparse_and_linear():
    kk = _kk()
    print("noalloc sparse / linear", flush=True)
    X, _ = ki.datasets.gaussian_mixture(9000, 16, 6, seed=15, sigma=1.5, box=5.0)
    offsets = np.array([0, 10, 10, 17, 30, 31, 40])
    coef = np.random.default_rng(1).uniform(0.2, 1.0, size=40)
    m = kk.kkm_model_create("rbf", d=16, C=6, max_support=40, dtype="f32", sigma=3.0)
    kk.kkm_model_load(m, X[:40], offsets, coef)
    _both(kk, m, X[40:], "fp32")
    _both(kk, m, X[40:777], "fp32")
    lin = kk.kkm_model_create("linear", d=16, C=5, dtype="f32")
    kk.kkm_model_load(lin, X[:5], np.arange(6), np.ones(5))
    _both(kk, lin, X[5:], "fp32")
    _both(kk, lin, X[5:64], "bf16x3")


def test_noalloc_assign_rmsd_frames():
    kk = _kk()
    print("noalloc rmsd", flush=True)
    X, _ = ki.datasets.md_frames(20_050, A=50, n_templates=10, seed=16)
    M = X[:50]
    m = kk.kkm_model_create("rmsd", d=150, C=50, dtype="f32", sigma=1.5, n_atoms=50)
    kk.kkm_model_load(m, M, np.arange(51), np.ones(50))
    _both(kk, m, X[50:], "fp32")
    _both(kk, m, X[50:3050], "fp32")


def test_noalloc_assign_refuses_sizes_beyond_its_scratch():
    kk = _kk()
    X, _ = ki.datasets.md_frames(60, A=50, n_templates=2, seed=17)
    m = kk.kkm_model_create("rmsd", d=150, C=2, dtype="f32", sigma=1.5, n_atoms=50)
    kk.kkm_model_load(m, X[:2], np.arange(3), np.ones(2))
    big = torch.zeros((100_000, 150), dtype=torch.float32, device="cuda")   # 100 000 frames > 48 MiB
    lab = torch.empty(100_000, dtype=torch.int32, device="cuda")
    with pytest.raises(kk.KkmError) as e:
        kk.kkm_assign_noalloc(m, big, lab)
    assert e.value.status == -6 and "scratch" in str(e.value)
