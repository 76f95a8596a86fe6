"""The (B, s) procedure of Sec. 4.2 with the single-batch timing replaced by a host model (no GPU):
start at (B_min, 1), lower s while it stays above the floor, then double B; B_min is the memory
knob's answer.  The clustering comparisons are checked on closed cases."""
import numpy as np
import pytest

import paper_1710_03013_amd as kk
from paper_1710_03013_amd import tuning


class _X:
    shape = (100_000, 16)
    dtype = None


def _budget(B):
    k = kk._kernel("rbf", 4.0)
    return kk.kkm_fit_workspace_bytes(100_000, 16, kk.KKM_F32, k, C=20, B=B, s=1.0, max_iter=20,
                                      sampling="stride", init="kmeans++", precision="fp32", seed=0,
                                      landmarks=None, kmpp_uniforms=None, init_labels=None, init_medoids=None)


@pytest.fixture
def fake_dtype(monkeypatch):
    monkeypatch.setattr(kk, "_dtype_code", lambda X: kk.KKM_F32)


def test_generous_budget_keeps_bmin_and_full_support(fake_dtype):
    mem = _budget(4)
    ch = tuning.choose_batches_and_fraction(_X(), 10.0, mem, sigma=4.0, C=20,
                                            single_batch_time=lambda B, s: 0.01)
    assert ch.B == ch.B_min and ch.s == 1.0 and ch.met
    assert ch.B_min == kk.kkm_fit_min_batches(100_000, 16, kk.KKM_F32, kk._kernel("rbf", 4.0), mem, C=20, s=1.0,
                                               max_iter=20, precision="fp32", seed=0, sampling="stride",
                                               init="kmeans++", landmarks=None, kmpp_uniforms=None, init_labels=None,
                                               init_medoids=None)


def test_lowers_s_before_raising_b(fake_dtype):
    # a single batch costs ~ s (n/B)^2: the budget forces s down to the floor, then B up
    model = lambda B, s: 1e-9 * s * (100_000 / B) ** 2
    ch = tuning.choose_batches_and_fraction(_X(), 0.05, _budget(4), sigma=4.0, C=20, s_factor=0.5, s_floor=0.2,
                                            single_batch_time=model)
    seq = [(t["B"], round(t["s"], 6)) for t in ch.trials]
    B0 = ch.B_min
    assert seq[:3] == [(B0, 1.0), (B0, 0.5), (B0, 0.25)]          # s halves while >= 0.2
    assert all(b >= B0 for b, _ in seq) and seq[3][0] == 2 * B0      # then B doubles, s kept
    assert ch.met and ch.expected_s <= 0.05
    assert ch.expected_s == pytest.approx(ch.B * model(ch.B, ch.s))


def test_unreachable_budget_is_reported(fake_dtype):
    ch = tuning.choose_batches_and_fraction(_X(), 1e-9, _budget(4), sigma=4.0, C=20, B_max=64,
                                            single_batch_time=lambda B, s: 1.0)
    assert not ch.met and ch.B <= 64


def test_nmi_and_accuracy_closed_cases():
    a = np.array([0, 0, 1, 1, 2, 2])
    assert tuning.nmi(a, np.array([5, 5, 9, 9, 7, 7])) == pytest.approx(1.0)
    assert tuning.nmi(np.array([0, 0, 1, 1]), np.array([0, 1, 0, 1])) == pytest.approx(0.0, abs=1e-12)
    assert tuning.majority_accuracy(a, np.array([1, 1, 0, 0, 0, 0])) == pytest.approx(4 / 6)
    assert tuning.majority_accuracy(a, np.array([3, 3, 1, 1, 2, 2])) == 1.0
