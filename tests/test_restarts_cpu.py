"""Selection rule of the best-of-restarts helper with the library calls replaced by host stand-ins
(no GPU): seeds seed .. seed + R - 1 in order, the lowest cost kept, the lowest seed on equal
costs, and the arguments the helper sets itself rejected."""
import pytest

import paper_1710_03013_amd.restarts as rs


def _fake(monkeypatch, costs):
    calls = []

    def fake_fit(X, seed=0, stream=None, **kw):
        calls.append(seed)
        return ("model", seed), ("labels", seed), {"seed": seed}

    def fake_cost(model, X, precision="fp64", stream=None):
        return costs[model[1]]

    monkeypatch.setattr(rs, "kkm_fit", fake_fit)
    monkeypatch.setattr(rs, "kkm_cost", fake_cost)
    return calls


def test_lowest_cost_wins(monkeypatch):
    calls = _fake(monkeypatch, {10: 5.0, 11: 3.0, 12: 4.0, 13: 3.5})
    model, labels, info = rs.fit_best_of(None, restarts=4, seed=10)
    assert calls == [10, 11, 12, 13]
    assert model == ("model", 11) and labels == ("labels", 11) and info["restart"] == 1
    assert info["restart_costs"] == [5.0, 3.0, 4.0, 3.5]


def test_equal_costs_keep_the_lowest_seed(monkeypatch):
    _fake(monkeypatch, {0: 2.0, 1: 1.0, 2: 1.0})
    _, _, info = rs.fit_best_of(None, restarts=3, seed=0)
    assert info["restart"] == 1


def test_arguments_the_helper_sets_are_rejected(monkeypatch):
    _fake(monkeypatch, {0: 1.0})
    for k in ("landmarks", "kmpp_uniforms", "init_labels"):
        with pytest.raises(ValueError):
            rs.fit_best_of(None, restarts=1, **{k: 1})
    with pytest.raises(ValueError):
        rs.fit_best_of(None, restarts=0)
