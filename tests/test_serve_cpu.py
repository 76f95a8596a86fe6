"""Scheduling logic of the serving loop with a host-only backend (no GPU): arrival-ordered
admission, the HBM budget, slot limits, coalescing of small assign requests, fit registration
and error reporting."""
import numpy as np
import pytest

from paper_1710_03013_amd.serve import Server


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


class FakeModel:
    def __init__(self, d, centres):
        self.d = d
        self.centres = np.asarray(centres, dtype=np.float64)

    def labels(self, X):
        d2 = ((X[:, None, :] - self.centres[None]) ** 2).sum(-1)
        return d2.argmin(1).astype(np.int32)


class FakeBackend:
    """Work finishes `latency` clock units after launch; memory is 8 bytes per row plus 100."""

    def __init__(self, clock, latency=1.0):
        self.clock, self.latency = clock, latency
        self.launches = []

    def assign_bytes(self, model, rows, concatenated):
        return 100 + 8 * rows + (4 * rows * model.d if concatenated else 0)

    def fit_bytes(self, X, kw):
        return 1000 + 16 * X.shape[0]

    def launch_assign(self, model, xs, slot, ready=None):
        X = np.concatenate(xs, 0)
        self.launches.append(("assign", [x.shape[0] for x in xs]))
        return {"t": self.clock() + self.latency, "labels": model.labels(X), "sizes": [x.shape[0] for x in xs]}

    def assign_done(self, h):
        return self.clock() >= h["t"]

    def assign_results(self, h):
        out, o = [], 0
        for n in h["sizes"]:
            out.append(h["labels"][o:o + n])
            o += n
        return out

    def start_fit(self, X, kw, slot, ready=None):
        self.launches.append(("fit", X.shape[0]))
        C = kw["C"]
        return {"t": self.clock() + 3 * self.latency, "model": FakeModel(X.shape[1], X[:C])}

    def fit_done(self, h):
        return self.clock() >= h["t"]

    def fit_result(self, h):
        return h["model"], None, {}


def _server(budget=10_000, slots=2, fits=1, **kw):
    clock = FakeClock()
    be = FakeBackend(clock)
    srv = Server(be, budget, assign_slots=slots, fit_workers=fits, clock=clock, **kw)
    srv.add_model("m", FakeModel(2, [[0.0, 0.0], [10.0, 10.0]]))
    return srv, be, clock


def _drain(srv, clock, step=0.5, limit=1000):
    for _ in range(limit):
        srv.poll()
        if srv.idle:
            return
        clock.t += step
    raise AssertionError("did not drain")


def test_results_match_standalone_and_arrival_order():
    srv, be, clock = _server()
    rng = np.random.default_rng(0)
    xs = [rng.normal(size=(n, 2)) * 6 for n in (5, 300, 17, 2, 900)]
    reqs = [srv.submit_assign("m", x) for x in xs]
    _drain(srv, clock)
    for r, x in zip(reqs, xs):
        assert r.error is None
        np.testing.assert_array_equal(r.result, srv.models["m"].labels(x))
        assert r.admitted >= r.arrival and r.finished >= r.admitted
    # admission follows arrival order
    adm = [r.admitted for r in reqs]
    assert adm == sorted(adm)


def test_small_requests_are_coalesced_up_to_the_row_cap():
    srv, be, clock = _server(batch_max_rows=100, batch_small_rows=50)
    xs = [np.full((n, 2), 1.0) for n in (10, 20, 30, 40, 60, 5)]
    reqs = [srv.submit_assign("m", x) for x in xs]
    srv.poll()
    sizes = [l[1] for l in be.launches if l[0] == "assign"]
    assert sizes[0] == [10, 20, 30, 40]          # 100 rows, then the cap stops the group
    _drain(srv, clock)
    assert all(r.done and r.error is None for r in reqs)
    total = sum(len(l[1]) for l in be.launches if l[0] == "assign")
    assert total == len(xs)


def test_budget_is_never_exceeded_and_slots_are_respected():
    srv, be, clock = _server(budget=3000, slots=2)
    xs = [np.zeros((200, 2)) for _ in range(12)]
    reqs = [srv.submit_assign("m", x) for x in xs]
    for _ in range(200):
        srv.poll()
        assert srv.in_use <= srv.budget
        assert sum(1 for t in srv.running if t[0] == "assign") <= 2
        if srv.idle:
            break
        clock.t += 0.25
    assert srv.idle and srv.peak_in_use <= 3000
    assert all(r.done and r.error is None for r in reqs)


def test_request_larger_than_the_budget_fails_alone():
    srv, be, clock = _server(budget=1000)
    big = srv.submit_assign("m", np.zeros((500, 2)))
    ok = srv.submit_assign("m", np.zeros((10, 2)))
    _drain(srv, clock)
    assert isinstance(big.error, MemoryError) and big.result is None
    assert ok.error is None and ok.result.shape == (10,)


def test_fit_registers_a_model_and_overlaps_with_assigns():
    srv, be, clock = _server(budget=100_000)
    X = np.arange(40, dtype=np.float64).reshape(20, 2)
    f = srv.submit_fit(X, register_as="new", C=3)
    a = srv.submit_assign("m", np.zeros((4, 2)))
    srv.poll()
    kinds = [t[0] for t in srv.running]
    assert kinds.count("fit") == 1 and kinds.count("assign") == 1   # both on the device at once
    _drain(srv, clock)
    assert f.error is None and "new" in srv.models
    b = srv.submit_assign("new", X[:3])
    _drain(srv, clock)
    np.testing.assert_array_equal(b.result, [0, 1, 2])
    assert a.latency == pytest.approx(1.0, abs=0.5)


def test_unknown_model_is_rejected_at_submission():
    srv, _, _ = _server()
    with pytest.raises(KeyError):
        srv.submit_assign("nope", np.zeros((1, 2)))


def test_a_waiting_fit_does_not_hold_back_assigns():
    srv, be, clock = _server(budget=100_000, fits=1)
    X = np.arange(40, dtype=np.float64).reshape(20, 2)
    f1 = srv.submit_fit(X, C=2)
    f2 = srv.submit_fit(X, C=2)          # waits for the single fit worker
    a = srv.submit_assign("m", np.zeros((4, 2)))
    srv.poll()
    assert f1.admitted is not None and f2.admitted is None
    assert a.admitted is not None
    _drain(srv, clock)
    assert f2.done and f2.admitted >= f1.finished
