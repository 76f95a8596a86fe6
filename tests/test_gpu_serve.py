"""Serving loop on the device: every request's result is the same alone and in the mix.

Assign requests of uneven sizes (coalesced when small) run on several streams while a fit job runs
on its own stream and thread; each assign result must equal a standalone kkm_assign of the same
rows bit for bit, and the fitted model must equal a standalone fit of the same job."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def setup():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import kkm_inputs as ki
    import paper_1710_03013_amd as kk
    X, _ = ki.datasets.gaussian_mixture(60_000, 64, 100, seed=1003, sigma=None)
    Xd = torch.from_numpy(X).cuda()
    model, _, _ = kk.kkm_fit(Xd[:20_000], "rbf", sigma=8.0, C=50, B=2, s=0.05, max_iter=20, seed=11)
    return kk, Xd, model


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_results_same_alone_and_in_the_mix(setup, precision):
    kk, Xd, model = setup
    from paper_1710_03013_amd.serve import KkmBackend, Server
    rng = np.random.default_rng(5)
    sizes = [1, 3, 17, 100, 255, 4096, 5000, 31, 2, 12_000, 64, 7]
    starts = [int(rng.integers(0, Xd.shape[0] - n)) for n in sizes]
    xs = [Xd[s:s + n] for s, n in zip(starts, sizes)]
    alone = [kk.kkm_assign(model, x, precision=precision).cpu().numpy() for x in xs]
    fit_kw = dict(kernel="rbf", sigma=8.0, C=10, B=3, s=0.05, max_iter=20, seed=23, precision=precision)
    Xf = Xd[20_000:50_000]
    ref_model, _, _ = kk.kkm_fit(Xf, **fit_kw)
    ref = kk.kkm_model_export(ref_model)
    torch.cuda.synchronize()

    srv = Server(KkmBackend(n_streams=3, precision=precision), budget_bytes=8 << 30, assign_slots=3,
                 fit_workers=1, batch_small_rows=4096)
    srv.add_model("m", model)
    reqs = []
    # a burst: everything queued before the first poll, the fit job in the middle
    for i, x in enumerate(xs):
        reqs.append(srv.submit_assign("m", x))
        if i == 4:
            fit_req = srv.submit_fit(Xf, register_as="fitted", **fit_kw)
    srv.run_until_idle(timeout=120)
    assert srv.peak_in_use <= srv.budget
    assert srv.launches < len(xs) + 1, "small requests were expected to be coalesced"
    for r, a in zip(reqs, alone):
        assert r.error is None
        np.testing.assert_array_equal(r.result.cpu().numpy(), a)
    assert fit_req.error is None
    got = kk.kkm_model_export(srv.models["fitted"])
    for key in ("medoid_index", "counts"):
        np.testing.assert_array_equal(got[key], ref[key])
    np.testing.assert_array_equal(got["support"], ref["support"])


def test_rows_written_on_the_submitting_stream(setup):
    """Rows produced by a kernel on the submitter's stream right before submission, with no host
    synchronisation: the server's streams must wait for them (a long matrix product runs first, and
    the rows are written after it)."""
    kk, Xd, model = setup
    from paper_1710_03013_amd.serve import KkmBackend, Server
    sizes, starts = [5000, 300, 20_000, 64], [100, 7000, 30_000, 55_000]
    alone = [kk.kkm_assign(model, Xd[s:s + n]).cpu().numpy() for s, n in zip(starts, sizes)]
    torch.cuda.synchronize()
    srv = Server(KkmBackend(n_streams=2), budget_bytes=8 << 30, assign_slots=2, fit_workers=1)
    srv.add_model("m", model)
    a = torch.randn(4096, 4096, device="cuda") / 64.0
    reqs = []
    for s, n in zip(starts, sizes):
        busy = a
        for _ in range(6):
            busy = busy @ a
        y = torch.empty_like(Xd[s:s + n])
        torch.add(Xd[s:s + n], busy[0, 0], alpha=0.0, out=y)   # written only after the products
        reqs.append(srv.submit_assign("m", y))
        del y, busy
    srv.run_until_idle(timeout=120)
    for r, want in zip(reqs, alone):
        assert r.error is None
        np.testing.assert_array_equal(r.result.cpu().numpy(), want)
