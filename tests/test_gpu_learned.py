"""Learned initial guess end to end on a small grid: solves used as training
targets converge, training lowers the loss, the solve started from the
learned x0 converges to the same solution as the solve from x0 = 0 (within
what the two stopping residuals allow), and a guess whose residual is not
below ||y|| is rejected so that the solve runs exactly as from x0 = 0."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _workload():
    from paper_2207_14222_amd import learned
    return learned.Workload((32, 32, 32), count=12, width=4, plane=6, w0=5.0)


def test_learned_pipeline_small_grid():
    _need_gpu()
    from paper_2207_14222_amd import learned, surrogate
    print("[gpu-case] learned pipeline 32^3", flush=True)
    wl = _workload()
    data = learned.make_dataset(wl, range(8))
    assert len(data) == 8
    net = surrogate.UNet3D(wl.shape, seed=3, scale=learned.target_scale(data))
    hist = learned.train(net, wl, data, epochs=6, lr=3e-3)
    assert all(np.isfinite(hist))
    assert np.mean(hist[-8:]) < 0.7 * np.mean(hist[:8])
    rows = learned.evaluate(net, wl, [100, 101], plain=True)
    for r in rows:
        assert r["converged"]
        # both solutions satisfy ||y - A x|| < 1e-6 ||y||
        assert r["diff"] < 1e-4, r
    s = learned.summarize(rows)
    assert s["media"] == 2 and s["all_converged"]


def test_rejected_guess_runs_as_zero_start():
    _need_gpu()
    from paper_2207_14222_amd import learned, surrogate
    print("[gpu-case] learned fallback 32^3", flush=True)
    wl = _workload()
    nre = next(wl.index_maps([7]))
    op, y = wl.operator(nre)
    r0 = wl.solve(op, y)
    net = surrogate.UNet3D(wl.shape, seed=4, scale=1e6)   # a guess far too large
    x0 = torch.empty_like(y)
    r1, rho0, used = learned.learned_solve(net, wl, op, y, nre, x0)
    assert rho0 >= 1.0 and not used
    assert r1.iterations == r0.iterations and torch.equal(r1.x, r0.x)
    op.close()


def test_judged_guess_plain_and_refined():
    """usp_solve with a judged guess: a good guess is kept (few iterations), a bad one is
    discarded and the solve equals the solve from zero bit for bit."""
    _need_gpu()
    from paper_2207_14222_amd import solver
    print("[gpu-case] judged guess 32^3 plain and refined", flush=True)
    wl = _workload()
    nre = next(wl.index_maps([5]))
    for refine in (False, True):
        op, y = wl.operator(nre, refine=refine)
        r0 = wl.solve(op, y)
        good = r0.x.clone()
        rg = op.solve(y, x=good, alpha=wl.alpha, tol=wl.tol, maxit=20000, check_every=wl.k, judge_guess=True)
        assert rg.converged and rg.iterations == 0 and rg.hist_true[0, 1] < wl.tol
        bad = (1e3 * torch.randn_like(y.real) + 0j).to(y.dtype).contiguous()
        rb = op.solve(y, x=bad, alpha=wl.alpha, tol=wl.tol, maxit=20000, check_every=wl.k, judge_guess=True)
        assert rb.hist_true[0, 1] >= 1.0
        assert rb.converged and rb.iterations == r0.iterations and torch.equal(rb.x, r0.x)
        op.close()
