"""Parity at the benchmark sizes, in the launch configuration bench.py times
(autotuned plans, refined complex64): K full iterations compared element by
element with the FP64 oracle's iterates, plus the solution against the
oracle's residual (a property that holds at any size); the batched workload
as bench.py runs it, with a sample of its solutions checked by the oracle's
residual."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from helpers import rel, to_np
from oracle import canon, operators, richardson as R
from paper_2207_14222_amd import media

pytestmark = pytest.mark.gpu


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def test_helmholtz_256cubed_iterates_and_solution():
    """256^3 spheres (seed 2): 3 complex64 iterations vs the oracle; refined solve's
    final x has oracle residual < 1e-6."""
    _need_gpu()
    from paper_2207_14222_amd import solver
    print("[gpu-case] 256^3 helmholtz full size", flush=True)
    p = media.helmholtz_spheres(shape=(256, 256, 256), seed=2)
    cp = canon.canonical_helmholtz(p.k2, p.source, p.spacing)
    op_o = operators.Operator(cp)
    K = 3
    xo, ho = R.iterate(op_o, cp.y, 0.8, K)
    can64 = solver.canonical_helmholtz(p.k2, p.source, p.spacing, dtype=torch.complex64)
    op64 = solver.Operator(can64.symbol, can64.B)
    xt = torch.zeros_like(can64.y)
    op64.autotune(can64.y, xt, alpha=0.8, reps=2)
    x, h = op64.iterate(can64.y, alpha=0.8, K=K)
    assert rel(to_np(x), xo) < 3e-5
    np.testing.assert_allclose(np.sqrt(h), ho, rtol=1e-4)
    del op64, can64, x
    can = solver.canonical_helmholtz(p.k2, p.source, p.spacing, dtype=torch.complex128)
    op = solver.Operator(can.symbol, can.B, refine=True)
    res = op.solve(can.y, alpha=0.8, tol=1e-6, maxit=2000, check_every=20)
    assert res.converged
    xs = to_np(res.x)
    assert R.relative_residual(op_o, xs, cp.y) < 1e-6


def test_diffusion_full_size_iterates():
    """256 x 256 x 128 frequency-domain diffusion (seed 3): complex64 iterates vs the oracle."""
    _need_gpu()
    from paper_2207_14222_amd import solver
    print("[gpu-case] diffusion 128x256x256 full size", flush=True)
    d = media.diffusion_blobs(seed=3)
    cp = canon.canonical_diffusion(d.mu_a, d.D, d.omega_over_v, d.source, d.spacing)
    op_o = operators.Operator(cp)
    xo, _ = R.iterate(op_o, cp.y, 1.0, 3)
    can = solver.canonical_diffusion(d.mu_a, d.D, d.omega_over_v, d.source, d.spacing, dtype=torch.complex64)
    op = solver.Operator(can.symbol, can.B)
    x, _ = op.iterate(can.y, alpha=1.0, K=3)
    assert rel(to_np(x), xo) < 3e-5


def test_batch_largest_size_iterates():
    """1024^2 disks (largest batched size): complex64 iterates vs the oracle."""
    _need_gpu()
    from paper_2207_14222_amd import solver
    print("[gpu-case] 1024^2 disks", flush=True)
    p = media.helmholtz_disks(n=1024, seed=4000)
    cp = canon.canonical_helmholtz(p.k2, p.source, p.spacing)
    op_o = operators.Operator(cp)
    xo, _ = R.iterate(op_o, cp.y, 0.8, 5)
    can = solver.canonical_helmholtz(p.k2, p.source, p.spacing, dtype=torch.complex64)
    op = solver.Operator(can.symbol, can.B)
    x, _ = op.iterate(can.y, alpha=0.8, K=5)
    assert rel(to_np(x), xo) < 3e-5


def test_batched_workload_solutions_by_oracle_residual():
    """The batched workload as bench.py runs it (96 problems, sides from
    {128, 256, 512, 1024} drawn with seed 4, disks with seeds 4000 + i; grouped
    schedule with the streamed fused-pass plan, refinement interval 150 with
    the final cycle predicted per problem, alpha 0.9, tol 1e-6): every problem
    converges, and for three problems of each size the solution's residual
    recomputed by the oracle is below 1e-6."""
    _need_gpu()
    from paper_2207_14222_amd import solver
    print("[gpu-case] batched workload 96 problems", flush=True)
    sizes = media.batch_sizes(96, seed=4)
    probs, cans, ops = [], [], []
    for i, n in enumerate(sizes):
        p = media.helmholtz_disks(n=n, seed=4000 + i)
        probs.append(p)
        cans.append(solver.canonical_helmholtz(p.k2, p.source, p.spacing, dtype=torch.complex128))
        ops.append(solver.Operator(cans[-1].symbol, cans[-1].B, refine=True))
    xs = [torch.zeros_like(c.y) for c in cans]
    b = solver.Batch(ops, [c.y for c in cans], xs, alpha=0.9, tol=1e-6, maxit=20000)
    out = b.solve(refine_every=150, use_graph=True, variant=2)
    assert out.worst == 0, out.status
    assert max(out.rho) < 1e-6
    for n in (128, 256, 512, 1024):
        for i in [j for j, m in enumerate(sizes) if m == n][:3]:
            p = probs[i]
            cp = canon.canonical_helmholtz(p.k2, p.source, p.spacing)
            rho = R.relative_residual(operators.Operator(cp), to_np(xs[i]), cp.y)
            assert rho < 1e-6, (i, n, rho)
            assert abs(rho - out.rho[i]) < 1e-9, (i, n, rho, out.rho[i])
