"""Batched solve of many uneven-size 2-D problems (grouped graph-captured
launches and the one-launch persistent schedule) against the single-problem
refined solve and the FP64 oracle: both schedules give the same iteration
counts and solutions, every fused-pass plan and graph replay reproduces the
eager launch bit for bit, and 1024^2 problems (column-tiled spectrum) match
the single-problem solve."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from helpers import oracle_helmholtz, rel, to_np
from oracle import richardson as R
from paper_2207_14222_amd import media

pytestmark = pytest.mark.gpu


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _problems(sizes, seed0=4000):
    from paper_2207_14222_amd import solver
    probs, cans, ops = [], [], []
    for i, n in enumerate(sizes):
        p = media.helmholtz_disks(n=n, seed=seed0 + i, width=max(2, n // 16), w0=max(2.0, n / 16), row=min(20, n // 4))
        can = solver.canonical_helmholtz(p.k2, p.source, p.spacing, dtype=torch.complex128)
        probs.append(p)
        cans.append(can)
        ops.append(solver.Operator(can.symbol, can.B, refine=True))
    return probs, cans, ops


def test_batched_equals_single_problem_solves():
    _need_gpu()
    from paper_2207_14222_amd import solver
    sizes = [16, 64, 32, 128, 8, 64, 256]
    print(f"[gpu-case] batch sizes {sizes}", flush=True)
    probs, cans, ops = _problems(sizes)
    xs = [torch.zeros_like(c.y) for c in cans]
    b = solver.Batch(ops, [c.y for c in cans], xs, alpha=0.8, tol=1e-10, maxit=4000)
    out = b.solve(refine_every=20, use_graph=True, variant=0)
    assert out.worst == 0, out.status
    xg = [x.clone() for x in xs]
    outp = b.solve(refine_every=20, use_graph=True, variant=4)
    assert outp.worst == 0, outp.status
    assert outp.iterations == out.iterations
    for a, r in zip(xs, xg):
        assert rel(to_np(a), to_np(r)) < 1e-9
    for i, (p, can, op) in enumerate(zip(probs, cans, ops)):
        single = op.solve(can.y, alpha=0.8, tol=1e-10, maxit=4000, check_every=20)
        assert single.converged
        assert abs(out.iterations[i] - single.iterations) <= 20
        # same passes; only the compiler's multiply-add contraction may differ
        # between the two kernels, so agreement is to rounding, not bitwise
        assert rel(to_np(xs[i]), to_np(single.x)) < 1e-9, i
        cp, op_o = oracle_helmholtz(p)
        ref = R.solve(op_o, cp.y, 0.8, 1e-12, 8000, 20)
        assert rel(to_np(xs[i]), ref.x) < 1e-6
        assert out.rho[i] < 1e-10 and out.t_done_ms[i] > 0


def test_batched_variants_and_graph_replays_identical():
    _need_gpu()
    from paper_2207_14222_amd import solver
    sizes = [32, 128, 64, 16]
    print(f"[gpu-case] batch variants {sizes}", flush=True)
    probs, cans, ops = _problems(sizes, seed0=4100)
    xs = [torch.zeros_like(c.y) for c in cans]
    b = solver.Batch(ops, [c.y for c in cans], xs, alpha=0.8, tol=1e-8, maxit=3000)
    ref = b.solve(use_graph=False, variant=0)
    xref = [x.clone() for x in xs]
    for v in (0, 1, 2, 3, 4, 7, 8, 11):
        outs = []
        for graph in (False, True, True):
            for x in xs:
                x.fill_(7.0)   # eager work between runs; the solve starts from zero
            torch.cuda.synchronize()
            out = b.solve(use_graph=graph, variant=v)
            outs.append((out.iterations, [x.clone() for x in xs]))
        # graph replays reproduce the eager launch exactly
        for it, xv in outs[1:]:
            assert it == outs[0][0]
            for a, r in zip(xv, outs[0][1]):
                assert torch.equal(a, r)
        for a, r in zip(outs[0][1], xref):
            assert rel(to_np(a), to_np(r)) < 1e-9
    best = b.autotune(refine_every=20)
    assert 0 <= best <= 11


def test_batched_1024_column_tiles_equal_single_solve():
    """The grouped schedule keeps the complex64 spectrum of 1024^2 problems in
    column tiles (a layout of its own, 8 or 4 columns wide); the solution must
    match the single-problem refined solve (row-major spectrum), with every
    fused-pass plan and both column-tile widths, and graph replays must
    reproduce the eager launch bit for bit."""
    _need_gpu()
    from paper_2207_14222_amd import solver
    sizes = [1024, 64, 512]
    print(f"[gpu-case] batch column tiles {sizes}", flush=True)
    probs, cans, ops = _problems(sizes, seed0=4200)
    xs = [torch.zeros_like(c.y) for c in cans]
    b = solver.Batch(ops, [c.y for c in cans], xs, alpha=0.9, tol=1e-10, maxit=8000)
    out = b.solve(refine_every=60, use_graph=False, variant=0)
    assert out.worst == 0, out.status
    xref = [x.clone() for x in xs]
    for i, (can, op) in enumerate(zip(cans, ops)):
        single = op.solve(can.y, alpha=0.9, tol=1e-10, maxit=8000, check_every=60)
        assert single.converged
        assert abs(out.iterations[i] - single.iterations) <= 60
        assert rel(to_np(xs[i]), to_np(single.x)) < 1e-8, i
        assert out.rho[i] < 1e-10
    for v in (1, 2, 3, 8, 9, 10, 11):
        runs = []
        for graph in (False, True, True):
            for x in xs:
                x.fill_(3.0)
            torch.cuda.synchronize()
            o = b.solve(refine_every=60, use_graph=graph, variant=v)
            assert o.worst == 0, o.status
            runs.append((o.iterations, [x.clone() for x in xs]))
        for it, xv in runs[1:]:
            assert it == runs[0][0]
            for a, r in zip(xv, runs[0][1]):
                assert torch.equal(a, r)
        for a, r in zip(runs[0][1], xref):
            assert rel(to_np(a), to_np(r)) < 1e-9


def test_batch_rejects_fields_that_do_not_fit_the_operators():
    """Batch checks dtype, shape, contiguity and device of every y and x before the
    library sees a pointer (the kernels would read n^2 complex128 values)."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2207_14222_amd import media, solver
    p = media.helmholtz_disks(n=128, seed=4000)
    can = solver.canonical_helmholtz(p.k2, p.source, p.spacing, dtype=torch.complex128)
    op = solver.Operator(can.symbol, can.B, refine=True)
    good = torch.zeros_like(can.y)
    for bad in (good.to(torch.complex64), torch.zeros((128, 64), dtype=torch.complex128, device="cuda"),
                torch.zeros((128, 256), dtype=torch.complex128, device="cuda")[:, ::2], good.cpu()):
        with pytest.raises(ValueError):
            solver.Batch([op], [can.y], [bad])
        with pytest.raises(ValueError):
            solver.Batch([op], [bad], [good])
    plain = solver.Operator(can.symbol, can.B)
    with pytest.raises(ValueError):
        solver.Batch([plain], [can.y], [good])
