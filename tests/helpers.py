"""Shared test helpers: build the same seeded problem for the oracle and the HIP path.

The oracle and the library canonicalise the same media arrays independently.
"""
import numpy as np

from oracle import canon, operators

try:
    import torch
except Exception:  # pragma: no cover
    torch = None


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def oracle_helmholtz(prob, bias="complex", given=None):
    cp = canon.canonical_helmholtz(prob.k2, prob.source, prob.spacing, bias=bias, given=given)
    return cp, operators.Operator(cp)


def gpu_helmholtz(prob, dtype, bias="complex", given=None, refine=False):
    from paper_2207_14222_amd import solver
    tdt = torch.complex64 if dtype == "c64" else torch.complex128
    can = solver.canonical_helmholtz(prob.k2, prob.source, prob.spacing, bias=bias, given=given, dtype=tdt)
    op = solver.Operator(can.symbol, can.B, refine=refine)
    return can, op


def to_np(t):
    return t.detach().cpu().numpy().astype(np.complex128)
