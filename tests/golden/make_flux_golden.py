"""Writes flux_ring256.json: iteration counts of the FP64 oracle (Algorithm 1 on
the flux-form diffusion system of Sec. 3.2) on the 256 x 256 anisotropic ring
medium.  Calls only the oracle and the seeded input generators.

    PYTHONPATH=. python tests/golden/make_flux_golden.py
"""
import json
import os

from oracle import flux as F
from oracle import richardson as R
from paper_2207_14222_amd import media

HERE = os.path.dirname(os.path.abspath(__file__))


def main():
    p = media.diffusion_ring(n=256)
    cp = F.canonical_flux(p.mu, p.D, p.source, p.h)
    op = F.FluxOperator(cp)
    out = {"medium": "media.diffusion_ring(n=256)", "c": cp.c, "s": cp.s.tolist(), "runs": []}
    for alpha, tol in ((1.0, 1e-3), (1.0, 1e-6)):
        r = R.solve(op, cp.y, alpha, tol, 20000, 10)
        out["runs"].append({"alpha": alpha, "tol": tol, "check_every": 10, "iterations": len(r.hist_pre),
                            "converged": bool(r.converged), "rho": r.hist_true[-1][1],
                            "delta0": float(r.hist_pre[0]), "delta_last": float(r.hist_pre[-1])})
        print(out["runs"][-1], flush=True)
    with open(os.path.join(HERE, "flux_ring256.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
