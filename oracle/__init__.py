"""FP64 CPU oracle for the universal split preconditioner (Vettenburg & Vellekoop,
arXiv 2207.14222).

TEST INFRASTRUCTURE ONLY.  Nothing in the library imports this package: only the
tests, the smoke check and the CPU-baseline leg of the benchmark call it.  It is
a plain, slow, obviously-correct NumPy implementation of what the GPU path
computes, written from the paper:

* ``canon``      -- conversion to canonical form (Sec. 2.2) and the Helmholtz,
                    diffusion and pantograph splittings (Sec. 3.1-3.3), including
                    the smallest-circle bias.
* ``operators``  -- the discrete operators L, V, B = I - V, A = L + V and the
                    Fourier inverse (L + I)^-1 (Eq. laplacian_inverse), plus
                    dense matrices for tiny grids.
* ``richardson`` -- Algorithm 1 (preconditioned fixed-point iteration with the
                    forward problem eliminated, Sec. 2.1) and the FP64 form of
                    outer iterative refinement.
* ``flux``       -- steady diffusion in flux form with a tensor diffusion
                    coefficient (Sec. 3.2): [u; J] system, 3 x 3 block symbol,
                    per-voxel blocks of V, equilibration and scaling.
* ``antisym``    -- the antisymmetrised canonical form for systems that are
                    not accretive (Sec. 2.2), built on a 1-D operator.
* ``krylov``     -- BiCGSTAB, restarted GMRES(m) and CG on the preconditioned
                    operator with the forward problem eliminated (the solver
                    comparison of Sec. 4, Table 1b).
* ``eigen``      -- lowest-energy Schrodinger eigenmodes with the shifted,
                    canonical operator (Sec. 4, Eq. schrodinger): dense
                    definition, energies, residuals, condition numbers.
* ``surrogate``  -- the learned initial guess's network, loss, input channels
                    and Adam in plain PyTorch CPU float64.
* ``theory``     -- dense-matrix quantities of the appendix theorems
                    (Lemma 2, Theorem 2, Corollary 1, condition number and rate
                    bounds) used as invariants.

Every floating-point quantity is complex128/float64.  FFTs are numpy.fft
(pocketfft), pinned against a naive DFT in the tests.  The oracle shares no
code with the HIP path; the only shared module is the seeded input generator
``paper_2207_14222_amd.media``, which holds none of the method's arithmetic and
is not imported here (inputs arrive as arrays).

Parity status: every function here is pinned by a CPU test (see
``tests/test_oracle_*.py``) except where its docstring says "parity unpinned".
"""
