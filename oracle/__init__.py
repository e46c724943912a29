"""CPU oracle for the ETD / embedded-boundary / level-set hot path.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously-correct
float64 implementation of what the GPU path computes, written from the paper
(Liu & Liu, "Integration factor combined with level set method for
reaction-diffusion systems with free boundary in high spatial dimensions",
arXiv 2209.15095).  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it.  The product path
(``paper_2209_15095_amd``) never imports, calls or links anything here, and
this package imports nothing from the product path except the seeded input
generators in ``paper_2209_15095_amd.inputs`` (which hold no arithmetic of
the method).

Modules
-------
phi          scalar phi_k, and three independent routes to sum_k phi_k(tA) b_k
geometry     node grid, point classification, interface crossings, closest points
operator     embedded-boundary matrix A (Cases 1-3 of Section 2) as scipy CSR
etd          ETD1 / ETD2RK (Section 3) built on exact phi-combinations
levelset     Aslam extrapolation, Stefan velocity + extension, HJ-WENO5
             advection, reinitialisation (Section 4.3 algorithm, Steps 1-2)
freeboundary one free-boundary step (Section 4.3 algorithm)
adjoint      discrete adjoint of ETD2RK on a frozen domain

Pinning status of every function is listed in the module docstrings; the
coupled free-boundary trajectory is "parity unpinned" beyond the invariants
tested in tests/test_oracle_levelset.py (see each function).
"""
