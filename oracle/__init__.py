"""Plain FP64 CPU oracle for the single-seed Lanczos-CG method.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this package:
only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import, call or execute anything under ``oracle/``.  It shares
no code with the HIP library (no kernels, headers, tables or helpers); inputs
come from the seeded generators in ``paper_0810_0330_amd/synth.py``, which hold
none of the method's arithmetic.

Every function is written in plain NumPy/SciPy, complex128 or float64, with
explicit Python loops over the method's steps, so that it can be read against
the paper (Abdel-Rehim, Morgan, Wilcox, "Improved seed methods for symmetric
positive definite linear equations with multiple right-hand sides").

Modules
-------
operators  -- the A-apply: 2D Laplacian, Wilson-Dirac D, D^H, D^H D, diagonal,
              and pure-Python dense builders for tiny lattices (pins only).
cg         -- plain conjugate gradient (Hestenes-Stiefel), the seeded-system
              solver of Section 2.2.
seed       -- the Lanczos version of single seed CG with periodic
              reorthogonalization (Section 3, algorithm steps 1-9), the
              batched Galerkin projection over the stored basis, and the LU
              solve of the Lanczos tridiagonal matrix.
seeded     -- the whole single-seed driver (seed, project, CG), the related
              right-hand-side variant of Section 2.3, and the multiple-seeding
              comparator of Section 2.1.
mixed      -- the mixed-precision path emulated in NumPy: CG with float32 /
              complex64 vectors and operator and FP64 reliable updates, and
              the seed phase with a single-precision basis and FP64 scalars.
grad       -- gradients of L = sum_j Re<eta_j, x_j> with respect to b and kappa.
indefinite -- the indefinite variant: gamma_5 D, the Lanczos seed without LU,
              minimum-residual guesses through the (m+1) x m tridiagonal matrix,
              and MINRES to finish each system.

Parity status of each function is stated in its module header.
"""
