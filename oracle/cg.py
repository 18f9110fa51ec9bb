"""Oracle conjugate gradient (Hestenes-Stiefel), FP64 / complex128.

Test infrastructure only (see ``oracle/__init__.py``).

Section 2.2: after seeding, every right-hand side other than the first is
finished with plain CG started from its projected guess.  Conventions:
  * relative residual is ||b - A x|| / ||b|| against the original b;
  * CG stops on the recursively updated residual; the true residual is then
    recomputed and, if it is still above tol, CG restarts from r = b - A x
    (the restart's A-apply is not counted as an iteration);
  * one iteration is one A-apply inside the loop (for A = D^H D that is two
    products with D, as counted in Section 4).

Parity pins (tests/test_oracle_cg.py): exact solution for diagonal A; finite
termination in k steps for k distinct eigenvalues; dense numpy.linalg.solve;
monotone A-norm error.
"""
import numpy as np


def _dot(a, b):
    return np.vdot(a, b)  # conj(a) . b


def cg(apply_a, b, x0=None, tol=1e-8, maxit=100000, max_restarts=5, history=None):
    """Solve A x = b.  Returns (x, iterations, true relative residual).

    ``history`` (a list), when given, receives x after every iteration.
    """
    b = np.asarray(b)
    dtype = np.result_type(b.dtype, np.float64)
    x = np.zeros(b.shape, dtype=dtype) if x0 is None else np.array(x0, dtype=dtype)
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return np.zeros_like(x), 0, 0.0
    it = 0
    restarts = 0
    while True:
        r = b - apply_a(x)
        rho = _dot(r, r).real
        if np.sqrt(rho) <= tol * bnorm:
            break
        p = r.copy()
        while it < maxit:
            q = apply_a(p)
            alpha = rho / _dot(p, q).real
            x = x + alpha * p
            r = r - alpha * q
            rho_new = _dot(r, r).real
            it += 1
            if history is not None:
                history.append(x.copy())
            if np.sqrt(rho_new) <= tol * bnorm:
                break
            beta = rho_new / rho
            rho = rho_new
            p = r + beta * p
        true_rel = np.linalg.norm(b - apply_a(x)) / bnorm
        if true_rel <= tol or it >= maxit or restarts >= max_restarts:
            return x, it, float(true_rel)
        restarts += 1
    return x, it, float(np.linalg.norm(b - apply_a(x)) / bnorm)


def cg_multi(apply_a, B, X0=None, tol=1e-8, maxit=100000):
    """CG on each column of B independently.  Returns (X, iters[list], relres[list])."""
    B = np.asarray(B)
    k = B.shape[1]
    X = np.zeros(B.shape, dtype=np.result_type(B.dtype, np.float64))
    iters, rel = [], []
    for j in range(k):
        x0 = None if X0 is None else X0[:, j]
        x, it, rr = cg(apply_a, B[:, j], x0, tol, maxit)
        X[:, j] = x
        iters.append(it)
        rel.append(rr)
    return X, iters, rel
