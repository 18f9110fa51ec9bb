"""Oracle gradients of L = sum_j Re<eta_j, x_j>, x_j = A^{-1} b_j, A = D^H D.

Test infrastructure only (see ``oracle/__init__.py``).

Not part of the paper's method: the differentiable solve wraps the seeded
solver so that the adjoint systems A lambda_j = eta_j are extra right-hand
sides.  With <a, b> = a^H b and the complex-gradient convention
grad = dL/dRe + i dL/dIm:

    dL/db_j   = lambda_j = A^{-1} eta_j              (A is Hermitian)
    dL/dkappa = sum_j Re[(H lambda_j)^H D x_j + (D lambda_j)^H H x_j]

since D = 1 - kappa H gives dA/dkappa = -(H^H D + D^H H).

Parity pins (tests/test_oracle_grad.py): exact linearity of L in b (the
central difference along any direction equals Re<lambda, u> with no truncation
error), central finite differences in kappa on a tiny lattice solved densely.
"""
import numpy as np

from .cg import cg
from .operators import WilsonNormalOp, wilson_dense


def loss(X, Eta):
    return float(sum(np.vdot(Eta[:, j], X[:, j]).real for j in range(X.shape[1])))


def solve_dense(U, kappa, B, antiperiodic=True):
    d = wilson_dense(U, kappa, antiperiodic)
    a = d.conj().T @ d
    return np.linalg.solve(a, B)


def grads(U, kappa, B, Eta, antiperiodic=True, tol=1e-13, dense=False):
    """Returns (L, X, dL/dB, dL/dkappa) with tight solves (dense when ``dense``)."""
    op = WilsonNormalOp(U, kappa, antiperiodic)
    k = B.shape[1]
    if dense:
        X = solve_dense(U, kappa, B, antiperiodic)
        Lam = solve_dense(U, kappa, Eta, antiperiodic)
    else:
        X = np.stack([cg(op, B[:, j], tol=tol)[0] for j in range(k)], axis=1)
        Lam = np.stack([cg(op, Eta[:, j], tol=tol)[0] for j in range(k)], axis=1)
    gk = 0.0
    for j in range(k):
        gk += np.vdot(op.H(Lam[:, j]), op.D(X[:, j])).real
        gk += np.vdot(op.D(Lam[:, j]), op.H(X[:, j])).real
    return loss(X, Eta), X, Lam, float(gk)
