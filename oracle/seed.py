"""Oracle for the seed phase: Lanczos version of single seed CG with periodic
reorthogonalization (Section 3, algorithm steps 1-9), and the Galerkin
projection of the other right-hand sides over the stored Lanczos basis.

Test infrastructure only (see ``oracle/__init__.py``).

Readings of points the paper leaves open:
  R1  v_2 is f / beta_1 after step 2; step 8 never runs at i = 1.
  R2  alpha_i = Re(v_i^H f): T is real symmetric tridiagonal for Hermitian A.
  R3  steps 5-7 use v_i as it was before step 8; step 8 then overwrites the
      stored v_i, which later steps (and the projection) use.
  R4  alpha and beta keep their recurrence values after reorthogonalization.
  R5  one pass of classical Gram-Schmidt: the coefficients of v_i and of f on
      v_1..v_{i-1} are formed first and subtracted, v_i is renormalised, and
      then the component of f along the new v_i is removed.
  R6  step 8 runs when i is a multiple of the frequency (i >= 2, i = m
      included); frequency 1 is full reorthogonalization, 0 is none.
  R7  breakdown when beta_i <= 1e-12 * max_k |alpha_k| (a roundoff-level norm
      for an invariant Krylov space): stop with m_done = i.
      A non-positive pivot delta_i means A is not positive definite.
  R8  exactly m steps are run (past convergence, Section 3); beta_m and
      v_{m+1} are formed but the projection uses T_m and V_m only.
  R9  the canonical seeded guess is the Galerkin projection over the stored
      basis, X0 + V_m T_m^{-1} V_m^H R0; the incremental w_i / eta recurrences
      of steps 3-7 give the same vectors up to loss of orthogonality.

Parity pins (tests/test_oracle_seed.py, tests/test_oracle_paper.py): basis
orthogonality with full reorthogonalization; the three-term Lanczos relation;
Ritz values against closed-form and dense eigenvalues; equality of the
Lanczos x^1 iterates with plain CG iterates; Galerkin optimality against a
dense solve; agreement of the incremental and batched projections; the LU
solve of T against scipy.linalg.solve_banded; the character of Table 3.1.
"""
from dataclasses import dataclass, field

import numpy as np


BREAKDOWN_TOL = 1e-12   # reading R7


def _dot(a, b):
    return np.vdot(a, b)


@dataclass
class SeedResult:
    V: np.ndarray            # n x (m_done + 1): v_1 .. v_{m_done+1}, post-reorthogonalization
    alpha: np.ndarray        # alpha_1 .. alpha_{m_done}
    beta: np.ndarray         # beta_0 .. beta_{m_done}
    X: np.ndarray            # incremental approximations x^j for every right-hand side
    m_done: int
    status: str = "ok"       # "ok" | "breakdown" | "not_pd"
    delta: np.ndarray = field(default=None)   # LU pivots delta_1 .. delta_{m_done}
    x1_history: list = field(default=None)    # x^1 after each step (when requested)


def _reorthogonalize(V, i, f):
    """Step 8 at step i (1-based): V[:, :i] holds v_1..v_i (v_i = V[:, i-1]).

    Classical Gram-Schmidt, one pass (reading R5).
    """
    prev = V[:, : i - 1]
    vi = V[:, i - 1]
    c_v = prev.conj().T @ vi
    c_f = prev.conj().T @ f
    vi = vi - prev @ c_v
    vi = vi / np.linalg.norm(vi)
    f = f - prev @ c_f
    f = f - vi * _dot(vi, f)
    V[:, i - 1] = vi
    return f


def seed_lanczos(apply_a, B, X0=None, m=100, freq=0, record_x1=False, callback=None):
    """Run the seed algorithm on right-hand side 1, seeding columns 2..nrhs of B.

    Follows the algorithm's steps 1-9 with the readings in the module header.
    ``callback(i, X)``, when given, sees the incremental approximations after
    step 7 of every step i (after step 4 for i = 1).  Returns a SeedResult.
    """
    B = np.asarray(B)
    if B.ndim == 1:
        B = B[:, None]
    n, nrhs = B.shape
    dtype = np.result_type(B.dtype, np.float64)
    X = np.zeros((n, nrhs), dtype=dtype) if X0 is None else np.array(X0, dtype=dtype)
    # step 1: initial residuals
    R0 = B - apply_a(X) if np.any(X) else B.astype(dtype).copy()

    V = np.zeros((n, m + 1), dtype=dtype)
    alpha = np.zeros(m)
    beta = np.zeros(m + 1)
    delta = np.zeros(m)
    hist = [] if record_x1 else None

    # step 2: first Lanczos iteration
    beta[0] = np.linalg.norm(R0[:, 0])
    V[:, 0] = R0[:, 0] / beta[0]
    f = apply_a(V[:, 0])
    alpha[0] = _dot(V[:, 0], f).real
    f = f - alpha[0] * V[:, 0]
    beta[1] = np.linalg.norm(f)
    # step 3: linear equations for the first iteration
    delta[0] = alpha[0]
    if delta[0] <= 0.0:
        return SeedResult(V[:, :1], alpha[:1], beta[:1], X, 0, "not_pd", delta[:1], hist)
    w = V[:, 0] / delta[0]
    zeta = beta[0]
    X[:, 0] = X[:, 0] + zeta * w
    # step 4: the other right-hand sides
    eta = np.array([_dot(V[:, 0], R0[:, j]) for j in range(1, nrhs)], dtype=dtype)
    for j in range(1, nrhs):
        X[:, j] = X[:, j] + eta[j - 1] * w
    if hist is not None:
        hist.append(X[:, 0].copy())
    if callback is not None:
        callback(1, X)

    amax = abs(alpha[0])
    if beta[1] <= BREAKDOWN_TOL * amax or m == 1:
        V[:, 1] = f / beta[1] if beta[1] > 0 else 0.0
        status = "breakdown" if beta[1] <= BREAKDOWN_TOL * amax else "ok"
        return SeedResult(V[:, :2], alpha[:1], beta[:2], X, 1, status, delta[:1], hist)
    V[:, 1] = f / beta[1]   # reading R1

    for i in range(2, m + 1):
        vi = V[:, i - 1].copy()        # v_i as used by steps 5-7 (reading R3)
        # step 5: Lanczos iteration
        f = apply_a(vi) - beta[i - 1] * V[:, i - 2]
        alpha[i - 1] = _dot(vi, f).real
        f = f - alpha[i - 1] * vi
        # step 6: linear equations
        gamma = beta[i - 1] / delta[i - 2]
        delta[i - 1] = alpha[i - 1] - gamma * beta[i - 1]
        if delta[i - 1] <= 0.0:
            return SeedResult(V[:, :i], alpha[:i], beta[:i], X, i - 1, "not_pd", delta[:i], hist)
        w = (vi - beta[i - 1] * w) / delta[i - 1]
        zeta = -gamma * zeta
        X[:, 0] = X[:, 0] + zeta * w
        # step 7: other right-hand sides
        for j in range(1, nrhs):
            eta[j - 1] = _dot(vi, R0[:, j]) - gamma * eta[j - 1]
            X[:, j] = X[:, j] + eta[j - 1] * w
        if hist is not None:
            hist.append(X[:, 0].copy())
        if callback is not None:
            callback(i, X)
        # step 8: periodic reorthogonalization (readings R5, R6)
        if freq > 0 and i % freq == 0:
            f = _reorthogonalize(V, i, f)
        # step 9: finish the iteration
        beta[i] = np.linalg.norm(f)
        amax = max(amax, abs(alpha[i - 1]))
        if beta[i] <= BREAKDOWN_TOL * amax:   # reading R7
            V[:, i] = 0.0
            return SeedResult(V[:, : i + 1], alpha[:i], beta[: i + 1], X, i, "breakdown", delta[:i], hist)
        V[:, i] = f / beta[i]
    return SeedResult(V, alpha, beta, X, m, "ok", delta, hist)


# ----------------------------------------------------------------------------
# Lanczos tridiagonal T and its LU solve
# ----------------------------------------------------------------------------
def tridiag_dense(alpha, beta, m):
    """T_m: diagonal alpha_1..alpha_m, off-diagonal beta_1..beta_{m-1} (beta[0] = beta_0 unused)."""
    t = np.diag(np.asarray(alpha[:m], dtype=np.float64))
    off = np.asarray(beta[1:m], dtype=np.float64)
    t += np.diag(off, 1) + np.diag(off, -1)
    return t


def tridiag_lu_solve(alpha, beta, m, G):
    """Solve T_m Y = G with the LU factorization the seed algorithm uses (step 6).

    T = L U, L unit lower bidiagonal with multipliers gamma_{i-1} = beta_{i-1} / delta_{i-1},
    U upper bidiagonal with pivots delta_i = alpha_i - gamma_{i-1} beta_{i-1} and
    superdiagonal beta_i.  No pivoting: T is positive definite for HPD A.
    """
    G = np.asarray(G)
    squeeze = G.ndim == 1
    if squeeze:
        G = G[:, None]
    Y = np.zeros(G.shape, dtype=np.result_type(G.dtype, np.float64))
    delta = np.zeros(m)
    gamma = np.zeros(m)
    delta[0] = alpha[0]
    for i in range(1, m):
        gamma[i] = beta[i] / delta[i - 1]
        delta[i] = alpha[i] - gamma[i] * beta[i]
    # forward: L z = G
    Y[0] = G[0]
    for i in range(1, m):
        Y[i] = G[i] - gamma[i] * Y[i - 1]
    # backward: U y = z
    Y[m - 1] = Y[m - 1] / delta[m - 1]
    for i in range(m - 2, -1, -1):
        Y[i] = (Y[i] - beta[i + 1] * Y[i + 1]) / delta[i]
    return Y[:, 0] if squeeze else Y


def project(V, alpha, beta, m, R0, X0=None):
    """Batched Galerkin projection over the stored basis: X0 + V_m T_m^{-1} V_m^H R0 (reading R9)."""
    R0 = np.asarray(R0)
    Vm = V[:, :m]
    G = Vm.conj().T @ R0
    Y = tridiag_lu_solve(alpha, beta, m, G)
    X = Vm @ Y
    if X0 is not None:
        X = X + X0
    return X


def seed_x1(V, alpha, beta, m, x0=None):
    """Lanczos-CG approximation of right-hand side 1 after m steps: x0 + V_m T_m^{-1} (beta_0 e_1)."""
    e = np.zeros(m)
    e[0] = beta[0]
    y = tridiag_lu_solve(alpha, beta, m, e)
    x = V[:, :m] @ y
    if x0 is not None:
        x = x + x0
    return x
