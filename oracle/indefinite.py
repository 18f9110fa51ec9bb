"""Oracle for the indefinite variant of the seed method: the gamma_5 D operator
(Section 4 names it as the alternative to A^H A) with a QR factorization of
the Lanczos tridiagonal matrix in place of its LU (Section 3 names QR or LQ
for indefinite systems), and MINRES to finish each system.

Test infrastructure only (see ``oracle/__init__.py``).

The paper gives no algorithm for this variant beyond those two remarks.  The
readings are:
  R21  Q = gamma_5 D, Hermitian and indefinite (gamma_5-hermiticity of D); it
       costs one product with D per iteration.  The system D x = b is Q x =
       gamma_5 b; the functions here solve Q x = b for the b they are given.
  R22  the seed phase is the Lanczos part of the algorithm (steps 1, 2, 5, 8, 9,
       with readings R1-R8) on Q; steps 3 and 6 (the LU of T and its pivots,
       which need not be positive here) are dropped.  The guesses are minimum
       residual solutions over span(V_m): x^j = x0 + V_m y_j with
       y_j = argmin_y || c_j - T~_m y ||, T~_m the (m+1) x m tridiagonal matrix
       (T_m with the row beta_m e_m^T appended), c_j = V_{m+1}^H r0^j, and
       c_1 = beta_0 e_1 for the seed system itself.  By the Lanczos relation
       Q V_m = V_{m+1} T~_m this minimises ||r0^j - Q V_m y|| over y.  A QR
       factorization of T~_m solves it; the oracle takes the plain definition
       (a dense least-squares solve).
  R23  each system is finished by MINRES (the QR-factorized Lanczos method for
       Hermitian indefinite matrices, Paige and Saunders) from its guess; it
       stops on its recursive residual norm and then verifies the true residual
       as the CG of Section 2.2 does (restart from r = b - Q x, at most 5).
  R24  no pivot check; breakdown as R7.

Parity pins (tests/test_oracle_indefinite.py): Q is Hermitian and indefinite
(dense matrix on a 2^4 lattice); MINRES against scipy.sparse.linalg.minres and
against a dense solve; the least-squares coefficients against the exact
solution when the Krylov space is the whole space; the minimum-residual
property against random competitors; seeding lowers the MINRES count on an
indefinite diagonal example.
"""
import numpy as np

from .operators import wilson_D

BREAKDOWN_TOL = 1e-12   # reading R7, as in the seed phase


def gamma5(psi):
    """gamma_5 = diag(1, 1, -1, -1) in spin (the chiral basis of the operators module)."""
    out = np.array(psi, copy=True)
    out[..., 2:, :] *= -1.0
    return out


class WilsonG5Op:
    """Q = gamma_5 D on flat complex vectors of length V*12 (site-major layout)."""

    def __init__(self, U, kappa, antiperiodic=True):
        self.U = np.asarray(U, dtype=np.complex128)
        self.kappa = float(kappa)
        self.antiperiodic = bool(antiperiodic)
        self.dims = tuple(self.U.shape[1:5])
        self.n = int(np.prod(self.dims)) * 12
        self.dtype = np.complex128

    def __call__(self, v):
        v = np.asarray(v)
        if v.ndim == 2:
            return np.stack([self(v[:, j]) for j in range(v.shape[1])], axis=1)
        psi = v.reshape(self.dims + (4, 3))
        return gamma5(wilson_D(psi, self.U, self.kappa, self.antiperiodic)).reshape(-1)

    def g5(self, v):
        """gamma_5 on a flat vector (for turning D x = b into Q x = gamma_5 b)."""
        v = np.asarray(v)
        if v.ndim == 2:
            return np.stack([self.g5(v[:, j]) for j in range(v.shape[1])], axis=1)
        return gamma5(v.reshape(self.dims + (4, 3))).reshape(-1)


def lanczos(apply_a, b, m, freq):
    """The Lanczos steps of the seed algorithm (readings R1-R8) without the LU.

    Returns (V n x (m_done+1), alpha (m_done), beta (m_done+1), m_done, status).
    """
    b = np.asarray(b)
    n = b.size
    dtype = np.result_type(b.dtype, np.float64)
    V = np.zeros((n, m + 1), dtype=dtype)
    alpha = np.zeros(m)
    beta = np.zeros(m + 1)
    beta[0] = np.linalg.norm(b)
    if beta[0] == 0.0:
        return V[:, :1], alpha[:0], beta[:1], 0, "breakdown"
    V[:, 0] = b / beta[0]
    amax = 0.0
    for i in range(1, m + 1):
        vi = V[:, i - 1].copy()
        f = apply_a(vi)
        if i > 1:
            f = f - beta[i - 1] * V[:, i - 2]
        alpha[i - 1] = np.vdot(vi, f).real
        f = f - alpha[i - 1] * vi
        if freq > 0 and i >= 2 and i % freq == 0:
            prev = V[:, : i - 1]
            c_v = prev.conj().T @ vi
            c_f = prev.conj().T @ f
            vi = vi - prev @ c_v
            vi = vi / np.linalg.norm(vi)
            f = f - prev @ c_f
            f = f - vi * np.vdot(vi, f)
            V[:, i - 1] = vi
        beta[i] = np.linalg.norm(f)
        amax = max(amax, abs(alpha[i - 1]))
        if beta[i] <= BREAKDOWN_TOL * amax:
            V[:, i] = 0.0
            return V[:, : i + 1], alpha[:i], beta[: i + 1], i, "breakdown"
        V[:, i] = f / beta[i]
    return V, alpha, beta, m, "ok"


def tridiag_ext(alpha, beta, m):
    """T~_m: (m+1) x m, diagonal alpha_1..alpha_m, off-diagonals beta_1..beta_m."""
    T = np.zeros((m + 1, m))
    for k in range(m):
        T[k, k] = alpha[k]
        T[k + 1, k] = beta[k + 1]
        if k + 1 < m:
            T[k, k + 1] = beta[k + 1]
    return T


def lstsq_coeffs(alpha, beta, m, C):
    """y_j = argmin || C[:, j] - T~_m y || (reading R22), one column per system."""
    T = tridiag_ext(alpha, beta, m)
    C = np.asarray(C)
    if C.ndim == 1:
        C = C[:, None]
    Y = np.zeros((m, C.shape[1]), dtype=np.result_type(C.dtype, np.float64))
    for j in range(C.shape[1]):
        Y[:, j] = np.linalg.lstsq(T.astype(Y.dtype), C[:, j], rcond=None)[0]
    return Y


def minres(apply_a, b, x0=None, tol=1e-8, maxit=100000, max_restarts=5):
    """MINRES (Paige-Saunders) for Hermitian A x = b.  Returns (x, iterations, true relres).

    One iteration is one product with A inside the loop.  The recursive residual
    norm |phi_k| decides when to stop; the true residual is then checked and the
    iteration restarted from r = b - A x while it is above tol (reading R23).
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
        beta = np.linalg.norm(r)
        if beta <= tol * bnorm:
            break
        v_prev = np.zeros_like(r)
        v = r / beta
        w_prev = np.zeros_like(r)
        w_prev2 = np.zeros_like(r)
        c_prev, s_prev = -1.0, 0.0
        delta1 = 0.0      # delta_k^(1)
        eps = 0.0         # epsilon_k^(1)
        phibar = beta
        while it < maxit:
            p = apply_a(v)
            alpha = np.vdot(v, p).real
            p = p - alpha * v - beta * v_prev
            beta_next = np.linalg.norm(p)
            # the previous rotation on column k of T~
            delta2 = c_prev * delta1 + s_prev * alpha
            gamma1 = s_prev * delta1 - c_prev * alpha
            eps_next = s_prev * beta_next
            delta1_next = -c_prev * beta_next
            # the new rotation, which zeroes beta_{k+1}
            gamma2 = np.hypot(gamma1, beta_next)
            c, s = gamma1 / gamma2, beta_next / gamma2
            tau = c * phibar
            phibar = s * phibar
            w = (v - delta2 * w_prev - eps * w_prev2) / gamma2
            x = x + tau * w
            it += 1
            if abs(phibar) <= tol * bnorm or beta_next == 0.0:
                break
            v_prev, v = v, p / beta_next
            beta = beta_next
            w_prev2, w_prev = w_prev, w
            c_prev, s_prev = c, s
            delta1, eps = delta1_next, eps_next
        true_rel = np.linalg.norm(b - apply_a(x)) / bnorm
        if true_rel <= tol or it >= maxit or restarts >= max_restarts:
            return x, it, float(true_rel)
        restarts += 1
    return x, it, float(np.linalg.norm(b - apply_a(x)) / bnorm)


def seeded_solve(apply_a, B, m, freq, tol, maxit=100000):
    """The indefinite variant: Lanczos seed on column 1 of B (from zero guesses),
    minimum-residual guesses for every column over its basis, MINRES to finish.

    Returns dict(X, X_seeded, iters (column 1: seed steps + its MINRES count),
    relres, m_done, alpha, beta, Y).
    """
    B = np.asarray(B)
    n, nrhs = B.shape
    dtype = np.result_type(B.dtype, np.float64)
    V, alpha, beta, md, status = lanczos(apply_a, B[:, 0], m, freq)
    Xg = np.zeros((n, nrhs), dtype=dtype)
    Y = None
    if md >= 1:
        C = V[:, : md + 1].conj().T @ B.astype(dtype)
        C[:, 0] = 0.0
        C[0, 0] = beta[0]
        Y = lstsq_coeffs(alpha, beta, md, C)
        Xg = V[:, :md] @ Y
    X = np.zeros_like(Xg)
    iters, relres = [], []
    for j in range(nrhs):
        x, it, rr = minres(apply_a, B[:, j], Xg[:, j], tol, maxit)
        X[:, j] = x
        iters.append(it + (md if j == 0 else 0))
        relres.append(rr)
    return {"X": X, "X_seeded": Xg, "iters": iters, "relres": relres, "m_done": md, "status": status,
            "alpha": alpha, "beta": beta, "Y": Y}
