"""Oracle emulation of the mixed-precision path: CG with single-precision
vectors and operator and FP64 reliable updates, and the seed phase with a
single-precision Lanczos basis.

Test infrastructure only (see ``oracle/__init__.py``).

The paper states no arithmetic precision.  The library's mixed mode keeps the
bulk of the work in single precision and everything that decides convergence in
FP64; this module writes that mode out plainly, in NumPy, so that the GPU's
iteration counts and errors in that mode have an oracle beside them.

What is single precision (float32 / complex64) and what is FP64:
  * single: the vectors r, p, q = A p and the increment of x since the last
    reliable update; the Lanczos vectors v_i, f and the stored basis V; the
    operator apply (``op.single()`` in ``operators.py``);
  * FP64: x, b, the true residual b - A x (with the FP64 operator) and every
    scalar: inner products and norms are summed in FP64 from the
    single-precision values; alpha, beta and rho are FP64 and rounded to single
    where they scale a single-precision vector; the projection over the basis
    and the LU solve of T are FP64 sums over the single-precision basis.

Reliable updates (CG):
  * a column is due when ||r||^2 of the single-precision recursion has fallen
    below 1e-8 times its largest value since the last update (a 1e4 drop of
    the norm);
  * the update: x += x_s; x_s = 0; r_true = b - A x in FP64; r = r_true
    rounded to single; rho = ||r_true||^2, which also becomes the new largest
    value; the direction p is kept, unless the true residual no longer follows
    the recursion: ||r_true||^2 has not halved since the smallest value seen
    at an update, or it is more than 4 times the recursive ||r||^2 just before
    the update (||r_true|| more than twice ||r||).  Either means that the FP64
    residual is at its rounding floor while the recursion kept falling; the
    kept p belongs to that recursion, and CG continued with it and with the
    true residual's rho diverges.  Then p = r;
  * when ||r|| <= tol ||b|| the single-precision recursion stops, x_s is folded
    into x and the true residual decides: at tol, the column is done; above it,
    CG restarts from r_true with p = r (at most 5 restarts, as ``cg.cg``).
  * Here a due update is made at the iteration where it falls due; the library
    makes it at its next host check, at most 8 iterations later (the recursion
    is then still three orders of magnitude above its rounding floor, so the
    delay changes the iterates by rounding only).

Parity pins (tests/test_oracle_mixed.py):
  * with FP64 arrays and updates switched off, ``cg_mixed`` is ``cg.cg``
    iterate by iterate;
  * with FP64 arrays and updates on, the iterates still equal plain CG's to
    rounding (a reliable update that keeps p changes nothing in exact
    arithmetic), so a wrong update rule (p restarted, x_s not cleared, a stale
    rho) is caught;
  * after every update the stored true residual equals b - A x recomputed
    independently, and the 1e4 drop held since the previous update;
  * the final FP64 true residual is <= tol on the paper's Example 1 and on a
    Wilson 4^4 lattice; on Wilson the count is within a few of FP64 CG's;
  * ``seed_lanczos_mixed`` with FP64 arrays reproduces ``seed.seed_lanczos``;
    in single precision its basis after a reorthogonalization event is
    orthonormal to single precision and the three-term relation holds to it.
"""
from dataclasses import dataclass

import numpy as np

from .seed import BREAKDOWN_TOL, project, seed_x1

UPDATE_DROP2 = 1e-8   # reliable update when ||r||^2 < 1e-8 * (largest ||r||^2 since the last one)


def _single_of(hi):
    return np.complex64 if np.issubdtype(hi, np.complexfloating) else np.float32


def _real_single(lo):
    return np.float32 if np.dtype(lo) in (np.dtype(np.complex64), np.dtype(np.float32)) else np.float64


def _dot64(a, b):
    """conj(a) . b summed in FP64 from the stored values."""
    hi = np.complex128 if np.iscomplexobj(a) or np.iscomplexobj(b) else np.float64
    return np.vdot(np.asarray(a, dtype=hi), np.asarray(b, dtype=hi))


def cg_mixed(apply64, apply_lo, b, x0=None, tol=1e-8, maxit=100000, lo=None, updates=True, max_restarts=5,
             history=None, events=None):
    """Solve A x = b by CG in precision ``lo`` with FP64 reliable updates.

    apply64: the FP64 operator; apply_lo: the operator in precision ``lo``
    (default: the single-precision counterpart of b's FP64 type).  Returns
    (x, iterations, true relative residual).  ``history`` (a list) receives x
    after every iteration; ``events`` (a list) receives one dict per reliable
    update (iteration, x, stored true residual, rho before and the largest
    rho since the previous update).
    """
    b = np.asarray(b)
    hi = np.result_type(b.dtype, np.float64)
    lo = _single_of(hi) if lo is None else lo
    rlo = _real_single(lo)
    x = np.zeros(b.shape, dtype=hi) if x0 is None else np.array(x0, dtype=hi)
    bnorm2 = float(_dot64(b, b).real)
    if bnorm2 == 0.0:
        return np.zeros_like(x), 0, 0.0
    tol2 = tol * tol * bnorm2
    it = 0
    restarts = 0
    r_true = b - apply64(x)
    rho = float(_dot64(r_true, r_true).real)
    while True:
        if rho <= tol2:
            break
        r = r_true.astype(lo)
        p = r.copy()
        xs = np.zeros(b.shape, dtype=lo)
        rmax = rho
        best_true = np.inf
        while it < maxit:
            q = apply_lo(p)
            pq = float(_dot64(p, q).real)
            alpha = rho / pq
            a_lo = rlo(alpha)
            xs = xs + a_lo * p
            r = r - a_lo * q
            rho_new = float(_dot64(r, r).real)
            it += 1
            if history is not None:
                history.append(x + xs.astype(hi))
            if not (rho_new > tol2) or not np.isfinite(rho_new):
                break
            beta = rho_new / rho
            rho = rho_new
            rmax = max(rmax, rho)
            p = r + rlo(beta) * p
            if updates and rho < UPDATE_DROP2 * rmax:
                x = x + xs.astype(hi)
                xs = np.zeros(b.shape, dtype=lo)
                r_true = b - apply64(x)
                rho_true = float(_dot64(r_true, r_true).real)
                if events is not None:
                    events.append({"iter": it, "x": x.copy(), "r_true": r_true.copy(), "rho_rec": rho,
                                   "rmax": rmax})
                consistent = rho_true <= 4.0 * rho
                rho = rho_true
                rmax = rho
                r = r_true.astype(lo)
                improved = rho_true < 0.5 * best_true
                if improved:
                    best_true = rho_true
                if not (improved and consistent):
                    p = r.copy()
        x = x + xs.astype(hi)
        r_true = b - apply64(x)
        rho = float(_dot64(r_true, r_true).real)
        if rho <= tol2 or it >= maxit or restarts >= max_restarts:
            break
        restarts += 1
    return x, it, float(np.sqrt(rho / bnorm2))


@dataclass
class MixedSeedResult:
    V: np.ndarray        # n x (m_done + 1) in the single-precision type: v_1 .. v_{m_done+1}
    alpha: np.ndarray    # FP64
    beta: np.ndarray     # FP64, beta_0 .. beta_{m_done}
    m_done: int
    status: str          # "ok" | "breakdown" | "not_pd"


def _reorthogonalize_lo(V, i, f, lo):
    """Step 8 at step i (1-based) with FP64 sums over the stored basis; results stored in ``lo``.

    One pass of classical Gram-Schmidt: the coefficients of v_i and f on
    v_1..v_{i-1}, then v_i renormalised, then f's component on the new v_i.
    """
    hi = np.complex128 if np.issubdtype(lo, np.complexfloating) else np.float64
    prev = V[:, : i - 1].astype(hi)
    vi = V[:, i - 1].astype(hi)
    fh = f.astype(hi)
    c_v = prev.conj().T @ vi
    c_f = prev.conj().T @ fh
    vi = (vi - prev @ c_v).astype(lo)
    vi = (vi.astype(hi) / np.linalg.norm(vi.astype(hi))).astype(lo)
    fh = (fh - prev @ c_f).astype(lo).astype(hi)
    vih = vi.astype(hi)
    f = (fh - vih * np.vdot(vih, fh)).astype(lo)
    V[:, i - 1] = vi
    return f


def seed_lanczos_mixed(apply_lo, b1, m, freq, lo=None):
    """The Lanczos steps of the seed algorithm (steps 1, 2, 5, 8, 9, with the
    pivot check of steps 3 and 6) on right-hand side 1 from x = 0, with
    single-precision vectors and basis and FP64 scalars.  The guesses are
    then the batched projection over the stored basis (``seeded_solve_mixed``).
    """
    b1 = np.asarray(b1)
    hi = np.result_type(b1.dtype, np.float64)
    lo = _single_of(hi) if lo is None else lo
    rlo = _real_single(lo)
    n = b1.shape[0]
    V = np.zeros((n, m + 1), dtype=lo)
    alpha = np.zeros(m)
    beta = np.zeros(m + 1)
    # step 1 (x0 = 0) and step 2
    beta[0] = float(np.linalg.norm(b1.astype(hi)))
    V[:, 0] = (b1.astype(hi) / beta[0]).astype(lo)
    f = apply_lo(V[:, 0])
    alpha[0] = float(_dot64(V[:, 0], f).real)
    f = f - rlo(alpha[0]) * V[:, 0]
    beta[1] = float(np.sqrt(_dot64(f, f).real))
    delta = alpha[0]
    if delta <= 0.0:
        return MixedSeedResult(V[:, :1], alpha[:1], beta[:1], 0, "not_pd")
    amax = abs(alpha[0])
    if beta[1] <= BREAKDOWN_TOL * amax or m == 1:
        V[:, 1] = (f.astype(hi) / beta[1]).astype(lo) if beta[1] > 0 else 0.0
        return MixedSeedResult(V[:, :2], alpha[:1], beta[:2], 1,
                               "breakdown" if beta[1] <= BREAKDOWN_TOL * amax else "ok")
    V[:, 1] = (f.astype(hi) / beta[1]).astype(lo)
    for i in range(2, m + 1):
        vi = V[:, i - 1].copy()
        # step 5
        f = apply_lo(vi) - rlo(beta[i - 1]) * V[:, i - 2]
        alpha[i - 1] = float(_dot64(vi, f).real)
        f = f - rlo(alpha[i - 1]) * vi
        # the pivot of step 6 (A must be positive definite)
        delta = alpha[i - 1] - beta[i - 1] ** 2 / delta
        if delta <= 0.0:
            return MixedSeedResult(V[:, :i], alpha[:i], beta[:i], i - 1, "not_pd")
        # step 8
        if freq > 0 and i % freq == 0:
            f = _reorthogonalize_lo(V, i, f, lo)
        # step 9
        beta[i] = float(np.sqrt(_dot64(f, f).real))
        amax = max(amax, abs(alpha[i - 1]))
        if beta[i] <= BREAKDOWN_TOL * amax:
            return MixedSeedResult(V[:, : i + 1], alpha[:i], beta[: i + 1], i, "breakdown")
        V[:, i] = (f.astype(hi) / beta[i]).astype(lo)
    return MixedSeedResult(V, alpha, beta, m, "ok")


def seeded_solve_mixed(apply64, apply_lo, B, m, freq, tol, maxit=100000, lo=None):
    """Single seeding in mixed precision from zero guesses: the seed phase on
    column 1 (``seed_lanczos_mixed``), every column's guess from the projection
    over the stored basis (x^1 = V T^{-1} beta_0 e_1, x^j = V T^{-1} V^H b^j,
    FP64 sums over the single-precision basis), then ``cg_mixed`` on every
    column.  Returns a dict like ``seeded.seeded_solve`` (X, iters with the seed
    steps counted for column 1, cg_iters, relres, X_seeded, seed).
    """
    B = np.asarray(B)
    n, nrhs = B.shape
    hi = np.result_type(B.dtype, np.float64)
    res = seed_lanczos_mixed(apply_lo, B[:, 0], m, freq, lo)
    md = res.m_done
    Vh = res.V.astype(hi)
    Xg = np.zeros((n, nrhs), dtype=hi)
    if md >= 1:
        Xg[:, 0] = seed_x1(Vh, res.alpha, res.beta, md)
        if nrhs > 1:
            Xg[:, 1:] = project(Vh, res.alpha, res.beta, md, B[:, 1:].astype(hi))
    X = np.zeros_like(Xg)
    iters, cg_iters, relres = [], [], []
    for j in range(nrhs):
        x, it, rr = cg_mixed(apply64, apply_lo, B[:, j], Xg[:, j], tol, maxit, lo)
        X[:, j] = x
        cg_iters.append(it)
        iters.append(it + (md if j == 0 else 0))
        relres.append(rr)
    return {"X": X, "X_seeded": Xg, "iters": iters, "cg_iters": cg_iters, "relres": relres, "seed": res}


def cg_mixed_multi(apply64, apply_lo, B, X0=None, tol=1e-8, maxit=100000, lo=None):
    """``cg_mixed`` on each column of B.  Returns (X, iters[list], relres[list])."""
    B = np.asarray(B)
    X = np.zeros(B.shape, dtype=np.result_type(B.dtype, np.float64))
    iters, rel = [], []
    for j in range(B.shape[1]):
        x, it, rr = cg_mixed(apply64, apply_lo, B[:, j], None if X0 is None else X0[:, j], tol, maxit, lo)
        X[:, j] = x
        iters.append(it)
        rel.append(rr)
    return X, iters, rel


def related_rhs_solve_mixed(apply64, apply_lo, B, m, freq, tol, maxit=100000, lo=None):
    """Single seeding of related right-hand sides (Section 2.3, steps 1-4) with
    the solves of ``seeded_solve_mixed``: system 1 seeded in mixed precision and
    finished by ``cg_mixed``, the others projected over its single-precision
    basis, then each system in turn by ``cg_mixed`` from its carried guess; the
    rank-1 projections over each system's CG correction and the carried
    residuals are FP64.  Returns (X, A-applies per system).
    """
    B = np.asarray(B)
    n, nrhs = B.shape
    hi = np.result_type(B.dtype, np.float64)
    res = seed_lanczos_mixed(apply_lo, B[:, 0], m, freq, lo)
    md = res.m_done
    Vh = res.V.astype(hi)
    X = np.zeros((n, nrhs), dtype=hi)
    if md >= 1:
        X[:, 0] = seed_x1(Vh, res.alpha, res.beta, md)
        if nrhs > 1:
            X[:, 1:] = project(Vh, res.alpha, res.beta, md, B[:, 1:].astype(hi))
    x, it, _ = cg_mixed(apply64, apply_lo, B[:, 0], X[:, 0], tol, maxit, lo)
    X[:, 0] = x
    mvps = [it + md]
    R = np.stack([B[:, i] - apply64(X[:, i]) for i in range(nrhs)], axis=1)
    x_bcg = np.zeros(n, dtype=hi)
    r_bcg = B[:, 0].astype(hi)
    for j in range(nrhs):
        if j > 0:
            x_bcg = X[:, j].copy()
            r_bcg = R[:, j].copy()
            x, it, _ = cg_mixed(apply64, apply_lo, B[:, j], x_bcg, tol, maxit, lo)
            X[:, j] = x
            mvps.append(it)
        x_cg = X[:, j] - x_bcg
        den = np.vdot(x_cg, r_bcg)
        if den == 0:
            continue
        for i in range(j + 1, nrhs):
            d = np.vdot(x_cg, R[:, i]) / den
            X[:, i] = X[:, i] + d * x_cg
            R[:, i] = R[:, i] - d * r_bcg
    return X, mvps
