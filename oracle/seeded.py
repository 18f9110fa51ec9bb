"""Oracle drivers: single seeding (Sections 2.2 and 3), single seeding of related
right-hand sides (Section 2.3), and multiple seeding (Section 2.1, the method the
paper argues against, kept as a comparator).

Test infrastructure only (see ``oracle/__init__.py``).

Reading R10: if right-hand side 1 is not at tol after the m seed steps, it is
finished with CG from its Lanczos approximation like the seeded systems.

Parity pins: tests/test_oracle_paper.py checks the character of Examples 1-5
(Tables 2.1 and 3.1); tests/test_oracle_seed.py pins the pieces.  The paper's
own matrices and right-hand sides are random with unknown seeds, so its printed
counts are matched in character (bands and orderings), not exactly.
"""
import numpy as np

from .cg import cg
from .seed import project, seed_lanczos, seed_x1


def seeded_solve(apply_a, B, m, freq, tol, X0=None, maxit=100000):
    """Single seed: Lanczos-CG on column 1 for m steps, project columns 2.., finish with CG.

    Returns a dict with X, per-RHS iterations (RHS 1: the seed steps plus any
    finishing CG iterations), true relative residuals, the seed result and the
    seeded guesses before CG.
    """
    B = np.asarray(B)
    n, nrhs = B.shape
    dtype = np.result_type(B.dtype, np.float64)
    X0 = np.zeros((n, nrhs), dtype=dtype) if X0 is None else np.asarray(X0, dtype=dtype)
    res = seed_lanczos(apply_a, B, X0, m, freq)
    md = res.m_done
    R0 = B - apply_a(X0) if np.any(X0) else B.astype(dtype)
    Xg = np.zeros((n, nrhs), dtype=dtype)
    Xg[:, 0] = seed_x1(res.V, res.alpha, res.beta, md, X0[:, 0])
    if nrhs > 1:
        Xg[:, 1:] = project(res.V, res.alpha, res.beta, md, R0[:, 1:], X0[:, 1:])
    X = np.zeros_like(Xg)
    iters = []
    relres = []
    for j in range(nrhs):
        x, it, rr = cg(apply_a, B[:, j], Xg[:, j], tol, maxit)
        X[:, j] = x
        iters.append(it + (md if j == 0 else 0))
        relres.append(rr)
    return {"X": X, "X_seeded": Xg, "iters": iters, "cg_iters": [i - (md if j == 0 else 0) for j, i in enumerate(iters)],
            "relres": relres, "seed": res}


def related_rhs_solve(apply_a, B, m, freq, tol, maxit=100000):
    """Single seeding of related right-hand sides (Section 2.3 algorithm, steps 1-4).

    Step 2 uses the Lanczos seed (m steps, reorthogonalization frequency freq)
    and finishes system 1 with CG if needed.  After each system j is solved, its
    CG correction x_cg = x^j - x^j_bcg seeds every later system by a Galerkin
    projection over that single vector.  Returns (X, mvps per RHS, before_cg)
    where before_cg[j] = (x^j_bcg, r^j_bcg), the state each system's CG started from.
    """
    B = np.asarray(B)
    n, nrhs = B.shape
    out = seeded_solve(apply_a, B[:, :1], m, freq, tol, maxit=maxit)
    dtype = np.result_type(B.dtype, np.float64)
    X = np.zeros((n, nrhs), dtype=dtype)
    X[:, 0] = out["X"][:, 0]
    mvps = [out["iters"][0]]
    # seed the others over the Lanczos basis of system 1
    if nrhs > 1:
        res = out["seed"]
        X[:, 1:] = project(res.V, res.alpha, res.beta, res.m_done, B[:, 1:])
    R = B - apply_a(X)
    # step 1: x_bcg^1 = 0, r_bcg^1 = b^1
    x_bcg = np.zeros(n, dtype=dtype)
    r_bcg = B[:, 0].astype(dtype)
    before_cg = [(x_bcg.copy(), r_bcg.copy())]
    for j in range(nrhs):
        if j > 0:
            # step 4: the next system starts from its current guess
            x_bcg = X[:, j].copy()
            r_bcg = R[:, j].copy()
            before_cg.append((x_bcg.copy(), r_bcg.copy()))
            x, it, _ = cg(apply_a, B[:, j], x_bcg, tol, maxit)
            X[:, j] = x
            mvps.append(it)
        # step 3: project the remaining systems over the CG correction
        x_cg = X[:, j] - x_bcg
        den = np.vdot(x_cg, r_bcg)
        if den == 0:
            continue
        for i in range(j + 1, nrhs):
            d = np.vdot(x_cg, R[:, i]) / den
            X[:, i] = X[:, i] + d * x_cg
            R[:, i] = R[:, i] - d * r_bcg
    return X, mvps, before_cg


def multiple_seed_solve(apply_a, B, tol, maxit=100000):
    """Standard seed CG (Section 2.1): solve each system by CG in turn, and during
    each solve project every later system over the CG directions (Galerkin
    projection over the Krylov subspace, through the A-conjugate directions p
    and q = A p).  Returns (X, mvps per RHS).
    """
    B = np.asarray(B)
    n, nrhs = B.shape
    dtype = np.result_type(B.dtype, np.float64)
    X = np.zeros((n, nrhs), dtype=dtype)
    R = B.astype(dtype).copy()
    mvps = []
    for j in range(nrhs):
        bnorm = np.linalg.norm(B[:, j])
        x = X[:, j].copy()
        r = B[:, j] - apply_a(x)
        rho = np.vdot(r, r).real
        p = r.copy()
        it = 0
        while np.sqrt(rho) > tol * bnorm and it < maxit:
            q = apply_a(p)
            pq = np.vdot(p, q).real
            a = rho / pq
            x = x + a * p
            r = r - a * q
            for i in range(j + 1, nrhs):
                c = np.vdot(p, R[:, i]) / pq
                X[:, i] = X[:, i] + c * p
                R[:, i] = R[:, i] - c * q
            rho_new = np.vdot(r, r).real
            it += 1
            if np.sqrt(rho_new) <= tol * bnorm:
                break
            p = r + (rho_new / rho) * p
            rho = rho_new
        X[:, j] = x
        mvps.append(it)
    return X, mvps
