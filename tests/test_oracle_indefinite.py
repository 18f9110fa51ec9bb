"""Pins of the indefinite-variant oracle (oracle/indefinite.py) against things
other than itself: a dense gamma_5 D built entry by entry, SciPy's MINRES and
dense solves, the exact solution when the Krylov space is the whole space, and
a least-squares solve with the explicit matrix Q V_m in place of the Lanczos
relation."""
import numpy as np
import scipy.sparse.linalg as sla

from oracle import indefinite as ind
from oracle import operators as ops
from oracle.operators import DenseOp
from paper_0810_0330_amd import synth


def _dense(op):
    n = op.n
    return np.stack([op(np.eye(n, dtype=np.complex128)[:, j]) for j in range(n)], axis=1)


def test_g5_d_is_hermitian_and_indefinite():
    dims = (2, 2, 2, 2)
    U = synth.su3_links(dims, synth.rng(61, 0))
    Q = _dense(ind.WilsonG5Op(U, 0.12))
    assert np.abs(Q - Q.conj().T).max() < 1e-13
    ev = np.linalg.eigvalsh(Q)
    assert ev.min() < -0.1 and ev.max() > 0.1
    # Q = gamma_5 D, with D the oracle's Wilson matrix built by its own dense builder
    D = ops.wilson_dense(U, 0.12)
    g5 = np.kron(np.eye(16), np.kron(np.diag([1.0, 1.0, -1.0, -1.0]), np.eye(3)))
    assert np.abs(Q - g5 @ D).max() < 1e-13


def test_minres_matches_scipy_and_dense_solve():
    g = np.random.default_rng(1)
    n = 60
    Qm, _ = np.linalg.qr(g.standard_normal((n, n)))
    ev = np.concatenate([-np.linspace(0.1, 2, n // 2), np.linspace(0.2, 3, n - n // 2)])
    A = (Qm * ev) @ Qm.T
    b = g.standard_normal(n)
    xs, info = sla.minres(A, b, rtol=1e-12, maxiter=1000)
    assert info == 0
    x, it, rr = ind.minres(DenseOp(A), b, tol=1e-12)
    assert rr <= 1e-12 and it <= 2 * n  # finite precision: a little past n
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) < 1e-9
    # complex Hermitian against a dense solve
    A = g.standard_normal((n, n)) + 1j * g.standard_normal((n, n))
    A = (A + A.conj().T) / 2
    b = g.standard_normal(n) + 1j * g.standard_normal(n)
    x, it, rr = ind.minres(DenseOp(A), b, tol=1e-12)
    xd = np.linalg.solve(A, b)
    assert rr <= 1e-12
    assert np.linalg.norm(x - xd) / np.linalg.norm(xd) < 1e-12 * np.linalg.cond(A) * 10


def test_minres_residual_is_monotone():
    # MINRES minimises the residual over a growing Krylov space: ||r_k|| never increases
    g = np.random.default_rng(2)
    d = np.concatenate([-np.linspace(0.05, 1.0, 100), np.linspace(0.1, 2.0, 100)])
    b = g.standard_normal(d.size)
    res = []
    for k in range(1, 40, 3):
        x, it, rr = ind.minres(ops.DiagOp(d), b, tol=1e-300, maxit=k, max_restarts=0)
        res.append(rr)
    assert all(res[i + 1] <= res[i] * (1 + 1e-12) for i in range(len(res) - 1))


def test_lstsq_guess_is_exact_on_the_whole_space():
    # 40 distinct eigenvalues of both signs: the Krylov space of b is the whole
    # space after 40 steps, and the minimum-residual guess is the solution
    d = np.concatenate([-np.linspace(0.5, 2.0, 20), np.linspace(0.3, 1.7, 20)])
    b = np.random.default_rng(3).standard_normal(d.size)
    out = ind.seeded_solve(ops.DiagOp(d), b[:, None], m=60, freq=1, tol=1e-10)
    assert out["m_done"] == 40 and out["status"] == "breakdown"
    np.testing.assert_allclose(out["X_seeded"][:, 0], b / d, rtol=1e-9)
    assert out["iters"][0] == 40


def test_lstsq_guess_minimises_the_residual_over_the_basis():
    # the T~ reduction (Lanczos relation) against the explicit matrix Q V_m
    dims = (4, 4, 4, 4)
    U = synth.su3_links(dims, synth.rng(62, 0))
    op = ind.WilsonG5Op(U, 0.12)
    B = synth.complex_gaussian(op.n, 3, synth.rng(62, 1))
    m = 30
    V, alpha, beta, md, _ = ind.lanczos(op, B[:, 0], m, 1)
    QV = op(V[:, :md])
    for j in range(3):
        c = V[:, : md + 1].conj().T @ B[:, j]
        if j == 0:
            c = np.zeros(md + 1, dtype=np.complex128)
            c[0] = beta[0]
        y = ind.lstsq_coeffs(alpha, beta, md, c)[:, 0]
        y_direct = np.linalg.lstsq(QV, B[:, j], rcond=None)[0]
        assert np.linalg.norm(y - y_direct) / np.linalg.norm(y_direct) < 1e-8
        r = np.linalg.norm(B[:, j] - QV @ y)
        gen = np.random.default_rng(j)
        for _ in range(5):
            dy = gen.standard_normal(md) * 1e-3 * np.linalg.norm(y)
            assert np.linalg.norm(B[:, j] - QV @ (y + dy)) >= r


def test_seeding_lowers_the_minres_count():
    # an indefinite diagonal example in the spirit of Examples 1 and 5: a few
    # eigenvalues of both signs close to zero slow MINRES down; a seed run to
    # past convergence resolves them and the seeded systems need about half
    # the iterations
    g = np.random.default_rng(4)
    small = np.array([0.002, 0.004, 0.006, 0.008, 0.01])
    d = np.sort(np.concatenate([-g.uniform(0.2, 1.0, 995), g.uniform(0.2, 1.0, 995), small, -small]))
    B = g.standard_normal((d.size, 3))
    op = ops.DiagOp(d)
    plain = [ind.minres(op, B[:, j], tol=1e-8)[1] for j in range(1, 3)]
    out = ind.seeded_solve(op, B, m=400, freq=10, tol=1e-8)
    assert max(out["relres"]) <= 1e-8
    for a, p in zip(out["iters"][1:], plain):
        assert a < 0.6 * p, (out["iters"], plain)
