"""Pins of the oracle seed phase (Lanczos version of single seed CG, Section 3)."""
import numpy as np
import pytest
import scipy.linalg

from oracle import operators as ops
from oracle.cg import cg
from oracle.seed import _reorthogonalize, project, seed_lanczos, seed_x1, tridiag_dense, tridiag_lu_solve
from paper_0810_0330_amd import synth


@pytest.fixture(scope="module")
def laplace_full():
    w = synth.laplace_32x32()
    B = synth.make_inputs(w)["B"]
    op = ops.Laplace2DOp(32, 32)
    return op, B, seed_lanczos(op, B, m=200, freq=1)


@pytest.fixture(scope="module")
def wilson_tiny():
    dims = (2, 2, 2, 4)
    U = synth.su3_links(dims, synth.rng(11, 0))
    op = ops.WilsonNormalOp(U, 0.12)
    d = ops.wilson_dense(U, 0.12)
    B = np.concatenate([synth.point_sources(dims, synth.ALL_SPIN_COLOUR[:2]),
                        synth.z4_noise(op.n, 2, synth.rng(11, 1))], axis=1)
    return op, d.conj().T @ d, B


def test_orthogonality_full_reorth(laplace_full):
    op, B, res = laplace_full
    V = res.V[:, :200]
    assert np.linalg.norm(V.T @ V - np.eye(200)) < 1e-12


def test_orthogonality_full_reorth_complex(wilson_tiny):
    op, a, B = wilson_tiny
    res = seed_lanczos(op, B, m=60, freq=1)
    V = res.V[:, :60]
    assert np.linalg.norm(V.conj().T @ V - np.eye(60)) < 1e-12


def test_orthogonality_lost_without_reorth(laplace_full):
    op, B, _ = laplace_full
    res = seed_lanczos(op, B[:, :1], m=200, freq=0)
    V = res.V[:, :200]
    assert np.linalg.norm(V.T @ V - np.eye(200)) > 1e-6


def test_three_term_relation():
    op = ops.Laplace2DOp(32, 32)
    B = synth.make_inputs(synth.laplace_32x32())["B"]
    m = 60
    res = seed_lanczos(op, B[:, :1], m=m, freq=0)
    V = res.V
    lhs = op(V[:, :m])
    rhs = V[:, :m] @ tridiag_dense(res.alpha, res.beta, m)
    rhs[:, m - 1] += res.beta[m] * V[:, m]
    assert np.abs(lhs - rhs).max() < 1e-13 * 8


def test_ritz_values_closed_form(laplace_full):
    _, _, res = laplace_full
    ev = np.linalg.eigvalsh(tridiag_dense(res.alpha, res.beta, 200))
    lmin = 4 - 4 * np.cos(np.pi / 33)
    lmax = 4 + 4 * np.cos(np.pi / 33)
    assert abs(ev[0] - lmin) < 1e-10
    assert abs(ev[-1] - lmax) < 1e-10


def test_ritz_values_dense(wilson_tiny):
    # with full reorthogonalization and m = n the Ritz values are the whole spectrum
    op, a, B = wilson_tiny
    b = synth.complex_gaussian(op.n, 1, synth.rng(11, 2))
    res = seed_lanczos(op, b, m=op.n, freq=1)
    md = res.m_done
    assert md >= op.n - 1
    ev = np.linalg.eigvalsh(tridiag_dense(res.alpha, res.beta, md))
    ref = np.linalg.eigvalsh(a)
    assert abs(ev[0] - ref[0]) < 1e-11 * ref[-1]
    assert abs(ev[-1] - ref[-1]) < 1e-11 * ref[-1]
    if md == op.n:
        np.testing.assert_allclose(ev, ref, atol=1e-10 * ref[-1])


def test_lanczos_equals_cg_iterates():
    op = ops.Laplace2DOp(32, 32)
    b = synth.make_inputs(synth.laplace_32x32())["B"][:, 0]
    res = seed_lanczos(op, b, m=120, freq=0, record_x1=True)
    hist = []
    cg(op, b, tol=1e-14, maxit=120, history=hist)
    for i in range(120):
        rel = np.linalg.norm(res.x1_history[i] - hist[i]) / np.linalg.norm(hist[i])
        assert rel < 1e-10, (i, rel)
    # residual norm of the Lanczos iterate: ||r_i|| = beta_i |zeta_i / delta_i|
    i = 80
    x = res.x1_history[i - 1]
    zeta = res.beta[0]
    for k in range(1, i):
        zeta = -(res.beta[k] / res.delta[k - 1]) * zeta
    np.testing.assert_allclose(np.linalg.norm(b - op(x)), res.beta[i] * abs(zeta / res.delta[i - 1]), rtol=1e-8)


def test_galerkin_optimality(wilson_tiny):
    op, a, B = wilson_tiny
    m = 30
    res = seed_lanczos(op, B, m=m, freq=1)
    V = res.V[:, :m]
    X = project(res.V, res.alpha, res.beta, m, B[:, 1:])
    ref = V @ np.linalg.solve(V.conj().T @ a @ V, V.conj().T @ B[:, 1:])
    np.testing.assert_allclose(X, ref, rtol=1e-10, atol=1e-12 * np.abs(ref).max())


def test_incremental_equals_batched(laplace_full):
    op, B, res = laplace_full
    Xb = project(res.V, res.alpha, res.beta, 200, B[:, 1:])
    for j in range(4):
        rel = np.linalg.norm(Xb[:, j] - res.X[:, j + 1]) / np.linalg.norm(Xb[:, j])
        assert rel < 1e-10
    x1 = seed_x1(res.V, res.alpha, res.beta, 200)
    assert np.linalg.norm(x1 - res.X[:, 0]) / np.linalg.norm(x1) < 1e-10


def test_lu_solve_matches_banded():
    gen = np.random.default_rng(7)
    m = 50
    alpha = gen.uniform(2.0, 3.0, m)
    beta = np.concatenate([[5.0], gen.uniform(0.1, 0.9, m)])
    G = gen.standard_normal((m, 3)) + 1j * gen.standard_normal((m, 3))
    ab = np.zeros((3, m))
    ab[0, 1:] = beta[1:m]
    ab[1] = alpha
    ab[2, :-1] = beta[1:m]
    ref = scipy.linalg.solve_banded((1, 1), ab, G)
    np.testing.assert_allclose(tridiag_lu_solve(alpha, beta, m, G), ref, rtol=1e-12)


def test_nested_subspace_monotone(laplace_full):
    op, B, res = laplace_full
    a = ops.laplace2d_dense(32, 32)
    xs = np.linalg.solve(a, B[:, 1])
    prev = np.inf
    for m in range(10, 201, 10):
        e = project(res.V, res.alpha, res.beta, m, B[:, 1:2])[:, 0] - xs
        en = np.sqrt(e @ a @ e)
        assert en <= prev * (1 + 1e-10)
        prev = en


def test_breakdown_on_few_distinct_eigenvalues():
    vals = np.array([0.2, 0.5, 1.1, 3.0, 7.0])
    d = np.repeat(vals, 20)
    gen = np.random.default_rng(8)
    B = gen.standard_normal((d.size, 3))
    res = seed_lanczos(ops.DiagOp(d), B, m=20, freq=1)
    assert res.status == "breakdown" and res.m_done == 5
    X = project(res.V, res.alpha, res.beta, res.m_done, B[:, 1:])
    # the Krylov space of b^1 is invariant, so other RHS are solved only on it;
    # the seeded residual is orthogonal to the basis (Galerkin condition)
    R = B[:, 1:] - d[:, None] * X
    assert np.abs(res.V[:, :5].T @ R).max() < 1e-11
    x1 = seed_x1(res.V, res.alpha, res.beta, res.m_done)
    np.testing.assert_allclose(x1, B[:, 0] / d, rtol=1e-10)


def test_not_pd_detected():
    d = -np.linspace(1, 2, 100)
    res = seed_lanczos(ops.DiagOp(d), np.ones((100, 1)), m=10)
    assert res.status == "not_pd"


def test_reorthogonalization_step_semantics():
    # step 8 on inputs with O(1) overlaps: v_i re-orthonormalised against
    # v_1..v_{i-1}, f orthogonalised against v_1..v_i (the new v_i included)
    gen = np.random.default_rng(12)
    n, i = 40, 6
    q, _ = np.linalg.qr(gen.standard_normal((n, i - 1)) + 1j * gen.standard_normal((n, i - 1)))
    V = np.zeros((n, i + 1), dtype=np.complex128)
    V[:, : i - 1] = q
    V[:, i - 1] = gen.standard_normal(n) + 1j * gen.standard_normal(n)
    f = gen.standard_normal(n) + 1j * gen.standard_normal(n)
    f_out = _reorthogonalize(V, i, f.copy())
    vi = V[:, i - 1]
    assert abs(np.linalg.norm(vi) - 1) < 1e-14
    assert np.abs(q.conj().T @ vi).max() < 1e-14
    assert np.abs(V[:, :i].conj().T @ f_out).max() < 1e-13
    # f only lost components inside span(v_1..v_i)
    resid = f - f_out
    coef = np.linalg.lstsq(V[:, :i], resid, rcond=None)[0]
    assert np.linalg.norm(V[:, :i] @ coef - resid) < 1e-12
