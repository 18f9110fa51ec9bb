"""Pins of the oracle CG against closed forms and dense solves."""
import numpy as np

from oracle import operators as ops
from oracle.cg import cg, cg_multi
from paper_0810_0330_amd import synth


def test_cg_diagonal_exact():
    gen = np.random.default_rng(1)
    d = gen.uniform(0.5, 2.0, 300)
    b = gen.standard_normal(300)
    x, it, rr = cg(ops.DiagOp(d), b, tol=1e-13)
    np.testing.assert_allclose(x, b / d, rtol=1e-11)
    assert rr <= 1e-13


def test_cg_finite_termination():
    # a diagonal with k distinct values: the Krylov space has dimension k
    vals = np.array([0.1, 0.7, 1.3, 2.0, 5.0])
    d = np.repeat(vals, 40)
    b = np.random.default_rng(2).standard_normal(d.size)
    x, it, rr = cg(ops.DiagOp(d), b, tol=1e-12)
    assert it == 5
    assert rr <= 1e-12


def test_cg_dense_spd():
    gen = np.random.default_rng(3)
    m = gen.standard_normal((60, 60))
    a = m @ m.T + 60 * np.eye(60)
    b = gen.standard_normal(60)
    x, it, rr = cg(ops.DenseOp(a), b, tol=1e-13)
    np.testing.assert_allclose(x, np.linalg.solve(a, b), rtol=1e-11)


def test_cg_complex_wilson_dense():
    dims = (2, 2, 2, 4)
    U = synth.su3_links(dims, synth.rng(5, 0))
    op = ops.WilsonNormalOp(U, 0.12)
    d = ops.wilson_dense(U, 0.12)
    b = synth.complex_gaussian(op.n, 2, synth.rng(5, 1))
    X, iters, rel = cg_multi(op, b, tol=1e-12)
    np.testing.assert_allclose(X, np.linalg.solve(d.conj().T @ d, b), rtol=1e-9, atol=1e-11)
    assert max(rel) <= 1e-12


def test_cg_a_norm_error_monotone():
    nx = ny = 32
    a = ops.laplace2d_dense(nx, ny)
    b = np.random.default_rng(4).standard_normal(nx * ny)
    xs = np.linalg.solve(a, b)
    hist = []
    cg(ops.Laplace2DOp(nx, ny), b, tol=1e-12, history=hist)
    e0 = np.sqrt(xs @ a @ xs)
    prev = e0
    for x in hist:
        e = x - xs
        en = np.sqrt(e @ a @ e)
        if en / e0 <= 1e-12:
            break
        assert en <= prev * (1 + 1e-10)
        prev = en


def test_cg_zero_rhs_and_converged_guess():
    d = np.linspace(1, 2, 50)
    x, it, rr = cg(ops.DiagOp(d), np.zeros(50))
    assert it == 0 and not x.any()
    b = np.ones(50)
    x, it, rr = cg(ops.DiagOp(d), b, x0=b / d, tol=1e-8)
    assert it == 0
