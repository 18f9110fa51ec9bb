"""Pins of the oracle gradients: exact linearity in b and central differences in kappa."""
import numpy as np

from oracle import grad
from paper_0810_0330_amd import synth


def _setup():
    dims = (2, 2, 2, 4)
    U = synth.su3_links(dims, synth.rng(21, 0))
    B = synth.point_sources(dims, synth.ALL_SPIN_COLOUR[:3])
    Eta = synth.complex_gaussian(B.shape[0], 3, synth.rng(21, 2))
    return U, B, Eta


def test_grad_b_is_exact_directional_derivative():
    U, B, Eta = _setup()
    L, X, Lam, gk = grad.grads(U, 0.12, B, Eta, dense=True)
    gen = synth.rng(21, 4)
    for _ in range(3):
        Udir = synth.complex_gaussian(B.shape[0], 3, gen)
        h = 1e-3  # L is linear in b: no truncation error at any h
        lp = grad.loss(grad.solve_dense(U, 0.12, B + h * Udir), Eta)
        lm = grad.loss(grad.solve_dense(U, 0.12, B - h * Udir), Eta)
        fd = (lp - lm) / (2 * h)
        an = sum(np.vdot(Lam[:, j], Udir[:, j]).real for j in range(3))
        assert abs(fd - an) <= 1e-9 * max(1.0, abs(an))


def test_grad_kappa_central_difference():
    U, B, Eta = _setup()
    kappa, h = 0.12, 1e-6
    L, X, Lam, gk = grad.grads(U, kappa, B, Eta, dense=True)
    lp = grad.loss(grad.solve_dense(U, kappa + h, B), Eta)
    lm = grad.loss(grad.solve_dense(U, kappa - h, B), Eta)
    fd = (lp - lm) / (2 * h)
    assert abs(fd - gk) <= 1e-6 * abs(gk)


def test_grad_cg_matches_dense():
    U, B, Eta = _setup()
    L1, X1, Lam1, gk1 = grad.grads(U, 0.12, B, Eta, dense=True)
    L2, X2, Lam2, gk2 = grad.grads(U, 0.12, B, Eta, tol=1e-13)
    np.testing.assert_allclose(Lam2, Lam1, rtol=1e-9, atol=1e-11)
    assert abs(gk1 - gk2) <= 1e-9 * abs(gk1)
