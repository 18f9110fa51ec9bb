"""Pins of the oracle operators against facts fixed outside the oracle."""
import numpy as np
import pytest

from oracle import operators as ops
from paper_0810_0330_amd import synth


def _rand_field(dims_xyzt, gen):
    X, Y, Z, T = dims_xyzt
    return gen.standard_normal((T, Z, Y, X, 4, 3)) + 1j * gen.standard_normal((T, Z, Y, X, 4, 3))


# ---------------------------------------------------------------- Laplacian
def test_laplace_closed_form_eigenpairs():
    nx, ny = 32, 32
    i = np.arange(1, nx + 1)
    j = np.arange(1, ny + 1)
    for p, q in [(1, 1), (1, 2), (5, 17), (32, 32), (13, 1)]:
        u = np.outer(np.sin(q * np.pi * j / (ny + 1)), np.sin(p * np.pi * i / (nx + 1))).reshape(-1)
        lam = 4 - 2 * np.cos(p * np.pi / (nx + 1)) - 2 * np.cos(q * np.pi / (ny + 1))
        np.testing.assert_allclose(ops.laplace2d_apply(u, nx, ny), lam * u, atol=1e-13)


def test_laplace_apply_matches_dense():
    gen = np.random.default_rng(0)
    for nx, ny in [(1, 1), (3, 5), (7, 4)]:
        a = ops.laplace2d_dense(nx, ny)
        x = gen.standard_normal((nx * ny, 3))
        np.testing.assert_allclose(ops.laplace2d_apply(x, nx, ny), a @ x, atol=1e-14)


# ---------------------------------------------------------------- gamma matrices
def test_gamma_algebra():
    g = ops.GAMMA
    for mu in range(4):
        np.testing.assert_allclose(g[mu], g[mu].conj().T)
        for nu in range(4):
            ac = g[mu] @ g[nu] + g[nu] @ g[mu]
            np.testing.assert_allclose(ac, 2.0 * (mu == nu) * np.eye(4), atol=1e-15)
    np.testing.assert_allclose(ops.GAMMA5, np.diag([1, 1, -1, -1]), atol=1e-15)


# ---------------------------------------------------------------- Wilson
@pytest.mark.parametrize("dims,antiperiodic", [((2, 3, 2, 4), True), ((3, 2, 2, 2), False), ((2, 2, 2, 2), True)])
def test_wilson_apply_matches_dense_loops(dims, antiperiodic):
    gen = synth.rng(99, 0)
    U = synth.su3_links(dims, gen)
    kappa = 0.13
    psi = _rand_field(dims, gen)
    d = ops.wilson_dense(U, kappa, antiperiodic)
    got = ops.wilson_D(psi, U, kappa, antiperiodic).reshape(-1)
    np.testing.assert_allclose(got, d @ psi.reshape(-1), atol=1e-13)
    dd = ops.wilson_dense(U, kappa, antiperiodic, dagger=True)
    np.testing.assert_allclose(dd, d.conj().T, atol=1e-14)
    got = ops.wilson_Ddag(psi, U, kappa, antiperiodic).reshape(-1)
    np.testing.assert_allclose(got, dd @ psi.reshape(-1), atol=1e-13)


def test_wilson_gamma5_hermiticity():
    dims = (4, 4, 2, 6)
    gen = synth.rng(98, 0)
    U = synth.su3_links(dims, gen)
    psi = _rand_field(dims, gen)
    g5 = lambda f: np.einsum("ab,...bc->...ac", ops.GAMMA5, f)
    np.testing.assert_allclose(ops.wilson_Ddag(psi, U, 0.12), g5(ops.wilson_D(g5(psi), U, 0.12)), atol=1e-13)


def test_wilson_adjoint_and_positivity():
    dims = (4, 2, 4, 4)
    gen = synth.rng(97, 0)
    U = synth.su3_links(dims, gen)
    op = ops.WilsonNormalOp(U, 0.125)
    x = _rand_field(dims, gen).reshape(-1)
    y = _rand_field(dims, gen).reshape(-1)
    np.testing.assert_allclose(np.vdot(y, op.D(x)), np.vdot(op.Ddag(y), x), rtol=1e-13)
    np.testing.assert_allclose(np.vdot(y, op(x)), np.conj(np.vdot(x, op(y))), rtol=1e-13)
    xax = np.vdot(x, op(x))
    assert abs(xax.imag) < 1e-10 * abs(xax.real)
    assert xax.real > 0
    np.testing.assert_allclose(xax.real, np.linalg.norm(op.D(x)) ** 2, rtol=1e-13)


def test_wilson_gauge_covariance():
    dims = (4, 4, 4, 4)
    gen = synth.rng(96, 0)
    U = synth.su3_links(dims, gen)
    g = synth.random_gauge(dims, synth.rng(96, 5))
    psi = _rand_field(dims, gen)
    Ug = np.empty_like(U)
    for mu in range(4):
        g_fwd = np.roll(g, -1, axis=3 - mu)  # g(x + mu), periodic
        Ug[mu] = np.einsum("...ab,...bc,...dc->...ad", g, U[mu], g_fwd.conj())
    gpsi = np.einsum("...ab,...sb->...sa", g, psi)
    lhs = ops.wilson_D(gpsi, Ug, 0.12)
    rhs = np.einsum("...ab,...sb->...sa", g, ops.wilson_D(psi, U, 0.12))
    np.testing.assert_allclose(lhs, rhs, atol=1e-12)


@pytest.mark.parametrize("antiperiodic", [True, False])
def test_wilson_free_field_plane_waves(antiperiodic):
    dims = (4, 6, 4, 8)
    X, Y, Z, T = dims
    U = synth.unit_links(dims)
    kappa = 0.12
    gen = np.random.default_rng(3)
    coords = np.meshgrid(np.arange(T), np.arange(Z), np.arange(Y), np.arange(X), indexing="ij")
    t, z, y, x = coords
    for n in [(0, 0, 0, 0), (1, 2, 3, 1), (3, 5, 1, 7)]:
        p = [2 * np.pi * n[0] / X, 2 * np.pi * n[1] / Y, 2 * np.pi * n[2] / Z,
             (np.pi * (2 * n[3] + 1) if antiperiodic else 2 * np.pi * n[3]) / T]
        phase = np.exp(1j * (p[0] * x + p[1] * y + p[2] * z + p[3] * t))
        u = gen.standard_normal((4, 3)) + 1j * gen.standard_normal((4, 3))
        psi = phase[..., None, None] * u
        dp = (1 - 2 * kappa * sum(np.cos(pm) for pm in p)) * np.eye(4) \
            + 2j * kappa * sum(ops.GAMMA[mu] * np.sin(p[mu]) for mu in range(4))
        np.testing.assert_allclose(ops.wilson_D(psi, U, kappa, antiperiodic), phase[..., None, None] * (dp @ u), atol=1e-12)
        lam = (1 - 2 * kappa * sum(np.cos(pm) for pm in p)) ** 2 + 4 * kappa ** 2 * sum(np.sin(pm) ** 2 for pm in p)
        np.testing.assert_allclose(ops.wilson_normal(psi, U, kappa, antiperiodic), lam * psi, atol=1e-12)


def test_wilson_free_field_dense_spectrum():
    dims = (2, 2, 2, 4)
    U = synth.unit_links(dims)
    d = ops.wilson_dense(U, 0.12, True)
    ev = np.sort(np.linalg.eigvalsh(d.conj().T @ d))
    ref = np.sort(np.repeat(ops.free_field_normal_eigenvalues(dims, 0.12, True), 12))
    np.testing.assert_allclose(ev, ref, atol=1e-12)


def test_free_field_extremes_8x4():
    ev = ops.free_field_normal_eigenvalues((8, 8, 8, 8), 0.12, True)
    # closed form: minimum at p = (0,0,0,pi/8), maximum at the corners of the zone
    pmin = (1 - 2 * 0.12 * (3 + np.cos(np.pi / 8))) ** 2 + 4 * 0.12 ** 2 * np.sin(np.pi / 8) ** 2
    np.testing.assert_allclose(ev.min(), pmin, rtol=1e-14)
    assert abs(ev.min() - 0.0118306) < 1e-6 and abs(ev.max() - 3.77875) < 1e-4


# ---------------------------------------------------------------- synthetic inputs
def test_su3_links_are_special_unitary():
    U = synth.su3_links((2, 2, 2, 2), synth.rng(1, 0))
    eye = np.einsum("...ab,...cb->...ac", U, U.conj())
    np.testing.assert_allclose(eye, np.broadcast_to(np.eye(3), eye.shape), atol=1e-13)
    np.testing.assert_allclose(np.linalg.det(U), 1.0, atol=1e-13)
    U2 = synth.su3_links((2, 2, 2, 2), synth.rng(1, 0))
    assert np.array_equal(U, U2)


def test_z4_and_point_sources():
    z = synth.z4_noise(1000, 2, synth.rng(2, 1))
    assert set(np.round(z.reshape(-1), 12).tolist()) <= {1, 1j, -1, -1j}
    b = synth.point_sources((2, 2, 2, 2), synth.ALL_SPIN_COLOUR)
    assert b.shape == (16 * 12, 12)
    np.testing.assert_array_equal(b[:12], np.eye(12))
    assert not b[12:].any()
