"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This module draws random numbers and builds inputs only; it holds none of the
solver's arithmetic.  Everything is produced on the host in float64 /
complex128 in the natural layout:

  * spinor fields as flat vectors of length V*12, site-major: index
    (site*4 + spin)*3 + colour with site = x + X*(y + Y*(z + Z*t));
  * links as arrays of shape (4, T, Z, Y, X, 3, 3), U[mu] the link x -> x + mu.

Random streams come from numpy's PCG64 seeded by SeedSequence([810330,
config_id, stream]); streams are 0 = links, 1 = right-hand sides, 2 = eta
(gradient weights), 3 = per-system draws (kappa, nrhs).

The paper's lattice test (Section 4) uses a quenched 20^3 x 32 gauge
configuration at beta = 6.0, which is not available; random SU(3) links stand
in for it.  Its diagonal examples (Section 2, Examples 1-5) are reproduced
with diagonal entries uniform on [0, 1] and N(0, 1) right-hand sides.
"""
from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 810330


def rng(config_id, stream):
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([SEED_BASE, int(config_id), int(stream)])))


# ----------------------------------------------------------------------------
# gauge links
# ----------------------------------------------------------------------------
def su3_links(dims_xyzt, gen, eps=0.4):
    """Random SU(3) links U = exp(i eps H), H traceless Hermitian with Gaussian entries.

    G_ab = N(0,1) + i N(0,1); H = (G + G^H)/2 - tr/3; U = Q diag(exp(i eps lambda)) Q^H
    from eigh(H), which is exactly unitary with det U = exp(i eps tr H) = 1.
    """
    X, Y, Z, T = dims_xyzt
    shape = (4, T, Z, Y, X)
    g = gen.standard_normal(shape + (3, 3)) + 1j * gen.standard_normal(shape + (3, 3))
    h = 0.5 * (g + np.conj(np.swapaxes(g, -1, -2)))
    tr = np.trace(h, axis1=-2, axis2=-1).real / 3.0
    h = h - tr[..., None, None] * np.eye(3)
    lam, q = np.linalg.eigh(h)
    ph = np.exp(1j * eps * lam)
    return np.einsum("...ab,...b,...cb->...ac", q, ph, q.conj())


def unit_links(dims_xyzt):
    X, Y, Z, T = dims_xyzt
    u = np.zeros((4, T, Z, Y, X, 3, 3), dtype=np.complex128)
    u[...] = np.eye(3)
    return u


def random_gauge(dims_xyzt, gen):
    """Random SU(3) field g(x), shape (T, Z, Y, X, 3, 3) (used by gauge-covariance tests)."""
    u = su3_links(dims_xyzt, gen, eps=2.0)
    return u[0]


# ----------------------------------------------------------------------------
# right-hand sides
# ----------------------------------------------------------------------------
def volume(dims_xyzt):
    X, Y, Z, T = dims_xyzt
    return X * Y * Z * T


def point_sources(dims_xyzt, spin_colour):
    """One column per (spin, colour): delta at the origin (site 0)."""
    n = volume(dims_xyzt) * 12
    b = np.zeros((n, len(spin_colour)), dtype=np.complex128)
    for j, (s, c) in enumerate(spin_colour):
        b[s * 3 + c, j] = 1.0
    return b


ALL_SPIN_COLOUR = [(s, c) for s in range(4) for c in range(3)]


def z4_noise(n, k, gen):
    """Each complex component uniform in {1, i, -1, -i}."""
    ph = gen.integers(0, 4, size=(n, k))
    return (1j ** ph).astype(np.complex128)


def complex_gaussian(n, k, gen):
    return (gen.standard_normal((n, k)) + 1j * gen.standard_normal((n, k))) / np.sqrt(2.0)


def real_gaussian(n, k, gen):
    return gen.standard_normal((n, k))


def diag_example(n, gen):
    """Diagonal entries uniform on [0, 1], sorted (Section 2, Example 1)."""
    return np.sort(gen.uniform(0.0, 1.0, n))


def related_rhs(u):
    """Related right-hand sides from the columns u^1, u^2, ... (Example 3's recipe):
    b^1 = u^1, b^j = b^{j-1} + 0.2^{j-1} u^j."""
    B = np.zeros_like(u)
    B[:, 0] = u[:, 0]
    for j in range(1, u.shape[1]):
        B[:, j] = B[:, j - 1] + 0.2 ** j * u[:, j]
    return B


# ----------------------------------------------------------------------------
# workload presets
# ----------------------------------------------------------------------------
@dataclass
class Workload:
    name: str
    op: str                      # "laplace2d" | "wilson"
    dims: tuple                  # (nx, ny) or (X, Y, Z, T)
    nrhs: int
    tol: float
    m: int
    freq: int
    kappa: float = 0.0
    precision: str = "f64"       # "f64" | "mixed"
    config_id: int = 0
    extra: dict = field(default_factory=dict)

    @property
    def n(self):
        if self.op == "laplace2d":
            return self.dims[0] * self.dims[1]
        if self.op == "diag":
            return self.dims[0]
        return volume(self.dims) * 12


def laplace_32x32():
    return Workload("laplace2d_32x32_5rhs_f64", "laplace2d", (32, 32), 5, 1e-10, 200, 1, config_id=0)


def wilson_8x4(m=200):
    return Workload("wilson_ddagd_8^4_12pt_c128", "wilson", (8, 8, 8, 8), 12, 1e-8, m, 1, kappa=0.12, config_id=1)


def wilson_16x3x32(m=1000, freq=100):
    return Workload("wilson_ddagd_16^3x32_12pt+12z4_mixed", "wilson", (16, 16, 16, 32), 24, 1e-8, m, freq,
                    kappa=0.12, precision="mixed", config_id=2)


def wilson_12x4(m=200):
    return Workload("wilson_ddagd_12^4_12pt_grad_c128", "wilson", (12, 12, 12, 12), 12, 1e-8, m, 1,
                    kappa=0.12, config_id=3)


def diag_5000():
    """Section 2, Example 1: diagonal n = 5000, entries uniform on [0, 1], 8 N(0, 1) right-hand sides,
    tol 1e-8; the seed runs to the first system's convergence (m = 430 for this draw) without
    reorthogonalization."""
    return Workload("diag_5000_8rhs_f64", "diag", (5000,), 8, 1e-8, 430, 0, config_id=100)


def make_inputs(w: Workload):
    """Returns dict with 'B' (n x nrhs natural layout) and, for Wilson, 'U' and 'kappa'; for diag, 'd'."""
    if w.op == "laplace2d":
        return {"B": real_gaussian(w.n, w.nrhs, rng(w.config_id, 1))}
    if w.op == "diag":
        return {"d": diag_example(w.dims[0], rng(w.config_id, 0)), "B": real_gaussian(w.dims[0], w.nrhs, rng(w.config_id, 1))}
    U = su3_links(w.dims, rng(w.config_id, 0))
    npt = min(w.nrhs, 12)
    B = point_sources(w.dims, ALL_SPIN_COLOUR[:npt])
    if w.nrhs > npt:
        B = np.concatenate([B, z4_noise(w.n, w.nrhs - npt, rng(w.config_id, 1))], axis=1)
    return {"B": B, "U": U, "kappa": w.kappa}


UNEVEN_LATTICES = [(8, 8, 8, 8), (8, 8, 8, 16), (12, 12, 12, 12), (12, 12, 12, 24), (16, 16, 16, 16), (16, 16, 16, 32)]


def uneven_batch(lattices=UNEVEN_LATTICES, config_id=4, nrhs_range=(4, 24), kappa_range=(0.10, 0.13)):
    """Independent Wilson systems of different sizes, each with its own links and kappa.

    Per system s (stream 3 of the config, then a per-system links stream):
    nrhs_s uniform on nrhs_range, kappa_s uniform on kappa_range; right-hand sides are
    the first min(nrhs_s, 12) point sources, then Z4 noise.  Returns a list of dicts
    with dims, kappa, U (natural layout), B (n x nrhs natural layout).
    """
    g = rng(config_id, 3)
    out = []
    for i, dims in enumerate(lattices):
        k = int(g.integers(nrhs_range[0], nrhs_range[1] + 1))
        kap = float(g.uniform(kappa_range[0], kappa_range[1]))
        U = su3_links(dims, rng(config_id, 10 + i))
        n = volume(dims) * 12
        npt = min(k, 12)
        B = point_sources(dims, ALL_SPIN_COLOUR[:npt])
        if k > npt:
            B = np.concatenate([B, z4_noise(n, k - npt, rng(config_id, 20 + i))], axis=1)
        out.append({"dims": dims, "kappa": kap, "U": U, "B": B, "nrhs": k})
    return out


def seed_steps(k1, cap=1000):
    """m from a plain-CG count: 2 k1 rounded up to a multiple of 50, capped."""
    return int(min(cap, max(50, -(-2 * k1 // 50) * 50)))
