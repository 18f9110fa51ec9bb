"""Oracle A-apply operators (FP64 / complex128, plain NumPy).

Test infrastructure only (see ``oracle/__init__.py``).

The method needs only an apply of a Hermitian positive definite A (Section 1).
The paper's large test (Section 4) uses the Wilson-Dirac matrix D of lattice
QCD through the normal-equations form A = D^H D, which makes A HPD at the
price of two products with D per CG iteration.  The paper cites D without
defining it; the textbook definition used here is

    (D psi)(x) = psi(x) - kappa * sum_mu [ (1 - gamma_mu) U_mu(x) psi(x + mu)
                                         + (1 + gamma_mu) U_mu(x - mu)^H psi(x - mu) ]

with periodic boundaries in x, y, z and antiperiodic boundaries in t (a hop
that wraps round the t direction picks up a factor -1).  Writing D = 1 - kappa H
defines the hopping matrix H, so dD/dkappa = -H.  Its adjoint swaps the two
spin projectors:

    (D^H psi)(x) = psi(x) - kappa * sum_mu [ (1 + gamma_mu) U_mu(x) psi(x + mu)
                                           + (1 - gamma_mu) U_mu(x - mu)^H psi(x - mu) ]

Conventions (shared with the library as a data format, not as code):
  * a spinor field is an array of shape (T, Z, Y, X, 4, 3): site coordinates
    with x fastest, then spin, then colour;
  * links have shape (4, T, Z, Y, X, 3, 3); U[mu] at site x is the link from x
    to x + mu, mu = 0, 1, 2, 3 for x, y, z, t;
  * gamma matrices are Hermitian in a chiral basis with gamma_5 = diag(1,1,-1,-1):
    gamma_k = [[0, -i sigma_k], [i sigma_k, 0]] (k = 1, 2, 3 for x, y, z),
    gamma_4 = [[0, 1], [1, 0]] (t).

Smaller operators: the unscaled 2D five-point Laplacian with zero Dirichlet
boundary, and a diagonal matrix (the paper's Examples 1-5 use a diagonal A).

Every operator also has a single-precision apply (``single()``: the same
formulas evaluated in float32 / complex64 arithmetic), which the emulation of
the mixed-precision solver in ``mixed.py`` uses.

Parity pins (tests/test_oracle_operators.py): a dense matrix built entry by
entry with pure-Python loops on tiny lattices; the closed-form free-field
spectrum (plane waves); gamma_5-hermiticity D^H = gamma_5 D gamma_5; gauge
covariance; the closed-form Laplacian eigenpairs.
"""
import numpy as np

# ----------------------------------------------------------------------------
# gamma matrices, chiral basis
# ----------------------------------------------------------------------------
_SIGMA = (
    np.array([[0, 1], [1, 0]], dtype=np.complex128),
    np.array([[0, -1j], [1j, 0]], dtype=np.complex128),
    np.array([[1, 0], [0, -1]], dtype=np.complex128),
)
_Z2 = np.zeros((2, 2), dtype=np.complex128)
_I2 = np.eye(2, dtype=np.complex128)


def _gamma_space(s):
    return np.block([[_Z2, -1j * s], [1j * s, _Z2]])


GAMMA = (
    _gamma_space(_SIGMA[0]),
    _gamma_space(_SIGMA[1]),
    _gamma_space(_SIGMA[2]),
    np.block([[_Z2, _I2], [_I2, _Z2]]),
)
GAMMA5 = GAMMA[0] @ GAMMA[1] @ GAMMA[2] @ GAMMA[3]
I4 = np.eye(4, dtype=np.complex128)


# ----------------------------------------------------------------------------
# 2D Laplacian (unscaled, zero Dirichlet halo)
# ----------------------------------------------------------------------------
def laplace2d_apply(x, nx, ny, dtype=np.float64):
    """y = 4 x - (north + south + east + west) on an nx-by-ny grid, zeros outside.

    ``x`` is a vector of length nx*ny (index i + nx*j, i fastest) or a matrix
    whose columns are such vectors.  Arithmetic in ``dtype``.
    """
    x = np.asarray(x, dtype=dtype)
    cols = x.reshape(ny, nx, -1)
    y = 4.0 * cols
    y[1:, :, :] -= cols[:-1, :, :]
    y[:-1, :, :] -= cols[1:, :, :]
    y[:, 1:, :] -= cols[:, :-1, :]
    y[:, :-1, :] -= cols[:, 1:, :]
    return y.reshape(x.shape)


def laplace2d_dense(nx, ny):
    """Dense Laplacian matrix built entry by entry (pins the apply)."""
    n = nx * ny
    a = np.zeros((n, n))
    for j in range(ny):
        for i in range(nx):
            row = i + nx * j
            a[row, row] = 4.0
            for di, dj in ((1, 0), (-1, 0), (0, 1), (0, -1)):
                ii, jj = i + di, j + dj
                if 0 <= ii < nx and 0 <= jj < ny:
                    a[row, ii + nx * jj] = -1.0
    return a


# ----------------------------------------------------------------------------
# diagonal operator (Examples 1-5)
# ----------------------------------------------------------------------------
def diag_apply(x, d):
    x = np.asarray(x)
    if x.ndim == 1:
        return d * x
    return d[:, None] * x


# ----------------------------------------------------------------------------
# Wilson-Dirac
# ----------------------------------------------------------------------------
def _site_axis(mu):
    # field axes are (T, Z, Y, X, ...): direction mu lives on axis 3 - mu
    return 3 - mu


def _shift_fwd(psi, mu, antiperiodic):
    """psi(x + mu) with the boundary phase of direction mu."""
    ax = _site_axis(mu)
    out = np.roll(psi, -1, axis=ax)
    if mu == 3 and antiperiodic:
        out[-1] *= -1.0
    return out


def _shift_bwd(psi, mu, antiperiodic):
    """psi(x - mu) with the boundary phase of direction mu."""
    ax = _site_axis(mu)
    out = np.roll(psi, 1, axis=ax)
    if mu == 3 and antiperiodic:
        out[0] *= -1.0
    return out


def _colour(u, chi):
    # (u chi)_{s,c} = sum_d u_{c,d} chi_{s,d}, i.e. chi u^T per site
    return np.matmul(chi, np.swapaxes(u, -1, -2))


def _colour_dag(u, chi):
    # (u^H chi)_{s,c} = sum_d conj(u_{d,c}) chi_{s,d}, i.e. chi conj(u) per site
    return np.matmul(chi, u.conj())


def _spin(p, chi):
    # (p chi)_{a,c} = sum_b p_{a,b} chi_{b,c}
    return np.matmul(p, chi)


def wilson_hop(psi, U, antiperiodic=True, dagger=False, dtype=np.complex128):
    """Hopping term H psi (or H^H psi when ``dagger``) on fields of shape (T,Z,Y,X,4,3).

    Arithmetic in ``dtype`` (complex128, or complex64 for the single-precision apply).
    """
    psi = np.asarray(psi, dtype=dtype)
    U = np.asarray(U, dtype=dtype)
    out = np.zeros_like(psi)
    for mu in range(4):
        pm = (I4 - GAMMA[mu]).astype(dtype)
        pp = (I4 + GAMMA[mu]).astype(dtype)
        p_fwd, p_bwd = (pp, pm) if dagger else (pm, pp)
        fwd = _colour(U[mu], _shift_fwd(psi, mu, antiperiodic))
        u_back = np.roll(U[mu], 1, axis=_site_axis(mu))  # U_mu(x - mu)
        bwd = _colour_dag(u_back, _shift_bwd(psi, mu, antiperiodic))
        out += _spin(p_fwd, fwd) + _spin(p_bwd, bwd)
    return out


def _real_of(dtype):
    return np.float32 if np.dtype(dtype) == np.complex64 else np.float64


def wilson_D(psi, U, kappa, antiperiodic=True, dtype=np.complex128):
    """D psi = psi - kappa H psi."""
    k = _real_of(dtype)(kappa)
    return np.asarray(psi, dtype=dtype) - k * wilson_hop(psi, U, antiperiodic, dtype=dtype)


def wilson_Ddag(psi, U, kappa, antiperiodic=True, dtype=np.complex128):
    """D^H psi = psi - kappa H^H psi."""
    k = _real_of(dtype)(kappa)
    return np.asarray(psi, dtype=dtype) - k * wilson_hop(psi, U, antiperiodic, dagger=True, dtype=dtype)


def wilson_normal(psi, U, kappa, antiperiodic=True, dtype=np.complex128):
    """A psi = D^H D psi (two D-applies, Section 4)."""
    return wilson_Ddag(wilson_D(psi, U, kappa, antiperiodic, dtype), U, kappa, antiperiodic, dtype)


class WilsonNormalOp:
    """A = D^H D acting on flat complex vectors of length V*12 (site-major layout)."""

    def __init__(self, U, kappa, antiperiodic=True):
        self.U = np.asarray(U, dtype=np.complex128)
        self.kappa = float(kappa)
        self.antiperiodic = bool(antiperiodic)
        self.dims = tuple(self.U.shape[1:5])  # (T, Z, Y, X)
        self.n = int(np.prod(self.dims)) * 12
        self.dtype = np.complex128

    def _field(self, v):
        return np.asarray(v).reshape(self.dims + (4, 3))

    def __call__(self, v):
        v = np.asarray(v)
        if v.ndim == 2:
            return np.stack([self(v[:, j]) for j in range(v.shape[1])], axis=1)
        return wilson_normal(self._field(v), self.U, self.kappa, self.antiperiodic).reshape(-1)

    def D(self, v):
        return wilson_D(self._field(v), self.U, self.kappa, self.antiperiodic).reshape(-1)

    def Ddag(self, v):
        return wilson_Ddag(self._field(v), self.U, self.kappa, self.antiperiodic).reshape(-1)

    def H(self, v):
        return wilson_hop(self._field(v), self.U, self.antiperiodic).reshape(-1)

    def Hdag(self, v):
        return wilson_hop(self._field(v), self.U, self.antiperiodic, dagger=True).reshape(-1)

    def single(self):
        """A = D^H D applied in complex64 arithmetic (links rounded to complex64)."""
        U32 = self.U.astype(np.complex64)

        def apply(v):
            v = np.asarray(v)
            if v.ndim == 2:
                return np.stack([apply(v[:, j]) for j in range(v.shape[1])], axis=1)
            f = v.astype(np.complex64).reshape(self.dims + (4, 3))
            return wilson_normal(f, U32, self.kappa, self.antiperiodic, np.complex64).reshape(-1)
        return apply


class Laplace2DOp:
    def __init__(self, nx, ny):
        self.nx, self.ny = int(nx), int(ny)
        self.n = self.nx * self.ny
        self.dtype = np.float64

    def __call__(self, v):
        return laplace2d_apply(v, self.nx, self.ny)

    def single(self):
        """The same stencil in float32 arithmetic."""
        return lambda v: laplace2d_apply(v, self.nx, self.ny, dtype=np.float32)


class DiagOp:
    def __init__(self, d):
        self.d = np.asarray(d, dtype=np.float64)
        self.n = self.d.size
        self.dtype = np.float64

    def __call__(self, v):
        return diag_apply(v, self.d)

    def single(self):
        """diag(d) in float32 arithmetic (d rounded to float32)."""
        d32 = self.d.astype(np.float32)
        return lambda v: diag_apply(np.asarray(v, dtype=np.float32), d32)


class DenseOp:
    def __init__(self, a):
        self.a = np.asarray(a)
        self.n = self.a.shape[0]
        self.dtype = self.a.dtype

    def __call__(self, v):
        return self.a @ v


def wilson_dense(U, kappa, antiperiodic=True, dagger=False):
    """Dense D (or D^H) built entry by entry with Python loops (tiny lattices only).

    Row and column index (site*4 + spin)*3 + colour, site = x + X*(y + Y*(z + Z*t)).
    Pins the vectorised apply: the neighbour index, the boundary sign and the
    placement of U vs U^H are all written out here independently of the rolls.
    """
    U = np.asarray(U, dtype=np.complex128)
    T, Z, Y, X = U.shape[1:5]
    dims = (X, Y, Z, T)
    vol = X * Y * Z * T
    n = vol * 12
    d = np.eye(n, dtype=np.complex128)

    def site_of(c):
        return c[0] + X * (c[1] + Y * (c[2] + Z * c[3]))

    for t in range(T):
        for z in range(Z):
            for y in range(Y):
                for x in range(X):
                    c = [x, y, z, t]
                    s = site_of(c)
                    for mu in range(4):
                        pm = I4 - GAMMA[mu]
                        pp = I4 + GAMMA[mu]
                        p_fwd, p_bwd = (pp, pm) if dagger else (pm, pp)
                        # forward neighbour
                        cf = list(c)
                        cf[mu] += 1
                        sign_f = 1.0
                        if cf[mu] == dims[mu]:
                            cf[mu] = 0
                            if mu == 3 and antiperiodic:
                                sign_f = -1.0
                        sf = site_of(cf)
                        u_f = U[mu, t, z, y, x]
                        # backward neighbour, link U_mu(x - mu) taken daggered
                        cb = list(c)
                        cb[mu] -= 1
                        sign_b = 1.0
                        if cb[mu] < 0:
                            cb[mu] = dims[mu] - 1
                            if mu == 3 and antiperiodic:
                                sign_b = -1.0
                        sb = site_of(cb)
                        u_b = U[mu, cb[3], cb[2], cb[1], cb[0]].conj().T
                        for a in range(4):
                            for b in range(4):
                                if p_fwd[a, b] == 0 and p_bwd[a, b] == 0:
                                    continue
                                for ci in range(3):
                                    for cj in range(3):
                                        row = (s * 4 + a) * 3 + ci
                                        d[row, (sf * 4 + b) * 3 + cj] -= kappa * sign_f * p_fwd[a, b] * u_f[ci, cj]
                                        d[row, (sb * 4 + b) * 3 + cj] -= kappa * sign_b * p_bwd[a, b] * u_b[ci, cj]
    return d


def free_field_normal_eigenvalues(dims_xyzt, kappa, antiperiodic=True):
    """Closed-form spectrum of D^H D for unit links (each value has multiplicity 12).

    For U = 1 a plane wave exp(i p.x) u is mapped by D to exp(i p.x) D(p) u with
    D(p) = 1 - 2 kappa sum_mu cos p_mu + 2 i kappa sum_mu gamma_mu sin p_mu, so
    D(p)^H D(p) = (1 - 2 kappa sum cos p_mu)^2 + 4 kappa^2 sum sin^2 p_mu.  Momenta
    are 2 pi n / L in periodic directions and pi (2n + 1) / L in the antiperiodic one.
    """
    grids = []
    for mu, L in enumerate(dims_xyzt):
        nvec = np.arange(L)
        if mu == 3 and antiperiodic:
            grids.append(np.pi * (2 * nvec + 1) / L)
        else:
            grids.append(2 * np.pi * nvec / L)
    P = np.meshgrid(*grids, indexing="ij")
    csum = sum(np.cos(p) for p in P)
    s2 = sum(np.sin(p) ** 2 for p in P)
    return ((1 - 2 * kappa * csum) ** 2 + 4 * kappa ** 2 * s2).reshape(-1)
