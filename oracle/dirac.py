"""Fine-grid twisted-mass Wilson-clover operator, written out from its definition.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Paper: Sec. 1 defines D(+-mu) = D_W +- i Gamma5 mu and the bound
D(mu)^dag D(mu) = D_W^dag D_W + mu^2; Sec. 2 fixes gamma5 = diag(-1,-1,1,1)
and the lexicographic site order TZYX, and leaves the other gamma matrices
free.  D_W itself is only named ("Wilson clover operator"); the form used here
is the textbook Wilson + Sheikholeslami-Wohlert operator in mass
normalisation:

  (D_W psi)(x) = (m0+4) psi(x)
                 - 1/2 sum_mu [ (1-gamma_mu) U_mu(x) psi(x+mu)
                              + (1+gamma_mu) U_mu(x-mu)^dag psi(x-mu) ]
                 + (i c_sw / 4) sum_{mu,nu} sigma_{mu nu} F_{mu nu}(x) psi(x)

  sigma_{mu nu} = (i/2)[gamma_mu, gamma_nu],  F_{mu nu} = (Q_{mu nu} - Q_{nu mu}) / 8,
  Q_{mu nu}(x) = sum of the four plaquette leaves at x in the (mu,nu) plane,
  m0 = 1/(2 kappa) - 4.

Gamma basis (Euclidean, chiral): gamma_k = [[0, -i s_k], [i s_k, 0]] for the
X, Y, Z directions (s_k Pauli), gamma_T = [[0, -1], [-1, 0]]; their product
gamma_X gamma_Y gamma_Z gamma_T is the paper's gamma5.

Pins (tests/test_oracle_dirac.py): free-field plane waves (closed form),
pure-gauge fields, constant diagonal links (per-colour momentum shift), a
constant abelian field strength (closed form of the clover term), Gamma5
hermiticity, the squared-operator identity, gauge covariance, dense
brute-force spectrum bound sigma_min >= mu.
"""
from __future__ import annotations

import numpy as np

# direction index: 0:T 1:Z 2:Y 3:X (lattice axis order T, Z, Y, X)
NDIM = 4

_s1 = np.array([[0, 1], [1, 0]], dtype=np.complex128)
_s2 = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
_s3 = np.array([[1, 0], [0, -1]], dtype=np.complex128)
_Z2 = np.zeros((2, 2), dtype=np.complex128)
_I2 = np.eye(2, dtype=np.complex128)


def _gamma_spatial(s):
    return np.block([[_Z2, -1j * s], [1j * s, _Z2]])


GAMMA_X = _gamma_spatial(_s1)
GAMMA_Y = _gamma_spatial(_s2)
GAMMA_Z = _gamma_spatial(_s3)
GAMMA_T = np.block([[_Z2, -_I2], [-_I2, _Z2]])
# gamma matrix belonging to each link direction mu = 0:T 1:Z 2:Y 3:X
GAMMA = np.stack([GAMMA_T, GAMMA_Z, GAMMA_Y, GAMMA_X])
GAMMA5 = np.diag([-1.0, -1.0, 1.0, 1.0]).astype(np.complex128)


def sigma_munu(mu: int, nu: int) -> np.ndarray:
    """sigma_{mu nu} = (i/2)[gamma_mu, gamma_nu] (4x4)."""
    g1, g2 = GAMMA[mu], GAMMA[nu]
    return 0.5j * (g1 @ g2 - g2 @ g1)


def m0_from_kappa(kappa: float) -> float:
    return 1.0 / (2.0 * kappa) - 4.0


def _dag(M):
    return np.conj(np.swapaxes(M, -1, -2))


def _shift(f, mu: int, sign: int):
    """f(x + sign*mu) on the periodic lattice (lattice axes are the first four)."""
    return np.roll(f, -sign, axis=mu)


def spin_mul(G, psi):
    """Apply a 4x4 spin matrix to psi[..., 4, 3]."""
    return np.einsum("st,...tc->...sc", G, psi)


def colour_mul(U, psi):
    """Apply per-site colour matrices U[...,3,3] to psi[...,4,3]."""
    return np.einsum("...ab,...sb->...sa", U, psi)


# ----------------------------------------------------------------------------
# clover term
# ----------------------------------------------------------------------------

def clover_leaves(U, mu: int, nu: int):
    """Q_{mu nu}(x): the four plaquettes in the (mu,nu) plane that touch x,
    all taken with the same orientation (mu first, then nu)."""
    Um = U[..., mu, :, :]
    Un = U[..., nu, :, :]
    sh = _shift
    # leaf 1: x -> x+mu -> x+mu+nu -> x+nu -> x
    q = Um @ sh(Un, mu, +1) @ _dag(sh(Um, nu, +1)) @ _dag(Un)
    # leaf 2: x -> x+nu -> x-mu+nu -> x-mu -> x
    q = q + Un @ _dag(sh(sh(Um, mu, -1), nu, +1)) @ _dag(sh(Un, mu, -1)) @ sh(Um, mu, -1)
    # leaf 3: x -> x-mu -> x-mu-nu -> x-nu -> x
    q = q + _dag(sh(Um, mu, -1)) @ _dag(sh(sh(Un, mu, -1), nu, -1)) @ sh(sh(Um, mu, -1), nu, -1) @ sh(Un, nu, -1)
    # leaf 4: x -> x-nu -> x+mu-nu -> x+mu -> x
    q = q + _dag(sh(Un, nu, -1)) @ sh(Um, nu, -1) @ sh(sh(Un, mu, +1), nu, -1) @ _dag(Um)
    return q


def field_strength(U, mu: int, nu: int):
    """F_{mu nu} = (Q_{mu nu} - Q_{nu mu}) / 8 (anti-Hermitian 3x3 per site)."""
    return (clover_leaves(U, mu, nu) - clover_leaves(U, nu, mu)) / 8.0


def clover_matrix(U, csw: float):
    """Clover term A(x) = (i c_sw/4) sum_{mu,nu} sigma_{mu nu} (x) F_{mu nu}(x)
    as a 12x12 matrix per site, index = 3*spin + colour.  Shape [T,Z,Y,X,12,12]."""
    dims = U.shape[:4]
    A = np.zeros(dims + (4, 3, 4, 3), dtype=np.complex128)
    for mu in range(4):
        for nu in range(4):
            if mu == nu:
                continue
            F = field_strength(U, mu, nu)
            A += np.einsum("st,...ab->...satb", sigma_munu(mu, nu), F)
    A *= 1j * csw / 4.0
    return A.reshape(dims + (12, 12))


def clover_blocks(A12):
    """The two 6x6 chirality blocks of a chirality-block-diagonal 12x12 matrix.
    Block 0 = spins 0,1 (gamma5 = -1), block 1 = spins 2,3 (gamma5 = +1);
    6-index = 3*(spin mod 2) + colour.  Shape [..., 2, 6, 6]."""
    return np.stack([A12[..., 0:6, 0:6], A12[..., 6:12, 6:12]], axis=-3)


def clover_from_blocks(Ab):
    """Inverse of clover_blocks: [...,2,6,6] -> [...,12,12]."""
    out = np.zeros(Ab.shape[:-3] + (12, 12), dtype=np.complex128)
    out[..., 0:6, 0:6] = Ab[..., 0, :, :]
    out[..., 6:12, 6:12] = Ab[..., 1, :, :]
    return out


# ----------------------------------------------------------------------------
# operator
# ----------------------------------------------------------------------------

def boundary_phase_links(U, theta):
    """Links that carry twisted boundary conditions psi(x + L_mu e_mu) =
    exp(i theta_mu) psi(x) (Sec. 2) on the periodic lattice: the forward hop
    from x_mu = L_mu - 1 reads psi(0) and must see exp(i theta_mu) psi(0), so
    U_mu(x) at x_mu = L_mu - 1 takes that factor (and the backward hop from
    x_mu = 0, through U^dag, its inverse)."""
    U = np.array(U, dtype=np.complex128, copy=True)
    for mu in range(4):
        idx = [slice(None)] * 4
        idx[mu] = -1
        U[tuple(idx) + (mu,)] *= np.exp(1j * theta[mu])
    return U


class WilsonClover:
    """D(mu) = D_W + i mu Gamma5 on a periodic lattice, or with twisted
    boundary conditions (theta, per direction T,Z,Y,X).

    U      links [T,Z,Y,X,4,3,3]
    kappa  hopping parameter (m0 = 1/(2 kappa) - 4)
    csw    clover coefficient (ignored if `clover` is given)
    mu     twisted mass (mass normalisation); with mu_odd, the twist of the
           even sites
    clover optional clover term [T,Z,Y,X,2,6,6] (A only, without m0+4)
    theta  optional boundary phases; the clover term is built from the
           unphased links (closed loops do not see the phases)
    mu_odd optional twist of the odd sites (Sec. 2: the library takes a
           different twisted mass on even and odd sites, which the Hasenbusch
           terms of Sec. 3.1 need): D = D_W + i mu(x) Gamma5 with mu(x) = mu
           on even and mu_odd on odd sites (parity of the coordinate sum).
           An explicit `mu` argument of the methods below overrides the
           twist with that one value on every site.
    """

    def __init__(self, U, kappa: float, csw: float, mu: float, clover=None, theta=None, mu_odd=None):
        self.U = np.asarray(U, dtype=np.complex128)
        self.dims = self.U.shape[:4]
        self.m0 = m0_from_kappa(kappa)
        self.mu = float(mu)
        self.mu_odd = None if mu_odd is None else float(mu_odd)
        if clover is None:
            self.A = clover_matrix(self.U, csw)
        else:
            self.A = clover_from_blocks(np.asarray(clover, dtype=np.complex128))
        if theta is not None:
            self.U = boundary_phase_links(self.U, theta)

    # --- twist ----------------------------------------------------------------
    def twist(self, mu=None):
        """The twisted mass of every site: the given value, the one twist, or
        with mu_odd the field mu(x) [T,Z,Y,X]."""
        if mu is not None:
            return float(mu)
        if self.mu_odd is None:
            return self.mu
        return self.mu + (self.mu_odd - self.mu) * odd_mask(self.dims)

    def mean_twist(self) -> float:
        """(mu_even + mu_odd) / 2: the twist the coarse levels carry."""
        return self.mu if self.mu_odd is None else 0.5 * (self.mu + self.mu_odd)

    # --- pieces -------------------------------------------------------------
    def hop(self, psi):
        """-1/2 sum_mu [(1-g_mu) U_mu(x) psi(x+mu) + (1+g_mu) U_mu(x-mu)^dag psi(x-mu)]."""
        out = np.zeros_like(psi)
        for mu in range(4):
            fwd = colour_mul(self.U[..., mu, :, :], _shift(psi, mu, +1))
            Ub = _shift(self.U[..., mu, :, :], mu, -1)
            bwd = colour_mul(_dag(Ub), _shift(psi, mu, -1))
            out -= 0.5 * (fwd - spin_mul(GAMMA[mu], fwd) + bwd + spin_mul(GAMMA[mu], bwd))
        return out

    def site(self, psi, mu=None):
        """T(x) psi(x) = (m0+4) psi + A psi + i mu gamma5 psi."""
        t = self.twist(mu)
        t = t[..., None, None] if np.ndim(t) else t
        flat = psi.reshape(psi.shape[:-2] + (12,))
        a = np.einsum("...ij,...j->...i", self.A, flat).reshape(psi.shape)
        return (self.m0 + 4.0) * psi + a + 1j * t * spin_mul(GAMMA5, psi)

    def site_matrix(self, mu=None):
        """T(x) as a 12x12 matrix per site."""
        t = self.twist(mu)
        t = t[..., None, None] if np.ndim(t) else t
        g5 = np.kron(GAMMA5, np.eye(3))
        return self.A + (self.m0 + 4.0) * np.eye(12) + 1j * t * g5

    def site_inv(self, psi, mu=None):
        """T(x)^{-1} psi(x) by a direct solve per site."""
        T = self.site_matrix(mu)
        flat = psi.reshape(psi.shape[:-2] + (12,))
        return np.linalg.solve(T, flat[..., None])[..., 0].reshape(psi.shape)

    # --- full operators -------------------------------------------------------
    def apply(self, psi, mu=None):
        """D(mu) psi.  Pass mu=-self.mu for D(-mu), mu=0 for D_W."""
        return self.site(psi, mu) + self.hop(psi)

    def apply_w(self, psi):
        return self.apply(psi, 0.0)

    def dense(self, mu=None):
        """Dense matrix of D(mu) (tiny lattices only); column index = site*12+comp."""
        V = int(np.prod(self.dims))
        n = V * 12
        M = np.zeros((n, n), dtype=np.complex128)
        e = np.zeros(self.dims + (4, 3), dtype=np.complex128)
        ef = e.reshape(-1)
        for k in range(n):
            ef[:] = 0
            ef[k] = 1
            M[:, k] = self.apply(e, mu).reshape(-1)
        return M


def gamma5_field(psi):
    """Gamma5 psi (spin index second-to-last)."""
    return spin_mul(GAMMA5, psi)


def odd_mask(dims):
    """1.0 on the odd sites (sum of the coordinates odd), 0.0 on the even ones."""
    return (np.indices(tuple(dims)).sum(axis=0) % 2).astype(np.float64)


def apply_odd_shifted(op, psi, rho: float, mu=None):
    """D(mu; rho) psi: D(mu) with the twist of the odd sites raised by rho
    (Sec. 3.1: the Hasenbusch-shifted operators carry an extra i rho Gamma5
    on one parity)."""
    m = odd_mask(op.dims)[..., None, None]
    return op.apply(psi, mu) + 1j * rho * m * spin_mul(GAMMA5, psi)


def schur_odd(op, psi, rho: float = 0.0, mu=None):
    """(Dhat(mu) + i rho Gamma5hat) psi_o with Dhat = D_oo - D_oe D_ee^-1 D_eo,
    the odd-site reduced operator (Sec. 3.1).  psi is a full-lattice field whose
    even sites are ignored; the result is zero on the even sites.  Hops link
    opposite parities only, so D_ee and D_oo are the site terms."""
    m = odd_mask(op.dims)[..., None, None]
    xo = m * psi
    t = (1.0 - m) * op.hop(xo)              # D_eo x_o
    u = (1.0 - m) * op.site_inv(t, mu)      # D_ee^-1 D_eo x_o
    w = m * op.hop(u)                       # D_oe D_ee^-1 D_eo x_o
    return m * op.site(xo, mu) + 1j * rho * m * spin_mul(GAMMA5, xo) - w


def plane_wave_symbol(p, m0: float, mu: float):
    """Closed form of D(mu) on psi(x) = exp(i p.x) u in the free field (U = 1):
    m0 + sum_mu (1 - cos p_mu) + i sum_mu gamma_mu sin p_mu + i mu gamma5.
    p is indexed by direction (T,Z,Y,X)."""
    M = (m0 + sum(1.0 - np.cos(pm) for pm in p)) * np.eye(4, dtype=np.complex128)
    for d in range(4):
        M = M + 1j * np.sin(p[d]) * GAMMA[d]
    return M + 1j * mu * GAMMA5


def apply_at_sites(U, psi, kappa, csw, mu, sites):
    """(D(mu) psi)(x) at a few sites of an arbitrarily large lattice.

    For each site the 3^4 neighbourhood (offsets -1..1 in every direction,
    periodic in the big lattice) of links and spinors is gathered and the
    operator is applied on that patch; at the patch centre every term of D
    (site term with its clover leaves, the eight hops) only touches sites
    inside the patch, so the centre value is the exact one.  U and psi may
    be numpy arrays or anything indexable the same way (e.g. memory maps).
    """
    dims = U.shape[:4]
    out = []
    for x in sites:
        idx = [np.array([(x[d] + o) % dims[d] for o in (-1, 0, 1)]) for d in range(4)]
        ix = np.ix_(*idx)
        Up = np.asarray(U[ix])
        pp = np.asarray(psi[ix])
        op = WilsonClover(Up, kappa, csw, mu)
        out.append(op.apply(pp)[1, 1, 1, 1])
    return np.stack(out)


def apply_t_slab(U, psi, kappa, csw, mu, t0, nt):
    """(D(mu) psi)(x) for the time slices t0 .. t0+nt-1 of a lattice of any size.

    The slices t0-1 .. t0+nt (periodic in T) of the links and the spinor are
    gathered and the operator is applied on that slab with its own periodic
    T extent nt+2; on the nt inner slices every term of D (the site term with
    its clover leaves, which reach one slice either way, and the eight hops)
    only touches slices of the slab, so they are the exact values.  Returns
    [nt, Z, Y, X, 4, 3].  U and psi may be any arrays indexable by a list of
    time slices (numpy arrays, memory maps)."""
    T = U.shape[0]
    rows = [(t0 + k) % T for k in range(-1, nt + 1)]
    Us = np.asarray(U[rows])
    ps = np.asarray(psi[rows])
    return WilsonClover(Us, kappa, csw, mu).apply(ps)[1:nt + 1]

