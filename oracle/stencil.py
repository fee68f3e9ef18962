"""Generic nearest-neighbour block stencil on a periodic 4D lattice.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Every level of the hierarchy is a stencil of this form (fine level: n = 12
spin-colour components; coarse levels: n = 2 N_v):

  (D y)(x) = S(x) y(x) + i mu Gamma5 y(x)
             + sum_mu [ F_mu(x) y(x+mu) + Gamma5 F_mu(x-mu)^dag Gamma5 y(x-mu) ]

with Gamma5 = diag(-1 (n/2 times), +1 (n/2 times)).  The backward blocks are
the Gamma5-conjugate transposes of the forward ones, which is how Gamma5
hermiticity D^dag = Gamma5 D Gamma5 of the fine operator (Sec. 1) carries over
to the coarse operator (Sec. 1: D_c^dag = Gamma5,c D_c Gamma5,c).  The twist
i mu Gamma5 is stored apart from S, as in D_c(mu) = D_c + i mu Gamma5,c (Sec. 1).

Fields are arrays [T, Z, Y, X, n]; S is [T,Z,Y,X,n,n]; F is [4,T,Z,Y,X,n,n].
"""
from __future__ import annotations

import numpy as np

from . import dirac


def gamma5_diag(n: int) -> np.ndarray:
    return np.concatenate([-np.ones(n // 2), np.ones(n // 2)])


def _dag(M):
    return np.conj(np.swapaxes(M, -1, -2))


def _mv(M, y):
    return np.einsum("...ij,...j->...i", M, y)


class Stencil:
    """dmu (optional, [T,Z,Y,X] real): a site-dependent addition to the twist,
    i (mu + dmu(x)) Gamma5 (the fine level with different twists on the two
    parities: mu their mean, dmu = -+ half their difference).  An explicit
    `mu` argument of the methods below drops it."""

    def __init__(self, S, F, mu: float, dmu=None):
        self.S = np.asarray(S, dtype=np.complex128)
        self.F = np.asarray(F, dtype=np.complex128)
        self.dims = self.S.shape[:4]
        self.n = self.S.shape[-1]
        self.mu = float(mu)
        self.dmu = None if dmu is None else np.asarray(dmu, dtype=np.float64)
        self.g5 = gamma5_diag(self.n)

    def with_mu(self, mu: float) -> "Stencil":
        return Stencil(self.S, self.F, mu)

    def _twist(self, mu):
        if mu is not None or self.dmu is None:
            return self.mu if mu is None else mu
        return (self.mu + self.dmu)[..., None]

    def backward_block(self, mu: int):
        """B_mu(x) = Gamma5 F_mu(x-mu)^dag Gamma5, coupling x to x-mu."""
        Fb = np.roll(self.F[mu], 1, axis=mu)
        return self.g5[:, None] * _dag(Fb) * self.g5[None, :]

    def site(self, y, mu=None):
        return _mv(self.S, y) + 1j * self._twist(mu) * self.g5 * y

    def site_matrix(self, mu=None):
        t = self._twist(mu)
        return self.S + 1j * (t[..., None] if np.ndim(t) else t) * np.diag(self.g5)

    def site_inv(self, y, mu=None):
        return np.linalg.solve(self.site_matrix(mu), y[..., None])[..., 0]

    def hop(self, y):
        out = np.zeros_like(y)
        for mu in range(4):
            out += _mv(self.F[mu], np.roll(y, -1, axis=mu))
            out += _mv(self.backward_block(mu), np.roll(y, 1, axis=mu))
        return out

    def apply(self, y, mu=None):
        return self.site(y, mu) + self.hop(y)

    def dense(self, mu=None):
        n = int(np.prod(self.dims)) * self.n
        M = np.zeros((n, n), dtype=np.complex128)
        e = np.zeros(self.dims + (self.n,), dtype=np.complex128)
        ef = e.reshape(-1)
        for k in range(n):
            ef[:] = 0
            ef[k] = 1
            M[:, k] = self.apply(e, mu).reshape(-1)
        return M


def wilson_stencil(op: "dirac.WilsonClover") -> Stencil:
    """The fine operator written as a 12x12 block stencil:
    S(x) = (m0+4) + A(x), F_mu(x) = -1/2 (1 - gamma_mu) (x) U_mu(x); the twist
    as its mean over the parities plus the site-dependent rest."""
    dims = op.dims
    S = op.A + (op.m0 + 4.0) * np.eye(12)
    F = np.zeros((4,) + dims + (12, 12), dtype=np.complex128)
    for mu in range(4):
        P = -0.5 * (np.eye(4) - dirac.GAMMA[mu])
        F[mu] = np.einsum("st,...ab->...satb", P, op.U[..., mu, :, :]).reshape(dims + (12, 12))
    mean = op.mean_twist()
    dmu = None if op.mu_odd is None else op.twist() - mean
    return Stencil(S, F, mean, dmu)


class FineLevel:
    """Flat-vector view [T,Z,Y,X,12] of the explicit Wilson-clover operator."""

    def __init__(self, op: "dirac.WilsonClover"):
        self.op = op
        self.dims = op.dims
        self.n = 12
        self.mu = op.mu
        self.g5 = gamma5_diag(12)

    def _s(self, y):
        return y.reshape(y.shape[:-1] + (4, 3))

    def _f(self, y):
        return y.reshape(y.shape[:-2] + (12,))

    def apply(self, y, mu=None):
        return self._f(self.op.apply(self._s(y), mu))

    def site(self, y, mu=None):
        return self._f(self.op.site(self._s(y), mu))

    def site_inv(self, y, mu=None):
        return self._f(self.op.site_inv(self._s(y), mu))

    def hop(self, y):
        return self._f(self.op.hop(self._s(y)))
