"""Galerkin coarse operator and the coarsest-level odd-even solve.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Paper, Sec. 1: D_c = P^dag D_W P (Eq. 1 context); with a Gamma5-compatible P
the twist stays diagonal, D_c(mu) = D_c + i mu Gamma5,c; on the coarsest grid
the twist is raised to mu_coarse = delta * mu with delta >= 1.  Sec. 2/3:
odd-even preconditioning is used on the coarsest level.

Assembly (stencil form, same as oracle.stencil):
  S_c(A)    = sum_{x in A} Q(x)^dag S(x) Q(x)
              + sum_{links x->x+mu inside A} [ X + Gamma5,c X^dag Gamma5,c ],
                X = Q(x)^dag F_mu(x) Q(x+mu)
  F_c,mu(A) = sum_{x in A, x+mu in A+mu} Q(x)^dag F_mu(x) Q(x+mu)
where Q(x) is the n x 2Nv matrix of P restricted to site x.  A link is
"inside A" when x is not on the upper mu-face of A; upper-face links always
go to F_c,mu (even when the coarse extent is 1 or 2, in which case A+mu may be
A-mu or A itself: forward and backward couplings are kept apart and summed
by the apply).

Reading on delta (paper says "on the coarsest grid"): mu_l = mu on
intermediate levels, delta*mu on the coarsest.

Pins: equality with brute force P^dag D(mu_c) P column by column, the
free-field closed form with constant test vectors, Gamma5,c hermiticity,
D_c(mu) - D_c(0) = i mu Gamma5,c, gauge invariance.
"""
from __future__ import annotations

import numpy as np

from . import aggregation as agg
from .stencil import Stencil, gamma5_diag


def _Qsite(Q):
    """Q[Nv,T,Z,Y,X,n] -> per-site interpolation blocks [T,Z,Y,X,n,2Nv]."""
    Nv = Q.shape[0]
    n = Q.shape[-1]
    q = np.moveaxis(Q, 0, -1)                 # [dims, n, Nv]
    out = np.zeros(q.shape[:-1] + (2 * Nv,), dtype=np.complex128)
    out[..., : n // 2, :Nv] = q[..., : n // 2, :]
    out[..., n // 2:, Nv:] = q[..., n // 2:, :]
    return out


def _dag(M):
    return np.conj(np.swapaxes(M, -1, -2))


def _block_sum(f, dims, bsize):
    """Sum a per-site quantity [dims, a, b] over each aggregate -> [cdims, a, b]."""
    shp = []
    for d, b in zip(dims, bsize):
        shp += [d // b, b]
    g = f.reshape(tuple(shp) + f.shape[4:])
    return g.sum(axis=(1, 3, 5, 7))


def assemble(st: Stencil, Q, bsize, mu_c: float) -> Stencil:
    """D_c(mu_c) = P^dag D P in stencil form (blocks per coarse site)."""
    dims = st.dims
    Nv = Q.shape[0]
    g5c = gamma5_diag(2 * Nv)
    Qs = _Qsite(Q)
    Qd = _dag(Qs)
    coords = np.indices(dims)
    S_site = Qd @ st.S @ Qs
    dmu = getattr(st, "dmu", None)
    if dmu is not None:
        # the site-dependent part of the twist, i dmu(x) Gamma5, enters the
        # coarse site term as its Galerkin product (mu_c carries the mean)
        S_site = S_site + 1j * dmu[..., None, None] * (Qd @ (st.g5[:, None] * Qs))
    X = np.zeros_like(S_site)
    Fc = []
    for mu in range(4):
        W = Qd @ st.F[mu] @ np.roll(Qs, -1, axis=mu)         # Q(x)^dag F Q(x+mu)
        upper = (coords[mu] % bsize[mu]) == bsize[mu] - 1
        X = X + W * (~upper)[..., None, None]
        Fc.append(_block_sum(W * upper[..., None, None], dims, bsize))
    Xc = _block_sum(X, dims, bsize)
    Sc = _block_sum(S_site, dims, bsize) + Xc + g5c[:, None] * _dag(Xc) * g5c[None, :]
    return Stencil(Sc, np.stack(Fc), mu_c)


def brute_force(level_op, Q, bsize, mu_c):
    """Dense P^dag D(mu_c) P by applying D to every prolongated coarse unit
    vector (tiny lattices only); mu_c None applies the operator's own twist
    (which may differ between the parities)."""
    dims = level_op.dims
    Nv = Q.shape[0]
    cd = agg.coarse_dims(dims, bsize)
    nc = int(np.prod(cd)) * 2 * Nv
    M = np.zeros((nc, nc), dtype=np.complex128)
    e = np.zeros(cd + (2 * Nv,), dtype=np.complex128)
    ef = e.reshape(-1)
    for k in range(nc):
        ef[:] = 0
        ef[k] = 1
        y = level_op.apply(agg.prolong(Q, e, bsize), mu_c)
        M[:, k] = agg.restrict(Q, y, bsize).reshape(-1)
    return M


# ----------------------------------------------------------------------------
# odd-even reduced coarsest-level system
# ----------------------------------------------------------------------------

def parity(dims):
    return np.indices(dims).sum(axis=0) % 2


class OddEven:
    """Schur complement on even sites, S = D_ee - D_eo D_oo^{-1} D_oe.

    D_ee, D_oo are the (block-diagonal) site terms including the twist.  Needs
    even extents in every direction so that hops connect opposite parities."""

    def __init__(self, st: Stencil):
        for d in st.dims:
            if d % 2:
                raise ValueError("odd-even needs even coarse extents")
        self.st = st
        self.par = parity(st.dims)
        self.E = (self.par == 0)[..., None]
        self.O = (self.par == 1)[..., None]

    def schur(self, v):
        st = self.st
        v = v * self.E
        w = self.O * st.site_inv(self.O * st.hop(v))
        return self.E * (st.site(v) - st.hop(w))

    def rhs(self, b):
        """b_e - D_eo D_oo^{-1} b_o."""
        st = self.st
        return self.E * (b - st.hop(self.O * st.site_inv(b * self.O)))

    def reconstruct(self, x_e, b):
        """x = x_e + D_oo^{-1} (b_o - D_oe x_e)."""
        st = self.st
        x_e = x_e * self.E
        x_o = self.O * st.site_inv(self.O * (b - st.hop(x_e)))
        return x_e + x_o
