"""Gamma5-compatible aggregation: interpolation P and restriction P^dagger.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Paper, Sec. 1: P is built by aggregating N_v test vectors v_i over small
blocks (local coherence) and is Gamma5-compatible, Gamma5 P = P Gamma5,c.
Sec. 2: standard aggregates are 4^4 (fine -> first coarse) and 2^4 (first ->
second coarse).  Reading taken here (paper silent on the construction):

  * an aggregate is a block A of sites times one chirality half s: s = 0 holds
    the first n/2 components of a site (fine: spins 0,1, gamma5 = -1), s = 1
    the last n/2 (spins 2,3, gamma5 = +1);
  * for each (A, s) the restricted test vectors form a matrix V_{A,s} (rows:
    sites of A x components of half s, columns: v_1..v_Nv); its thin QR
    factorisation V = Q R with real positive diag(R) gives the columns of P
    on that aggregate (unique for full-rank V);
  * coarse dof at aggregate A: index s*N_v + i, so Gamma5,c = diag(-1_Nv, +1_Nv).

Fields are [T,Z,Y,X,n]; test vectors [Nv,T,Z,Y,X,n]; coarse fields
[Tc,Zc,Yc,Xc,2Nv].  P itself is stored as the orthonormalised test vectors Q
with the same shape as the test vectors.

Pins: P^dag P = I, Gamma5 P = P Gamma5,c, V = Q R with R upper triangular and
positive diagonal, P P^dag is an orthogonal projector (tests/test_oracle_mg.py).
"""
from __future__ import annotations

import numpy as np


def coarse_dims(dims, bsize):
    return tuple(d // b for d, b in zip(dims, bsize))


def _to_blocks(f, dims, bsize):
    """[..., T,Z,Y,X, n] -> [..., Tc,Zc,Yc,Xc, bT,bZ,bY,bX, n]."""
    lead = f.shape[: f.ndim - 5]
    n = f.shape[-1]
    shp = []
    for d, b in zip(dims, bsize):
        shp += [d // b, b]
    g = f.reshape(lead + tuple(shp) + (n,))
    k = len(lead)
    perm = list(range(k)) + [k + 0, k + 2, k + 4, k + 6, k + 1, k + 3, k + 5, k + 7, k + 8]
    return g.transpose(perm)


def _from_blocks(g, dims):
    """Inverse of _to_blocks."""
    lead = g.shape[: g.ndim - 9]
    k = len(lead)
    perm = list(range(k)) + [k + 0, k + 4, k + 1, k + 5, k + 2, k + 6, k + 3, k + 7, k + 8]
    h = g.transpose(perm)
    return h.reshape(lead + tuple(dims) + (g.shape[-1],))


def _aggregate_matrices(V, dims, bsize):
    """Test vectors [Nv,T,Z,Y,X,n] -> per-aggregate-half matrices
    [Tc,Zc,Yc,Xc, 2, rows, Nv] with rows = block sites x n/2."""
    Nv = V.shape[0]
    n = V.shape[-1]
    B = _to_blocks(V, dims, bsize)  # [Nv, Tc..Xc, bT..bX, n]
    cd = B.shape[1:5]
    bs = int(np.prod(bsize))
    B = B.reshape((Nv,) + cd + (bs, 2, n // 2))          # split comps into halves
    B = np.moveaxis(B, 0, -1)                             # [cd, bs, 2, n/2, Nv]
    B = np.moveaxis(B, -4, -3)                            # [cd, 2, bs, n/2, Nv]
    return B.reshape(cd + (2, bs * (n // 2), Nv))


def _from_aggregate_matrices(M, dims, bsize, n):
    cd = M.shape[:4]
    Nv = M.shape[-1]
    bs = int(np.prod(bsize))
    B = M.reshape(cd + (2, bs, n // 2, Nv))
    B = np.moveaxis(B, -4, -3)                            # [cd, bs, 2, n/2, Nv]
    B = np.moveaxis(B, -1, 0)                             # [Nv, cd, bs, 2, n/2]
    B = B.reshape((Nv,) + cd + tuple(bsize) + (n,))
    return _from_blocks(B, dims)


def orthonormalise(V, bsize):
    """Q with Q_{A,s} R_{A,s} = V_{A,s}, diag(R) real positive, for every
    aggregate half.  Raises ValueError on a rank-deficient aggregate."""
    dims = V.shape[1:5]
    n = V.shape[-1]
    M = _aggregate_matrices(V, dims, bsize)
    Q, R = np.linalg.qr(M)                    # Householder QR (LAPACK)
    d = np.diagonal(R, axis1=-2, axis2=-1)
    if np.any(np.abs(d) <= 1e-12 * np.linalg.norm(M, axis=(-2, -1))[..., None]):
        raise ValueError("rank-deficient aggregate")
    ph = d / np.abs(d)
    Q = Q * ph[..., None, :]
    return _from_aggregate_matrices(Q, dims, bsize, n)


def qr_factors(V, bsize):
    """(Q, R) per aggregate half, with the positive-diagonal convention."""
    dims = V.shape[1:5]
    M = _aggregate_matrices(V, dims, bsize)
    Q, R = np.linalg.qr(M)
    d = np.diagonal(R, axis1=-2, axis2=-1)
    ph = d / np.abs(d)
    return Q * ph[..., None, :], np.conj(ph)[..., :, None] * R


def restrict(Q, r, bsize):
    """P^dag r: (r_c)_{A, s*Nv+i} = sum over aggregate-half rows conj(Q_i) r."""
    dims = Q.shape[1:5]
    n = Q.shape[-1]
    Nv = Q.shape[0]
    Qb = _to_blocks(Q, dims, bsize)                       # [Nv, cd, bs..., n]
    rb = _to_blocks(r, dims, bsize)                       # [cd, bs..., n]
    prod = np.conj(Qb) * rb[None]
    s0 = prod[..., : n // 2].sum(axis=(-5, -4, -3, -2, -1))
    s1 = prod[..., n // 2:].sum(axis=(-5, -4, -3, -2, -1))
    return np.concatenate([np.moveaxis(s0, 0, -1), np.moveaxis(s1, 0, -1)], axis=-1)


def prolong(Q, e, bsize):
    """P e_c: x = sum_i Q_i e_c(A, s(comp)*Nv + i)."""
    dims = Q.shape[1:5]
    n = Q.shape[-1]
    Nv = Q.shape[0]
    Qb = _to_blocks(Q, dims, bsize)                       # [Nv, cd, bs..., n]
    e0 = np.moveaxis(e[..., :Nv], -1, 0)                  # [Nv, cd]
    e1 = np.moveaxis(e[..., Nv:], -1, 0)
    ex = (slice(None),) * 5 + (None,) * 4
    x0 = (Qb[..., : n // 2] * e0[ex][..., None]).sum(axis=0)
    x1 = (Qb[..., n // 2:] * e1[ex][..., None]).sum(axis=0)
    xb = np.concatenate([x0, x1], axis=-1)
    return _from_blocks(xb, dims)


def dense_P(Q, bsize):
    """Dense interpolation matrix (tiny lattices): columns = coarse unit vectors."""
    dims = Q.shape[1:5]
    Nv = Q.shape[0]
    cd = coarse_dims(dims, bsize)
    nc = int(np.prod(cd)) * 2 * Nv
    cols = []
    e = np.zeros(cd + (2 * Nv,), dtype=np.complex128)
    ef = e.reshape(-1)
    for k in range(nc):
        ef[:] = 0
        ef[k] = 1
        cols.append(prolong(Q, e, bsize).reshape(-1))
    return np.stack(cols, axis=1)
