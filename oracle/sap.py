"""Schwarz alternating procedure (SAP) smoother with block-local MR solves.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Paper: Sec. 1 names SAP as the smoother M of Eq. (1) that damps the UV modes;
Sec. 3 states that odd-even preconditioning is used in the smoother (and on
the coarsest level) only.  The paper gives no further detail, so the reading
taken here is the multiplicative Schwarz method with two colours:

  * the lattice is cut into blocks of size bsize (4 numbers, T,Z,Y,X); block
    colour = parity of the sum of block coordinates; an even number of blocks
    per direction is required (so that same-colour blocks never touch);
  * one SAP iteration:  for colour in (0, 1):
        r = b - D x;  for every block B of that colour: x_B += D_B^{-1} r_B
    where D_B = (restriction of D to B, hops leaving B dropped);
  * the block solve D_B^{-1} is approximate: on the fine level, n_MR minimal
    residual steps on the even-site Schur complement
        S = T_ee - D_eo T_oo^{-1} D_oe
    followed by the odd-site reconstruction; on coarse levels (schur=False)
    n_MR minimal residual steps on D_B itself.
  * MR step (Saad, Iterative Methods, Sec. 5.3.2):
        q = S rho;  alpha = <q,rho>/<q,q>;  e += alpha rho;  rho -= alpha q.
    A block with <q,q> = 0 takes alpha = 0.

All blocks of one colour are handled at once with masks; dot products are
summed per block.

Pins: brute-force dense Schur complement + MR on every block (tiny lattice),
exact block solves annihilate the residual on the just-solved colour,
gauge covariance of one SAP iteration.
"""
from __future__ import annotations

import numpy as np


def site_coords(dims):
    return np.indices(dims)  # [4, T, Z, Y, X]


def site_parity(dims):
    return site_coords(dims).sum(axis=0) % 2


def block_layout(dims, bsize):
    """(block id per site, colour per site, number of blocks)."""
    dims = tuple(dims)
    bsize = tuple(bsize)
    nb = [d // b for d, b in zip(dims, bsize)]
    for d, b in zip(dims, bsize):
        if d % b != 0:
            raise ValueError("lattice extent not divisible by block size")
    for n in nb:
        if n % 2 != 0:
            raise ValueError("SAP needs an even number of blocks per direction")
    c = site_coords(dims)
    bc = [c[i] // bsize[i] for i in range(4)]
    bid = ((bc[0] * nb[1] + bc[1]) * nb[2] + bc[2]) * nb[3] + bc[3]
    col = (bc[0] + bc[1] + bc[2] + bc[3]) % 2
    return bid, col, int(np.prod(nb))


def _block_sum(vals, bid, nblocks):
    """Sum of complex per-site values over each block."""
    re = np.bincount(bid.ravel(), weights=vals.real.ravel(), minlength=nblocks)
    im = np.bincount(bid.ravel(), weights=vals.imag.ravel(), minlength=nblocks)
    return re + 1j * im


def _mr(apply_S, rho, bid, nblocks, n_mr):
    e = np.zeros_like(rho)
    for _ in range(n_mr):
        q = apply_S(rho)
        qr = _block_sum(np.sum(np.conj(q) * rho, axis=-1), bid, nblocks)
        qq = _block_sum(np.sum(np.abs(q) ** 2, axis=-1), bid, nblocks).real
        alpha = np.where(qq > 0, qr / np.where(qq > 0, qq, 1.0), 0.0)
        a = alpha[bid][..., None]
        e = e + a * rho
        rho = rho - a * q
    return e


def block_solve(op, r, colour, bid, col, nblocks, n_mr, schur=True):
    """Approximate D_B^{-1} r_B on every block of the given colour (r may be
    nonzero elsewhere; only the colour's blocks are read and written)."""
    M = (col == colour)[..., None]
    if not schur:
        rho = r * M
        return _mr(lambda v: M * op.apply(v), rho, bid, nblocks, n_mr)
    par = site_parity(op.dims)
    E = M & (par == 0)[..., None]
    O = M & (par == 1)[..., None]
    r_e = r * E
    r_o = r * O
    # right-hand side of the Schur system: r_e - D_eo T_oo^{-1} r_o
    t_o = O * op.site_inv(r_o)
    rt = r_e - E * op.hop(t_o)

    def apply_S(v):
        w = O * op.site_inv(O * op.hop(v))
        return E * (op.site(v) - op.hop(w))

    e_e = _mr(apply_S, rt, bid, nblocks, n_mr)
    e_o = O * op.site_inv(r_o - O * op.hop(e_e))
    return e_e + e_o


def sap_iteration(op, b, x, bsize, n_mr, schur=True):
    """One SAP iteration (both colours) on D x = b; returns the new x."""
    bid, col, nblocks = block_layout(op.dims, bsize)
    x = x.copy()
    for colour in (0, 1):
        r = b - op.apply(x)
        x = x + block_solve(op, r, colour, bid, col, nblocks, n_mr, schur)
    return x


def sap(op, b, x, bsize, n_mr, iters, schur=True):
    for _ in range(iters):
        x = sap_iteration(op, b, x, bsize, n_mr, schur)
    return x
