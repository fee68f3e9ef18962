"""Gauge-covariant parallel-transport network proposing the setup's test vectors.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Not a method of the paper: the paper's adaptive setup (Sec. 1) starts from
random test vectors; this network replaces that random start, and the plain
adaptive setup stays the fallback.  Definition (FP64 here):

  input  x^0_c(x), c = 1..C: C spin(4) x colour(3) fields (Gaussian noise)
  layer  z_c(x) = sum_{d=0..8} sum_{c'} W_{d,c,c'} (T_d x_{c'})(x)
           T_0 = 1, T_{+mu} x(x) = U_mu(x) x(x+mu), T_{-mu} x(x) = U_mu(x-mu)^dag x(x-mu)
           W_{d,c,c'} is a 4x4 complex spin matrix (acts on spin, commutes with
           colour, so the layer is gauge covariant); no additive bias.
  gate   y_c(x) = z_c(x) * sigmoid(a_c |z_c(x)|^2 + b_c)  (|.| over spin and
           colour: gauge invariant); the last layer is not gated.
  output the C fields of the last layer -> block orthonormalisation -> P.

Offsets d: 0 identity, 1..4 forward T,Z,Y,X, 5..8 backward T,Z,Y,X.

Loss (invariant to the basis chosen inside each aggregate half):
  L = sum_{A,s} || (I - Pi_{Y_{A,s}}) Q*_{A,s} ||_F^2 / sum ||Q*_{A,s}||_F^2,
  Pi_Y = Y (Y^dag Y)^{-1} Y^dag,  Y_{A,s} = network output restricted to the
  aggregate half, Q* = orthonormal targets from the plain adaptive setup.

Gradients are the hand-derived adjoints (G = dL/dRe + i dL/dIm):
  loss   G_Y = -2 (I - Pi_Y) Q* C^dag G^{-1} / norm,  G = Y^dag Y, C = Y^dag Q*
  gate   G_z = s G_y + 2 t s' z,  t = Re <z, G_y>_{site,channel},
         s' = a s (1-s);  G_a = sum t s(1-s) |z|^2, G_b = sum t s(1-s)
  mixing G_W[d,c,c'] = sum_{x,colour} G_z[c] (T_d x_{c'})^dag (4x4 in spin),
         G_{T_d x}[c'] = sum_c W[d,c,c']^dag G_z[c]
  transport G_x = sum_d T_d^dag G_{T_d x}.
Pins (tests/test_oracle_net.py): central finite differences of every
parameter kind, exact gauge equivariance, loss = 0 for Y = Q*, invariance of
the loss under a change of basis inside an aggregate.
"""
from __future__ import annotations

import numpy as np

from . import aggregation as agg

NOFF = 9


def _dag(M):
    return np.conj(np.swapaxes(M, -1, -2))


def transport(U, x, d):
    """T_d applied to fields x[..., T,Z,Y,X, 4, 3] (leading channel axes allowed)."""
    if d == 0:
        return x
    mu = (d - 1) % 4
    lead = x.ndim - 6
    ax = lead + mu
    if d <= 4:
        xs = np.roll(x, -1, axis=ax)
        return np.einsum("...ab,...sb->...sa", U[..., mu, :, :], xs)
    Ub = np.roll(U[..., mu, :, :], 1, axis=mu)
    xs = np.roll(x, 1, axis=ax)
    return np.einsum("...ba,...sb->...sa", np.conj(Ub), xs)


def transport_adj(U, g, d):
    """T_d^dag applied to fields g (the adjoint of transport)."""
    if d == 0:
        return g
    mu = (d - 1) % 4
    lead = g.ndim - 6
    ax = lead + mu
    if d <= 4:
        # (T_{+mu} x)(x) = U(x) x(x+mu)  ->  (T^dag g)(y) = U(y-mu)^dag g(y-mu)
        Ub = np.roll(U[..., mu, :, :], 1, axis=mu)
        gs = np.roll(g, 1, axis=ax)
        return np.einsum("...ba,...sb->...sa", np.conj(Ub), gs)
    # (T_{-mu} x)(x) = U(x-mu)^dag x(x-mu)  ->  (T^dag g)(y) = U(y) g(y+mu)
    gs = np.roll(g, -1, axis=ax)
    return np.einsum("...ab,...sb->...sa", U[..., mu, :, :], gs)


def sigmoid(u):
    return 1.0 / (1.0 + np.exp(-u))


class Net:
    """W: list of arrays [9, C, C, 4, 4] complex; a, b: lists of [C] real
    (gates of layers 0..L-2)."""

    def __init__(self, W, a, b):
        self.W = [np.asarray(w, dtype=np.complex128) for w in W]
        self.a = [np.asarray(v, dtype=np.float64) for v in a]
        self.b = [np.asarray(v, dtype=np.float64) for v in b]

    @property
    def nlayers(self):
        return len(self.W)

    def forward(self, U, x0, keep=False):
        """x0: [C, T,Z,Y,X, 4, 3].  Returns the output (and the cache)."""
        x = x0
        cache = []
        for l, W in enumerate(self.W):
            TX = np.stack([transport(U, x, d) for d in range(NOFF)])   # [9, C', ..., 4, 3]
            z = np.einsum("dcpst,dp...tk->c...sk", W, TX)
            if l < self.nlayers - 1:
                n = np.sum(np.abs(z) ** 2, axis=(-2, -1))              # [C, dims]
                u = self.a[l][(slice(None),) + (None,) * 4] * n + self.b[l][(slice(None),) + (None,) * 4]
                s = sigmoid(u)
                y = z * s[..., None, None]
            else:
                n = s = None
                y = z
            if keep:
                cache.append((x, TX, z, n, s))
            x = y
        return (x, cache) if keep else x

    def backward(self, U, cache, G_out):
        """G_out = dL/dRe(y) + i dL/dIm(y) of the output.  Returns (G_W, G_a, G_b)."""
        GW = [None] * self.nlayers
        Ga = [None] * (self.nlayers - 1)
        Gb = [None] * (self.nlayers - 1)
        G = G_out
        for l in range(self.nlayers - 1, -1, -1):
            x, TX, z, n, s = cache[l]
            if l < self.nlayers - 1:
                t = np.real(np.sum(np.conj(G) * z, axis=(-2, -1)))     # [C, dims]
                sp = s * (1.0 - s)
                Gz = s[..., None, None] * G + (2.0 * t * self.a[l][(slice(None),) + (None,) * 4] * sp)[..., None, None] * z
                Ga[l] = np.sum(t * sp * n, axis=(1, 2, 3, 4))
                Gb[l] = np.sum(t * sp, axis=(1, 2, 3, 4))
            else:
                Gz = G
            nc = Gz.shape[0]
            Gz_r = Gz.reshape(nc, -1, 4, 3)
            TX_r = TX.reshape(TX.shape[0], TX.shape[1], -1, 4, 3)
            GW[l] = np.einsum("cvsk,dpvtk->dcpst", Gz_r, np.conj(TX_r))
            GTX = np.einsum("dcpst,c...sk->dp...tk", np.conj(self.W[l]), Gz)
            G = sum(transport_adj(U, GTX[d], d) for d in range(NOFF))
        return GW, Ga, Gb


def subspace_loss(Y, Qstar, bsize, grad=False):
    """Y, Qstar: [C, T,Z,Y,X, 12] (flat spin-colour).  Returns L (and G_Y)."""
    dims = Y.shape[1:5]
    My = agg._aggregate_matrices(Y, dims, bsize)      # [cd, 2, rows, C]
    Mq = agg._aggregate_matrices(Qstar, dims, bsize)
    G = _dag(My) @ My
    C = _dag(My) @ Mq
    Ginv_C = np.linalg.solve(G, C)
    proj = My @ Ginv_C                                  # Pi_Y Q*
    R = Mq - proj
    norm = np.sum(np.abs(Mq) ** 2)
    L = np.sum(np.abs(R) ** 2) / norm
    if not grad:
        return L
    Ginv = np.linalg.inv(G)
    GY = -2.0 * (R @ _dag(C) @ Ginv) / norm
    GYf = agg._from_aggregate_matrices(GY, dims, bsize, Y.shape[-1])
    return L, GYf
