"""Seeded synthetic inputs shared by the GPU path's tests/bench and the CPU oracle.

This module holds input generation only: SU(3) gauge fields, Gaussian complex
fields, Haar-random gauge transformations.  It contains none of the method's
arithmetic (no Dirac operator, no smoother, no aggregation), so both sides of
a parity test may draw their inputs from here without sharing any code path.

Array conventions (host side), lattice axes ordered (T, Z, Y, X):
  links   complex128 [T, Z, Y, X, 4, 3, 3], link direction 0:T 1:Z 2:Y 3:X
  spinor  complex128 [T, Z, Y, X, 4, 3]     (spin, colour)
"""
from __future__ import annotations

import numpy as np

# Gell-Mann matrices, the standard basis of traceless Hermitian 3x3 matrices.
_GM = np.zeros((8, 3, 3), dtype=np.complex128)
_GM[0][0, 1] = _GM[0][1, 0] = 1
_GM[1][0, 1] = -1j
_GM[1][1, 0] = 1j
_GM[2][0, 0], _GM[2][1, 1] = 1, -1
_GM[3][0, 2] = _GM[3][2, 0] = 1
_GM[4][0, 2] = -1j
_GM[4][2, 0] = 1j
_GM[5][1, 2] = _GM[5][2, 1] = 1
_GM[6][1, 2] = -1j
_GM[6][2, 1] = 1j
_GM[7][0, 0] = _GM[7][1, 1] = 1 / np.sqrt(3)
_GM[7][2, 2] = -2 / np.sqrt(3)


def su3_near_identity(n: int, eps: float, rng: np.random.Generator, chunk: int = 1 << 22) -> np.ndarray:
    """n matrices U = exp(i*eps*H), H = sum_a h_a lambda_a / 2 with h_a ~ N(0,1).

    The matrix exponential is taken in FP64 with torch.matrix_exp on the CPU
    (batched, multithreaded) in fixed-size chunks, so a field is a pure
    function of (n, eps, seed).  exp of a traceless Hermitian matrix times i
    lies in SU(3) up to rounding; the determinant phase is divided out.
    """
    import torch

    out = np.empty((n, 3, 3), dtype=np.complex128)
    for a in range(0, n, chunk):
        m = min(chunk, n - a)
        h = rng.standard_normal((m, 8))
        H = np.einsum("na,aij->nij", h, _GM) * 0.5
        U = torch.matrix_exp(torch.from_numpy(1j * eps * H)).numpy()
        det = (U[:, 0, 0] * (U[:, 1, 1] * U[:, 2, 2] - U[:, 1, 2] * U[:, 2, 1])
               - U[:, 0, 1] * (U[:, 1, 0] * U[:, 2, 2] - U[:, 1, 2] * U[:, 2, 0])
               + U[:, 0, 2] * (U[:, 1, 0] * U[:, 2, 1] - U[:, 1, 1] * U[:, 2, 0]))
        out[a:a + m] = U / (det ** (1.0 / 3.0))[:, None, None]
    return out


def gauge_field(dims, eps: float, seed: int) -> np.ndarray:
    """Links U_mu(x) for a lattice dims=(T,Z,Y,X), shape [T,Z,Y,X,4,3,3]."""
    dims = tuple(int(d) for d in dims)
    rng = np.random.default_rng(seed)
    V = int(np.prod(dims))
    U = su3_near_identity(V * 4, eps, rng)
    return U.reshape(dims + (4, 3, 3))


def gaussian(shape, seed: int) -> np.ndarray:
    """Complex Gaussian field, N(0,1) independently on real and imaginary parts."""
    rng = np.random.default_rng(seed)
    shape = tuple(int(s) for s in shape)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def spinor(dims, seed: int, nvec: int | None = None) -> np.ndarray:
    """Gaussian spinor field(s): [T,Z,Y,X,4,3] or [nvec,T,Z,Y,X,4,3]."""
    dims = tuple(int(d) for d in dims)
    shape = dims + (4, 3) if nvec is None else (nvec,) + dims + (4, 3)
    return gaussian(shape, seed)


def haar_su3(n: int, rng: np.random.Generator) -> np.ndarray:
    """n Haar-distributed SU(3) matrices (QR of a complex Gaussian, phase fixed)."""
    z = rng.standard_normal((n, 3, 3)) + 1j * rng.standard_normal((n, 3, 3))
    q, r = np.linalg.qr(z)
    d = np.diagonal(r, axis1=1, axis2=2)
    q = q * (d / np.abs(d))[:, None, :]
    det = np.linalg.det(q)
    return q / (det ** (1.0 / 3.0))[:, None, None]


def gauge_transform(dims, seed: int) -> np.ndarray:
    """A random gauge transformation Omega(x) in SU(3), shape [T,Z,Y,X,3,3]."""
    dims = tuple(int(d) for d in dims)
    rng = np.random.default_rng(seed)
    return haar_su3(int(np.prod(dims)), rng).reshape(dims + (3, 3))


def transform_links(U: np.ndarray, Om: np.ndarray) -> np.ndarray:
    """U^Omega_mu(x) = Omega(x) U_mu(x) Omega(x+mu)^dagger (periodic lattice)."""
    out = np.empty_like(U)
    for mu in range(4):
        Om_fwd = np.roll(Om, -1, axis=mu)
        out[..., mu, :, :] = Om @ U[..., mu, :, :] @ np.conj(np.swapaxes(Om_fwd, -1, -2))
    return out


def transform_spinor(psi: np.ndarray, Om: np.ndarray) -> np.ndarray:
    """(Omega psi)(x) acting on colour; psi has shape [..., T,Z,Y,X,4,3]."""
    return np.einsum("...ab,...sb->...sa", Om, psi)


def mean_plaquette(U: np.ndarray) -> float:
    """Average of Re tr(U_mu U_nu U_mu^dag U_nu^dag)/3 over sites and planes."""
    acc = 0.0
    n = 0
    for mu in range(4):
        for nu in range(mu + 1, 4):
            Umu = U[..., mu, :, :]
            Unu = U[..., nu, :, :]
            P = Umu @ np.roll(Unu, -1, axis=mu) @ np.conj(np.swapaxes(np.roll(Umu, -1, axis=nu), -1, -2)) \
                @ np.conj(np.swapaxes(Unu, -1, -2))
            acc += np.trace(P, axis1=-2, axis2=-1).real.mean() / 3.0
            n += 1
    return acc / n


# ----------------------------------------------------------------------------
# device-side generators (torch, seeded CUDA generator): the same distributions
# for lattices whose host-side generation would take minutes (48^3 x 96 test
# vectors are tens of GB).  Deterministic for a given (shape, seed, device).

def gaussian_device(shape, seed: int, device="cuda", dtype="complex128"):
    """Complex Gaussian field (N(0,1) real and imaginary parts) drawn on the
    device with a seeded torch generator; dtype complex128 or complex64."""
    import torch

    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    shape = tuple(int(s) for s in shape)
    rt = torch.float64 if dtype == "complex128" else torch.float32
    re = torch.randn(shape, generator=gen, device=device, dtype=rt)
    im = torch.randn(shape, generator=gen, device=device, dtype=rt)
    return torch.complex(re, im)


def gauge_field_device(dims, eps: float, seed: int, device="cuda", chunk: int = 1 << 22):
    """Links exp(i eps H) with H = sum_a h_a lambda_a / 2, h_a ~ N(0,1), computed
    on the device in chunks; shape [T,Z,Y,X,4,3,3] complex128."""
    import torch

    dims = tuple(int(d) for d in dims)
    n = int(np.prod(dims)) * 4
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    gm = torch.from_numpy(_GM).to(device)
    out = torch.empty((n, 3, 3), dtype=torch.complex128, device=device)
    for a in range(0, n, chunk):
        m = min(chunk, n - a)
        h = torch.randn((m, 8), generator=gen, device=device, dtype=torch.float64).to(torch.complex128)
        H = torch.einsum("na,aij->nij", h, gm) * 0.5
        U = torch.linalg.matrix_exp(1j * eps * H)
        det = torch.linalg.det(U)
        out[a:a + m] = U / (det ** (1.0 / 3.0))[:, None, None]
    return out.reshape(dims + (4, 3, 3))


def net_init_weights(C: int, nlayers: int, seed: int, scale: float = 1.0):
    """Seeded initial weights of the gauge-covariant network (an input to both
    the GPU kernels and the oracle): W_{d,c,c'} complex Gaussian scaled by
    scale/sqrt(2*9*C*4), the identity offset shifted by 0.5 * identity in
    channel and spin; gates a = 0, b = 0.  Shapes: W [9, C, C, 4, 4]."""
    rng = np.random.default_rng(seed)
    W, a, b = [], [], []
    for l in range(nlayers):
        w = rng.standard_normal((9, C, C, 4, 4)) + 1j * rng.standard_normal((9, C, C, 4, 4))
        w *= scale / np.sqrt(2.0 * 9 * C * 4)
        w[0] += np.einsum("cp,st->cpst", np.eye(C), np.eye(4)) * 0.5
        W.append(w)
        if l < nlayers - 1:
            a.append(np.zeros(C))
            b.append(np.zeros(C))
    return W, a, b
