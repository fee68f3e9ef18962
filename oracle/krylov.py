"""Krylov solvers: GMRES(m) and flexible GMRES(m), textbook form.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Paper, Sec. 1: a flexible Krylov method is preconditioned at every step by the
multigrid cycle of Eq. (1) (Fig. 3 caption: FGMRES).  The paper gives no
further detail; this follows Saad, "A flexible inner-outer preconditioned
GMRES algorithm" (1993) and Saad, Iterative Methods, Alg. 6.9/9.6:

  r0 = b - A x0, beta = |r0|, v1 = r0/beta
  for j = 1..m:  z_j = M(v_j);  w = A z_j   (GMRES: z_j = v_j)
                 orthogonalise w against v_1..v_j (classical Gram-Schmidt, twice)
                 h_{j+1,j} = |w|, v_{j+1} = w / h_{j+1,j}
                 apply the previous Givens rotations to column j, form the next
                 one, update the least-squares residual estimate |g_{j+1}|
  x = x0 + Z y with H y = g (upper-triangular solve);  restart from the true
  residual.

The vectors are arbitrary-shape complex arrays; inner products are summed
over all entries.  `tol` is relative to |b|; `fixed=True` runs exactly
max_iter iterations without testing the tolerance (deterministic
preconditioner for element-wise comparisons).

Pins: GMRES equals numpy.linalg.solve on small dense systems, FGMRES with the
identity preconditioner equals GMRES, residual estimates are non-increasing.
"""
from __future__ import annotations

import numpy as np


def _dot(a, b):
    return np.vdot(a, b)


def _norm(a):
    return float(np.sqrt(np.vdot(a, a).real))


def fgmres(A, b, M=None, x0=None, tol=1e-10, restart=10, max_iter=1000,
           fixed=False, true_residual=True):
    """Returns (x, info) with info = dict(iters, resid (relative, true),
    converged, history)."""
    if M is None:
        M = lambda v: v  # noqa: E731
    x = np.zeros_like(b) if x0 is None else x0.copy()
    bnorm = _norm(b)
    hist = []
    if bnorm == 0.0:
        return x, dict(iters=0, resid=0.0, converged=True, history=hist)
    it = 0
    r = b - A(x)
    beta = _norm(r)
    while True:
        if not fixed and beta <= tol * bnorm:
            break
        if it >= max_iter:
            break
        m = restart if not fixed else min(restart, max_iter - it)
        V = [r / beta]
        Z = []
        H = np.zeros((m + 1, m), dtype=np.complex128)
        cs = np.zeros(m)
        sn = np.zeros(m, dtype=np.complex128)
        g = np.zeros(m + 1, dtype=np.complex128)
        g[0] = beta
        j_done = 0
        for j in range(m):
            z = M(V[j])
            Z.append(z)
            w = A(z)
            for _ in range(2):  # CGS2
                h = np.array([_dot(V[i], w) for i in range(j + 1)])
                for i in range(j + 1):
                    w = w - h[i] * V[i]
                H[: j + 1, j] += h
            H[j + 1, j] = _norm(w)
            # previous rotations
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -np.conj(sn[i]) * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            a, bb = H[j, j], H[j + 1, j]
            den = np.sqrt(abs(a) ** 2 + abs(bb) ** 2)
            if den == 0.0:
                cs[j], sn[j] = 1.0, 0.0
            elif a == 0:
                cs[j], sn[j] = 0.0, 1.0
            else:
                cs[j] = abs(a) / den
                sn[j] = (a / abs(a)) * np.conj(bb) / den
            H[j, j] = cs[j] * a + sn[j] * bb
            H[j + 1, j] = 0.0
            g[j + 1] = -np.conj(sn[j]) * g[j]
            g[j] = cs[j] * g[j]
            it += 1
            j_done = j + 1
            est = abs(g[j + 1])
            hist.append(est / bnorm)
            hn = _norm(w)
            if hn > 0:
                V.append(w / hn)
            else:
                V.append(np.zeros_like(w))
            if not fixed and est <= tol * bnorm:
                break
            if it >= max_iter:
                break
            if hn == 0:
                break
        # solve the triangular least-squares system
        y = np.zeros(j_done, dtype=np.complex128)
        for i in range(j_done - 1, -1, -1):
            s = g[i] - np.dot(H[i, i + 1: j_done], y[i + 1: j_done])
            y[i] = s / H[i, i] if H[i, i] != 0 else 0.0
        for i in range(j_done):
            x = x + y[i] * Z[i]
        r = b - A(x)
        beta = _norm(r)
        if fixed and it >= max_iter:
            break
        if beta == 0.0:
            break
    resid = beta / bnorm
    return x, dict(iters=it, resid=resid, converged=resid <= tol, history=hist)


def gmres(A, b, x0=None, tol=1e-10, restart=30, max_iter=1000, fixed=False):
    return fgmres(A, b, None, x0, tol, restart, max_iter, fixed)


def mr(A, b, n_steps):
    """Plain minimal-residual iteration from x = 0 (Saad, Sec. 5.3.2)."""
    x = np.zeros_like(b)
    rho = b.copy()
    for _ in range(n_steps):
        q = A(rho)
        qq = np.vdot(q, q).real
        alpha = np.vdot(q, rho) / qq if qq > 0 else 0.0
        x = x + alpha * rho
        rho = rho - alpha * q
    return x
