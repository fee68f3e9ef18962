"""Learned initial test vectors for the adaptive setup: training, inference,
evaluation and the fallback to the plain setup.

The paper's adaptive setup (Sec. 1) starts from random test vectors; here a
gauge-covariant network (libddamg's ddamg_net_* kernels) maps Gaussian noise to
the starting vectors, followed by one refinement iteration of the setup.  It is
trained on the block-orthonormalised test vectors that the plain setup
(MGSetupIter iterations) produces on seeded synthetic fields.  Every
arithmetic step runs in the library's kernels; this module only sequences
calls and moves fields.

Judged by multigrid outcomes: the V-cycle error-reduction factor
  rho = (|(I - M D)^n e| / |e|)^(1/n)
and the FGMRES iteration count to a 1e-10 true residual.  Fallback: when the
probe rho of the learned start exceeds `margin` times the reference rho of the
plain setup, the plain setup is run instead (decide_fallback).
"""
from __future__ import annotations

import time

import numpy as np

from . import ddamg, synth

KAPPA, CSW, MU = 0.13729, 1.57551, 0.0009


def decide_fallback(rho_probe: float, rho_ref: float, margin: float = 1.25) -> bool:
    """True when the learned start must be replaced by the plain setup."""
    if not np.isfinite(rho_probe):
        return True
    return rho_probe > margin * rho_ref


def init_torch_device():
    """torch's HIP context must exist before the library's first call."""
    import torch
    torch.cuda.init()
    return torch


def _torch_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def error_reduction(ctx: ddamg.DDAMG, dims, n: int = 10, seed: int = 0) -> float:
    """rho of the fine-level V-cycle on D(mu): e <- e - M D e, n times, from a
    Gaussian e (host arrays, FP64)."""
    e = synth.spinor(dims, seed)
    n0 = np.linalg.norm(e)
    for _ in range(n):
        e = e - ctx.vcycle(ctx.apply_dirac(e))
    return float((np.linalg.norm(e) / n0) ** (1.0 / n))


def mg_params(levels=2, nvec=(24,), block=(4, 4, 4, 4), setup_iters=1, precision="fp32", delta=5.0):
    blocks = [block] + [(2, 2, 2, 2)] * (levels - 2)
    return ddamg.default_params(levels=levels, block=blocks, nvec=list(nvec), setup_iters=setup_iters,
                                precision=precision, coarse_mu_factor=delta)


def make_targets(dims, block, seeds, eps_list, nvec=24, setup_iters=5, stream=None):
    """Plain setups on seeded fields; returns [(U, Q)] with Q the block
    orthonormalised level-0 test vectors (host FP64, spinor layout)."""
    out = []
    for i, s in enumerate(seeds):
        eps = eps_list[i % len(eps_list)]
        U = synth.gauge_field(dims, eps, s)
        with ddamg.DDAMG(dims, block, KAPPA, CSW, MU, stream=stream) as ctx:
            ctx.set_gauge(U)
            V0 = synth.spinor(dims, s + 100000, nvec=nvec)
            ctx.setup(mg_params(nvec=(nvec,), block=block, setup_iters=setup_iters, precision="fp32"), [V0])
            Q = ctx.get_interpolation(0)
        out.append((U, Q))
    return out


def train(dims, block, data, C=24, L=4, epochs=8, lr=2e-3, seed=4242, log=print, on_device=True):
    """Adam on the subspace loss over the (U, Q) pairs of `data`; a fresh noise
    draw per step.  Returns (parameter vector, loss history)."""
    if on_device:
        init_torch_device()
    W, a, b = synth.net_init_weights(C, L, seed)
    params = ddamg.pack_net(W, a, b)
    hist = []
    with ddamg.DDAMG(dims, block, KAPPA, CSW, MU) as ctx:
        ctx.net_create(L, C)
        ctx.net_set_params(params)
        tgts = [_torch_dev(Q) if on_device else Q for (_, Q) in data]
        step = 0
        for ep in range(epochs):
            t0 = time.time()
            losses = []
            for i, (U, _) in enumerate(data):
                ctx.set_gauge(U)
                noise = synth.spinor(dims, seed + 7919 * step + 1, nvec=C)
                nz = _torch_dev(noise) if on_device else noise
                losses.append(ctx.net_train_step(nz, tgts[i], lr))
                step += 1
            hist.append(float(np.mean(losses)))
            log(f"epoch {ep}: mean loss {hist[-1]:.4f} ({time.time() - t0:.1f} s)")
        params = ctx.net_get_params()
    return params, hist


def learned_vectors(ctx: ddamg.DDAMG, params, C, L, dims, seed):
    """Network output on the context's gauge field for a seeded noise draw."""
    ctx.net_create(L, C)
    ctx.net_set_params(params)
    return ctx.net_forward(synth.spinor(dims, seed, nvec=C))


def evaluate(dims, block, seeds, eps, params, C=24, L=4, nvec=24, tol=1e-10, log=print):
    """For each held-out field: learned + 1 refinement, random + 1 refinement,
    plain 5-iteration setup.  Returns a list of per-field dicts."""
    rows = []
    for s in seeds:
        U = synth.gauge_field(dims, eps, s)
        b = synth.spinor(dims, s + 200000)
        row = {"seed": s}
        with ddamg.DDAMG(dims, block, KAPPA, CSW, MU) as ctx:
            ctx.set_gauge(U)
            Vr = synth.spinor(dims, s + 100000, nvec=nvec)
            Vl = learned_vectors(ctx, params, C, L, dims, s + 300000)
            for name, vecs, it in (("learned+1", Vl, 1), ("random+1", Vr, 1), ("plain5", Vr, 5)):
                t0 = time.time()
                ctx.setup(mg_params(nvec=(nvec,), block=block, setup_iters=it), [vecs])
                ts = time.time() - t0
                rho = error_reduction(ctx, dims, n=10, seed=s + 400000)
                x, st = ctx.solve(b, tol=tol)
                row[name] = {"rho": rho, "iters": st["iters"], "setup_s": ts, "solve_s": st["seconds"]}
        log(row)
        rows.append(row)
    return rows
