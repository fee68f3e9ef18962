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
and the FGMRES iteration count to a 1e-10 true residual.  Fallback
(setup_with_fallback): when the learned start fails or its probe rho
(ddamg_error_reduction, on the device) exceeds `margin` times a reference
rho, the plain setup is run instead (decide_fallback).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

from . import ddamg, synth

KAPPA, CSW, MU = 0.13729, 1.57551, 0.0009


def decide_fallback(rho_probe: float, rho_ref: float, margin: float = 1.25) -> bool:
    """True when the learned start must be replaced by the plain setup."""
    if not np.isfinite(rho_probe):
        return True
    return rho_probe > margin * rho_ref


def setup_with_fallback(ctx: ddamg.DDAMG, params, noise, coarse_init, plain_vectors, probe, rho_ref=0.9,
                        margin=1.0, n_probe=2, plain_params=None):
    """The learned setup with the plain adaptive setup as its fallback.

    Runs ddamg_setup_learned, then probes the resulting cycle's error
    reduction rho on `probe` (n_probe applications of I - M D on the device).
    When the learned start fails (a rank-deficient aggregate: NUMERICAL) or
    decide_fallback(rho, rho_ref, margin) holds, the plain setup runs instead
    on plain_vectors() (a callable, so that its random vectors are only made
    when needed) with plain_params (default: params).  Returns
    {"fallback": bool, "rho_learned": float, "rho": float}."""
    try:
        ctx.setup_learned(params, noise, coarse_init)
        rho_l = ctx.error_reduction(probe, n_probe)
    except ddamg.DDAMGError as e:
        if e.status != ddamg.NUMERICAL:
            raise
        rho_l = float("nan")
    if not decide_fallback(rho_l, rho_ref, margin):
        return {"fallback": False, "rho_learned": rho_l, "rho": rho_l}
    ctx.setup(plain_params if plain_params is not None else params, plain_vectors())
    return {"fallback": True, "rho_learned": rho_l, "rho": ctx.error_reduction(probe, n_probe)}


def init_torch_device():
    """Select device 0 in torch; returns torch's current stream handle, which
    every context created here uses."""
    import torch
    torch.cuda.set_device(0)
    return torch.cuda.current_stream().cuda_stream


def _ctx(dims, block):
    return ddamg.DDAMG(dims, block, KAPPA, CSW, MU, stream=init_torch_device())


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


def make_targets(dims, block, seeds, eps_list, nvec=24, setup_iters=5, log=print):
    """Plain setups on seeded fields; returns [(U, Q)] with Q the block
    orthonormalised level-0 test vectors (host FP64, spinor layout)."""
    out = []
    t0 = time.time()
    for i, s in enumerate(seeds):
        if i % 8 == 0:
            log(f"targets: field {i}/{len(seeds)} ({time.time() - t0:.1f} s)")
        eps = eps_list[i % len(eps_list)]
        U = synth.gauge_field(dims, eps, s)
        with _ctx(dims, block) as ctx:
            ctx.set_gauge(U)
            V0 = synth.spinor(dims, s + 100000, nvec=nvec)
            ctx.setup(mg_params(nvec=(nvec,), block=block, setup_iters=setup_iters, precision="fp32"), [V0])
            Q = ctx.get_interpolation(0)
        out.append((U, Q))
    return out


def train(dims, block, data, C=24, L=4, epochs=8, lr=2e-3, seed=4242, log=print, on_device=True):
    """Adam on the subspace loss over the (U, Q) pairs of `data`; a fresh noise
    draw per step.  Returns (parameter vector, loss history)."""
    W, a, b = synth.net_init_weights(C, L, seed)
    params = ddamg.pack_net(W, a, b)
    hist = []
    with _ctx(dims, block) as ctx:
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


def VARIANTS(Vl, Vr):
    """(name, initial vectors, setup iterations) of the comparison: learned or
    random start with 0 or 1 refinement iterations, and the plain 5-iteration
    setup from the random start."""
    return (("learned+0", Vl, 0), ("random+0", Vr, 0), ("learned+1", Vl, 1), ("random+1", Vr, 1),
            ("plain5", Vr, 5))


def evaluate(dims, block, seeds, eps, params, C=24, L=4, nvec=24, tol=1e-10, log=print):
    """For each held-out field: learned + 1 refinement, random + 1 refinement,
    plain 5-iteration setup.  Returns a list of per-field dicts."""
    rows = []
    for s in seeds:
        U = synth.gauge_field(dims, eps, s)
        b = synth.spinor(dims, s + 200000)
        row = {"seed": s}
        with _ctx(dims, block) as ctx:
            ctx.set_gauge(U)
            Vr = synth.spinor(dims, s + 100000, nvec=nvec)
            Vl = learned_vectors(ctx, params, C, L, dims, s + 300000)
            for name, vecs, it in VARIANTS(Vl, Vr):
                t0 = time.time()
                ctx.setup(mg_params(nvec=(nvec,), block=block, setup_iters=it), [vecs])
                ts = time.time() - t0
                rho = error_reduction(ctx, dims, n=10, seed=s + 400000)
                x, st = ctx.solve(b, tol=tol)
                row[name] = {"rho": rho, "iters": st["iters"], "setup_s": ts, "solve_s": st["seconds"]}
        log(row)
        rows.append(row)
    return rows


def save_weights(path, params, C, L, meta=None):
    """Parameter vector (FP32, the precision the network computes in) and
    shape in a plain .npz (no pickled objects)."""
    np.savez(path, params=np.asarray(params, dtype=np.float32), C=np.int64(C), L=np.int64(L),
             meta=np.array(json.dumps(meta or {})))


def load_weights(path):
    with np.load(path, allow_pickle=False) as z:
        return z["params"].astype(np.float64), int(z["C"]), int(z["L"]), json.loads(str(z["meta"]))


WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights", "net_l4_c24.npz")


def _seeds(spec):
    a, b = (int(x) for x in spec.split(":"))
    return list(range(a, b))


def _tuple(spec):
    return tuple(int(x) for x in spec.split(","))


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    sp = ap.add_subparsers(dest="mode", required=True)
    t = sp.add_parser("train")
    t.add_argument("--dims", default="16,8,8,8", help="T,Z,Y,X")
    t.add_argument("--block", default="4,4,4,4")
    t.add_argument("--seeds", default="4000:4064")
    t.add_argument("--eps", default="0.2,0.3,0.4")
    t.add_argument("--nvec", type=int, default=24)
    t.add_argument("--layers", type=int, default=4)
    t.add_argument("--epochs", type=int, default=20)
    t.add_argument("--lr", type=float, default=2e-3)
    t.add_argument("--out", default=WEIGHTS)
    e = sp.add_parser("evaluate")
    e.add_argument("--dims", default="48,24,24,24")
    e.add_argument("--block", default="4,4,4,4")
    e.add_argument("--seeds", default="4100:4116")
    e.add_argument("--eps", type=float, default=0.3)
    e.add_argument("--weights", default=WEIGHTS)
    e.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    if a.mode == "train":
        dims, block = _tuple(a.dims), _tuple(a.block)
        eps = [float(x) for x in a.eps.split(",")]
        t0 = time.time()
        data = make_targets(dims, block, _seeds(a.seeds), eps, nvec=a.nvec)
        t_targets = time.time() - t0
        print(f"targets: {len(data)} fields in {t_targets:.1f} s", flush=True)
        t0 = time.time()
        params, hist = train(dims, block, data, C=a.nvec, L=a.layers, epochs=a.epochs, lr=a.lr)
        t_train = time.time() - t0
        meta = {"dims": dims, "block": block, "seeds": a.seeds, "eps": eps, "epochs": a.epochs, "lr": a.lr,
                "loss_history": hist, "targets_s": t_targets, "train_s": t_train,
                "targets": "block-orthonormalised level-0 test vectors of the plain 5-iteration FP32 setup"}
        os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
        save_weights(a.out, params, a.nvec, a.layers, meta)
        print(json.dumps({k: v for k, v in meta.items() if k != "loss_history"}), flush=True)
    else:
        params, C, L, meta = load_weights(a.weights)
        rows = evaluate(_tuple(a.dims), _tuple(a.block), _seeds(a.seeds), a.eps, params, C=C, L=L, nvec=C)
        summary = {}
        for k in [v[0] for v in VARIANTS(None, None)]:
            summary[k] = {m: float(np.mean([r[k][m] for r in rows])) for m in ("rho", "iters", "setup_s", "solve_s")}
        out = {"dims": _tuple(a.dims), "eps": a.eps, "seeds": a.seeds, "summary": summary, "rows": rows}
        print(json.dumps(summary), flush=True)
        if a.out:
            with open(a.out, "w") as fh:
                json.dump(out, fh, indent=1)


if __name__ == "__main__":
    sys.exit(main())
