"""Benchmark: DD-alpha-AMG time to a 1e-10 true residual at 48^3 x 96, mixed
precision vs FP64, with the fine operator's D(mu) bandwidth against the HBM
roofline.

One step = the whole hot path on one batch of synthetic input: adaptive setup
(test vectors, block QR, Galerkin coarse operators on every level) followed by
the preconditioned FGMRES solve of every right-hand side to a true relative
residual <= 1e-10.  Inputs (SU(3) links exp(i 0.3 H), Gaussian sources and
initial test vectors, all seeded) are generated on the device before the
timed region.

    python bench.py [--gpus 1] [--steps 1] [--warmup 0] [--nrhs 2]
                    [--dims 96,48,48,48] [--fp64-compare 1]

Prints one JSON line.  `value` is the mixed-precision step time in seconds
(lower is better); the plain FP64 form is run once after the timed steps on
the same inputs and reported as fp64_step_s.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "D(μ) GB/s; DD-αAMG time to 1e-10 residual at 48^3×96, mixed vs FP64"
HBM_PEAK_GBS = 8000.0
KAPPA, CSW, MU = 0.13729, 1.57551, 0.0009
# algorithmic bytes per site of one FP64 D(mu) apply: spinor in + out (2 x 192),
# links (4 x 9 complex), clover (two Hermitian 6x6 = 72 reals)
DIRAC_FP64_BYTES_PER_SITE = 2 * 192 + 576 + 576


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=0)
    ap.add_argument("--nrhs", type=int, default=2)
    ap.add_argument("--dims", type=str, default="96,48,48,48")
    ap.add_argument("--precision", type=str, default="bf16")
    ap.add_argument("--setup-iters", type=int, default=1)
    ap.add_argument("--fp64-compare", type=int, default=1)
    ap.add_argument("--fp64-setup-iters", type=int, default=5)
    ap.add_argument("--cpu-baseline", type=int, default=1)
    ap.add_argument("--rhs-batch", type=int, default=2)
    ap.add_argument("--learned", type=int, default=1)
    ap.add_argument("--batch", type=int, default=16)
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(nrhs, V_target):
    """The oracle timed on a bounded sample: one 2-level setup + solve of the
    4^4 configuration (Nv 8, 2^4 aggregates, 3 setup iterations, tol 1e-10),
    scaled linearly by volume and by the number of right-hand sides."""
    try:
        from threadpoolctl import threadpool_limits
    except ImportError:  # pragma: no cover
        threadpool_limits = None
    import numpy as np

    from oracle import dirac, mg
    from paper_1611_01034_amd import synth

    dims = (4, 4, 4, 4)
    U = synth.gauge_field(dims, 0.3, 1001)
    V0 = synth.gaussian((8,) + dims + (12,), 1501)
    b = synth.spinor(dims, 1101).reshape(dims + (12,))
    ctx = threadpool_limits(1) if threadpool_limits else None
    t = time.time()
    op = dirac.WilsonClover(U, KAPPA, CSW, MU)
    h = mg.Hierarchy(op, mg.Params(levels=2, blocks=[(2, 2, 2, 2)], nvec=[8], setup_iters=3)).setup([V0])
    x, info = h.solve(b, tol=1e-10)
    dt = time.time() - t
    if ctx is not None:
        ctx.unregister() if hasattr(ctx, "unregister") else None
    V = int(np.prod(dims))
    return {"value": dt * (V_target / V) * nrhs, "unit": "s", "cores": 1, "kind": "oracle",
            "sample": f"numpy FP64 oracle, 2-level setup (3 iterations) + 1 solve to 1e-10 on 4^4 "
                      f"({dt:.2f} s measured, {info['iters']} FGMRES iterations), scaled by volume "
                      f"x{V_target // V} and by {nrhs} right-hand sides"}


DIRAC_SOURCES = ["dirac.hip", "finedev.hpp", "common.hpp"]


def dirac_sources_sha256():
    """Hash of the sources the D(mu) kernel is built from (same recipe as
    paper_1611_01034_amd.profsum.sources_sha256)."""
    h = hashlib.sha256()
    for f in DIRAC_SOURCES:
        with open(os.path.join(ROOT, "paper_1611_01034_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def traffic_for(kernel_src_hash):
    p = os.path.join(ROOT, "profiles", "dirac_fp64_48x48x48x96_traffic.json")
    if not os.path.exists(p):
        return None
    with open(p) as f:
        d = json.load(f)
    if d.get("source_sha256") != kernel_src_hash:
        return None
    return d.get("bytes_per_launch")


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); multi-GPU runs are not part of "
              "this build", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_1611_01034_amd import ddamg, synth

    dims = tuple(int(x) for x in args.dims.split(","))
    V = int(np.prod(dims))
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    block = (4, 4, 4, 4)
    cd = tuple(d // 4 for d in dims)
    nv = [24, 32]
    levels = 3

    log("generating inputs on the device")
    U = synth.gauge_field_device(dims, 0.3, 5001)
    b = synth.gaussian_device((args.nrhs,) + dims + (4, 3), 5101)
    x = torch.empty_like(b)
    V1 = synth.gaussian_device((nv[1],) + cd + (2 * nv[0],), 5502)
    if args.learned:
        from paper_1611_01034_amd import learned_setup
        wts, C, L, _ = learned_setup.load_weights(learned_setup.WEIGHTS)
        if C != nv[0]:
            raise SystemExit("network channels must equal the level-0 test vector count")
        noise = synth.gaussian_device((C,) + dims + (4, 3), 5501, dtype="complex64")
        V0 = None
    else:
        V0 = synth.gaussian_device((nv[0],) + dims + (4, 3), 5501)
    torch.cuda.synchronize()

    def make_ctx(net=False):
        c = ddamg.DDAMG(dims, block, KAPPA, CSW, MU, stream=stream.cuda_stream)
        c.set_gauge(U)
        if net:
            c.net_create(L, C)
            c.net_set_params(wts)
        return c

    def params(prec, setup_iters, rhs_batch, batch):
        return ddamg.default_params(levels=levels, block=[block, (2, 2, 2, 2)], nvec=nv, setup_iters=setup_iters,
                                    coarse_setup_iters=3, precision=prec, coarse_mu_factor=5.0, batch=batch,
                                    rhs_batch=rhs_batch)

    ctx = make_ctx(net=bool(args.learned))
    p_mixed = params(args.precision, args.setup_iters, min(args.rhs_batch, args.nrhs), args.batch)

    def step(c, tag):
        t = time.time()
        if args.learned:
            c.setup_learned(p_mixed, noise, V1)
        else:
            c.setup(p_mixed, [V0, V1])
        log(f"{tag}: setup issued ({time.time() - t:.1f} s)")
        _, st = c.solve(b, tol=1e-10, x=x)
        log(f"{tag}: solve done ({time.time() - t:.1f} s, {st['iters']} iterations)")
        return st

    for i in range(args.warmup):
        step(ctx, f"warmup {i}")
    torch.cuda.synchronize()
    ctx.timing(True)
    t0 = time.time()
    stats = None
    for i in range(args.steps):
        stats = step(ctx, f"step {i}")
    torch.cuda.synchronize()
    dt = (time.time() - t0) / args.steps
    n_d, ms_d = ctx.timing_query(0)
    kinds = {k: ctx.timing_query(i) for i, k in enumerate(["dirac_fp64", "fine_sap", "coarse_apply",
                                                            "transfer", "dirac_reduced", "coarsest_schur"])}
    # the D(mu) FP64 launches of the residual check below are not in the timed region
    ctx.timing(False)
    log(f"mixed step {dt:.2f} s, stats {stats}")

    # true residual of the last solve, checked in FP64 on the device
    resid = 0.0
    for i in range(args.nrhs):
        r = ctx.apply_dirac(x[i])
        resid = max(resid, float(torch.linalg.vector_norm(b[i] - r) / torch.linalg.vector_norm(b[i])))

    # D(mu) FP64 bandwidth inside the timed steps (HIP events around every launch)
    avg_ms = ms_d / max(n_d, 1)
    bytes_launch = DIRAC_FP64_BYTES_PER_SITE * V
    achieved = bytes_launch / (avg_ms * 1e-3) / 1e9 if n_d else None
    src_hash = dirac_sources_sha256()
    ctx.close()
    del ctx
    torch.cuda.empty_cache()

    fp64_s = None
    fp64_stats = None
    if args.fp64_compare:
        if V0 is None:
            del noise
            torch.cuda.empty_cache()
            V0 = synth.gaussian_device((nv[0],) + dims + (4, 3), 5501)
        c64 = make_ctx()
        # FP64 fine fields are twice the size: 4 test vectors per setup batch
        p64 = params("fp64", args.fp64_setup_iters, 1, min(args.batch, 4))
        torch.cuda.synchronize()
        t1 = time.time()
        c64.setup(p64, [V0, V1])
        log(f"fp64: setup issued ({time.time() - t1:.1f} s)")
        _, fp64_stats = c64.solve(b, tol=1e-10, x=x)
        torch.cuda.synchronize()
        fp64_s = time.time() - t1
        c64.close()
        log(f"fp64 step {fp64_s:.2f} s, stats {fp64_stats}")

    cpu = None
    if args.cpu_baseline:
        log("timing the oracle on the host")
        cpu = cpu_baseline(args.nrhs, V)

    out = {
        "metric": METRIC,
        "value": round(dt, 4),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt * 1e3, 2),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else args.precision.replace("fp", "f"),
        "data": "synthetic",
        "config": {"workload": f"{'x'.join(str(d) for d in reversed(dims))} twisted-mass Wilson-clover, "
                               f"kappa {KAPPA}, c_sw {CSW}, mu {MU}, delta 5, 3 levels (4^4, 2^4 aggregates, "
                               f"Nv 24/32), {args.nrhs} rhs ({min(args.rhs_batch, args.nrhs)} in lock step), "
                               f"{'learned' if args.learned else 'random'} initial test vectors + "
                               f"{args.setup_iters} setup iteration(s) on batches of {args.batch} test vectors, "
                               f"preconditioner {args.precision}, outer FGMRES FP64, tol 1e-10",
                   "global_batch": args.nrhs, "parallelism": "none"},
        "roofline": {"bound": "hbm", "kernel": "D(mu) FP64 full-lattice apply",
                     "achieved": round(achieved, 1) if achieved else None, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4) if achieved else None,
                     "traffic": traffic_for(src_hash), "algorithmic_bytes_per_launch": bytes_launch,
                     "launches": n_d, "avg_launch_ms": round(avg_ms, 4)},
        "cpu_baseline": cpu,
        "mixed_stats": stats,
        "true_residual_max": resid,
        "fp64_step_s": round(fp64_s, 3) if fp64_s else None,
        "fp64_stats": fp64_stats,
        "speedup_mixed_vs_fp64": round(fp64_s / dt, 3) if fp64_s else None,
        "kernel_ms": {k: {"launches": v[0], "ms": round(v[1], 2)} for k, v in kinds.items()},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
