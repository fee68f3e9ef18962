"""Benchmark: DD-alpha-AMG time to a 1e-10 true residual at 48^3 x 96 with 12
right-hand sides, mixed precision vs FP64, with the fine operator's D(mu) and
the SAP smoother's bandwidth against the HBM roofline.

One step = the whole hot path on one batch of synthetic input: the adaptive
setup (learned initial test vectors, one refinement iteration, block QR,
Galerkin coarse operators on every level) followed by the preconditioned
FGMRES solve of every right-hand side to a true relative residual <= 1e-10
(lock-step groups of --rhs-batch).  Inputs (SU(3) links exp(i 0.3 H),
Gaussian sources, network noise and level-1 test vectors, all seeded) are
generated on the device before the timed region.

    python bench.py [--gpus 1] [--steps 1] [--warmup 0] [--nrhs 12]
                    [--rhs-batch 6] [--restart 4] [--fp64-compare 1] [--cpu-baseline 1]

Prints one JSON line.  `value` is the mixed-precision step time in seconds
(lower is better).  After the timed steps:
  * the plain FP64 form (random start, 5-iteration setup) runs once on the
    same right-hand sides when it fits --time-budget (seconds since start),
    else the line says it was skipped;
  * the oracle leg (cpu_baseline): the FP64 CPU oracle applies D(mu) to the
    solution of the first right-hand side over the whole 48^3 x 96 lattice in
    time slabs on the host's cores, which times the oracle (GB/s with the
    same algorithmic bytes as the device kernel) and gives the oracle's own
    true residual of that solution and its agreement with the library's D(mu).
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

T_START = time.time()
METRIC = "D(μ) GB/s; DD-αAMG time to 1e-10 residual at 48^3×96, mixed vs FP64"
HBM_PEAK_GBS = 8000.0
FP32_VALU_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12  # 78.6
KAPPA, CSW, MU = 0.13729, 1.57551, 0.0009
# algorithmic bytes per site of one FP64 D(mu) apply: spinor in + out (2 x 192),
# links (4 x 9 complex), clover (two Hermitian 6x6 = 72 reals)
DIRAC_FP64_BYTES_PER_SITE = 2 * 192 + 576 + 576


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=0)
    ap.add_argument("--nrhs", type=int, default=12)
    ap.add_argument("--dims", type=str, default="96,48,48,48")
    ap.add_argument("--precision", type=str, default="bf16")
    ap.add_argument("--setup-iters", type=int, default=1)
    ap.add_argument("--fp64-compare", type=int, default=1)
    ap.add_argument("--fp64-setup-iters", type=int, default=5)
    ap.add_argument("--fp64-rhs-batch", type=int, default=2)
    ap.add_argument("--cpu-baseline", type=int, default=1)
    ap.add_argument("--rhs-batch", type=int, default=6)
    ap.add_argument("--restart", type=int, default=4,
                    help="outer FGMRES restart of the mixed form (its FP64 basis of restart+1 fields per "
                         "right-hand side is what bounds the lock-step group at 48^3x96)")
    ap.add_argument("--learned", type=int, default=1)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--time-budget", type=float, default=540.0,
                    help="seconds since start beyond which the FP64 leg is skipped")
    ap.add_argument("--set", action="append", default=[], metavar="KEY=VALUE",
                    help="override a solver parameter of the mixed form (ddamg_params field)")
    return ap.parse_args()


def log(*a):
    print(f"[{time.time() - T_START:6.1f} s]", *a, file=sys.stderr, flush=True)


def oracle_leg(U, x0, b0, y_lib, budget_s=25.0):
    """The FP64 oracle on the host: D(mu) x0 over the whole lattice in time
    slabs of two slices (one halo slice each side), on as many threads as the
    host offers (at most 16).  Returns the cpu_baseline record and the
    oracle's check of the device result (true residual of x0, agreement of
    the library's D(mu) x0 with the oracle's)."""
    import numpy as np
    from concurrent.futures import ThreadPoolExecutor

    try:
        from threadpoolctl import threadpool_limits
    except ImportError:  # pragma: no cover
        threadpool_limits = None
    from oracle import dirac

    T = U.shape[0]
    nt = 2
    slabs = list(range(0, T, nt))
    sites_slab = nt * int(np.prod(U.shape[1:4]))
    cores = max(1, min(16, os.cpu_count() or 1))

    def work(t0):
        t = time.time()
        Dx = dirac.apply_t_slab(U, x0, KAPPA, CSW, MU, t0, nt)
        dt = time.time() - t
        rows = list(range(t0, t0 + nt))
        r = b0[rows] - Dx
        d = Dx - y_lib[rows]
        return (dt, float(np.vdot(r, r).real), float(np.vdot(b0[rows], b0[rows]).real),
                float(np.abs(d).max()), float(np.abs(Dx).max()))

    ctx = threadpool_limits(1) if threadpool_limits else None
    # one core: slabs one after another until the bounded sample is used
    t1 = time.time()
    one = []
    for t0 in slabs:
        one.append(work(t0))
        if time.time() - t1 > budget_s / 2:
            break
    t1 = time.time() - t1
    # all cores: the whole lattice (the slabs done above are not repeated)
    rest = slabs[len(one):]
    tp = time.time()
    with ThreadPoolExecutor(max_workers=cores) as ex:
        many = list(ex.map(work, rest))
    tp = time.time() - tp
    if ctx is not None and hasattr(ctx, "unregister"):
        ctx.unregister()
    allr = one + many
    r2 = sum(v[1] for v in allr)
    b2 = sum(v[2] for v in allr)
    dmax = max(v[3] for v in allr)
    ymax = max(v[4] for v in allr)
    gbs1 = len(one) * sites_slab * DIRAC_FP64_BYTES_PER_SITE / t1 / 1e9
    gbsp = len(rest) * sites_slab * DIRAC_FP64_BYTES_PER_SITE / tp / 1e9 if rest else None
    cpu = {"value": round(gbsp if gbsp else gbs1, 3), "unit": "GB/s", "cores": cores if gbsp else 1,
           "kind": "oracle",
           "sample": f"numpy FP64 oracle D(mu) on the 48^3x96 solution of the first right-hand side, time slabs "
                     f"of {nt} slices with one halo slice each side: {len(rest)} slabs on {cores} threads in "
                     f"{tp:.1f} s (whole lattice with the {len(one)} slabs timed on one thread in {t1:.1f} s, "
                     f"{gbs1:.3f} GB/s); bytes counted as the device kernel's {DIRAC_FP64_BYTES_PER_SITE} B/site",
           "one_core_gbs": round(gbs1, 4)}
    check = {"oracle_true_residual_rhs0": float(np.sqrt(r2 / b2)),
             "dirac_max_abs_diff_over_max": dmax / ymax,
             "sites_checked": len(allr) * sites_slab}
    return cpu, check


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
    kb = min(args.rhs_batch, args.nrhs)

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

    def make_ctx(Ug, net=False):
        c = ddamg.DDAMG(dims, block, KAPPA, CSW, MU, stream=stream.cuda_stream)
        c.set_gauge(Ug)
        if net:
            c.net_create(L, C)
            c.net_set_params(wts)
        return c

    def params(prec, setup_iters, rhs_batch, batch):
        return ddamg.default_params(levels=levels, block=[block, (2, 2, 2, 2)], nvec=nv, setup_iters=setup_iters,
                                    coarse_setup_iters=3, precision=prec, coarse_mu_factor=5.0, batch=batch,
                                    rhs_batch=rhs_batch)

    ctx = make_ctx(U, net=bool(args.learned))
    # the device copy of the links is the library's from here on; the host
    # oracle leg regenerates the same seeded field
    del U
    torch.cuda.empty_cache()
    p_mixed = params(args.precision, args.setup_iters, kb, args.batch)
    p_mixed.restart = args.restart
    overrides = {}
    for kv in args.set:
        k, v = kv.split("=", 1)
        overrides[k] = float(v) if "." in v or "e" in v else int(v)
        setattr(p_mixed, k, overrides[k])

    def step(c, tag):
        t = time.time()
        if args.learned:
            c.setup_learned(p_mixed, noise, V1)
        else:
            c.setup(p_mixed, [V0, V1])
        log(f"{tag}: setup issued ({time.time() - t:.1f} s)")
        _, st = c.solve(b, tol=1e-10, x=x)
        log(f"{tag}: solve done ({time.time() - t:.1f} s, {st['iters']} iterations over {st['nrhs']} rhs, "
            f"{st['iters_min']}-{st['iters_max']} per rhs)")
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
    # the D(mu) FP64 launches of the checks below are not in the timed region
    ctx.timing(False)
    log(f"mixed step {dt:.2f} s, stats {stats}")

    # the solve's workspaces go back to the device for the checks below
    ctx.release_memory()
    # true residuals of the last solve, checked in FP64 on the device
    resid = 0.0
    for i in range(args.nrhs):
        r = ctx.apply_dirac(x[i])
        resid = max(resid, float(torch.linalg.vector_norm(b[i] - r) / torch.linalg.vector_norm(b[i])))
    y0 = ctx.apply_dirac(x[0]).cpu().numpy() if args.cpu_baseline else None

    # D(mu) FP64 bandwidth inside the timed steps (HIP events around every launch)
    avg_ms = ms_d / max(n_d, 1)
    bytes_launch = DIRAC_FP64_BYTES_PER_SITE * V
    achieved = bytes_launch / (avg_ms * 1e-3) / 1e9 if n_d else None
    src_hash = dirac_sources_sha256()
    # fine SAP colour sweeps inside the timed steps: every launch sweeps the
    # blocks of one colour for K fields (K = the setup's batch or the rhs
    # group); the library adds up each launch's algorithmic bytes
    n_s, ms_s = kinds["fine_sap"]
    bytes_s = ctx.timing_bytes(1)
    flops_s = ctx.timing_flops(1)
    sap = None
    if n_s and ms_s > 0:
        # bound by instruction issue: FP32 flops against the FP32 vector peak
        # without packed math (the build disables packed FP32 instructions):
        # 256 CUs x 4 SIMDs x 16 lanes x 2 (fused multiply-add) x 2.4 GHz
        a = flops_s / (ms_s * 1e-3) / 1e12
        gbs = bytes_s / (ms_s * 1e-3) / 1e9
        sap = {"bound": "alu", "kernel": f"fine SAP colour sweep ({args.precision} links, FP32 arithmetic, "
                                         f"4 MR steps), K fields per launch",
               "achieved": round(a, 2), "peak": FP32_VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
               "frac": round(a / FP32_VALU_PEAK_TFLOPS, 4), "traffic": None, "algorithmic_flops": flops_s,
               "hbm_gbs": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4), "algorithmic_bytes": bytes_s,
               "launches": n_s, "avg_launch_ms": round(ms_s / n_s, 4)}
    ctx.close()
    del ctx
    torch.cuda.empty_cache()

    fp64_s = None
    fp64_stats = None
    fp64_note = None
    if args.fp64_compare:
        elapsed = time.time() - T_START
        # the FP64 form has run ~20x the mixed step on this lattice
        projected = 20.0 * dt * max(1.0, args.nrhs / 12.0)
        if elapsed + projected > args.time_budget:
            fp64_note = (f"skipped: {elapsed:.0f} s elapsed + about {projected:.0f} s projected exceeds the "
                         f"{args.time_budget:.0f} s budget of this run")
            log("fp64:", fp64_note)
        else:
            if args.learned:
                del noise
                torch.cuda.empty_cache()
            V0 = synth.gaussian_device((nv[0],) + dims + (4, 3), 5501)
            U = synth.gauge_field_device(dims, 0.3, 5001)
            c64 = make_ctx(U)
            del U
            torch.cuda.empty_cache()
            # FP64 fine fields are twice the size: 4 test vectors per setup batch
            p64 = params("fp64", args.fp64_setup_iters, min(args.fp64_rhs_batch, args.nrhs), min(args.batch, 4))
            torch.cuda.synchronize()
            t1 = time.time()
            c64.setup(p64, [V0, V1])
            del V0
            torch.cuda.empty_cache()
            log(f"fp64: setup done ({time.time() - t1:.1f} s)")
            # the right-hand sides group by group (one call each, so that the
            # run reports progress); statistics summed as one call would
            kb64 = p64.rhs_batch
            fp64_stats = None
            for g0 in range(0, args.nrhs, kb64):
                _, st = c64.solve(b[g0:g0 + kb64], tol=1e-10, x=x[g0:g0 + kb64])
                if fp64_stats is None:
                    fp64_stats = st
                else:
                    for k in ("iters", "vcycles", "nrhs"):
                        fp64_stats[k] += st[k]
                    fp64_stats["coarse_iters"] = [a + c for a, c in zip(fp64_stats["coarse_iters"],
                                                                         st["coarse_iters"])]
                    fp64_stats["converged"] = fp64_stats["converged"] and st["converged"]
                    fp64_stats["resid"] = max(fp64_stats["resid"], st["resid"])
                    fp64_stats["iters_min"] = min(fp64_stats["iters_min"], st["iters_min"])
                    fp64_stats["iters_max"] = max(fp64_stats["iters_max"], st["iters_max"])
                    fp64_stats["seconds"] += st["seconds"]
                log(f"fp64: right-hand sides {g0}..{g0 + kb64 - 1} solved ({time.time() - t1:.1f} s)")
            torch.cuda.synchronize()
            fp64_s = time.time() - t1
            c64.close()
            log(f"fp64 step {fp64_s:.2f} s, stats {fp64_stats}")

    cpu = None
    check = None
    if args.cpu_baseline:
        log("oracle leg on the host")
        U_host = synth.gauge_field_device(dims, 0.3, 5001).cpu().numpy()
        x0 = x[0].cpu().numpy()
        b0 = b[0].cpu().numpy()
        cpu, check = oracle_leg(U_host, x0, b0, y0)
        log(f"oracle: {cpu['value']} GB/s on {cpu['cores']} threads, check {check}")

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
                               f"Nv 24/32), {args.nrhs} rhs ({kb} in lock step, outer restart {args.restart}), "
                               f"{'learned' if args.learned else 'random'} initial test vectors + "
                               f"{args.setup_iters} setup iteration(s) on batches of {args.batch} test vectors, "
                               f"preconditioner {args.precision}, outer FGMRES FP64, tol 1e-10"
                               + (f", overrides {overrides}" if overrides else ""),
                   "global_batch": args.nrhs, "parallelism": "none"},
        "roofline": {"bound": "hbm", "kernel": "D(mu) FP64 full-lattice apply",
                     "achieved": round(achieved, 1) if achieved else None, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4) if achieved else None,
                     "traffic": traffic_for(src_hash), "algorithmic_bytes_per_launch": bytes_launch,
                     "launches": n_d, "avg_launch_ms": round(avg_ms, 4)},
        "roofline_sap": sap,
        "cpu_baseline": cpu,
        "oracle_check": check,
        "mixed_stats": stats,
        "iters_per_rhs": round(stats["iters"] / max(1, stats["nrhs"]), 2) if stats else None,
        "true_residual_max": resid,
        "fp64_step_s": round(fp64_s, 3) if fp64_s else None,
        "fp64_stats": fp64_stats,
        "fp64_note": fp64_note,
        "speedup_mixed_vs_fp64": round(fp64_s / dt, 3) if fp64_s else None,
        "kernel_ms": {k: {"launches": v[0], "ms": round(v[1], 2)} for k, v in kinds.items()},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
