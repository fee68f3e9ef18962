"""Benchmark: DD-alpha-AMG time to a 1e-10 true residual at 48^3 x 96 with 12
right-hand sides, mixed precision vs FP64, with the fine operator's D(mu) and
the SAP smoother's bandwidth against the HBM roofline.

One step = the whole hot path on one batch of synthetic input: the adaptive
setup (initial test vectors from Gaussian noise or from the learned network,
one refinement iteration, block QR, Galerkin coarse operators on every level)
followed by the preconditioned
FGMRES solve of every right-hand side to a true relative residual <= 1e-10
(lock-step groups of --rhs-batch).  Inputs (SU(3) links exp(i 0.3 H),
Gaussian sources, network noise and level-1 test vectors, all seeded) are
generated on the device before the timed region.

    python bench.py [--gpus 1] [--steps 1] [--warmup 0] [--nrhs 12]
                    [--rhs-batch 6] [--restart 4] [--fp64-compare 1] [--cpu-baseline 1]

Prints one JSON line.  `value` is the mixed-precision step time in seconds
(lower is better).  After the timed steps:
  * with --alt-start 1, one untimed step with the other initial test vectors
    (learned <-> random) on the same inputs ran before the warm-up steps
    (`other_start`);
  * the plain FP64 form (random start, 5-iteration setup) runs once on the
    same right-hand sides when it fits --time-budget (seconds since start),
    else the line says it was skipped;
  * the oracle leg (cpu_baseline), which runs on the host while the GPU
    works: the FP64 CPU oracle applies D(mu) to the first right-hand side on
    single time slices, one slice on one thread, then --oracle-procs slices on
    as many processes (GB/s with the device kernel's algorithmic bytes); the
    slices are compared with the library's D(mu), and at --oracle-sites
    random sites the oracle computes b - D x of the first solution.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

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
SAP_POST = 2  # fine post-smoothing sweeps (k of Eq. (1)) of both forms


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
    ap.add_argument("--oracle-procs", type=int, default=8,
                    help="worker processes of the oracle leg (one time slice each)")
    ap.add_argument("--oracle-sites", type=int, default=512,
                    help="random sites at which the oracle checks b - D x of the first solution")
    ap.add_argument("--rhs-batch", type=int, default=6)
    ap.add_argument("--restart", type=int, default=4,
                    help="outer FGMRES restart of the mixed form (its FP64 basis of restart+1 fields per "
                         "right-hand side is what bounds the lock-step group at 48^3x96)")
    ap.add_argument("--learned", type=int, default=0,
                    help="1: the network proposes the initial test vectors; 0: Gaussian random vectors "
                         "(the faster start at this roughness after one setup iteration; --alt-start 1 "
                         "times the other one in an untimed step)")
    ap.add_argument("--alt-start", type=int, default=0,
                    help="one untimed step with the other initial vectors before the warm-up steps")
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--time-budget", type=float, default=540.0,
                    help="seconds since start beyond which the FP64 leg is skipped")
    ap.add_argument("--set", action="append", default=[], metavar="KEY=VALUE",
                    help="override a solver parameter (ddamg_params field) of both forms")
    return ap.parse_args()


def log(*a):
    print(f"[{time.time() - T_START:6.1f} s]", *a, file=sys.stderr, flush=True)


def _oracle_slab(args):
    """One oracle D(mu) apply on one time slice: Us, bs hold the slices
    t-1, t, t+1 of the links and of the spinor; returns (seconds, D bs on t).
    Module level, so that worker processes can import it."""
    Us, bs = args
    try:
        from threadpoolctl import threadpool_limits
    except ImportError:  # pragma: no cover
        threadpool_limits = None
    from oracle import dirac
    lim = threadpool_limits(1) if threadpool_limits else None
    t = time.time()
    y = dirac.apply_t_slab(Us, bs, KAPPA, CSW, MU, 1, 1)[0]
    dt = time.time() - t
    if lim is not None and hasattr(lim, "unregister"):
        lim.unregister()
    return dt, y


class OracleLeg:
    """The FP64 CPU oracle timed on the host while the GPU runs the steps.

    D(mu) b_0 on single time slices of the lattice (the oracle's
    slab apply: slices t-1..t+1 gathered, the operator applied on that slab,
    the middle slice kept): first one slice on one thread, then `nproc` slices
    on `nproc` worker processes at once.  GB/s counts the device kernel's
    algorithmic bytes for the sites produced.  The slices' values are checked
    against the library's D(mu) b_0 after the steps (`check`)."""

    def __init__(self, U_dev, b0_dev, nproc):
        import threading
        T = U_dev.shape[0]
        self.nproc = nproc
        self.T = T
        # slice 0 on one thread, then nproc slices spread over T
        self.ts = [0] + [1 + k * (T // nproc) for k in range(nproc)]
        self.inputs = []
        for t in self.ts:
            rows = [(t - 1) % T, t, (t + 1) % T]
            self.inputs.append((U_dev[rows].cpu().numpy(), b0_dev[rows].cpu().numpy()))
        self.sites_slice = int(np.prod(U_dev.shape[1:4]))
        self.lattice = "x".join(str(d) for d in reversed(tuple(U_dev.shape[:4])))
        self.res = {}
        self.th = threading.Thread(target=self._run, daemon=True)
        self.th.start()

    def _run(self):
        try:
            from concurrent.futures import ProcessPoolExecutor
            import multiprocessing as mp
            dt1, y1 = _oracle_slab(self.inputs[0])
            self.res["one"] = (dt1, y1)
            log(f"oracle leg: one slice on one thread in {dt1:.1f} s")
            tp = time.time()
            ex = ProcessPoolExecutor(max_workers=self.nproc, mp_context=mp.get_context("spawn"))
            try:
                many = list(ex.map(_oracle_slab, self.inputs[1:], timeout=900))
            finally:
                ex.shutdown(wait=False, cancel_futures=True)
            tp = time.time() - tp
            self.res["many"] = (tp, many)
            log(f"oracle leg: {self.nproc} slices on {self.nproc} processes in {tp:.1f} s")
        except Exception as e:  # reported in the JSON line
            self.res["error"] = repr(e)
        finally:
            self.inputs = None

    def result(self, yb_slices):
        """Join; yb_slices[t] = the library's D(mu) b_0 on slice t."""
        self.th.join(timeout=600)
        if self.th.is_alive():
            return None, {"error": "the oracle leg did not finish within 600 s of the GPU work"}
        if "error" in self.res:
            return None, {"error": self.res["error"]}
        dt1, y1 = self.res["one"]
        tp, many = self.res["many"]
        bps = self.sites_slice * DIRAC_FP64_BYTES_PER_SITE
        gbs1 = bps / dt1 / 1e9
        gbsp = self.nproc * bps / tp / 1e9
        ys = [y1] + [m[1] for m in many]
        dmax = max(float(np.abs(y - yb_slices[t]).max()) for t, y in zip(self.ts, ys))
        ymax = max(float(np.abs(yb_slices[t]).max()) for t in self.ts)
        cpu = {"value": round(gbsp, 4), "unit": "GB/s", "cores": self.nproc, "kind": "oracle",
               "sample": f"numpy FP64 oracle D(mu) b_0 on single time slices of the {self.lattice} lattice (slab of 3 "
                         f"slices gathered, middle slice kept; {self.sites_slice} sites each): {self.nproc} slices "
                         f"on {self.nproc} worker processes in {tp:.1f} s; bytes counted as the device kernel's "
                         f"{DIRAC_FP64_BYTES_PER_SITE} B/site; run on the host while the GPU ran the steps",
               "one_core_gbs": round(gbs1, 5), "one_core_s_per_slice": round(dt1, 2)}
        check = {"dirac_slices_max_abs_diff_over_max": dmax / ymax,
                 "dirac_sites_checked": len(ys) * self.sites_slice}
        return cpu, check


def oracle_sites(U_dev, x0_dev, b0_dev, yx_dev, nsites, seed=7):
    """b - D x of the device solution at random sites, by the oracle: the
    3^4 neighbourhood of each site (links and x_0) is gathered from the
    device and the oracle's site apply gives (D x_0)(site); compared with the
    library's D(mu) x_0 at the same sites."""
    import torch
    from oracle import dirac
    dims = tuple(U_dev.shape[:4])
    rng = np.random.default_rng(seed)
    sites = np.stack([rng.integers(0, d, nsites) for d in dims], axis=1)
    t = time.time()
    # every site's 3^4 neighbourhood in one gather: index [site, o_T, o_Z, o_Y, o_X]
    off = np.arange(-1, 2)
    idx = []
    for d in range(4):
        shape = [nsites, 1, 1, 1, 1]
        shape[1 + d] = 3
        v = (sites[:, d][:, None] + off[None, :]) % dims[d]
        idx.append(torch.as_tensor(v.reshape(shape), device=U_dev.device))
    Up = U_dev[tuple(idx)].cpu().numpy()
    xp = x0_dev[tuple(idx)].cpu().numpy()
    centre = tuple(torch.as_tensor(sites[:, d], device=U_dev.device) for d in range(4))
    bs_all = b0_dev[centre].cpu().numpy()
    ys_all = yx_dev[centre].cpu().numpy()
    num = den = dlib = 0.0
    for k in range(nsites):
        Dx = dirac.apply_at_sites(Up[k], xp[k], KAPPA, CSW, MU, [(1, 1, 1, 1)])[0]
        bs, ys = bs_all[k], ys_all[k]
        num += float(np.sum(np.abs(bs - Dx) ** 2))
        den += float(np.sum(np.abs(bs) ** 2))
        dlib = max(dlib, float(np.abs(ys - Dx).max()) / max(float(np.abs(Dx).max()), 1e-300))
    return {"sites_sampled": int(nsites), "oracle_residual_at_sites": float(np.sqrt(num / den)),
            "dirac_x0_max_rel_diff_at_sites": dlib, "seconds": round(time.time() - t, 1)}


DIRAC_SOURCES = ["dirac.hip", "finedev.hpp", "common.hpp"]


def dirac_sources_sha256():
    """Hash of the sources the D(mu) kernel is built from (same recipe as
    paper_1611_01034_amd.profsum.sources_sha256)."""
    h = hashlib.sha256()
    for f in DIRAC_SOURCES:
        with open(os.path.join(ROOT, "paper_1611_01034_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def traffic_for(kernel_src_hash, nfields):
    """Calibrated HBM bytes per launch of the FP64 D(mu) kernel on nfields
    fields at 48^3x96, from the committed counter record of that launch shape,
    or None when there is none or the kernel sources changed since."""
    tag = f"{nfields}fields_" if nfields > 1 else ""
    p = os.path.join(ROOT, "profiles", f"dirac_fp64_{tag}48x48x48x96_traffic.json")
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
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}): the library runs on one GPU; "
              "how the path would shard is described in the design notes", file=sys.stderr)
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
    need_net = bool(args.learned or args.alt_start)
    if need_net:
        from paper_1611_01034_amd import learned_setup
        wts, C, L, _ = learned_setup.load_weights(learned_setup.WEIGHTS)
        if C != nv[0]:
            raise SystemExit("network channels must equal the level-0 test vector count")

    def start_input(learned):
        """The fine-level input of a start: the network's noise (learned) or
        the Gaussian initial vectors, both complex64 (the setup stores them in
        FP32 or lower) and drawn from the same seed."""
        v = synth.gaussian_device((nv[0],) + dims + (4, 3), 5501, dtype="complex64")
        # the real and imaginary parts it was built from go back to the device
        torch.cuda.empty_cache()
        return v
    torch.cuda.synchronize()

    def make_ctx(Ug, net=False):
        c = ddamg.DDAMG(dims, block, KAPPA, CSW, MU, stream=stream.cuda_stream)
        c.set_gauge(Ug)
        if net:
            c.net_create(L, C)
            c.net_set_params(wts)
        return c

    # two fine post-smoothing sweeps in both forms: on this synthetic field
    # one, three and four sweeps all take more outer iterations
    def params(prec, setup_iters, rhs_batch, batch):
        return ddamg.default_params(levels=levels, block=[block, (2, 2, 2, 2)], nvec=nv, setup_iters=setup_iters,
                                    coarse_setup_iters=3, precision=prec, coarse_mu_factor=5.0, batch=batch,
                                    rhs_batch=rhs_batch, sap_post=SAP_POST)

    ctx = make_ctx(U, net=need_net)
    # the oracle leg takes its slices of the inputs now and runs on the host
    # while the GPU works
    leg = OracleLeg(U, b[0], args.oracle_procs) if args.cpu_baseline else None
    # the device copy of the links is the library's from here on; the site
    # check after the steps regenerates the same seeded field
    del U
    torch.cuda.empty_cache()
    p_mixed = params(args.precision, args.setup_iters, kb, args.batch)
    p_mixed.restart = args.restart
    overrides = {}
    for kv in args.set:
        k, v = kv.split("=", 1)
        overrides[k] = float(v) if "." in v or "e" in v else int(v)
        setattr(p_mixed, k, overrides[k])

    def step(c, tag, learned, init):
        t = time.time()
        if learned:
            c.setup_learned(p_mixed, init, V1)
        else:
            c.setup(p_mixed, [init, V1])
        log(f"{tag}: setup issued ({time.time() - t:.1f} s)")
        _, st = c.solve(b, tol=1e-10, x=x)
        log(f"{tag}: solve done ({time.time() - t:.1f} s, {st['iters']} iterations over {st['nrhs']} rhs, "
            f"{st['iters_min']}-{st['iters_max']} per rhs)")
        return st

    # the other start first (one untimed step on the same inputs), so that it
    # runs with the memory the timed steps use
    other_start = None
    if args.alt_start:
        o_learned = not args.learned
        init = start_input(o_learned)
        torch.cuda.synchronize()
        t = time.time()
        st_o = step(ctx, "other start", o_learned, init)
        torch.cuda.synchronize()
        dt_o = time.time() - t
        other_start = {"start": ("learned" if o_learned else "random") + f"+{args.setup_iters}",
                       "step_s": round(dt_o, 3), "iters_per_rhs": round(st_o["iters"] / max(1, st_o["nrhs"]), 2),
                       "iters_min": st_o["iters_min"], "iters_max": st_o["iters_max"], "resid": st_o["resid"],
                       "note": "one untimed step before the warm-up steps, same inputs; its first-call "
                               "allocations are in its time"}
        init = None
        torch.cuda.empty_cache()
        ctx.release_memory()
    init = start_input(bool(args.learned))
    torch.cuda.synchronize()
    for i in range(args.warmup):
        step(ctx, f"warmup {i}", bool(args.learned), init)
    torch.cuda.synchronize()
    ctx.timing(True)
    t0 = time.time()
    stats = None
    for i in range(args.steps):
        stats = step(ctx, f"step {i}", bool(args.learned), init)
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
    yb_slices = None
    sites_check = None
    if leg is not None:
        # the library's D(mu) b_0 on the oracle's slices, and the oracle's
        # b - D x at random sites of the first solution
        yb = ctx.apply_dirac(b[0])
        yb_slices = {t: yb[t].cpu().numpy() for t in leg.ts}
        del yb
        yx = ctx.apply_dirac(x[0])
        Ud = synth.gauge_field_device(dims, 0.3, 5001)
        sites_check = oracle_sites(Ud, x[0], b[0], yx, args.oracle_sites)
        del yx, Ud
        torch.cuda.empty_cache()
        log(f"oracle at {args.oracle_sites} random sites: {sites_check}")

    # D(mu) FP64 bandwidth inside the timed steps (HIP events around every
    # launch); each launch applies the operator to the K fields of a lock-step
    # group and reads the links and clover once: (1152 + 384 K) B per site
    avg_ms = ms_d / max(n_d, 1)
    bytes_d = ctx.timing_bytes(0)
    bytes_launch = bytes_d / max(n_d, 1)
    d_fields = int(round((bytes_launch / V - 1152) / 384)) if n_d else 0
    achieved = bytes_d / (ms_d * 1e-3) / 1e9 if n_d else None
    src_hash = dirac_sources_sha256()
    d_traffic = traffic_for(src_hash, d_fields)
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

    # the one-field D(mu) launch (ddamg_apply_dirac's form) on resident
    # fields, after the timed steps and outside them: the D(mu) GB/s of a
    # single application
    ctx.timing(True)
    ctx.bench_dirac(10, "fp64")
    n_1, ms_1 = ctx.timing_query(0)
    bytes_1 = ctx.timing_bytes(0)
    ctx.timing(False)
    one_field = None
    if n_1 and ms_1 > 0:
        a1 = bytes_1 / (ms_1 * 1e-3) / 1e9
        t1 = traffic_for(src_hash, 1)
        one_field = {"kernel": "D(mu) FP64 full-lattice apply, one field per launch (10 launches after the steps)",
                     "achieved": round(a1, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(a1 / HBM_PEAK_GBS, 4), "traffic": t1,
                     "algorithmic_bytes_per_launch": bytes_1 / n_1, "avg_launch_ms": round(ms_1 / n_1, 4)}

    ctx.close()
    del ctx
    torch.cuda.empty_cache()

    fp64_s = None
    fp64_stats = None
    fp64_note = None
    if args.fp64_compare:
        elapsed = time.time() - T_START
        # the FP64 form has run 21-25x the mixed step on this lattice; 26x
        # keeps a margin so that the leg never overruns the budget
        projected = 26.0 * dt * max(1.0, args.nrhs / 12.0)
        if elapsed + projected > args.time_budget:
            fp64_note = (f"skipped: {elapsed:.0f} s elapsed + about {projected:.0f} s projected exceeds the "
                         f"{args.time_budget:.0f} s budget of this run")
            log("fp64:", fp64_note)
        else:
            init = None
            torch.cuda.empty_cache()
            V0 = synth.gaussian_device((nv[0],) + dims + (4, 3), 5501)
            U = synth.gauge_field_device(dims, 0.3, 5001)
            c64 = make_ctx(U)
            del U
            torch.cuda.empty_cache()
            c64.set_progress(lambda stage, level, i: log(
                f"fp64: setup level {level} " + ("initial phase done" if stage == 0 else f"iteration {i + 1} done")))
            # FP64 fine fields are twice the size: 4 test vectors per setup batch
            p64 = params("fp64", args.fp64_setup_iters, min(args.fp64_rhs_batch, args.nrhs), min(args.batch, 4))
            for k, v in overrides.items():  # the same solver parameters in both forms
                setattr(p64, k, v)
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
    if leg is not None:
        cpu, check = leg.result(yb_slices)
        check.update(sites_check)
        log(f"oracle: {cpu and cpu['value']} GB/s on {cpu and cpu['cores']} processes, check {check}")

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
                               f"Nv 24/32, {SAP_POST} fine post-smoothing SAP sweeps), {args.nrhs} rhs ({kb} in lock step, "
                               f"outer restart {args.restart}), "
                               f"{'learned' if args.learned else 'random'} initial test vectors + "
                               f"{args.setup_iters} setup iteration(s) on batches of {args.batch} test vectors, "
                               f"preconditioner {args.precision}, outer FGMRES FP64, tol 1e-10"
                               + (f", overrides {overrides}" if overrides else ""),
                   "global_batch": args.nrhs, "parallelism": "none"},
        "roofline": {"bound": "hbm", "kernel": f"D(mu) FP64 full-lattice apply on the {d_fields} fields of a "
                                               f"lock-step group per launch",
                     "achieved": round(achieved, 1) if achieved else None, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4) if achieved else None,
                     "traffic": d_traffic, "algorithmic_bytes_per_launch": bytes_launch,
                     "traffic_gbs": round(d_traffic / (avg_ms * 1e-3) / 1e9, 1) if d_traffic and n_d else None,
                     "fields_per_launch": d_fields, "launches": n_d, "avg_launch_ms": round(avg_ms, 4),
                     "ms_per_field": round(avg_ms / max(d_fields, 1), 4), "one_field": one_field},
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
        "other_start": other_start,
        "kernel_ms": {k: {"launches": v[0], "ms": round(v[1], 2)} for k, v in kinds.items()},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
