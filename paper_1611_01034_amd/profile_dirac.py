"""Profiling driver for the fine operator: a fixed number of D(mu) applies on
a seeded synthetic field (or, with --nfields K > 1, on K Gaussian fields in
one launch each, as the lock-step outer solve applies it), followed by a
plain device copy of known size.

The copy calibrates rocprofv3's HBM byte counters (FETCH_SIZE, WRITE_SIZE):
it reads and writes exactly `--copy-mib` MiB, so counter / known bytes is the
scale factor applied to the D(mu) readings.  Run under rocprofv3, e.g.

    rocprofv3 --pmc FETCH_SIZE -f csv -d OUT -o fetch -- \\
        python -m paper_1611_01034_amd.profile_dirac --dims 96,48,48,48

Every step runs in libddamg (D(mu)) or is a single torch elementwise kernel
(the copy); nothing here computes the operator.
"""
import argparse
import sys

KAPPA, CSW, MU = 0.13729, 1.57551, 0.0009


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--dims", type=str, default="96,48,48,48", help="T,Z,Y,X")
    ap.add_argument("--napply", type=int, default=10)
    ap.add_argument("--precision", type=str, default="fp64")
    ap.add_argument("--copy-mib", type=int, default=2048)
    ap.add_argument("--eps", type=float, default=0.3)
    ap.add_argument("--seed", type=int, default=5001)
    ap.add_argument("--nfields", type=int, default=1)
    a = ap.parse_args()

    import torch

    from . import ddamg, synth

    dims = tuple(int(x) for x in a.dims.split(","))
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    U = synth.gauge_field_device(dims, a.eps, a.seed)
    with ddamg.DDAMG(dims, (4, 4, 4, 4), KAPPA, CSW, MU, stream=stream.cuda_stream) as ctx:
        ctx.set_gauge(U)
        del U
        torch.cuda.synchronize()
        if a.nfields == 1:
            ctx.bench_dirac(a.napply, a.precision)
        else:
            psis = synth.gaussian_device((a.nfields,) + dims + (4, 3), a.seed + 1)
            torch.cuda.empty_cache()
            for _ in range(a.napply):
                ctx.apply_dirac_multi(psis, precision=a.precision)
        torch.cuda.synchronize()
    n = a.copy_mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()
    print(f"profile_dirac: dims {dims}, {a.napply} x D(mu) {a.precision} on {a.nfields} field(s), "
          f"copy {a.copy_mib} MiB read + {a.copy_mib} MiB written x 3", flush=True)


if __name__ == "__main__":
    sys.exit(main())
