"""Profiling driver for the fine SAP smoother: a fixed number of SAP iterations
(two colour sweeps each) on --nfields fields at once (one launch per colour
for all of them, as in the setup and the lock-step solve) on a seeded
synthetic field.  Run under rocprofv3, e.g.

    rocprofv3 --pmc SQ_WAVES SQ_INSTS_VALU -f csv -d OUT -o sq -- \\
        python -m paper_1611_01034_amd.profile_sap --dims 96,48,48,48

Every sweep runs in libddamg (the SAP entry point uploads b and x0 and
converts them to the requested precision on the device); nothing here
computes the smoother.
"""
import argparse

KAPPA, CSW, MU = 0.13729, 1.57551, 0.0009


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--dims", type=str, default="96,48,48,48", help="T,Z,Y,X")
    ap.add_argument("--iters", type=int, default=2)
    ap.add_argument("--mr-steps", type=int, default=4)
    ap.add_argument("--precision", type=str, default="fp32")
    ap.add_argument("--eps", type=float, default=0.3)
    ap.add_argument("--seed", type=int, default=5001)
    ap.add_argument("--nfields", type=int, default=1)
    a = ap.parse_args()

    import numpy as np
    import torch

    from . import ddamg, synth

    dims = tuple(int(x) for x in a.dims.split(","))
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    U = synth.gauge_field_device(dims, a.eps, a.seed)
    b = np.stack([synth.spinor(dims, a.seed + 1 + k) for k in range(a.nfields)])
    x0 = np.zeros_like(b)
    with ddamg.DDAMG(dims, (4, 4, 4, 4), KAPPA, CSW, MU, stream=stream.cuda_stream) as ctx:
        ctx.set_gauge(U)
        del U
        torch.cuda.synchronize()
        x = ctx.sap_multi(b, x0, a.iters, a.mr_steps, a.precision)
        torch.cuda.synchronize()
    print(f"profile_sap: dims {dims}, {a.nfields} field(s), {a.iters} SAP iterations ({a.mr_steps} MR steps) "
          f"{a.precision}, "
          f"|x| = {float(np.linalg.norm(x)):.6e}", flush=True)


if __name__ == "__main__":
    main()
