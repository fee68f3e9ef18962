"""Profiling driver for the coarse operators: a three-level hierarchy on a
seeded synthetic field (injected random test vectors, no setup iterations:
only the operators matter here), then timed applications of the K-column
coarse operator of each coarse level, the full stencil and the coarsest
odd-even reduced operator, for several K.

Algorithmic bytes of one K-column stencil application (each datum once):
  per coarse site  5 n^2 s  (self + 4 forward blocks, s bytes per complex entry)
                 + 2 K n 8  (FP32 complex input and output, K fields)
and of the odd-even reduced operator (two passes, hop blocks of both parities
and the odd-site inverses once, input, intermediate and output fields):
  5 n^2 s N + n^2 8 N/2 + 4 K n 8 N/2     (N coarse sites).

    python -m paper_1611_01034_amd.profile_coarse --dims 64,32,32,32 --precision bf16
"""
import argparse
import json
import sys

KAPPA, CSW, MU = 0.13729, 1.57551, 0.0009
SBYTES = {"fp64": 16, "fp32": 8, "fp16": 4, "bf16": 4}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--dims", default="64,32,32,32", help="T,Z,Y,X")
    ap.add_argument("--precision", default="bf16")
    ap.add_argument("--nvec", default="24,32")
    ap.add_argument("--ks", default="1,4,8,12,16")
    ap.add_argument("--napply", type=int, default=20)
    a = ap.parse_args()

    import numpy as np
    import torch

    from . import ddamg, synth

    dims = tuple(int(x) for x in a.dims.split(","))
    nv = [int(x) for x in a.nvec.split(",")]
    torch.cuda.set_device(0)
    st = torch.cuda.current_stream()
    cd = tuple(d // 4 for d in dims)
    U = synth.gauge_field_device(dims, 0.3, 5001)
    V0 = synth.gaussian_device((nv[0],) + dims + (4, 3), 5501)
    V1 = synth.gaussian_device((nv[1],) + cd + (2 * nv[0],), 5502)
    rows = []
    with ddamg.DDAMG(dims, (4, 4, 4, 4), KAPPA, CSW, MU, stream=st.cuda_stream) as ctx:
        ctx.set_gauge(U)
        p = ddamg.default_params(levels=3, block=[(4, 4, 4, 4), (2, 2, 2, 2)], nvec=nv, precision=a.precision,
                                 coarse_mu_factor=5.0)
        ctx.set_test_vectors(p, [V0, V1])
        del V0
        torch.cuda.synchronize()
        s = SBYTES[a.precision]
        for level, which in ((1, 0), (2, 0), (2, 1)):
            n = 2 * nv[level - 1]
            N = int(np.prod(cd)) if level == 1 else int(np.prod(cd)) // 16
            for K in (int(k) for k in a.ks.split(",")):
                ctx.bench_coarse(level, K, 2, which)
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                torch.cuda.synchronize()
                e0.record(st)
                ctx.bench_coarse(level, K, a.napply, which)
                e1.record(st)
                torch.cuda.synchronize()
                ms = e0.elapsed_time(e1) / a.napply
                if which == 0:
                    byts = N * (5 * n * n * s + 2 * K * n * 8)
                else:
                    byts = 5 * n * n * s * N + n * n * 8 * N // 2 + 4 * K * n * 8 * N // 2
                flops = 8.0 * K * (9 * n * n * N + (n * n * N / 2 if which else 0))
                row = {"level": level, "op": "stencil" if which == 0 else "odd-even", "n": n, "sites": N, "K": K,
                       "ms": ms, "GB/s": byts / ms / 1e6, "TFLOP/s": flops / ms / 1e9,
                       "ms_per_rhs": ms / K}
                rows.append(row)
                print(json.dumps(row), flush=True)
    print(json.dumps({"precision": a.precision, "dims": dims, "rows": len(rows)}), flush=True)


if __name__ == "__main__":
    sys.exit(main())
