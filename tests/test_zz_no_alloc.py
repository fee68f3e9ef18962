"""ddamg_apply_dirac_noalloc against ddamg_apply_dirac (FP64, Sec. 1 D(+-mu)),
through the C interface on the GPU: two calls in a row on two lattices, the
second smaller, each bit-identical to the allocating entry point (same
kernels) and within 1e-12 of it by the FP64 operator bar; no device memory
is taken by the call; a lattice above the scratch limit is rejected."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

KAPPA, CSW, MU = 0.13729, 1.57551, 0.0009


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    return torch.device("cuda:0")


def _case(dims, block, seed):
    from paper_1611_01034_amd import ddamg, synth
    dev = _dev()
    U = synth.gauge_field_device(dims, 0.3, seed)
    psi = synth.gaussian_device(dims + (4, 3), seed + 1)
    stream = torch.cuda.current_stream().cuda_stream
    ctx = ddamg.DDAMG(dims, block, KAPPA, CSW, MU, stream=stream)
    ctx.set_gauge(U)
    return ctx, psi


def test_noalloc_matches_allocating_entry_point_two_calls():
    _dev()
    cases = [((32, 16, 16, 16), (4, 4, 4, 4), 7101, +1),   # 131072 sites: the scratch limit
             ((8, 4, 4, 8), (2, 2, 2, 2), 7201, -1)]       # a smaller lattice afterwards
    for dims, block, seed, sign in cases:
        print(f"no-alloc D(mu): dims {dims}, sign {sign}", flush=True)
        ctx, psi = _case(dims, block, seed)
        try:
            ref = ctx.apply_dirac(psi, sign=sign)
            out = torch.full_like(psi, complex(np.nan, np.nan))
            torch.cuda.synchronize()
            free0 = torch.cuda.mem_get_info()[0]
            ctx.apply_dirac_noalloc(psi, out, sign=sign)
            torch.cuda.synchronize()
            free1 = torch.cuda.mem_get_info()[0]
            assert free1 == free0, "the no-allocation entry point took device memory"
            assert torch.equal(out, ref)
            rel = float(torch.linalg.vector_norm(out - ref) / torch.linalg.vector_norm(ref))
            assert rel <= 1e-12
        finally:
            ctx.close()


def test_noalloc_rejects_lattice_above_limit():
    from paper_1611_01034_amd import ddamg
    ctx, psi = _case((48, 16, 16, 16), (4, 4, 4, 4), 7301)
    try:
        out = torch.empty_like(psi)
        with pytest.raises(ddamg.DDAMGError) as e:
            ctx.apply_dirac_noalloc(psi, out)
        assert e.value.status == ddamg.INVALID_ARG
    finally:
        ctx.close()
