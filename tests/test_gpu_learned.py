"""What the trained network gains over the method without it.

The committed weights (trained on the GPU by the library's own forward,
backward and Adam kernels on 64 fields with eps in {0.2, 0.3, 0.4}) propose the
initial test vectors of the adaptive setup on held-out fields (seeds 4100..,
not used in training; eps 0.48 is not a training roughness at all).  Judged by
multigrid outcomes only: FGMRES iterations to a 1e-10 true residual and the
V-cycle error-reduction factor rho, against Gaussian initial vectors with the
same number of refinement iterations."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ls():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1611_01034_amd import learned_setup
    return learned_setup


@pytest.mark.parametrize("eps", [0.3, 0.48])
def test_learned_start_beats_random_start(ls, eps):
    params, C, L, _ = ls.load_weights(ls.WEIGHTS)
    rows = ls.evaluate((16, 8, 8, 8), (4, 4, 4, 4), range(4100, 4104), eps, params, C=C, L=L, nvec=C,
                       log=lambda *a: None)
    it = {k: np.array([r[k]["iters"] for r in rows]) for k in rows[0] if k != "seed"}
    rho = {k: np.array([r[k]["rho"] for r in rows]) for k in rows[0] if k != "seed"}
    # no refinement: the network's vectors against smoothed noise
    assert np.all(it["learned+0"] < it["random+0"]), (it["learned+0"], it["random+0"])
    assert it["learned+0"].mean() <= 0.8 * it["random+0"].mean()
    assert rho["learned+0"].mean() < rho["random+0"].mean()
    if eps == 0.48:
        # one refinement iteration, roughness outside the training set
        assert np.all(it["learned+1"] <= it["random+1"]), (it["learned+1"], it["random+1"])
        assert it["learned+1"].mean() < it["random+1"].mean()
        assert rho["learned+1"].mean() < rho["random+1"].mean()


def test_setup_learned_equals_setup_on_network_output(ls):
    # the fused entry point (noise -> network -> setup on the device) gives the
    # hierarchy of the plain setup started from the network's output; complex64
    # and complex128 noise reach the FP32 network identically
    from paper_1611_01034_amd import ddamg, synth
    params, C, L, _ = ls.load_weights(ls.WEIGHTS)
    dims, block = (8, 8, 8, 8), (2, 2, 2, 2)
    U = synth.gauge_field(dims, 0.3, 4200)
    noise = synth.spinor(dims, 4201, nvec=C)
    p = ddamg.default_params(levels=2, block=[block], nvec=[C], setup_iters=1, precision="fp32",
                             coarse_mu_factor=5.0)
    Q = []
    with ddamg.DDAMG(dims, block, ls.KAPPA, ls.CSW, ls.MU) as ctx:
        ctx.set_gauge(U)
        ctx.net_create(L, C)
        ctx.net_set_params(params)
        ctx.setup(p, [ctx.net_forward(noise)])
        Q.append(ctx.get_interpolation(0))
        ctx.setup_learned(p, noise)
        Q.append(ctx.get_interpolation(0))
        ctx.setup_learned(p, noise.astype(np.complex64))
        Q.append(ctx.get_interpolation(0))
    assert np.linalg.norm(Q[1] - Q[0]) <= 1e-6 * np.linalg.norm(Q[0])
    assert np.array_equal(Q[2], Q[1])


def test_fallback_to_plain_setup(ls):
    # a network that maps everything to zero cannot start the setup (every
    # aggregate is rank deficient): the plain setup runs instead and the solve
    # converges; the trained network on a near-critical field keeps its start
    from oracle import dirac
    from paper_1611_01034_amd import ddamg, synth
    params, C, L, _ = ls.load_weights(ls.WEIGHTS)
    dims, block = (8, 8, 8, 8), (4, 4, 4, 4)
    U = synth.gauge_field(dims, 0.48, 4210)
    noise = synth.spinor(dims, 4211, nvec=C)
    probe = synth.spinor(dims, 4212)
    plain = lambda: [synth.spinor(dims, 4213, nvec=C)]
    p = ddamg.default_params(levels=2, block=[block], nvec=[C], setup_iters=1, precision="fp32", coarse_mu_factor=5.0)
    b = synth.spinor(dims, 4214)
    op = dirac.WilsonClover(U, ls.KAPPA, ls.CSW, ls.MU)
    with ddamg.DDAMG(dims, block, ls.KAPPA, ls.CSW, ls.MU) as ctx:
        ctx.set_gauge(U)
        ctx.net_create(L, C)
        ctx.net_set_params(np.zeros_like(params))
        info = ls.setup_with_fallback(ctx, p, noise, None, plain, probe)
        assert info["fallback"] and not np.isfinite(info["rho_learned"]) and info["rho"] < 0.9
        x, st = ctx.solve(b, tol=1e-10)
        assert np.linalg.norm(b - op.apply(x)) <= 1e-10 * np.linalg.norm(b)
        # a finite but useless start: the probe rejects it against a tight reference
        ctx.net_set_params(params)
        info = ls.setup_with_fallback(ctx, p, noise, None, plain, probe, rho_ref=1e-3)
        assert info["fallback"] and np.isfinite(info["rho_learned"]) and info["rho_learned"] > 1e-3
        # the trained network keeps its start at the default reference
        info = ls.setup_with_fallback(ctx, p, noise, None, plain, probe)
        assert not info["fallback"] and info["rho_learned"] < 0.9
        x, st = ctx.solve(b, tol=1e-10)
        assert np.linalg.norm(b - op.apply(x)) <= 1e-10 * np.linalg.norm(b)
