"""GPU parity: the HIP path through the C interface against the CPU oracle.

Tolerances: FP64 operator applies <= 1e-12 relative (element by element over
the whole field); FP64 compositions of a few operators (SAP, V-cycle with
fixed iteration counts) <= 1e-10; FP32 storage: the relative error of one
apply is bounded by a few units of 2^-24 times the number of terms summed,
<= 2e-6; FP16 / BF16 links: <= 4e-3 / 3e-2.
"""
import numpy as np
import pytest

from oracle import aggregation as agg
from oracle import coarse, dirac, mg, sap, stencil
from paper_1611_01034_amd import synth

pytestmark = pytest.mark.gpu

KAPPA, CSW, MU = 0.13729, 1.57551, 0.0009


def rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b))


@pytest.fixture(scope="module")
def dd():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1611_01034_amd import ddamg
    return ddamg


def make(dd, dims, block, seed=1001, mu=MU, eps=0.3):
    U = synth.gauge_field(dims, eps, seed)
    ctx = dd.DDAMG(dims, block, KAPPA, CSW, mu)
    ctx.set_gauge(U)
    return ctx, dirac.WilsonClover(U, KAPPA, CSW, mu), U


CASES = [((4, 4, 4, 4), (2, 2, 2, 2)), ((4, 8, 4, 12), (2, 2, 2, 2)), ((8, 8, 8, 16), (4, 4, 4, 4)),
         ((8, 4, 8, 8), (4, 2, 4, 2))]


@pytest.mark.parametrize("dims,block", CASES)
def test_clover_term(dd, dims, block):
    ctx, op, _ = make(dd, dims, block)
    got = ctx.get_clover()
    want = dirac.clover_blocks(op.A)
    assert np.abs(got - want).max() < 1e-13


@pytest.mark.parametrize("dims,block", CASES)
@pytest.mark.parametrize("sign", [1, -1])
def test_dirac_fp64(dd, dims, block, sign):
    ctx, op, _ = make(dd, dims, block, mu=0.05)
    psi = synth.spinor(dims, 7)
    got = ctx.apply_dirac(psi, sign=sign)
    want = op.apply(psi, sign * op.mu)
    assert rel(got, want) < 1e-12
    assert np.abs(got - want).max() < 1e-12 * np.abs(want).max()


# K fields per launch: the first case sweeps blocks per XCD range, the other
# two in XCD groups of two block rows (both block sizes)
MULTI_CASES = [((8, 8, 8, 16), (4, 4, 4, 4)), ((16, 8, 8, 16), (4, 4, 4, 4)), ((4, 8, 4, 12), (2, 2, 2, 2))]


@pytest.mark.parametrize("dims,block", MULTI_CASES)
@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
def test_dirac_multi_fields(dd, dims, block, prec):
    """D(-mu) on K = 3 fields in one launch: every field bit-identical to the
    one-field apply; in FP64 element by element against the oracle."""
    ctx, op, _ = make(dd, dims, block, mu=0.05)
    K = 3
    psis = np.stack([synth.spinor(dims, 20 + k) for k in range(K)])
    got = ctx.apply_dirac_multi(psis, sign=-1, precision=prec)
    for k in range(K):
        assert np.array_equal(got[k], ctx.apply_dirac(psis[k], sign=-1, precision=prec))
        if prec == "fp64":
            want = op.apply(psis[k], -op.mu)
            assert rel(got[k], want) < 1e-12
            assert np.abs(got[k] - want).max() < 1e-12 * np.abs(want).max()


def test_dirac_multi_device_fields_and_limits(dd):
    torch = pytest.importorskip("torch")
    dims, block = (16, 8, 8, 16), (4, 4, 4, 4)
    ctx, op, _ = make(dd, dims, block)
    psis = np.stack([synth.spinor(dims, 30 + k) for k in range(5)])
    got = ctx.apply_dirac_multi(torch.from_numpy(psis).cuda()).cpu().numpy()
    assert np.array_equal(got, ctx.apply_dirac_multi(psis))
    assert rel(got[4], op.apply(psis[4])) < 1e-12
    with pytest.raises(dd.DDAMGError):
        ctx.apply_dirac_multi(np.zeros((17,) + dims + (4, 3), np.complex128))


@pytest.mark.parametrize("prec,tol", [("fp32", 2e-6), ("fp16", 4e-3), ("bf16", 3e-2)])
def test_dirac_reduced(dd, prec, tol):
    dims, block = (8, 8, 8, 16), (4, 4, 4, 4)
    ctx, op, _ = make(dd, dims, block)
    psi = synth.spinor(dims, 8)
    err = rel(ctx.apply_dirac(psi, precision=prec), op.apply(psi))
    assert err < tol, err


@pytest.mark.parametrize("dims,block", CASES)
def test_sap_fp64(dd, dims, block):
    ctx, op, _ = make(dd, dims, block, mu=0.02)
    fl = stencil.FineLevel(op)
    b = synth.spinor(dims, 9)
    x0 = synth.spinor(dims, 10)
    got = ctx.sap(b, x0, iters=2, mr_steps=4)
    want = sap.sap(fl, b.reshape(dims + (12,)), x0.reshape(dims + (12,)), block, 4, 2)
    assert rel(got.reshape(dims + (12,)), want) < 1e-11


def test_sap_fp32(dd):
    dims, block = (8, 8, 8, 16), (4, 4, 4, 4)
    ctx, op, _ = make(dd, dims, block)
    fl = stencil.FineLevel(op)
    b = synth.spinor(dims, 11)
    x0 = np.zeros_like(b)
    got = ctx.sap(b, x0, iters=1, mr_steps=4, precision="fp32")
    want = sap.sap(fl, b.reshape(dims + (12,)), x0.reshape(dims + (12,)), block, 4, 1)
    assert rel(got.reshape(dims + (12,)), want) < 1e-5


def _two_level(dd, dims, block, nv, delta=1.0, mu=MU, **kw):
    ctx, op, U = make(dd, dims, block, mu=mu)
    V = synth.gaussian((nv,) + dims + (12,), 1501)
    p = dd.default_params(levels=2, block=[block], nvec=[nv], coarse_mu_factor=delta, **kw)
    ctx.set_test_vectors(p, [V.reshape((nv,) + dims + (4, 3))])
    op_params = mg.Params(levels=2, blocks=[block], nvec=[nv], delta=delta,
                          coarse_max_iter=p.coarse_max_iter, coarse_restart=p.coarse_restart,
                          coarse_tol=p.coarse_tol, sap_post=p.sap_post, mr_steps=p.mr_steps,
                          fixed=bool(p.fixed_iters))
    h = mg.Hierarchy(op, op_params).set_test_vectors([V])
    return ctx, op, h, V


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
@pytest.mark.parametrize("K", [1, 2, 3, 5, 6, 8])
def test_transfers_k_columns(dd, prec, tol, K):
    """The K-column fine restriction and prolongation of the lock-step cycle
    (column groups of 1, 2, 4 and 6, one or two passes over P) against the
    oracle's P^dag and P with its own test vectors, column by column,
    relative and element-wise."""
    dims, block, nv = (8, 8, 8, 16), (4, 4, 4, 4), 20
    ctx, op, h, V = _two_level(dd, dims, block, nv, delta=5.0, precision=prec)
    Q = h.levels[0].Q
    rs = np.stack([synth.gaussian(dims + (12,), 40 + k) for k in range(K)])
    got = ctx.restrict_multi(0, rs.reshape((K,) + dims + (4, 3)))
    es = np.stack([synth.gaussian(got.shape[1:], 60 + k) for k in range(K)])
    xs = ctx.prolong_multi(0, es).reshape((K,) + dims + (12,))
    for k in range(K):
        want = agg.restrict(Q, rs[k], block)
        assert rel(got[k], want) < tol
        assert np.abs(got[k] - want).max() < tol * np.abs(want).max()
        want = agg.prolong(Q, es[k], block)
        assert rel(xs[k], want) < tol
        assert np.abs(xs[k] - want).max() < tol * np.abs(want).max()


@pytest.mark.parametrize("dims,block,nv", [((4, 4, 4, 4), (2, 2, 2, 2), 8), ((8, 8, 8, 16), (4, 4, 4, 4), 20),
                                          ((8, 4, 8, 8), (4, 2, 4, 2), 12)])
def test_interpolation_transfer_and_coarse_operator(dd, dims, block, nv):
    ctx, op, h, V = _two_level(dd, dims, block, nv, delta=5.0)
    Q = ctx.get_interpolation(0).reshape((nv,) + dims + (12,))
    assert rel(Q, h.levels[0].Q) < 1e-12
    r = synth.gaussian(dims + (12,), 21)
    rc = ctx.restrict(0, r.reshape(dims + (4, 3)))
    assert rel(rc, agg.restrict(h.levels[0].Q, r, block)) < 1e-12
    e = synth.gaussian(rc.shape, 22)
    x = ctx.prolong(0, e).reshape(dims + (12,))
    assert rel(x, agg.prolong(h.levels[0].Q, e, block)) < 1e-12
    S, F = ctx.get_coarse_op(1)
    Dc = h.levels[1].op
    assert rel(S, Dc.S) < 1e-12
    assert rel(F, Dc.F) < 1e-12
    y = synth.gaussian(Dc.dims + (Dc.n,), 23)
    assert rel(ctx.apply_coarse(1, y), Dc.apply(y)) < 1e-12


def test_coarsest_solve_fixed_iterations(dd):
    dims, block, nv = (8, 8, 8, 16), (4, 4, 4, 4), 8
    ctx, op, h, V = _two_level(dd, dims, block, nv, delta=3.0, fixed_iters=1, coarse_max_iter=40,
                               coarse_restart=15)
    Dc = h.levels[1].op
    b = synth.gaussian(Dc.dims + (Dc.n,), 31)
    got = ctx.coarse_solve(1, b)
    want = h.coarse_solve(1, b)
    assert rel(got, want) < 1e-10


def test_vcycle_fixed_iterations(dd):
    dims, block, nv = (8, 8, 8, 16), (4, 4, 4, 4), 8
    ctx, op, h, V = _two_level(dd, dims, block, nv, delta=5.0, fixed_iters=1, coarse_max_iter=20,
                               coarse_restart=10)
    v = synth.gaussian(dims + (12,), 41)
    got = ctx.vcycle(v.reshape(dims + (4, 3))).reshape(dims + (12,))
    want = h.vcycle(0, v)
    assert rel(got, want) < 1e-10


def test_solve_c1_matches_dense_lu(dd):
    # 4^4, eps 0.3, mu 0.0009, delta 1, Nv 8, 2^4 aggregates, 3 setup iterations
    dims, block = (4, 4, 4, 4), (2, 2, 2, 2)
    ctx, op, _ = make(dd, dims, block)
    V0 = synth.spinor(dims, 1501, nvec=8)
    ctx.setup(dd.default_params(levels=2, block=[block], nvec=[8], setup_iters=3), [V0])
    b = synth.spinor(dims, 1101)
    x, st = ctx.solve(b, tol=1e-10)
    r = rel(op.apply(x), b)
    assert st["converged"] and r <= 1e-10
    D = op.dense()
    xs = np.linalg.solve(D, b.reshape(-1)).reshape(b.shape)
    sv = np.linalg.svd(D, compute_uv=False)
    assert rel(x, xs) <= (sv.max() / sv.min()) * 1e-10


@pytest.mark.parametrize("prec", ["fp32", "fp16", "bf16"])
def test_solve_reduced_precision_reaches_fp64_tolerance(dd, prec):
    dims, block = (8, 8, 8, 16), (4, 4, 4, 4)
    ctx, op, _ = make(dd, dims, block)
    V0 = synth.spinor(dims, 2501, nvec=12)
    ctx.setup(dd.default_params(levels=2, block=[block], nvec=[12], setup_iters=2, precision=prec,
                                coarse_mu_factor=5.0), [V0])
    b = synth.spinor(dims, 2101)
    x, st = ctx.solve(b, tol=1e-10)
    assert st["converged"] and rel(op.apply(x), b) <= 1e-10


def test_minus_mu_reuses_setup(dd):
    dims, block = (8, 8, 8, 16), (4, 4, 4, 4)
    ctx, op, _ = make(dd, dims, block)
    V0 = synth.spinor(dims, 2501, nvec=12)
    ctx.setup(dd.default_params(levels=2, block=[block], nvec=[12], setup_iters=2, coarse_mu_factor=3.0), [V0])
    b = synth.spinor(dims, 2102)
    x1, s1 = ctx.solve(b, tol=1e-10)
    ctx.set_mu(-MU)
    x2, s2 = ctx.solve(b, tol=1e-10)
    assert rel(op.apply(x1, MU), b) <= 1e-10 and rel(op.apply(x2, -MU), b) <= 1e-10
    assert abs(s1["iters"] - s2["iters"]) <= max(2, 0.2 * s1["iters"])


def test_squared_operator_as_two_solves(dd):
    # D^dag D x = b as x = D(mu)^-1 G5 D(-mu)^-1 G5 b with one setup for both
    # signs (Sec. 3: the squared operator is inverted by two solves of D;
    # D(mu)^dag = G5 D(-mu) G5)
    dims, block = (8, 8, 8, 16), (4, 4, 4, 4)
    ctx, op, _ = make(dd, dims, block)
    ctx.setup(dd.default_params(levels=2, block=[block], nvec=[12], setup_iters=2, coarse_mu_factor=3.0),
              [synth.spinor(dims, 2511, nvec=12)])
    g5 = np.array([-1.0, -1.0, 1.0, 1.0])[:, None]
    b = synth.spinor(dims, 2512)
    ctx.set_mu(-MU)
    y, s1 = ctx.solve(g5 * b, tol=1e-11)
    ctx.set_mu(MU)
    x, s2 = ctx.solve(g5 * y, tol=1e-11)
    assert s1["converged"] and s2["converged"]
    r = b - g5 * op.apply(g5 * op.apply(x, MU), -MU)
    # r = G5 e1 + D^dag e2 with |e1| <= 1e-11 |b|, |e2| <= 1e-11 |y| and
    # |y| <= |b| / mu (D^dag D = D_W^dag D_W + mu^2); |D| < 16
    assert np.linalg.norm(r) / np.linalg.norm(b) <= 1e-11 * (1 + 16.0 / MU)


@pytest.mark.parametrize("prec", ["fp64", "bf16"])
def test_hasenbusch_shifted_odd_even_systems(dd, prec):
    # (Dhat(mu) + i rho G5hat) x_o = b_o and (G5hat Dhat(-mu) G5hat - i rho G5hat) x_o = b_o
    # through the full operator with the odd-site twist raised by rho (Sec. 3.1)
    dims, block = (8, 8, 8, 16), (4, 4, 4, 4)
    ctx, op, _ = make(dd, dims, block)
    ctx.setup(dd.default_params(levels=2, block=[block], nvec=[12], setup_iters=2, precision=prec,
                                coarse_mu_factor=3.0), [synth.spinor(dims, 2521, nvec=12)])
    g5 = np.array([-1.0, -1.0, 1.0, 1.0])[:, None]
    odd = dirac.odd_mask(dims)[..., None, None]
    b = synth.spinor(dims, 2522)
    _, s0 = ctx.solve(b, tol=1e-10)
    for rho in (0.0, 0.01, 0.1):
        x, st = ctx.solve_odd_shifted(b, rho, tol=1e-10)
        assert st["converged"]
        assert rel(dirac.apply_odd_shifted(op, x, rho), odd * b) <= 1e-10
        assert rel(dirac.schur_odd(op, x, rho), odd * b) <= 1e-9
    # the setup's own twist is back: the plain solve repeats itself
    x, s1 = ctx.solve(b, tol=1e-10)
    assert s1["iters"] == s0["iters"] and rel(op.apply(x), b) <= 1e-10
    rho = 0.01
    ctx.set_mu(-MU)
    y, st = ctx.solve_odd_shifted(g5 * b, -rho, tol=1e-10)
    ctx.set_mu(MU)
    assert st["converged"]
    x = g5 * y
    # G5hat (Dhat(-mu) - i rho G5hat) G5hat x_o = b_o
    assert rel(g5 * dirac.schur_odd(op, g5 * x, -rho, -MU), odd * b) <= 1e-9


# ------------------------------------------------------------------ twisted boundary conditions (Sec. 2)

THETA = (np.pi, 0.4, -1.3, 2.0)


@pytest.mark.parametrize("dims,block", CASES[2:])
def test_dirac_and_sap_twisted_boundary(dd, dims, block):
    U = synth.gauge_field(dims, 0.3, 1001)
    op = dirac.WilsonClover(U, KAPPA, CSW, 0.05, theta=THETA)
    psi = synth.spinor(dims, 8)
    ctx = dd.DDAMG(dims, block, KAPPA, CSW, 0.05)
    ctx.set_boundary_phases(THETA)
    ctx.set_gauge(U)
    assert rel(ctx.apply_dirac(psi), op.apply(psi)) < 1e-12
    assert rel(ctx.apply_dirac(psi, sign=-1), op.apply(psi, -op.mu)) < 1e-12
    assert np.abs(ctx.get_clover() - dirac.clover_blocks(op.A)).max() < 1e-13
    x0 = np.zeros_like(psi)
    got = ctx.sap(psi, x0, iters=2, mr_steps=4, precision="fp64")
    want = sap.sap(stencil.FineLevel(op), psi.reshape(dims + (12,)), x0.reshape(dims + (12,)), block, 4, 2)
    assert rel(got.reshape(dims + (12,)), want) < 1e-11
    # phases changed with the field in place
    ctx.set_boundary_phases((0.3, 0.0, 0.0, 0.0))
    ctx.set_boundary_phases(THETA)
    assert rel(ctx.apply_dirac(psi), op.apply(psi)) < 1e-12
    ctx.set_boundary_phases((0.0, 0.0, 0.0, 0.0))
    assert rel(ctx.apply_dirac(psi), dirac.WilsonClover(U, KAPPA, CSW, 0.05).apply(psi)) < 1e-12
    with pytest.raises(dd.DDAMGError):
        ctx.set_boundary_phases((np.nan, 0.0, 0.0, 0.0))
    ctx.close()


def test_coarse_operator_twisted_boundary(dd):
    dims, block, nv = (8, 4, 8, 8), (4, 2, 4, 2), 8
    U = synth.gauge_field(dims, 0.3, 1001)
    op = dirac.WilsonClover(U, KAPPA, CSW, MU, theta=THETA)
    ctx = dd.DDAMG(dims, block, KAPPA, CSW, MU)
    ctx.set_boundary_phases(THETA)
    ctx.set_gauge(U)
    V = synth.gaussian((nv,) + dims + (12,), 2903)
    ctx.set_test_vectors(dd.default_params(levels=2, block=[block], nvec=[nv], coarse_mu_factor=5.0),
                         [V.reshape((nv,) + dims + (4, 3))])
    h = mg.Hierarchy(op, mg.Params(levels=2, blocks=[block], nvec=[nv], delta=5.0)).set_test_vectors([V])
    S, F = ctx.get_coarse_op(1)
    assert rel(S, h.levels[1].op.S) < 1e-12
    assert rel(F, h.levels[1].op.F) < 1e-12
    ctx.close()


@pytest.mark.parametrize("prec", ["fp64", "bf16"])
def test_solve_twisted_boundary(dd, prec):
    dims, block = (8, 8, 8, 16), (4, 4, 4, 4)
    U = synth.gauge_field(dims, 0.3, 1001)
    op = dirac.WilsonClover(U, KAPPA, CSW, MU, theta=THETA)
    ctx = dd.DDAMG(dims, block, KAPPA, CSW, MU)
    ctx.set_boundary_phases(THETA)
    ctx.set_gauge(U)
    ctx.setup(dd.default_params(levels=2, block=[block], nvec=[12], setup_iters=2, precision=prec,
                                coarse_mu_factor=3.0), [synth.spinor(dims, 2901, nvec=12)])
    b = synth.spinor(dims, 2902)
    x, st = ctx.solve(b, tol=1e-10)
    assert st["converged"] and rel(op.apply(x), b) <= 1e-10
    ctx.close()


# ------------------------------------------------------------------ setup update (Sec. 3.1)

def _perturbed(U, eta, seed):
    """exp(i eta H') U on every link: a small random step of the field."""
    W = synth.gauge_field(U.shape[:4], eta, seed)
    return np.einsum("...ab,...bc->...ac", W, U)


def test_update_gauge_without_iterations_is_galerkin_of_old_interpolation(dd):
    dims, block, nv = (8, 8, 8, 16), (4, 4, 4, 4), 12
    ctx, op, U = make(dd, dims, block)
    p = dd.default_params(levels=2, block=[block], nvec=[nv], setup_iters=1, coarse_mu_factor=3.0)
    ctx.setup(p, [synth.spinor(dims, 2601, nvec=nv)])
    Q = ctx.get_interpolation(0).reshape((nv,) + dims + (12,))
    U2 = _perturbed(U, 0.05, 2602)
    ctx.update_gauge(U2, dd.default_params(levels=2, block=[block], nvec=[nv], setup_iters=0, init_sap_iters=0,
                                           coarse_mu_factor=3.0))
    op2 = dirac.WilsonClover(U2, KAPPA, CSW, MU)
    psi = synth.spinor(dims, 2603)
    assert rel(ctx.apply_dirac(psi), op2.apply(psi)) < 1e-12
    h = mg.Hierarchy(op2, mg.Params(levels=2, blocks=[block], nvec=[nv], delta=3.0)).set_test_vectors([Q])
    # the old basis is already orthonormal per aggregate half: QR keeps it
    assert rel(h.levels[0].Q, Q) < 1e-13
    assert rel(ctx.get_interpolation(0).reshape(Q.shape), Q) < 1e-12
    S, F = ctx.get_coarse_op(1)
    assert rel(S, h.levels[1].op.S) < 1e-12
    assert rel(F, h.levels[1].op.F) < 1e-12


@pytest.mark.parametrize("prec", ["fp64", "bf16"])
def test_update_gauge_iteration_counts(dd, prec):
    # after small changes of the field, one fine setup iteration on the kept
    # test vectors gives the outer iteration count of a new full setup
    dims, block, nv = (8, 8, 8, 16), (4, 4, 4, 4), 12
    ctx, op, U = make(dd, dims, block)
    kw = dict(levels=2, block=[block], nvec=[nv], coarse_mu_factor=3.0, precision=prec, keep_test_vectors=1)
    V0 = synth.spinor(dims, 2701, nvec=nv)
    ctx.setup(dd.default_params(setup_iters=3, **kw), [V0])
    b = synth.spinor(dims, 2702)
    U2 = U
    for step in range(3):
        U2 = _perturbed(U2, 0.02, 2710 + step)
        ctx.update_gauge(U2, dd.default_params(setup_iters=1, init_sap_iters=0, **kw))
        x, s = ctx.solve(b, tol=1e-10)
        op2 = dirac.WilsonClover(U2, KAPPA, CSW, MU)
        assert s["converged"] and rel(op2.apply(x), b) <= 1e-10
        fresh = dd.DDAMG(dims, block, KAPPA, CSW, MU)
        fresh.set_gauge(U2)
        fresh.setup(dd.default_params(setup_iters=3, **kw), [V0])
        _, sf = fresh.solve(b, tol=1e-10)
        fresh.close()
        assert s["iters"] <= sf["iters"] + max(2, 0.2 * sf["iters"]), (step, s["iters"], sf["iters"])


def test_update_gauge_rejects_other_shapes(dd):
    dims, block = (8, 8, 8, 16), (4, 4, 4, 4)
    ctx, op, U = make(dd, dims, block)
    with pytest.raises(dd.DDAMGError):
        ctx.update_gauge(U, dd.default_params(levels=2, block=[block], nvec=[8]))  # no setup yet
    ctx.setup(dd.default_params(levels=2, block=[block], nvec=[8], setup_iters=0),
              [synth.spinor(dims, 2801, nvec=8)])
    with pytest.raises(dd.DDAMGError):
        ctx.update_gauge(U, dd.default_params(levels=2, block=[block], nvec=[10], setup_iters=0))
    bad = U.copy()
    bad[0, 0, 0, 0, 0, 0, 0] = np.nan
    with pytest.raises(dd.DDAMGError):
        ctx.update_gauge(bad, dd.default_params(levels=2, block=[block], nvec=[8], setup_iters=0))
    # the failed calls left the setup in place
    b = synth.spinor(dims, 2802)
    x, st = ctx.solve(b, tol=1e-10)
    assert rel(op.apply(x), b) <= 1e-10


def test_update_gauge_three_levels(dd):
    # the paper's use (Sec. 3.1): one fine and three first-coarse iterations per
    # field change; on three levels a fine iteration without level-1 iterations
    # is rejected with the setup intact
    dims, b0, b1 = (8, 8, 8, 8), (2, 2, 2, 2), (2, 2, 2, 2)
    ctx, op, U = make(dd, dims, b0)
    kw = dict(levels=3, block=[b0, b1], nvec=[6, 8], coarse_mu_factor=5.0, keep_test_vectors=1)
    V0 = synth.spinor(dims, 2901, nvec=6)
    V1 = synth.gaussian((8,) + agg.coarse_dims(dims, b0) + (12,), 2902)
    ctx.setup(dd.default_params(setup_iters=3, **kw), [V0, V1])
    b = synth.spinor(dims, 2903)
    with pytest.raises(dd.DDAMGError) as e:
        ctx.update_gauge(U, dd.default_params(setup_iters=1, coarse_setup_iters=0, init_sap_iters=0, **kw))
    assert e.value.status == dd.INVALID_ARG
    x, _ = ctx.solve(b, tol=1e-10)
    assert rel(op.apply(x), b) <= 1e-10
    U2 = U
    for step in range(2):
        U2 = _perturbed(U2, 0.02, 2910 + step)
        ctx.update_gauge(U2, dd.default_params(setup_iters=1, coarse_setup_iters=3, init_sap_iters=0, **kw))
        x, s = ctx.solve(b, tol=1e-10)
        op2 = dirac.WilsonClover(U2, KAPPA, CSW, MU)
        assert s["converged"] and rel(op2.apply(x), b) <= 1e-10
        fresh = dd.DDAMG(dims, b0, KAPPA, CSW, MU)
        fresh.set_gauge(U2)
        fresh.setup(dd.default_params(setup_iters=3, **kw), [V0, V1])
        _, sf = fresh.solve(b, tol=1e-10)
        fresh.close()
        # the three-level counts of this small hierarchy scatter by ~20 % between setups
        assert s["iters"] <= 1.5 * sf["iters"] + 2, (step, s["iters"], sf["iters"])


# ------------------------------------------------------------------ 3 levels

def _three_level(dd, **kw):
    dims, b0, b1 = (8, 8, 8, 8), (2, 2, 2, 2), (2, 2, 2, 2)
    nv0, nv1 = 6, 8
    ctx, op, U = make(dd, dims, b0)
    V0 = synth.gaussian((nv0,) + dims + (12,), 3501)
    cd = agg.coarse_dims(dims, b0)
    V1 = synth.gaussian((nv1,) + cd + (2 * nv0,), 3502)
    p = dd.default_params(levels=3, block=[b0, b1], nvec=[nv0, nv1], coarse_mu_factor=5.0, **kw)
    ctx.set_test_vectors(p, [V0.reshape((nv0,) + dims + (4, 3)), V1])
    op_params = mg.Params(levels=3, blocks=[b0, b1], nvec=[nv0, nv1], delta=5.0, fixed=bool(p.fixed_iters),
                          coarse_max_iter=p.coarse_max_iter, coarse_restart=p.coarse_restart,
                          inter_max_iter=p.inter_max_iter, inter_restart=p.inter_restart,
                          coarse_sap_post=p.coarse_sap_post, coarse_mr_steps=p.coarse_mr_steps)
    h = mg.Hierarchy(op, op_params).set_test_vectors([V0, V1])
    return ctx, op, h


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
@pytest.mark.parametrize("K", [1, 3, 6, 9])
def test_coarse_transfers_k_columns(dd, prec, tol, K):
    """Level 1 <-> level 2 restriction and prolongation of K columns in one
    launch each (column groups of 4 and 8) against the oracle's P^dag and P of
    level 1, column by column, relative and element-wise."""
    ctx, op, h = _three_level(dd, precision=prec)
    Q1, b1 = h.levels[1].Q, (2, 2, 2, 2)
    shape1 = Q1.shape[1:]
    rs = np.stack([synth.gaussian(shape1, 70 + k) for k in range(K)])
    got = ctx.restrict_multi(1, rs)
    es = np.stack([synth.gaussian(got.shape[1:], 80 + k) for k in range(K)])
    xs = ctx.prolong_multi(1, es)
    for k in range(K):
        want = agg.restrict(Q1, rs[k], b1)
        assert rel(got[k], want) < tol
        assert np.abs(got[k] - want).max() < tol * np.abs(want).max()
        want = agg.prolong(Q1, es[k], b1)
        assert rel(xs[k], want) < tol
        assert np.abs(xs[k] - want).max() < tol * np.abs(want).max()


def test_three_level_operators(dd):
    ctx, op, h = _three_level(dd)
    for l in (1, 2):
        S, F = ctx.get_coarse_op(l)
        assert rel(S, h.levels[l].op.S) < 1e-12
        assert rel(F, h.levels[l].op.F) < 1e-12
    Q1 = ctx.get_interpolation(1)
    assert rel(Q1, h.levels[1].Q) < 1e-12
    st1 = h.levels[1].op
    b = synth.gaussian(st1.dims + (st1.n,), 51)
    x0 = synth.gaussian(st1.dims + (st1.n,), 52)
    got = ctx.coarse_sap(1, b, x0, 2)
    want = sap.sap(st1, b, x0, (2, 2, 2, 2), h.p.coarse_mr_steps, 2, schur=False)
    assert rel(got, want) < 1e-11


def test_three_level_vcycle_fixed(dd):
    ctx, op, h = _three_level(dd, fixed_iters=1, coarse_max_iter=8, coarse_restart=8, inter_max_iter=3,
                              inter_restart=3)
    v = synth.gaussian(op.dims + (12,), 61)
    got = ctx.vcycle(v.reshape(op.dims + (4, 3))).reshape(op.dims + (12,))
    want = h.vcycle(0, v)
    assert rel(got, want) < 1e-10


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_rank_deficient_test_vectors_rejected(dd, prec):
    # one test vector is i times another (exact in both precisions): every
    # aggregate half is rank-deficient and the block orthonormalisation must
    # refuse the set, as the oracle's does
    dims, block, nv = (4, 4, 4, 8), (2, 2, 2, 2), 6
    ctx, op, U = make(dd, dims, block)
    V = synth.gaussian((nv,) + dims + (12,), 1601)
    V[3] = 1j * V[1]
    with pytest.raises(ValueError):
        agg.orthonormalise(V, block)
    p = dd.default_params(levels=2, block=[block], nvec=[nv], precision=prec)
    with pytest.raises(dd.DDAMGError) as e:
        ctx.set_test_vectors(p, [V.reshape((nv,) + dims + (4, 3))])
    assert e.value.status == dd.NUMERICAL


def test_setup_progress_notifications(dd):
    # one notification per finished initial phase and setup iteration, in
    # order; none after the callback is removed
    dims = (8, 8, 8, 8)
    ctx, op, U = make(dd, dims, (2, 2, 2, 2))
    calls = []
    ctx.set_progress(lambda stage, level, i: calls.append((stage, level, i)))
    V0 = synth.gaussian((6,) + dims + (4, 3), 1701)
    p = dd.default_params(levels=2, block=[(2, 2, 2, 2)], nvec=[6], setup_iters=2, precision="fp32")
    ctx.setup(p, [V0])
    assert calls == [(0, 0, 0), (1, 0, 0), (1, 0, 1)]
    calls.clear()
    V1 = synth.gaussian((8,) + (4, 4, 4, 4) + (12,), 1702)
    p3 = dd.default_params(levels=3, block=[(2, 2, 2, 2), (2, 2, 2, 2)], nvec=[6, 8], setup_iters=1,
                           coarse_setup_iters=2, precision="fp32")
    ctx.setup(p3, [V0, V1])
    assert calls == [(0, 0, 0), (0, 1, 0), (1, 1, 0), (1, 1, 1), (1, 0, 0)]
    calls.clear()
    ctx.set_progress(None)
    ctx.setup(p, [V0])
    assert calls == []
    ctx.close()


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_setup_from_complex64_initial_vectors(dd, prec):
    # the fine initial vectors passed as complex64 give the hierarchy of the
    # same values passed as complex128 (the setup stores them in FP32 or
    # lower either way)
    dims, block, nv = (8, 8, 8, 8), (4, 4, 4, 4), 8
    ctx, op, _ = make(dd, dims, block)
    V = synth.spinor(dims, 1801, nvec=nv).astype(np.complex64)
    p = dd.default_params(levels=2, block=[block], nvec=[nv], setup_iters=1, precision=prec)
    ctx.setup(p, [V.astype(np.complex128)])
    Q128 = ctx.get_interpolation(0)
    ctx.setup(p, [V])
    Q64 = ctx.get_interpolation(0)
    assert np.array_equal(Q64, Q128)
    ctx.close()
