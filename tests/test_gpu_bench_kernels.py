"""Parity of the kernels the 48^3 x 96 benchmark spends its time in, against
the FP64 oracle, through the C interface: the fine SAP sweep with FP16/BF16
links on one and on K fields, the coarsest odd-even reduced operator on K
columns (matrix cores at n = 16..64), the K-field SAP of an intermediate
level on the matrix cores (n = 48, 64), the Galerkin assembly from FP32 test vectors and the
FP32-output block orthonormalisation, the adaptive setup itself (element by
element in the fixed-iteration mode) and the benchmark's own hierarchy shape
(4^4 then 2^4 aggregates, N_v 24 / 32, BF16) on a 16^4 lattice.

Bars (each derived from the arithmetic of the device path; u = 2^-11 for
FP16, 2^-8 for BF16, 2^-24 for FP32):
  * fine SAP with 16-bit links: the device rounds every link once to nearest
    even and computes in FP32; the oracle runs in FP64 on the same rounded
    links (rounded here by numpy, correctly rounded like the device's
    conversion), so the two differ by FP32 arithmetic only: relative and
    element-wise <= 1e-5, the bar of the FP32 sweep.  K fields in one launch
    equal K one-field sweeps bit for bit.
  * coarsest odd-even operator S x = D_ee x - D_eo D_oo^-1 D_oe x: the
    operator entries, the input and the odd-site intermediate are each
    rounded once to the storage format before FP32 accumulation, D_oo^-1 is
    FP32 from FP64.  Componentwise, |S_gpu x - S x| <= 4u (|D_ee||x| +
    |D_eo||t| + |D_eo||D_oo^-1||D_oe||x|), t = D_oo^-1 D_oe x (each product
    carries 2u + FP32 accumulation <= 3u; the 4th u covers the inverse).
  * K-field SAP of an intermediate level with 16-bit storage: every one of the
    2 iters (n_MR + 1) operator applications of the sweep rounds its operator
    and input (2u); first order the relative error stays below
    2u * 2 iters (n_MR + 1) = 16u * iters; checked in norm and element-wise
    (relative to the largest entry).
  * Galerkin assembly from FP32 test vectors: the vectors are widened and
    the products summed in FP64, so the blocks equal the oracle's FP64
    assembly of the same FP32 vectors to FP64 rounding (<= 1e-12 of the
    largest entry), and differ from the oracle's FP64 vectors only by the
    FP32 rounding of Q (<= 2e-6 relative, cond(V_A) ~ 10, so <= 1e-5 in D_c).
  * setup in FP64 with fixed iteration counts: deterministic on both sides,
    element-wise <= 1e-9 (rounding amplified through the iterations).
"""
import copy

import numpy as np
import pytest

from oracle import aggregation as agg
from oracle import coarse, dirac, mg, sap, stencil
from paper_1611_01034_amd import synth

pytestmark = pytest.mark.gpu

KAPPA, CSW, MU = 0.13729, 1.57551, 0.0009
U16 = {"fp16": 2.0 ** -11, "bf16": 2.0 ** -8}


def rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b))


def max_rel(a, b):
    """Largest element-wise difference over the largest entry of b."""
    a, b = np.asarray(a), np.asarray(b)
    return np.abs(a - b).max() / np.abs(b).max()


def round16(x, prec):
    """Round real and imaginary parts to FP16 / BF16, nearest even (values of
    links and coarse operators are far inside both exponent ranges)."""
    x = np.asarray(x, dtype=np.complex128)
    if prec == "fp16":
        f = lambda v: v.astype(np.float16).astype(np.float64)
    else:
        def f(v):
            m, e = np.frexp(v)
            return np.ldexp(np.round(m * 256.0) / 256.0, e)
    return f(x.real) + 1j * f(x.imag)


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


# ---------------------------------------------------------------------------
# fine SAP with 16-bit links
@pytest.mark.parametrize("prec", ["fp16", "bf16"])
def test_fine_sap_16bit_links(dd, prec):
    dims, block = (8, 8, 8, 16), (4, 4, 4, 4)
    ctx, op, U = make(dd, dims, block)
    print(f"fine SAP {prec} one field {dims}", flush=True)
    b = synth.spinor(dims, 11)
    x0 = synth.spinor(dims, 12) * 0.1
    got = ctx.sap(b, x0, iters=2, mr_steps=4, precision=prec).reshape(dims + (12,))
    opr = copy.copy(op)
    opr.U = round16(U, prec)
    want = sap.sap(stencil.FineLevel(opr), b.reshape(dims + (12,)), x0.reshape(dims + (12,)), block, 4, 2)
    assert rel(got, want) <= 1e-5
    assert max_rel(got, want) <= 1e-5
    # and against the unrounded operator: the link rounding itself, a few u
    exact = sap.sap(stencil.FineLevel(op), b.reshape(dims + (12,)), x0.reshape(dims + (12,)), block, 4, 2)
    assert rel(got, exact) <= 8 * U16[prec]
    ctx.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
@pytest.mark.parametrize("K", [2, 5, 16])
def test_fine_sap_k_fields(dd, prec, K):
    dims, block = (8, 8, 8, 8), (4, 4, 4, 4)
    ctx, op, U = make(dd, dims, block)
    print(f"fine SAP {prec} K={K}", flush=True)
    bs = np.stack([synth.spinor(dims, 20 + k) for k in range(K)])
    xs = np.stack([synth.spinor(dims, 60 + k) * 0.1 for k in range(K)])
    got = ctx.sap_multi(bs, xs, iters=1, mr_steps=4, precision=prec)
    for k in (0, K // 2, K - 1):
        one = ctx.sap(bs[k], xs[k], iters=1, mr_steps=4, precision=prec)
        assert np.array_equal(got[k], one), k
    opr = op
    if prec == "bf16":
        opr = copy.copy(op)
        opr.U = round16(U, prec)
    bar = 1e-11 if prec == "fp64" else 1e-5
    for k in (0, K - 1):
        want = sap.sap(stencil.FineLevel(opr), bs[k].reshape(dims + (12,)), xs[k].reshape(dims + (12,)), block, 4, 1)
        assert rel(got[k].reshape(dims + (12,)), want) <= bar
        assert max_rel(got[k].reshape(dims + (12,)), want) <= bar
    ctx.close()


# ---------------------------------------------------------------------------
# coarse levels
def _hier2(dd, dims, block, nv, prec, delta=5.0, mu=MU, seed=1501):
    ctx, op, U = make(dd, dims, block, mu=mu)
    V = synth.gaussian((nv,) + dims + (12,), seed)
    p = dd.default_params(levels=2, block=[block], nvec=[nv], coarse_mu_factor=delta, precision=prec)
    ctx.set_test_vectors(p, [V.reshape((nv,) + dims + (4, 3))])
    h = mg.Hierarchy(op, mg.Params(levels=2, blocks=[block], nvec=[nv], delta=delta)).set_test_vectors([V])
    return ctx, op, h


def _hier3(dd, dims, b0, b1, nv0, nv1, prec, delta=5.0, mu=MU, seed=3501, csb=(2, 2, 2, 2), **kw):
    ctx, op, U = make(dd, dims, b0, mu=mu)
    V0 = synth.gaussian((nv0,) + dims + (12,), seed)
    V1 = synth.gaussian((nv1,) + agg.coarse_dims(dims, b0) + (2 * nv0,), seed + 1)
    p = dd.default_params(levels=3, block=[b0, b1], nvec=[nv0, nv1], coarse_mu_factor=delta, precision=prec,
                          coarse_sap_block=csb, **kw)
    ctx.set_test_vectors(p, [V0.reshape((nv0,) + dims + (4, 3)), V1])
    op_params = mg.Params(levels=3, blocks=[b0, b1], nvec=[nv0, nv1], delta=delta, coarse_sap_block=csb,
                          coarse_mr_steps=p.coarse_mr_steps)
    return ctx, op, mg.Hierarchy(op, op_params).set_test_vectors([V0, V1]), p


def abs_apply(st, y):
    """|D_c| |y|: every block replaced by its entrywise absolute value."""
    a = np.abs(y)
    out = np.einsum("...ij,...j->...i", np.abs(st.S), a) + abs(st.mu) * a
    for mu in range(4):
        out += np.einsum("...ij,...j->...i", np.abs(st.F[mu]), np.roll(a, -1, axis=mu))
        Fb = np.roll(np.abs(st.F[mu]), 1, axis=mu)
        out += np.einsum("...ji,...j->...i", Fb, np.roll(a, 1, axis=mu))
    return out


def _schur_bound_terms(st):
    """Dense |D_ee|, |D_eo|, |D_oe|, |D_oo^-1| (even / odd site masks in the
    dense lexicographic ordering) and D_oo^-1 of a coarse stencil."""
    D = st.dense()
    n = st.n
    par = coarse.parity(st.dims).reshape(-1)
    ev = np.repeat(par == 0, n)
    od = ~ev
    Dee, Deo, Doe, Doo = D[np.ix_(ev, ev)], D[np.ix_(ev, od)], D[np.ix_(od, ev)], D[np.ix_(od, od)]
    Mi = np.linalg.inv(Doo)
    return ev, Dee, Deo, Doe, Mi


def _check_schur(ctx, st, level, prec, Ks, seed):
    # FP32 / FP64 vector path: one rounding per operator entry plus accumulation
    # over <= 9n terms, bounded here by 32 units of the format
    u = U16[prec] if prec in U16 else (2.0 ** -24 if prec == "fp32" else 2.0 ** -53) * 32
    oe = coarse.OddEven(st)
    ev, Dee, Deo, Doe, Mi = _schur_bound_terms(st)
    for K in Ks:
        print(f"coarsest odd-even operator {prec} n={st.n} K={K}", flush=True)
        xs = synth.gaussian((K,) + st.dims + (st.n,), seed + K)
        got = ctx.apply_coarse_schur_multi(level, xs)
        for k in range(K):
            want = oe.schur(xs[k])
            g, w = got[k].reshape(-1), want.reshape(-1)
            assert np.all(g[~ev] == 0)
            xe = xs[k].reshape(-1)[ev]
            t = Mi @ (Doe @ xe)
            bound = 4 * u * (np.abs(Dee) @ np.abs(xe) + np.abs(Deo) @ np.abs(t)
                             + np.abs(Deo) @ (np.abs(Mi) @ (np.abs(Doe) @ np.abs(xe))))
            err = np.abs(g[ev] - w[ev])
            assert np.all(err <= bound), (K, k, float((err / bound).max()))
            if prec in ("fp64",):
                assert rel(g, w) <= 1e-12


@pytest.mark.parametrize("prec", ["fp16", "bf16"])
@pytest.mark.parametrize("nv", [8, 16, 24, 32])
def test_coarsest_odd_even_operator_k_columns(dd, prec, nv):
    ctx, op, h = _hier2(dd, (8, 8, 8, 16), (4, 4, 4, 4), nv, prec)
    _check_schur(ctx, h.levels[1].op, 1, prec, (1, 2, 12, 16), 900 + nv)
    ctx.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_coarsest_odd_even_operator_k_columns_vector_path(dd, prec):
    ctx, op, h = _hier2(dd, (8, 8, 8, 16), (4, 4, 4, 4), 12, prec)
    _check_schur(ctx, h.levels[1].op, 1, prec, (1, 3), 950)
    ctx.close()


@pytest.mark.parametrize("prec", ["fp16", "bf16", "fp32"])
@pytest.mark.parametrize("nv0,nv1", [(24, 32), (32, 24)])
def test_intermediate_sap_k_fields(dd, prec, nv0, nv1):
    # level 1 of n = 2 nv0 = 48 or 64 on a 4^4 coarse lattice, 2^4 SAP blocks
    ctx, op, h, p = _hier3(dd, (8, 8, 8, 8), (2, 2, 2, 2), (2, 2, 2, 2), nv0, nv1, prec)
    st = h.levels[1].op
    iters = 2
    for K in (1, 2, 16):
        print(f"intermediate SAP {prec} n={st.n} K={K}", flush=True)
        bs = synth.gaussian((K,) + st.dims + (st.n,), 970 + K)
        xs = synth.gaussian((K,) + st.dims + (st.n,), 990 + K) * 0.1
        got = ctx.coarse_sap_multi(1, bs, xs, iters)
        bar = 1e-5 if prec == "fp32" else 16 * U16[prec] * iters
        for k in range(K):
            want = sap.sap(st, bs[k], xs[k], p.coarse_sap_block, p.coarse_mr_steps, iters, schur=False)
            assert rel(got[k], want) <= bar, (K, k, rel(got[k], want))
            assert max_rel(got[k], want) <= bar, (K, k, max_rel(got[k], want))
    ctx.close()


@pytest.mark.parametrize("nv0,nv1", [(24, 32), (32, 24)])
def test_coarsest_odd_even_operator_three_levels(dd, nv0, nv1):
    ctx, op, h, p = _hier3(dd, (8, 8, 8, 8), (2, 2, 2, 2), (2, 2, 2, 2), nv0, nv1, "bf16")
    _check_schur(ctx, h.levels[2].op, 2, "bf16", (2, 12, 16), 1100)
    ctx.close()


# ---------------------------------------------------------------------------
# FP32 assembly and FP32-output orthonormalisation
def _coarse_blocks(st):
    """S [T,Z,Y,X][n][n] and F [4][T,Z,Y,X][n][n] of an oracle stencil, the
    layout of ddamg_get_coarse_op."""
    return np.asarray(st.S), np.stack([np.asarray(st.F[m]) for m in range(4)])


def test_fp32_orthonormalisation_and_assembly(dd):
    dims, block, nv = (8, 8, 8, 16), (4, 4, 4, 4), 24
    ctx, op, h = _hier2(dd, dims, block, nv, "fp32")
    Q = ctx.get_interpolation(0).reshape((nv,) + dims + (12,))
    Qo = h.levels[0].Q
    assert max_rel(Q, Qo) <= 2e-6
    S, F = ctx.get_coarse_op(1)
    # against the FP64 assembly of the device's own FP32 vectors: the assembly arithmetic
    st_own = coarse.assemble(stencil.wilson_stencil(op), Q, block, 5 * MU)
    So, Fo = _coarse_blocks(st_own)
    scale = max(np.abs(So).max(), np.abs(Fo).max())
    assert np.abs(S - So).max() <= 1e-12 * scale
    assert np.abs(F - Fo).max() <= 1e-12 * scale
    # against the oracle's FP64 vectors: adds the rounding of Q to FP32
    Sw, Fw = _coarse_blocks(h.levels[1].op)
    assert np.abs(S - Sw).max() <= 1e-5 * scale
    assert np.abs(F - Fw).max() <= 1e-5 * scale
    ctx.close()


def test_fp32_three_level_assembly(dd):
    ctx, op, h, p = _hier3(dd, (8, 8, 8, 8), (2, 2, 2, 2), (2, 2, 2, 2), 12, 16, "fp32")
    for lev in (1, 2):
        S, F = ctx.get_coarse_op(lev)
        Sw, Fw = _coarse_blocks(h.levels[lev].op)
        scale = max(np.abs(Sw).max(), np.abs(Fw).max())
        assert np.abs(S - Sw).max() <= 2e-5 * scale, lev
        assert np.abs(F - Fw).max() <= 2e-5 * scale, lev
    Q1 = ctx.get_interpolation(1)
    assert max_rel(Q1, h.levels[1].Q) <= 1e-5
    ctx.close()


# ---------------------------------------------------------------------------
# the adaptive setup, element by element (FP64, fixed iteration counts)
@pytest.mark.parametrize("levels,setup_iters", [(2, 1), (2, 2), (3, 1)])
def test_setup_matches_oracle_fixed_iterations(dd, levels, setup_iters):
    dims = (8, 8, 8, 8)
    b0 = (2, 2, 2, 2) if levels == 3 else (4, 4, 4, 4)
    nv0, nv1 = 8, 8
    ctx, op, U = make(dd, dims, b0, mu=0.02)
    print(f"setup levels={levels} iters={setup_iters}", flush=True)
    V0 = synth.gaussian((nv0,) + dims + (12,), 4401)
    vecs = [V0.reshape((nv0,) + dims + (4, 3))]
    kw = dict(coarse_max_iter=12, coarse_restart=6, inter_max_iter=3, inter_restart=3, fixed_iters=1,
              init_sap_iters=2, setup_iters=setup_iters, coarse_setup_iters=1, coarse_mu_factor=3.0)
    oracle_vecs = [V0]
    if levels == 3:
        V1 = synth.gaussian((nv1,) + agg.coarse_dims(dims, b0) + (2 * nv0,), 4402)
        vecs.append(V1)
        oracle_vecs.append(V1)
        p = dd.default_params(levels=3, block=[b0, (2, 2, 2, 2)], nvec=[nv0, nv1], precision="fp64", batch=4, **kw)
        op_p = mg.Params(levels=3, blocks=[b0, (2, 2, 2, 2)], nvec=[nv0, nv1])
    else:
        p = dd.default_params(levels=2, block=[b0], nvec=[nv0], precision="fp64", batch=4, **kw)
        op_p = mg.Params(levels=2, blocks=[b0], nvec=[nv0])
    op_p = mg.Params(**{**op_p.__dict__, **dict(coarse_max_iter=12, coarse_restart=6, inter_max_iter=3,
                                               inter_restart=3, fixed=True, init_sap_iters=2, setup_iters=setup_iters,
                                               coarse_setup_iters=1, delta=3.0, sap_post=p.sap_post,
                                               mr_steps=p.mr_steps, coarse_sap_post=p.coarse_sap_post,
                                               coarse_mr_steps=p.coarse_mr_steps)})
    ctx.setup(p, vecs)
    h = mg.Hierarchy(op, op_p).setup(oracle_vecs)
    Q0 = ctx.get_interpolation(0).reshape(h.levels[0].Q.shape)
    assert max_rel(Q0, h.levels[0].Q) <= 1e-9
    for lev in range(1, levels):
        S, F = ctx.get_coarse_op(lev)
        Sw, Fw = _coarse_blocks(h.levels[lev].op)
        scale = max(np.abs(Sw).max(), np.abs(Fw).max())
        assert np.abs(S - Sw).max() <= 1e-9 * scale, lev
        assert np.abs(F - Fw).max() <= 1e-9 * scale, lev
    if levels == 3:
        assert max_rel(ctx.get_interpolation(1), h.levels[1].Q) <= 1e-9
    ctx.close()


# ---------------------------------------------------------------------------
# the benchmark's hierarchy shape on 16^4
@pytest.fixture(scope="module")
def bench_shape(dd):
    dims = (16, 16, 16, 16)
    print("bench-shaped hierarchy 16^4, 4^4 / 2^4 aggregates, Nv 24/32, BF16", flush=True)
    ctx, op, h, p = _hier3(dd, dims, (4, 4, 4, 4), (2, 2, 2, 2), 24, 32, "bf16", seed=5501, rhs_batch=2,
                           setup_iters=1, coarse_setup_iters=1)
    yield ctx, op, h, p
    ctx.close()


def test_bench_shape_coarse_operators(dd, bench_shape):
    ctx, op, h, p = bench_shape
    # level 1 (n = 48): FP32 assembly; level 2 (n = 64): assembled from level 1
    for lev in (1, 2):
        S, F = ctx.get_coarse_op(lev)
        Sw, Fw = _coarse_blocks(h.levels[lev].op)
        scale = max(np.abs(Sw).max(), np.abs(Fw).max())
        assert np.abs(S - Sw).max() <= 2e-5 * scale, lev
        assert np.abs(F - Fw).max() <= 2e-5 * scale, lev


def test_bench_shape_k_column_kernels(dd, bench_shape):
    ctx, op, h, p = bench_shape
    u = U16["bf16"]
    st1 = h.levels[1].op
    ys = synth.gaussian((16,) + st1.dims + (st1.n,), 5601)
    got = ctx.apply_coarse_multi(1, ys)
    for k in range(16):
        err = np.abs(got[k] - st1.apply(ys[k]))
        assert np.all(err <= 3 * u * abs_apply(st1, ys[k]) + 1e-5 * np.abs(ys[k]).max()), k
    _check_schur(ctx, h.levels[2].op, 2, "bf16", (2, 12, 16), 5700)
    iters = 2
    bs = synth.gaussian((16,) + st1.dims + (st1.n,), 5801)
    xs = np.zeros_like(bs)
    got = ctx.coarse_sap_multi(1, bs, xs, iters)
    for k in (0, 7, 15):
        want = sap.sap(st1, bs[k], xs[k], p.coarse_sap_block, p.coarse_mr_steps, iters, schur=False)
        assert rel(got[k], want) <= 16 * u * iters
        assert max_rel(got[k], want) <= 16 * u * iters


def test_bench_shape_fine_sap_and_solve(dd, bench_shape):
    ctx, op, h, p = bench_shape
    dims = op.dims
    bs = np.stack([synth.spinor(dims, 5901 + k) for k in range(16)])
    xs = np.zeros_like(bs)
    got = ctx.sap_multi(bs, xs, iters=1, mr_steps=4, precision="bf16")
    opr = copy.copy(op)
    opr.U = round16(op.U, "bf16")
    for k in (15,):
        want = sap.sap(stencil.FineLevel(opr), bs[k].reshape(dims + (12,)), xs[k].reshape(dims + (12,)),
                       (4, 4, 4, 4), 4, 1)
        assert rel(got[k].reshape(dims + (12,)), want) <= 1e-5
        assert max_rel(got[k].reshape(dims + (12,)), want) <= 1e-5
    # an adaptive setup of the same shape (one iteration), then two right-hand
    # sides in lock step to a true residual of 1e-10, checked with the oracle's D
    V0 = synth.gaussian((24,) + dims + (12,), 5501).reshape((24,) + dims + (4, 3))
    V1 = synth.gaussian((32,) + agg.coarse_dims(dims, (4, 4, 4, 4)) + (48,), 5502)
    ctx.setup(p, [V0, V1])
    b = np.stack([synth.spinor(dims, 6001 + k) for k in range(2)])
    x, st = ctx.solve(b, tol=1e-10)
    for k in range(2):
        r = np.linalg.norm(b[k] - op.apply(x[k])) / np.linalg.norm(b[k])
        assert r <= 1e-10, (k, r)
