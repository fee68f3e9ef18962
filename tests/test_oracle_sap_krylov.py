"""Pins of the oracle's SAP smoother and Krylov solvers.

SAP (Sec. 1 smoother; odd-even inside it, Sec. 3) is checked block by block
against dense linear algebra on explicitly extracted block matrices; the
Krylov solvers against numpy.linalg.solve and textbook properties.
"""
import numpy as np
import pytest

from oracle import dirac, krylov, sap, stencil
from paper_1611_01034_amd import synth

KAPPA, CSW, MU = 0.13729, 1.57551, 0.0009


def _site_index(dims):
    return np.arange(int(np.prod(dims))).reshape(dims)


def _dense_mr(S, rho, n):
    e = np.zeros_like(rho)
    for _ in range(n):
        q = S @ rho
        qq = np.vdot(q, q).real
        a = np.vdot(q, rho) / qq
        e = e + a * rho
        rho = rho - a * q
    return e


@pytest.mark.parametrize("bsize", [(2, 2, 2, 2), (2, 4, 2, 2)])
def test_block_solve_matches_dense_schur_mr(bsize):
    dims = (4, 8, 4, 4)
    U = synth.gauge_field(dims, 0.3, 101)
    op = dirac.WilsonClover(U, KAPPA, CSW, 0.02)
    fl = stencil.FineLevel(op)
    r = synth.gaussian(dims + (12,), 102)
    bid, col, nb = sap.block_layout(dims, bsize)
    n_mr = 3
    got = sap.block_solve(fl, r, 1, bid, col, nb, n_mr)
    # brute force on two blocks of colour 1
    par = sap.site_parity(dims)
    idx = _site_index(dims)
    for B in np.unique(bid[col == 1])[:2]:
        sites = idx[bid == B]
        # dense D restricted to the block (Dirichlet): apply D to unit vectors on the block
        nloc = len(sites) * 12
        DB = np.zeros((nloc, nloc), dtype=np.complex128)
        e = np.zeros(dims + (12,), dtype=np.complex128)
        ef = e.reshape(-1, 12)
        for k in range(nloc):
            ef[:] = 0
            ef[sites[k // 12], k % 12] = 1
            y = fl.apply(e).reshape(-1, 12)
            DB[:, k] = y[sites].reshape(-1)
        pe = np.repeat(par.reshape(-1)[sites] == 0, 12)
        po = ~pe
        Dee, Deo = DB[np.ix_(pe, pe)], DB[np.ix_(pe, po)]
        Doe, Doo = DB[np.ix_(po, pe)], DB[np.ix_(po, po)]
        S = Dee - Deo @ np.linalg.solve(Doo, Doe)
        rb = r.reshape(-1, 12)[sites].reshape(-1)
        rt = rb[pe] - Deo @ np.linalg.solve(Doo, rb[po])
        ee = _dense_mr(S, rt, n_mr)
        eo = np.linalg.solve(Doo, rb[po] - Doe @ ee)
        want = np.zeros(nloc, dtype=np.complex128)
        want[pe] = ee
        want[po] = eo
        assert np.abs(got.reshape(-1, 12)[sites].reshape(-1) - want).max() < 1e-12
    # nothing written outside colour-1 blocks
    assert np.abs(got[col == 0]).max() == 0.0


def test_block_mr_without_schur_matches_dense():
    dims = (4, 4, 4, 4)
    rng = np.random.default_rng(7)
    n = 6
    S = rng.standard_normal(dims + (n, n)) + 1j * rng.standard_normal(dims + (n, n))
    S = S + 6 * np.eye(n)
    F = 0.3 * (rng.standard_normal((4,) + dims + (n, n)) + 1j * rng.standard_normal((4,) + dims + (n, n)))
    st = stencil.Stencil(S, F, 0.1)
    r = synth.gaussian(dims + (n,), 8)
    bsize = (2, 2, 2, 2)
    bid, col, nb = sap.block_layout(dims, bsize)
    got = sap.block_solve(st, r, 0, bid, col, nb, 4, schur=False)
    idx = _site_index(dims)
    B = np.unique(bid[col == 0])[3]
    sites = idx[bid == B]
    nloc = len(sites) * n
    DB = np.zeros((nloc, nloc), dtype=np.complex128)
    e = np.zeros(dims + (n,), dtype=np.complex128)
    ef = e.reshape(-1, n)
    for k in range(nloc):
        ef[:] = 0
        ef[sites[k // n], k % n] = 1
        DB[:, k] = st.apply(e).reshape(-1, n)[sites].reshape(-1)
    want = _dense_mr(DB, r.reshape(-1, n)[sites].reshape(-1), 4)
    assert np.abs(got.reshape(-1, n)[sites].reshape(-1) - want).max() < 1e-12


def test_exact_block_solves_kill_the_residual_on_the_solved_colour():
    dims = (4, 4, 4, 4)
    U = synth.gauge_field(dims, 0.3, 111)
    fl = stencil.FineLevel(dirac.WilsonClover(U, KAPPA, CSW, MU))
    b = synth.gaussian(dims + (12,), 112)
    bsize = (2, 2, 2, 2)
    bid, col, nb = sap.block_layout(dims, bsize)
    x = np.zeros_like(b)
    r = b - fl.apply(x)
    x = x + sap.block_solve(fl, r, 0, bid, col, nb, 150)
    r = b - fl.apply(x)
    assert np.abs(r[col == 0]).max() < 1e-9 * np.abs(b).max()
    assert np.abs(r[col == 1]).max() > 1e-3


def test_sap_gauge_covariant():
    dims = (4, 4, 4, 4)
    U = synth.gauge_field(dims, 0.3, 121)
    Om = synth.gauge_transform(dims, 122)
    f1 = stencil.FineLevel(dirac.WilsonClover(U, KAPPA, CSW, MU))
    f2 = stencil.FineLevel(dirac.WilsonClover(synth.transform_links(U, Om), KAPPA, CSW, MU))
    b = synth.spinor(dims, 123)
    x1 = sap.sap(f1, b.reshape(dims + (12,)), np.zeros(dims + (12,), complex), (2, 2, 2, 2), 4, 2)
    b2 = synth.transform_spinor(b, Om).reshape(dims + (12,))
    x2 = sap.sap(f2, b2, np.zeros(dims + (12,), complex), (2, 2, 2, 2), 4, 2)
    assert np.abs(synth.transform_spinor(x1.reshape(dims + (4, 3)), Om).reshape(dims + (12,)) - x2).max() < 1e-12


def test_sap_damps_a_rough_residual():
    # SAP is a smoother, not a convergent solver on its own: on a Gaussian
    # (UV-dominated) right-hand side the first sweeps cut the residual
    # sharply, later sweeps stall on the low modes.
    dims = (4, 4, 4, 4)
    U = synth.gauge_field(dims, 0.3, 131)
    fl = stencil.FineLevel(dirac.WilsonClover(U, KAPPA, CSW, MU))
    b = synth.gaussian(dims + (12,), 132)
    x = np.zeros_like(b)
    res = [np.linalg.norm(b)]
    for _ in range(2):
        x = sap.sap_iteration(fl, b, x, (2, 2, 2, 2), 4)
        res.append(np.linalg.norm(b - fl.apply(x)))
    assert res[1] < 0.5 * res[0] and res[2] < res[1]


def test_odd_block_count_rejected():
    with pytest.raises(ValueError):
        sap.block_layout((4, 4, 4, 6), (2, 2, 2, 2))


# ---------------------------------------------------------------- Krylov

def _rand_system(n, seed, shift=4.0):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    A = A / np.sqrt(n) + shift * np.eye(n)
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    return A, b


def test_gmres_matches_dense_solve():
    A, b = _rand_system(60, 1)
    x, info = krylov.gmres(lambda v: A @ v, b, tol=1e-12, restart=10, max_iter=500)
    xs = np.linalg.solve(A, b)
    kappa = np.linalg.cond(A)
    assert info["converged"]
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) < kappa * 1e-12
    h = info["history"]
    # within one restart cycle the residual estimates never increase
    assert all(h[i + 1] <= h[i] * (1 + 1e-12) for i in range(min(9, len(h) - 1)))


def test_fgmres_identity_preconditioner_equals_gmres():
    A, b = _rand_system(40, 2, shift=2.0)
    x1, i1 = krylov.fgmres(lambda v: A @ v, b, M=lambda v: v, tol=1e-10, restart=8, max_iter=200)
    x2, i2 = krylov.gmres(lambda v: A @ v, b, tol=1e-10, restart=8, max_iter=200)
    assert i1["iters"] == i2["iters"]
    assert np.abs(x1 - x2).max() < 1e-13


def test_fgmres_exact_preconditioner_one_step():
    A, b = _rand_system(30, 3)
    Ainv = np.linalg.inv(A)
    x, info = krylov.fgmres(lambda v: A @ v, b, M=lambda v: Ainv @ v, tol=1e-10, restart=5, max_iter=10)
    assert info["iters"] == 1 and info["resid"] < 1e-12


def test_mr_scalar_one_step():
    a = 2.0 - 0.7j
    x = krylov.mr(lambda v: a * v, np.array([1.5 + 0.2j]), 1)
    assert abs(x[0] - (1.5 + 0.2j) / a) < 1e-15


def test_fgmres_fixed_mode_runs_exact_count():
    A, b = _rand_system(50, 4, shift=1.0)
    x, info = krylov.fgmres(lambda v: A @ v, b, tol=1e-30, restart=7, max_iter=17, fixed=True)
    assert info["iters"] == 17
