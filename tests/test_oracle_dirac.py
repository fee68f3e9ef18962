"""Pins of the oracle's fine operator against closed forms and exact identities.

Paper: Sec. 1 (D(+-mu) = D_W +- i Gamma5 mu, D^dag D = D_W^dag D_W + mu^2),
Sec. 2 (gamma5 = diag(-1,-1,1,1), TZYX order).  D_W is the textbook
Wilson-clover operator (the paper only names it).
"""
import os

import numpy as np
import pytest

from oracle import dirac, stencil
from paper_1611_01034_amd import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")
KAPPA, CSW, MU = 0.13729, 1.57551, 0.0009


def _free_links(dims):
    U = np.zeros(tuple(dims) + (4, 3, 3), dtype=np.complex128)
    U[..., :, :, :] = np.eye(3)
    return U


def test_gamma_basis_matches_paper_gamma5():
    g5 = np.loadtxt(os.path.join(GOLD, "gamma5.txt"))
    G = dirac.GAMMA
    for a in range(4):
        assert np.allclose(G[a], G[a].conj().T)
        for b in range(4):
            ac = G[a] @ G[b] + G[b] @ G[a]
            assert np.allclose(ac, 2.0 * (a == b) * np.eye(4))
    # gamma_X gamma_Y gamma_Z gamma_T, direction index 3,2,1,0
    prod = G[3] @ G[2] @ G[1] @ G[0]
    assert np.allclose(prod, g5)
    assert np.allclose(dirac.GAMMA5, g5)


@pytest.mark.parametrize("mu", [0.0, MU, 0.3])
def test_free_field_plane_wave(mu):
    dims = (4, 6, 2, 8)           # T, Z, Y, X all different
    op = dirac.WilsonClover(_free_links(dims), KAPPA, CSW, mu)
    rng = np.random.default_rng(3)
    x = np.indices(dims)
    for n in [(0, 0, 0, 0), (1, 0, 0, 0), (0, 1, 1, 3), (3, 5, 1, 7), (2, 2, 0, 1)]:
        p = [2 * np.pi * n[d] / dims[d] for d in range(4)]
        phase = np.exp(1j * sum(p[d] * x[d] for d in range(4)))
        u = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
        psi = phase[..., None, None] * u
        got = op.apply(psi)
        sym = dirac.plane_wave_symbol(p, op.m0, mu)
        want = phase[..., None, None] * (sym @ u)
        assert np.abs(got - want).max() < 1e-13


@pytest.mark.parametrize("theta", [(np.pi, 0.0, 0.0, 0.0), (0.7, -1.9, 2.6, np.pi)])
def test_free_field_plane_wave_twisted_boundary(theta):
    # psi(x + L_mu) = exp(i theta_mu) psi(x) admits the momenta
    # p_mu = (2 pi n_mu + theta_mu) / L_mu, with the free-field symbol
    dims = (4, 6, 2, 8)
    op = dirac.WilsonClover(_free_links(dims), KAPPA, CSW, MU, theta=theta)
    rng = np.random.default_rng(4)
    x = np.indices(dims)
    for n in [(0, 0, 0, 0), (1, 0, 0, 0), (0, 1, 1, 3), (3, 5, 1, 7)]:
        p = [(2 * np.pi * n[d] + theta[d]) / dims[d] for d in range(4)]
        phase = np.exp(1j * sum(p[d] * x[d] for d in range(4)))
        u = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
        got = op.apply(phase[..., None, None] * u)
        want = phase[..., None, None] * (dirac.plane_wave_symbol(p, op.m0, MU) @ u)
        assert np.abs(got - want).max() < 1e-13


def test_twisted_boundary_equals_uniform_abelian_phase():
    # Omega(x) = exp(-i sum_mu theta_mu x_mu / L_mu) maps the twisted operator
    # to the periodic one on links exp(i theta_mu / L_mu) U_mu(x):
    # D_theta = Omega^-1 D_per[U'] Omega
    dims = (4, 2, 6, 4)
    theta = (np.pi, 0.4, -1.3, 2.0)
    U = synth.gauge_field(dims, 0.4, 17)
    op = dirac.WilsonClover(U, KAPPA, CSW, MU, theta=theta)
    U1 = U * np.exp(1j * np.array([theta[d] / dims[d] for d in range(4)]))[:, None, None]
    per = dirac.WilsonClover(U1, KAPPA, CSW, MU)
    x = np.indices(dims)
    om = np.exp(-1j * sum(theta[d] * x[d] / dims[d] for d in range(4)))[..., None, None]
    psi = synth.spinor(dims, 18)
    assert np.abs(op.apply(psi) - per.apply(om * psi) / om).max() < 1e-13
    assert np.abs(op.A - per.A).max() < 1e-13


def test_odd_shifted_operator_and_schur_complement_dense():
    # D(mu; rho) = D(mu) + i rho Gamma5 on the odd sites; its odd-site Schur
    # complement from the dense blocks equals schur_odd, and the odd part of
    # the full solve of D(mu; rho) x = (0, b_o) solves the reduced system
    dims = (4, 2, 2, 4)
    rho = 0.07
    op = dirac.WilsonClover(synth.gauge_field(dims, 0.4, 19), KAPPA, CSW, 0.05)
    D = op.dense()
    odd = np.repeat(dirac.odd_mask(dims).reshape(-1) > 0.5, 12)
    g5 = np.tile(np.repeat([-1.0, -1.0, 1.0, 1.0], 3), int(np.prod(dims)))
    Ds = D + np.diag(1j * rho * g5 * odd)
    e = synth.spinor(dims, 20)
    assert np.abs(dirac.apply_odd_shifted(op, e, rho).reshape(-1) - Ds @ e.reshape(-1)).max() < 1e-13
    o, ev = np.where(odd)[0], np.where(~odd)[0]
    S = Ds[np.ix_(o, o)] - Ds[np.ix_(o, ev)] @ np.linalg.solve(Ds[np.ix_(ev, ev)], Ds[np.ix_(ev, o)])
    got = dirac.schur_odd(op, e, rho).reshape(-1)
    assert np.abs(got[o] - S @ e.reshape(-1)[o]).max() < 1e-12
    assert np.abs(got[ev]).max() == 0.0
    b = np.where(odd, e.reshape(-1), 0.0)
    x = np.linalg.solve(Ds, b)
    r = dirac.schur_odd(op, x.reshape(e.shape), rho).reshape(-1)[o] - e.reshape(-1)[o]
    assert np.abs(r).max() < 1e-12


def test_constant_diagonal_links_shift_momentum_per_colour():
    dims = (4, 4, 6, 2)
    alpha = np.array([[0.3, -0.1, -0.2], [0.05, 0.4, -0.45], [-0.7, 0.2, 0.5], [0.11, 0.13, -0.24]])
    U = np.zeros(dims + (4, 3, 3), dtype=np.complex128)
    for mu in range(4):
        U[..., mu, :, :] = np.diag(np.exp(1j * alpha[mu]))
    op = dirac.WilsonClover(U, KAPPA, CSW, MU)
    assert np.abs(op.A).max() < 1e-14           # abelian constant links: no field strength
    x = np.indices(dims)
    n = (1, 3, 2, 1)
    p = np.array([2 * np.pi * n[d] / dims[d] for d in range(4)])
    phase = np.exp(1j * sum(p[d] * x[d] for d in range(4)))
    rng = np.random.default_rng(5)
    for a in range(3):
        s = rng.standard_normal(4) + 1j * rng.standard_normal(4)
        u = np.zeros((4, 3), dtype=np.complex128)
        u[:, a] = s
        psi = phase[..., None, None] * u
        sym = dirac.plane_wave_symbol(p + alpha[:, a], op.m0, MU)
        want = np.zeros_like(u)
        want[:, a] = sym @ s
        assert np.abs(op.apply(psi) - phase[..., None, None] * want).max() < 1e-13


def test_constant_abelian_field_clover_closed_form():
    # U_X(x) = diag(e^{i a y}, e^{-i a y}, 1), a = 2 pi n / L_Y, all other links 1:
    # every XY plaquette is diag(e^{-ia}, e^{ia}, 1), so F_XY = -i sin(a) diag(1,-1,0)
    # and the clover term is (c_sw/2) sin(a) sigma_XY (x) diag(1,-1,0).
    dims = (2, 2, 6, 4)
    a = 2 * np.pi * 1 / dims[2]
    U = _free_links(dims)
    y = np.indices(dims)[2]
    U[..., 3, 0, 0] = np.exp(1j * a * y)
    U[..., 3, 1, 1] = np.exp(-1j * a * y)
    csw = 1.7
    op = dirac.WilsonClover(U, KAPPA, csw, 0.0)
    sig = dirac.sigma_munu(3, 2)
    want = 0.5 * csw * np.sin(a) * np.kron(sig, np.diag([1.0, -1.0, 0.0]))
    assert np.abs(op.A - want).max() < 1e-14
    Q = dirac.clover_leaves(U, 3, 2)
    assert np.allclose(Q[..., 0, 0], 4 * np.exp(-1j * a))


def test_pure_gauge_field():
    dims = (4, 2, 4, 6)
    Om = synth.gauge_transform(dims, 11)
    U = synth.transform_links(_free_links(dims), Om)
    op = dirac.WilsonClover(U, KAPPA, CSW, MU)
    free = dirac.WilsonClover(_free_links(dims), KAPPA, CSW, MU)
    assert np.abs(op.A).max() < 1e-13
    psi = synth.spinor(dims, 12)
    got = op.apply(psi)
    Omd = np.conj(np.swapaxes(Om, -1, -2))
    want = synth.transform_spinor(free.apply(synth.transform_spinor(psi, Omd)), Om)
    assert np.abs(got - want).max() < 1e-12


def test_gauge_covariance_random_field():
    dims = (4, 4, 2, 4)
    U = synth.gauge_field(dims, 0.4, 21)
    Om = synth.gauge_transform(dims, 22)
    op = dirac.WilsonClover(U, KAPPA, CSW, MU)
    opt = dirac.WilsonClover(synth.transform_links(U, Om), KAPPA, CSW, MU)
    psi = synth.spinor(dims, 23)
    lhs = opt.apply(synth.transform_spinor(psi, Om))
    rhs = synth.transform_spinor(op.apply(psi), Om)
    assert np.abs(lhs - rhs).max() < 1e-12
    A2 = opt.A.reshape(dims + (4, 3, 4, 3))
    A1 = op.A.reshape(dims + (4, 3, 4, 3))
    Omd = np.conj(np.swapaxes(Om, -1, -2))
    rot = np.einsum("...ab,...sbtc,...cd->...satd", Om, A1, Omd)
    assert np.abs(A2 - rot).max() < 1e-12


def test_gamma5_hermiticity_and_twist():
    dims = (4, 4, 4, 2)
    U = synth.gauge_field(dims, 0.3, 31)
    op = dirac.WilsonClover(U, KAPPA, CSW, 0.05)
    x = synth.spinor(dims, 32)
    y = synth.spinor(dims, 33)
    g5 = dirac.gamma5_field
    lhs = np.vdot(x, op.apply(y))
    rhs = np.vdot(g5(op.apply(g5(x), -op.mu)), y)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
    # D(mu) - D(-mu) = 2 i mu Gamma5
    d = op.apply(y) - op.apply(y, -op.mu)
    assert np.abs(d - 2j * op.mu * g5(y)).max() < 1e-13


def test_squared_operator_identity():
    dims = (4, 2, 4, 4)
    U = synth.gauge_field(dims, 0.3, 41)
    op = dirac.WilsonClover(U, KAPPA, CSW, 0.07)
    x = synth.spinor(dims, 42)
    lhs = np.vdot(op.apply(x), op.apply(x)).real
    rhs = np.vdot(op.apply_w(x), op.apply_w(x)).real + op.mu ** 2 * np.vdot(x, x).real
    assert abs(lhs - rhs) < 1e-12 * lhs


def test_dense_twisted_mass_bound():
    dims = (2, 2, 2, 2)
    U = synth.gauge_field(dims, 0.3, 51)
    mu = 0.04
    op = dirac.WilsonClover(U, KAPPA, CSW, mu)
    D = op.dense()
    DW = op.dense(0.0)
    lhs = D.conj().T @ D
    rhs = DW.conj().T @ DW + mu ** 2 * np.eye(D.shape[0])
    assert np.abs(lhs - rhs).max() < 1e-12
    assert np.linalg.svd(D, compute_uv=False).min() >= mu * (1 - 1e-12)


def test_clover_structure():
    dims = (4, 2, 2, 4)
    U = synth.gauge_field(dims, 0.5, 61)
    A = dirac.clover_matrix(U, CSW)
    assert np.abs(A - np.conj(np.swapaxes(A, -1, -2))).max() < 1e-14
    assert np.abs(A[..., 0:6, 6:12]).max() == 0.0 and np.abs(A[..., 6:12, 0:6]).max() == 0.0
    Ab = dirac.clover_blocks(A)
    # traceless in spin within each chirality block
    sp = Ab[..., 0:3, 0:3] + Ab[..., 3:6, 3:6]
    assert np.abs(sp).max() < 1e-14
    assert np.abs(dirac.clover_matrix(U, 0.0)).max() == 0.0


def test_stencil_form_equals_explicit_operator():
    dims = (2, 4, 4, 4)
    U = synth.gauge_field(dims, 0.3, 71)
    op = dirac.WilsonClover(U, KAPPA, CSW, MU)
    st = stencil.wilson_stencil(op)
    fl = stencil.FineLevel(op)
    y = synth.gaussian(dims + (12,), 72)
    assert np.abs(st.apply(y) - fl.apply(y)).max() < 1e-13
    assert np.abs(st.apply(y, -MU) - fl.apply(y, -MU)).max() < 1e-13
