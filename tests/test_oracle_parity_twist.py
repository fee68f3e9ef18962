"""Pins of the oracle with different twisted masses on even and odd sites
(Sec. 2: the library's TM operator takes a different twist on the two
parities; Sec. 3.1: the Hasenbusch terms D^(mu) + i rho G^5 are odd-even
reduced operators of such an operator)."""
import numpy as np
import pytest

from oracle import aggregation as agg
from oracle import coarse, dirac, mg, stencil
from paper_1611_01034_amd import synth

KAPPA, CSW = 0.13729, 1.57551


@pytest.fixture(scope="module")
def field():
    dims = (4, 2, 2, 4)
    return dims, synth.gauge_field(dims, 0.4, 3101)


def _dense_g5(V):
    return np.kron(np.eye(V), np.kron(dirac.GAMMA5, np.eye(3)))


def test_equal_twists_are_the_one_twist_operator(field):
    dims, U = field
    psi = synth.spinor(dims, 3102)
    a = dirac.WilsonClover(U, KAPPA, CSW, 0.05).apply(psi)
    b = dirac.WilsonClover(U, KAPPA, CSW, 0.05, mu_odd=0.05).apply(psi)
    assert np.array_equal(a, b)


def test_odd_site_schur_complement_is_the_hasenbusch_term(field):
    # dense odd-odd Schur complement of D(mu, mu + rho) = that of D(mu, mu)
    # plus i rho Gamma5 on the odd sites: fixes which parity carries mu_odd
    dims, U = field
    mu, rho = 0.03, 0.2
    V = int(np.prod(dims))
    odd = np.repeat(dirac.odd_mask(dims).reshape(-1) > 0.5, 12)
    ev = ~odd

    def schur(M):
        return M[np.ix_(odd, odd)] - M[np.ix_(odd, ev)] @ np.linalg.solve(M[np.ix_(ev, ev)], M[np.ix_(ev, odd)])

    D1 = dirac.WilsonClover(U, KAPPA, CSW, mu, mu_odd=mu + rho).dense()
    D0 = dirac.WilsonClover(U, KAPPA, CSW, mu).dense()
    g5o = _dense_g5(V)[np.ix_(odd, odd)]
    assert np.abs(schur(D1) - (schur(D0) + 1j * rho * g5o)).max() < 1e-12
    # and the even-even complement is untouched by rho
    D1e = D1[np.ix_(ev, ev)] - D1[np.ix_(ev, odd)] @ np.linalg.solve(D1[np.ix_(odd, odd)], D1[np.ix_(odd, ev)])
    D2 = dirac.WilsonClover(U, KAPPA, CSW, mu, mu_odd=mu).dense()
    assert np.abs(D1[np.ix_(ev, ev)] - D2[np.ix_(ev, ev)]).max() == 0.0
    assert np.abs(D1e - (D2[np.ix_(ev, ev)] - D2[np.ix_(ev, odd)] @ np.linalg.solve(
        D1[np.ix_(odd, odd)], D2[np.ix_(odd, ev)]))).max() < 1e-12


def test_gamma5_hermiticity_flips_both_twists(field):
    dims, U = field
    V = int(np.prod(dims))
    D = dirac.WilsonClover(U, KAPPA, CSW, 0.02, mu_odd=-0.07).dense()
    Dm = dirac.WilsonClover(U, KAPPA, CSW, -0.02, mu_odd=0.07).dense()
    G = _dense_g5(V)
    assert np.abs(D.conj().T - G @ Dm @ G).max() < 1e-13


def test_translation_by_one_site_swaps_the_parities(field):
    # shifting the lattice by one site in X maps even sites to odd ones: the
    # operator with (mu_e, mu_o) on U equals the shifted one with (mu_o, mu_e)
    dims, U = field
    psi = synth.spinor(dims, 3103)
    a = dirac.WilsonClover(U, KAPPA, CSW, 0.01, mu_odd=0.3).apply(psi)
    Us = np.roll(U, 1, axis=3)
    b = dirac.WilsonClover(Us, KAPPA, CSW, 0.3, mu_odd=0.01).apply(np.roll(psi, 1, axis=3))
    assert np.abs(np.roll(a, 1, axis=3) - b).max() < 1e-13
    # and the parities are not interchangeable without the shift
    c = dirac.WilsonClover(U, KAPPA, CSW, 0.3, mu_odd=0.01).apply(psi)
    assert np.abs(a - c).max() > 1e-3


def test_coarse_operator_is_the_galerkin_product(field):
    # D_c from the stencil assembly (mean twist + folded parity rest) equals
    # P^dag D(mu_e, mu_o) P formed column by column
    dims, U = field
    op = dirac.WilsonClover(U, KAPPA, CSW, 0.05, mu_odd=0.25)
    bsize, nv = (2, 2, 2, 2), 3
    Q = agg.orthonormalise(synth.gaussian((nv,) + dims + (12,), 3104), bsize)
    st = stencil.wilson_stencil(op)
    Dc = coarse.assemble(st, Q, bsize, op.mean_twist())
    bf = coarse.brute_force(stencil.FineLevel(op), Q, bsize, None)
    assert np.abs(Dc.dense() - bf).max() < 1e-12
    # the rest is not a multiple of Gamma5,c: a mean-twist operator differs
    bf0 = coarse.brute_force(stencil.FineLevel(op), Q, bsize, op.mean_twist())
    assert np.abs(bf - bf0).max() > 1e-3


def test_two_level_solve_and_the_reduced_solution():
    # the full operator D(mu, mu + rho) solved by the hierarchy built for it;
    # with b = (0, b_o) the odd part of x solves (D^(mu) + i rho G^5) x_o = b_o
    dims, bsize, nv = (4, 4, 4, 4), (2, 2, 2, 2), 8
    U = synth.gauge_field(dims, 0.3, 3105)
    mu, rho = 0.02, 0.3
    op = dirac.WilsonClover(U, KAPPA, CSW, mu, mu_odd=mu + rho)
    h = mg.Hierarchy(op, mg.Params(levels=2, blocks=[bsize], nvec=[nv], setup_iters=2))
    h.setup([synth.gaussian((nv,) + dims + (12,), 3106)])
    m = dirac.odd_mask(dims)[..., None, None]
    b = m * synth.spinor(dims, 3107)
    x, info = h.solve(b.reshape(dims + (12,)), tol=1e-11)
    x = x.reshape(dims + (4, 3))
    assert np.linalg.norm(b - op.apply(x)) <= 1e-11 * np.linalg.norm(b)
    op0 = dirac.WilsonClover(U, KAPPA, CSW, mu)
    r = b - dirac.schur_odd(op0, m * x, rho)
    assert np.linalg.norm(r) <= 1e-9 * np.linalg.norm(b)
