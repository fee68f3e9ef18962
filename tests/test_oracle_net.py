"""Pins of the learned-setup network oracle: hand-derived gradients against
central finite differences, gauge equivariance, loss invariances."""
import numpy as np
import pytest

from oracle import aggregation as agg
from oracle import net
from paper_1611_01034_amd import synth

DIMS = (4, 2, 2, 4)
BS = (2, 2, 2, 2)
C = 3


def _setup(seed=0):
    U = synth.gauge_field(DIMS, 0.4, 700 + seed)
    W, a, b = synth.net_init_weights(C, 3, 701 + seed, scale=1.5)
    rng = np.random.default_rng(702 + seed)
    a = [0.3 * rng.standard_normal(C) for _ in a]
    b = [0.5 * rng.standard_normal(C) for _ in b]
    N = net.Net(W, a, b)
    x0 = synth.gaussian((C,) + DIMS + (4, 3), 703 + seed)
    Q = agg.orthonormalise(synth.gaussian((C,) + DIMS + (12,), 704 + seed), BS)
    return U, N, x0, Q


def _loss(N, U, x0, Q):
    y = N.forward(U, x0)
    return net.subspace_loss(y.reshape((C,) + DIMS + (12,)), Q, BS)


def test_transport_adjoint():
    U = synth.gauge_field(DIMS, 0.4, 1)
    x = synth.gaussian((2,) + DIMS + (4, 3), 2)
    g = synth.gaussian((2,) + DIMS + (4, 3), 3)
    for d in range(net.NOFF):
        lhs = np.vdot(g, net.transport(U, x, d))
        rhs = np.vdot(net.transport_adj(U, g, d), x)
        assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_gradients_match_central_differences():
    U, N, x0, Q = _setup()
    y, cache = N.forward(U, x0, keep=True)
    L, GY = net.subspace_loss(y.reshape((C,) + DIMS + (12,)), Q, BS, grad=True)
    GW, Ga, Gb = N.backward(U, cache, GY.reshape(y.shape))
    h = 1e-6
    rng = np.random.default_rng(5)
    for l in range(N.nlayers):
        for _ in range(4):
            idx = tuple(rng.integers(0, s) for s in N.W[l].shape)
            for unit in (1.0, 1j):
                N.W[l][idx] += h * unit
                Lp = _loss(N, U, x0, Q)
                N.W[l][idx] -= 2 * h * unit
                Lm = _loss(N, U, x0, Q)
                N.W[l][idx] += h * unit
                fd = (Lp - Lm) / (2 * h)
                an = GW[l][idx].real if unit == 1.0 else GW[l][idx].imag
                assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)) + 1e-8, (l, idx, unit, fd, an)
    for l in range(N.nlayers - 1):
        for arr, G in ((N.a, Ga), (N.b, Gb)):
            k = 1
            arr[l][k] += h
            Lp = _loss(N, U, x0, Q)
            arr[l][k] -= 2 * h
            Lm = _loss(N, U, x0, Q)
            arr[l][k] += h
            fd = (Lp - Lm) / (2 * h)
            assert abs(fd - G[l][k]) <= 1e-6 * max(1.0, abs(G[l][k])) + 1e-8


def test_network_is_gauge_equivariant():
    U, N, x0, Q = _setup(1)
    Om = synth.gauge_transform(DIMS, 9)
    y1 = N.forward(U, x0)
    y2 = N.forward(synth.transform_links(U, Om), synth.transform_spinor(x0, Om))
    assert np.abs(synth.transform_spinor(y1, Om) - y2).max() < 1e-12 * np.abs(y1).max()


def test_loss_invariances():
    U, N, x0, Q = _setup(2)
    assert net.subspace_loss(Q, Q, BS) < 1e-24
    # any invertible change of basis inside each aggregate half leaves the loss unchanged
    y = N.forward(U, x0).reshape((C,) + DIMS + (12,))
    M = agg._aggregate_matrices(y, DIMS, BS)
    rng = np.random.default_rng(3)
    R = rng.standard_normal(M.shape[:-2] + (C, C)) + 1j * rng.standard_normal(M.shape[:-2] + (C, C)) + 3 * np.eye(C)
    y2 = agg._from_aggregate_matrices(M @ R, DIMS, BS, 12)
    assert abs(net.subspace_loss(y, Q, BS) - net.subspace_loss(y2, Q, BS)) < 1e-12
    # and a gauge transformation of both output and target too
    Om = synth.gauge_transform(DIMS, 10)
    yt = synth.transform_spinor(y.reshape((C,) + DIMS + (4, 3)), Om).reshape(y.shape)
    Qt = synth.transform_spinor(Q.reshape((C,) + DIMS + (4, 3)), Om).reshape(Q.shape)
    assert abs(net.subspace_loss(y, Q, BS) - net.subspace_loss(yt, Qt, BS)) < 1e-12
