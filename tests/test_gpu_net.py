"""GPU parity of the learned-setup network (forward, loss, hand-written
backward) against the FP64 oracle.  Bars: FP32 forward <= 2e-5 relative;
loss <= 1e-5 relative; gradients <= 2e-4 relative per parameter block (sums
over all sites in FP32 partials with FP64 final reduction)."""
import numpy as np
import pytest

from oracle import aggregation as agg
from oracle import net
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


def _case(dd, C, L, dims, block, seed=0):
    U = synth.gauge_field(dims, 0.3, 800 + seed)
    W, a, b = synth.net_init_weights(C, L, 801 + seed, scale=1.5)
    rng = np.random.default_rng(802 + seed)
    a = [0.02 * rng.standard_normal(C) for _ in a]
    b = [0.5 * rng.standard_normal(C) for _ in b]
    ctx = dd.DDAMG(dims, block, KAPPA, CSW, MU)
    ctx.set_gauge(U)
    ctx.net_create(L, C)
    ctx.net_set_params(dd.pack_net(W, a, b))
    noise = synth.spinor(dims, 803 + seed, nvec=C)
    Q = agg.orthonormalise(synth.gaussian((C,) + dims + (12,), 804 + seed), block)
    return ctx, net.Net(W, a, b), U, noise, Q


@pytest.mark.parametrize("C,L,dims,block", [(4, 3, (4, 4, 4, 8), (2, 2, 2, 2)),
                                            (8, 2, (8, 4, 4, 8), (4, 2, 2, 2)),
                                            (24, 4, (4, 4, 4, 8), (2, 2, 2, 2))])
def test_network_forward(dd, C, L, dims, block):
    ctx, N, U, noise, Q = _case(dd, C, L, dims, block)
    got = ctx.net_forward(noise)
    want = N.forward(U, noise)
    assert rel(got, want) < 2e-5


@pytest.mark.parametrize("C,L,dims,block", [(4, 3, (4, 4, 4, 8), (2, 2, 2, 2)),
                                            (12, 3, (8, 4, 4, 8), (4, 2, 2, 2))])
def test_network_loss_and_gradients(dd, C, L, dims, block):
    ctx, N, U, noise, Q = _case(dd, C, L, dims, block, seed=1)
    loss, g = ctx.net_loss_grad(noise, Q.reshape((C,) + dims + (4, 3)))
    y, cache = N.forward(U, noise, keep=True)
    Lw, GY = net.subspace_loss(y.reshape((C,) + dims + (12,)), Q, block, grad=True)
    GW, Ga, Gb = N.backward(U, cache, GY.reshape(y.shape))
    assert abs(loss - Lw) <= 1e-5 * abs(Lw)
    Wg, ag, bg = dd.unpack_net(g, C, L)
    for l in range(L):
        assert rel(Wg[l], GW[l]) < 2e-4, l
    for l in range(L - 1):
        assert rel(ag[l], Ga[l]) < 2e-4 and rel(bg[l], Gb[l]) < 2e-4, l


def test_network_gauge_equivariant_on_gpu(dd):
    C, L, dims, block = 8, 3, (4, 4, 4, 8), (2, 2, 2, 2)
    ctx, N, U, noise, Q = _case(dd, C, L, dims, block, seed=2)
    y1 = ctx.net_forward(noise)
    Om = synth.gauge_transform(dims, 55)
    ctx.set_gauge(synth.transform_links(U, Om))
    y2 = ctx.net_forward(synth.transform_spinor(noise, Om))
    assert rel(synth.transform_spinor(y1, Om), y2) < 2e-5


def test_adam_steps_reduce_the_loss(dd):
    C, L, dims, block = 8, 3, (4, 4, 4, 8), (2, 2, 2, 2)
    ctx, N, U, noise, Q = _case(dd, C, L, dims, block, seed=3)
    tgt = Q.reshape((C,) + dims + (4, 3))
    losses = [ctx.net_train_step(noise, tgt, 3e-3) for _ in range(30)]
    assert losses[-1] < 0.8 * losses[0]
