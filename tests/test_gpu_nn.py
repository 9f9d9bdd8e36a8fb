"""GPU tests of the learned coarse correction (include/vlbm_nn.h) against the FP64
oracle (oracle/conv_ref.py) and against the plain VLBM sweep.

Tolerances: a single convolution fed BF16-exact inputs and weights is exact up to
FP32 accumulation (rel <= 1e-5); the full network and its gradients keep BF16
activations (the oracle rounds its stored activations the same way, but not the
back-propagated gradients), so they agree to BF16 precision (rel-L2 a few 1e-3 for
the forward pass, <= 3e-2 for the gradients)."""
import numpy as np
import pytest

import oracle
import oracle.conv_ref as C
import synth
from test_gpu_parity import gpu_params

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    from paper_2606_00641_amd import nn, vlbm
    return torch, vlbm, nn


def flat(params):
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in params]).astype(np.float32)


def unflat(w, layers, cin=8, width=32, dim=2):
    out, off = [], 0
    for Ws, bs in C.Net.shapes(cin, width, layers, dim=dim):
        nW, nb = int(np.prod(Ws)), int(np.prod(bs))
        out.append((w[off:off + nW].reshape(Ws).astype(np.float64), w[off + nW:off + nW + nb].astype(np.float64)))
        off += nW + nb
    return out


def rand_params(rng, layers, bf16=True, dim=2):
    ps = []
    for Ws, bs in C.Net.shapes(8, 32, layers, dim=dim):
        fan = Ws[1] * 3 ** dim
        W = rng.normal(0, np.sqrt(2.0 / fan), Ws)
        b = rng.normal(0, 0.05, bs)
        ps.append((C.bf16_round(W) if bf16 else W, b.astype(np.float32).astype(np.float64)))
    return ps


def cm(torch, a):
    """Batch-major [B, C, (D,) H, W] numpy -> channel-major [C, B, (D,) H, W] FP32 device tensor."""
    return torch.tensor(np.ascontiguousarray(np.swapaxes(a, 0, 1)), dtype=torch.float32, device="cuda")


def bm(t):
    """Channel-major device tensor -> batch-major numpy."""
    return np.swapaxes(t.cpu().numpy(), 0, 1)


def rel_l2(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))


def make_net(env, layers, params, dim=2):
    torch, vlbm, nn = env
    net = nn.Net(8, 32, layers, stream=torch.cuda.current_stream().cuda_stream, dim=dim)
    net.vlbm_nn_set_weights(flat(params))
    return net


def test_single_conv_forward_exact(env):
    torch = env[0]
    rng = np.random.default_rng(0)
    params = rand_params(rng, 1)
    X = C.bf16_round(rng.normal(size=(2, 8, 32, 48)))
    net = make_net(env, 1, params)
    Y = torch.empty((8, 2, 32, 48), dtype=torch.float32, device="cuda")
    net.vlbm_nn_forward(cm(torch, X), Y)
    want = C.Net(params, layers=1).forward(X)
    assert rel_l2(bm(Y), want) < 1e-5


def test_full_forward_matches_quantised_oracle(env):
    torch = env[0]
    rng = np.random.default_rng(1)
    params = rand_params(rng, 4)
    X = rng.normal(size=(2, 8, 32, 32))
    net = make_net(env, 4, params)
    Y = torch.empty((8, 2, 32, 32), dtype=torch.float32, device="cuda")
    net.vlbm_nn_forward(cm(torch, X), Y)
    want = C.Net(params, layers=4, quantize=True).forward(X)
    assert rel_l2(bm(Y), want) < 1e-2


def test_normalisation(env):
    """dQ = out_mean + out_std * net((X - in_mean) / in_std)."""
    torch = env[0]
    rng = np.random.default_rng(2)
    params = rand_params(rng, 1)
    mu_in, sd_in = rng.normal(size=8), rng.uniform(0.5, 2, 8)
    mu_out, sd_out = rng.normal(size=8), rng.uniform(0.5, 2, 8)
    Xs = C.bf16_round(rng.normal(size=(1, 8, 16, 16)))
    X = Xs * sd_in[None, :, None, None] + mu_in[None, :, None, None]
    net = make_net(env, 1, params)
    net.vlbm_nn_set_norm(mu_in, sd_in, mu_out, sd_out)
    Y = torch.empty((8, 1, 16, 16), dtype=torch.float32, device="cuda")
    net.vlbm_nn_forward(cm(torch, X), Y)
    want = C.Net(params, layers=1, quantize=True).forward((X - mu_in[None, :, None, None]) / sd_in[None, :, None, None])
    want = want * sd_out[None, :, None, None] + mu_out[None, :, None, None]
    assert rel_l2(bm(Y), want) < 1e-2


@pytest.mark.parametrize("layers", [1, 2, 4])
def test_gradients_match_oracle(env, layers):
    torch = env[0]
    rng = np.random.default_rng(3 + layers)
    params = rand_params(rng, layers)
    X = rng.normal(size=(2, 8, 32, 32))
    T = rng.normal(size=(2, 8, 32, 32))
    net = make_net(env, layers, params)
    loss, g = net.vlbm_nn_loss_grad(cm(torch, X), cm(torch, T))
    oloss, ograds = C.Net(params, layers=layers, quantize=True).loss_and_grads(X, T)
    assert abs(loss - oloss) <= 1e-2 * oloss
    gp = unflat(g, layers)
    for l in range(layers):
        assert rel_l2(gp[l][0], ograds[l][0]) < 3e-2, (l, "W")
        assert rel_l2(gp[l][1], ograds[l][1]) < 3e-2, (l, "b")


def test_adam_step_matches_oracle(env):
    torch = env[0]
    rng = np.random.default_rng(9)
    params = rand_params(rng, 2, bf16=False)
    X = cm(torch, rng.normal(size=(1, 8, 16, 16)))
    T = cm(torch, rng.normal(size=(1, 8, 16, 16)))
    net = make_net(env, 2, params)
    w0 = net.vlbm_nn_get_weights()
    ad = C.Adam(unflat(w0, 2), lr=1e-3)
    cur = unflat(w0, 2)
    for _ in range(3):
        _, g = net.vlbm_nn_loss_grad(X, T)
        net.vlbm_nn_adam_step(1e-3)
        cur = ad.step(cur, unflat(g, 2))
    w = net.vlbm_nn_get_weights()
    assert np.allclose(w, flat(cur), rtol=1e-5, atol=1e-7)


def test_training_reduces_loss(env):
    torch = env[0]
    rng = np.random.default_rng(10)
    params = rand_params(rng, 4, bf16=False)
    for l in range(4):  # start near zero output
        params[l] = (params[l][0] * (0.1 if l == 3 else 1.0), params[l][1] * 0)
    X = rng.normal(size=(4, 8, 32, 32))
    T = 0.5 * np.roll(X, 1, axis=3) - 0.3 * X  # a learnable local linear map
    net = make_net(env, 4, params)
    Xt = cm(torch, X)
    Tt = cm(torch, T)
    l0, _ = net.vlbm_nn_loss_grad(Xt, Tt, want_grad=False)
    for _ in range(150):
        net.vlbm_nn_train_step(Xt, Tt, 3e-3)
    l1, _ = net.vlbm_nn_loss_grad(Xt, Tt, want_grad=False)
    assert l1 < 0.3 * l0, (l0, l1)


def test_restriction_matches_oracle(env):
    torch, vlbm, nn = env
    rng = np.random.default_rng(11)
    Qf = rng.normal(size=(8, 1, 64, 48)).astype(np.float32)
    out = torch.empty((8, 1, 16, 12), dtype=torch.float32, device="cuda")
    nn.vlbm_restrict(torch.tensor(Qf, device="cuda"), 4, out)
    want = C.restrict(Qf.astype(np.float64), 4)
    assert np.allclose(out.cpu().numpy(), want, rtol=1e-6, atol=1e-7)
    Q3 = rng.normal(size=(8, 8, 8, 16)).astype(np.float32)
    out3 = torch.empty((8, 4, 4, 8), dtype=torch.float32, device="cuda")
    nn.vlbm_restrict(torch.tensor(Q3, device="cuda"), 2, out3)
    assert np.allclose(out3.cpu().numpy(), C.restrict(Q3.astype(np.float64), 2), rtol=1e-6, atol=1e-7)
    # a batch of 2D fields (rz = 1) minus a field
    Qb = rng.normal(size=(8, 3, 32, 16)).astype(np.float32)
    mn = rng.normal(size=(8, 3, 8, 4)).astype(np.float32)
    outb = torch.empty((8, 3, 8, 4), dtype=torch.float32, device="cuda")
    nn.vlbm_restrict(torch.tensor(Qb, device="cuda"), 4, outb, rz=1, minus=torch.tensor(mn, device="cuda"))
    want = np.stack([C.restrict(Qb[:, j:j + 1].astype(np.float64), 4)[:, 0] for j in range(3)], axis=1) - mn
    assert np.allclose(outb.cpu().numpy(), want, rtol=1e-6, atol=1e-6)


# --- 3x3x3 network (3D lattices) -----------------------------------------------

@pytest.mark.parametrize("nz", [1, 2, 5])
def test_conv3_single_layer_forward_exact(env, nz):
    """One 3x3x3 layer, BF16-exact inputs and weights: exact up to FP32 accumulation.
    nz = 1 and 2 are the degenerate periodic cases (z-1 and z+1 the same slice)."""
    torch = env[0]
    rng = np.random.default_rng(20 + nz)
    params = rand_params(rng, 1, dim=3)
    X = C.bf16_round(rng.normal(size=(2, 8, nz, 16, 32)))
    net = make_net(env, 1, params, dim=3)
    Y = torch.empty((8, 2, nz, 16, 32), dtype=torch.float32, device="cuda")
    net.vlbm_nn_forward(cm(torch, X), Y)
    want = C.Net(params, layers=1, dim=3).forward(X)
    assert rel_l2(bm(Y), want) < 1e-5


def test_conv3_full_forward_matches_quantised_oracle(env):
    torch = env[0]
    rng = np.random.default_rng(24)
    params = rand_params(rng, 4, dim=3)
    X = rng.normal(size=(1, 8, 6, 16, 32))
    net = make_net(env, 4, params, dim=3)
    Y = torch.empty((8, 1, 6, 16, 32), dtype=torch.float32, device="cuda")
    net.vlbm_nn_forward(cm(torch, X), Y)
    want = C.Net(params, layers=4, quantize=True, dim=3).forward(X)
    assert rel_l2(bm(Y), want) < 1e-2


@pytest.mark.parametrize("layers", [1, 2, 4])
def test_conv3_gradients_match_oracle(env, layers):
    """Loss and every layer's weight and bias gradient (weight gradient over three
    z-slabs, data gradient through the mirrored 27-tap weights) against the FP64
    oracle on BF16-rounded activations."""
    torch = env[0]
    rng = np.random.default_rng(30 + layers)
    params = rand_params(rng, layers, dim=3)
    X = rng.normal(size=(2, 8, 3, 16, 16))
    T = rng.normal(size=(2, 8, 3, 16, 16))
    net = make_net(env, layers, params, dim=3)
    loss, g = net.vlbm_nn_loss_grad(cm(torch, X), cm(torch, T))
    oloss, ograds = C.Net(params, layers=layers, quantize=True, dim=3).loss_and_grads(X, T)
    assert abs(loss - oloss) <= 1e-2 * oloss
    gp = unflat(g, layers, dim=3)
    for l in range(layers):
        assert rel_l2(gp[l][0], ograds[l][0]) < 3e-2, (l, "W")
        assert rel_l2(gp[l][1], ograds[l][1]) < 3e-2, (l, "b")


def test_conv3_gradient_exact_single_layer(env):
    """One layer on BF16-exact inputs and weights with a loss gradient that is
    BF16-exact up to the FP32 rounding of the target (y - t a BF16 value times a
    power of two): the weight gradient of every tap of all three z-slabs then agrees
    to 1e-3, against 3e-2 where the activations are rounded."""
    torch = env[0]
    rng = np.random.default_rng(35)
    params = rand_params(rng, 1, dim=3)
    X = C.bf16_round(rng.normal(size=(1, 8, 4, 16, 16)))
    Y = C.Net(params, layers=1, dim=3).forward(X)
    n = Y.size  # dZ = 2 (y - t) / n: pick y - t = n/2 * BF16 values
    D = C.bf16_round(rng.normal(size=Y.shape)) * (n / 2.0) * 2.0 ** -20
    T = Y - D
    net = make_net(env, 1, params, dim=3)
    _, g = net.vlbm_nn_loss_grad(cm(torch, X), cm(torch, T))
    _, ograds = C.Net(params, layers=1, dim=3).loss_and_grads(X, T)
    gp = unflat(g, 1, dim=3)
    # the GPU's y is the FP32 forward, so y - t differs from D by FP32 rounding of y
    assert rel_l2(gp[0][0], ograds[0][0]) < 1e-3
    assert rel_l2(gp[0][1], ograds[0][1]) < 1e-3


@pytest.mark.parametrize("dim", [2, 3])
def test_weight_gradient_exact_on_bf16_exact_operands(env, dim):
    """One layer with zero weights and biases: the output is exactly 0 on both sides,
    so the loss gradient dZ = -2 T / n is BF16-exact for T a BF16 value times n / 2 and
    a power of two, and the inputs are BF16-exact: the weight and bias gradients are
    then exact up to the FP32 accumulation (<= 1e-5), every tap of every slab."""
    torch = env[0]
    rng = np.random.default_rng(37 + dim)
    shape = (2, 8, 16, 32) if dim == 2 else (1, 8, 3, 16, 16)
    params = [(np.zeros(Ws), np.zeros(bs)) for Ws, bs in C.Net.shapes(8, 32, 1, dim=dim)]
    X = C.bf16_round(rng.normal(size=shape))
    n = int(np.prod(shape))
    T = C.bf16_round(rng.normal(size=shape)) * (n / 2.0) * 2.0 ** -12
    net = make_net(env, 1, params, dim=dim)
    loss, g = net.vlbm_nn_loss_grad(cm(torch, X), cm(torch, T))
    oloss, ograds = C.Net(params, layers=1, dim=dim).loss_and_grads(X, T)
    assert abs(loss - oloss) <= 1e-6 * oloss
    gp = unflat(g, 1, dim=dim)
    assert rel_l2(gp[0][0], ograds[0][0]) < 1e-5
    assert rel_l2(gp[0][1], ograds[0][1]) < 1e-5


@pytest.mark.parametrize("dim,shape,layers", [(2, (3, 8, 256, 256), 3), (3, (1, 8, 40, 64, 64), 2)])
def test_gradients_match_oracle_many_tiles(env, dim, shape, layers):
    """More 16 x 16 tiles than weight-gradient workgroups (768 and 640 against 512), so
    every workgroup walks several tiles and reuses its LDS across the loop's barrier:
    loss and every layer's gradients against the oracle at the BF16 tolerance."""
    torch = env[0]
    rng = np.random.default_rng(50 + dim)
    params = rand_params(rng, layers, dim=dim)
    X = rng.normal(size=shape)
    T = rng.normal(size=shape)
    net = make_net(env, layers, params, dim=dim)
    loss, g = net.vlbm_nn_loss_grad(cm(torch, X), cm(torch, T))
    oloss, ograds = C.Net(params, layers=layers, quantize=True, dim=dim).loss_and_grads(X, T)
    assert abs(loss - oloss) <= 1e-2 * oloss
    gp = unflat(g, layers, dim=dim)
    for l in range(layers):
        assert rel_l2(gp[l][0], ograds[l][0]) < 3e-2, (l, "W")
        assert rel_l2(gp[l][1], ograds[l][1]) < 3e-2, (l, "b")


@pytest.mark.parametrize("dim,shape", [(2, (3, 8, 256, 256)), (3, (1, 8, 40, 64, 64))])
def test_weight_gradient_exact_many_tiles(env, dim, shape):
    """The exact weight-gradient case (zero layer, BF16-exact operands: agreement up to
    FP32 accumulation) with several tiles per workgroup (768 / 640 tiles, 512
    workgroups)."""
    torch = env[0]
    rng = np.random.default_rng(57 + dim)
    params = [(np.zeros(Ws), np.zeros(bs)) for Ws, bs in C.Net.shapes(8, 32, 1, dim=dim)]
    X = C.bf16_round(rng.normal(size=shape))
    n = int(np.prod(shape))
    T = C.bf16_round(rng.normal(size=shape)) * (n / 2.0) * 2.0 ** -16
    net = make_net(env, 1, params, dim=dim)
    loss, g = net.vlbm_nn_loss_grad(cm(torch, X), cm(torch, T))
    oloss, ograds = C.Net(params, layers=1, dim=dim).loss_and_grads(X, T)
    assert abs(loss - oloss) <= 1e-6 * oloss
    gp = unflat(g, 1, dim=dim)
    assert rel_l2(gp[0][0], ograds[0][0]) < 1e-5
    assert rel_l2(gp[0][1], ograds[0][1]) < 1e-5


def test_conv3_training_reduces_loss(env):
    torch = env[0]
    rng = np.random.default_rng(36)
    params = rand_params(rng, 4, bf16=False, dim=3)
    for l in range(4):
        params[l] = (params[l][0] * (0.1 if l == 3 else 1.0), params[l][1] * 0)
    X = rng.normal(size=(2, 8, 4, 16, 16))
    T = 0.5 * np.roll(X, 1, axis=2) - 0.3 * X  # a local linear map along z
    net = make_net(env, 4, params, dim=3)
    Xt, Tt = cm(torch, X), cm(torch, T)
    l0, _ = net.vlbm_nn_loss_grad(Xt, Tt, want_grad=False)
    for _ in range(150):
        net.vlbm_nn_train_step(Xt, Tt, 3e-3)
    l1, _ = net.vlbm_nn_loss_grad(Xt, Tt, want_grad=False)
    assert l1 < 0.3 * l0, (l0, l1)


def test_network_dimension_checks(env):
    torch, vlbm, nn = env
    net2 = nn.Net(8, 32, 1, stream=torch.cuda.current_stream().cuda_stream)
    X = torch.zeros((8, 1, 2, 16, 16), dtype=torch.float32, device="cuda")
    with pytest.raises(vlbm.VlbmError):  # a 3x3 network takes nz = 1 only
        nn._check(nn._lib.vlbm_nn_forward(net2.h, nn._dev(X), nn._dev(X), 1, 16, 16, 2), net2.h)
    with pytest.raises(vlbm.VlbmError):
        nn.Net(8, 32, 1, dim=4)
    net3 = nn.Net(8, 32, 1, stream=torch.cuda.current_stream().cuda_stream, dim=3)
    assert net3.vlbm_nn_num_params() == 8 * 8 * 27 + 8
    sim = coarse_sim(env, "f32", n=32)
    with pytest.raises(vlbm.VlbmError):  # corrected 2D stepping needs the 3x3 network
        nn.vlbm_step_corrected(sim, net3, 1, np.full(8, 1e30), 0.1)


# --- corrected coarse stepping ----------------------------------------------------

def coarse_sim(env, storage="f64", n=64, powell=1, seed=0):
    torch, vlbm, nn = env
    w = synth.workload_fourier_2d(n=n)
    w["powell"] = powell
    sim = vlbm.Vlbm(gpu_params(vlbm, w, storage))
    sim.vlbm_init_fields(synth.fourier_2d(n, seed=seed))
    return sim


def test_zero_weights_corrected_run_is_the_plain_run(env):
    torch, vlbm, nn = env
    a = coarse_sim(env)
    b = coarse_sim(env)
    net = nn.Net(8, 32, 4, stream=torch.cuda.current_stream().cuda_stream)  # weights zero
    nfb = nn.vlbm_step_corrected(a, net, 25, np.full(8, 1e30), 0.1)
    b.vlbm_step(25)
    assert nfb == 0
    assert np.array_equal(a.vlbm_get_populations()[0], b.vlbm_get_populations()[0])


def test_zero_bound_falls_back_every_step(env):
    torch, vlbm, nn = env
    rng = np.random.default_rng(12)
    a = coarse_sim(env, "f32")
    b = coarse_sim(env, "f32")
    net = make_net(env, 4, rand_params(rng, 4))
    nfb = nn.vlbm_step_corrected(a, net, 17, np.zeros(8), 0.1)
    b.vlbm_step(17)
    assert nfb == 17
    assert np.array_equal(a.vlbm_get_populations()[0], b.vlbm_get_populations()[0])


def test_huge_weights_fall_back(env):
    torch, vlbm, nn = env
    rng = np.random.default_rng(13)
    params = [(W * 1e4, b) for W, b in rand_params(rng, 4)]
    a = coarse_sim(env, "f32")
    net = make_net(env, 4, params)
    nfb = nn.vlbm_step_corrected(a, net, 9, np.full(8, 10.0), 0.1)
    assert nfb == 9


def test_uniform_correction_matches_oracle_emulation(env):
    """A network whose only nonzero parameters are the last layer's biases outputs a
    uniform correction c; the corrected run then equals the plain run with
    f_{k,i} += w_i c_k after every step (oracle), and totals grow by N c_k per step."""
    torch, vlbm, nn = env
    n, steps = 32, 12
    c = np.array([1e-4, 2e-5, -1e-5, 3e-5, 2e-4, 0.0, 0.0, 1e-5])  # no change of B_x, B_y: div B unchanged
    params = [(np.zeros(Ws), np.zeros(bs)) for Ws, bs in C.Net.shapes(8, 32, 4)]
    params[3] = (params[3][0], c.astype(np.float32).astype(np.float64))
    net = make_net(env, 4, params)
    sim = coarse_sim(env, "f64", n=n, powell=0)
    nfb = nn.vlbm_step_corrected(sim, net, steps, np.full(8, 1.0), 0.1, project_totals=False)
    assert nfb == 0
    Qg, tg = sim.vlbm_moments()
    w = synth.workload_fourier_2d(n=n)
    op = oracle.make_params(dim=2, shape=(n, n, 1), tau=w["tau"], s=w["s"], powell=0)
    f = oracle.init(op, synth.fourier_2d(n, seed=0))
    wts = np.array([1 / 3, 1 / 6, 1 / 6, 1 / 6, 1 / 6])
    cf = c.astype(np.float32).astype(np.float64)
    for _ in range(steps):
        oracle.run(op, f, 1)
        f += (cf[:, None] * wts[None, :])[:, :, None]
    Qo, _, to = oracle.moments(op, f)
    assert np.abs(Qg - Qo).max() <= 1e-10
    _, _, t0 = oracle.moments(op, oracle.init(op, synth.fourier_2d(n, seed=0)))
    assert np.allclose(tg[:8] - t0[:8], steps * n * n * cf, rtol=1e-6, atol=1e-9)


def test_projected_uniform_correction_is_the_plain_run(env):
    """Projected to zero lattice totals, a uniform correction vanishes exactly: the run
    is bitwise the plain run."""
    torch, vlbm, nn = env
    c = np.array([1e-4, 2e-5, -1e-5, 3e-5, 2e-4, 1e-5, -2e-5, 1e-5])
    params = [(np.zeros(Ws), np.zeros(bs)) for Ws, bs in C.Net.shapes(8, 32, 4)]
    params[3] = (params[3][0], c.astype(np.float32).astype(np.float64))
    net = make_net(env, 4, params)
    a = coarse_sim(env, "f32", n=32)
    b = coarse_sim(env, "f32", n=32)
    assert nn.vlbm_step_corrected(a, net, 11, np.full(8, 1.0), 0.1) == 0
    b.vlbm_step(11)
    assert np.array_equal(a.vlbm_get_populations()[0], b.vlbm_get_populations()[0])


def test_projection_keeps_each_lattice_total(env):
    """A random network's correction, projected, leaves the total mass of every lattice
    of the batch where the plain VLBM keeps it, up to the FP32 rounding of the
    correction itself (|sum dQ| <= N 2^-24 max|dQ| per step: here below 1e-9 of the
    mass after 13 steps), while the unprojected correction moves it by 1e-3."""
    torch, vlbm, nn = env
    rng = np.random.default_rng(31)
    params = [(W * 0.05, b * 0.01) for W, b in rand_params(rng, 4)]
    net = make_net(env, 4, params)
    n, B = 32, 3
    w = synth.workload_fourier_2d(n=n)
    Q0 = np.concatenate([synth.fourier_2d(n, seed=40 + j) for j in range(B)], axis=1)

    def lattice_mass(sim):
        Q, _ = sim.vlbm_moments()
        return np.asarray(Q).reshape(8, B, n * n)[0].sum(axis=1)

    out = {}
    for proj in (True, False):
        sim = vlbm.Vlbm(gpu_params(vlbm, w, "f64", shape=(n, n, B)))
        sim.vlbm_init_fields(Q0)
        m0 = lattice_mass(sim)
        nn.vlbm_step_corrected(sim, net, 13, np.full(8, 10.0), 10.0, 1.0, project_totals=proj)
        out[proj] = np.abs(lattice_mass(sim) - m0).max() / np.abs(m0).max()
    assert out[True] <= 1e-9, out
    assert out[False] > 1e5 * max(out[True], 1e-16), out


def test_replayed_steps_equal_single_steps(env):
    """Long calls replay a captured pair of corrected steps; the result is bitwise the
    result of the same steps taken one call at a time (eager), fallbacks included."""
    torch, vlbm, nn = env
    rng = np.random.default_rng(21)
    params = [(W * 0.05, b * 0.01) for W, b in rand_params(rng, 4)]
    net = make_net(env, 4, params)
    bound = np.full(8, 0.02)
    a = coarse_sim(env, "f32", n=32, seed=4)
    b = coarse_sim(env, "f32", n=32, seed=4)
    nfa = nn.vlbm_step_corrected(a, net, 15, bound, 0.1, 1e-6)
    nfb = sum(nn.vlbm_step_corrected(b, net, 1, bound, 0.1, 1e-6) for _ in range(15))
    assert a.vlbm_get_step() == b.vlbm_get_step() == 15
    assert nfa == nfb
    # single calls inject their correction at the end of each call rather than
    # before the next collision: compare the moments, to FP32 rounding
    qa, _ = a.vlbm_moments()
    qb, _ = b.vlbm_moments()
    assert np.abs(qa - qb).max() <= 1e-5 * np.abs(qb).max()


def _moderate_net(env, seed):
    rng = np.random.default_rng(seed)
    return make_net(env, 4, [(W * 0.05, b * 0.01) for W, b in rand_params(rng, 4)])


def test_graph_kept_between_calls_equals_fresh_handles(env):
    """The handle keeps the captured pair of steps from call to call.  Calls 2 and 3 on
    one handle (its graph replayed, also after another context used the handle in
    between, which makes it capture again) give bitwise the populations of the same
    calls made each with a fresh handle of the same weights (fresh capture)."""
    torch, vlbm, nn = env
    bound = np.full(8, 0.02)
    a = coarse_sim(env, "f32", n=32, seed=4)
    other = coarse_sim(env, "f32", n=32, seed=5)
    ref = coarse_sim(env, "f32", n=32, seed=4)
    net = _moderate_net(env, 21)
    nfa = nfr = 0
    for call in range(3):
        nfa += nn.vlbm_step_corrected(a, net, 8, bound, 0.1, 1e-6)
        if call == 1:
            nn.vlbm_step_corrected(other, net, 6, bound, 0.1, 1e-6)
        nfr += nn.vlbm_step_corrected(ref, _moderate_net(env, 21), 8, bound, 0.1, 1e-6)
    assert a.vlbm_get_step() == ref.vlbm_get_step() == 24
    assert nfa == nfr
    assert np.array_equal(a.vlbm_get_populations()[0], ref.vlbm_get_populations()[0])


def test_graph_captured_again_after_reinit(env):
    """FP16 storage: initialising the context again changes its codec (rest state and
    scales), which the sweep takes by value; the handle's graph must not be replayed
    with the old one.  Result bitwise that of a fresh context and handle."""
    torch, vlbm, nn = env
    bound = np.full(8, 1e30)
    a = coarse_sim(env, "f16", n=32, seed=4)
    net = _moderate_net(env, 22)
    nn.vlbm_step_corrected(a, net, 8, bound, 10.0, 1.0)
    q2 = synth.fourier_2d(32, seed=9)
    q2[0] *= 1.5  # another density level: another rest state
    a.vlbm_init_fields(q2)
    nfa = nn.vlbm_step_corrected(a, net, 8, bound, 10.0, 1.0)
    b = coarse_sim(env, "f16", n=32, seed=4)
    b.vlbm_init_fields(q2)
    nfb = nn.vlbm_step_corrected(b, _moderate_net(env, 22), 8, bound, 10.0, 1.0)
    assert nfa == nfb == 0
    assert a.vlbm_get_step() == b.vlbm_get_step() == 8
    assert np.array_equal(a.vlbm_get_populations()[0], b.vlbm_get_populations()[0])


def test_gate_bounds_change_under_a_kept_graph(env):
    """The gate reads its bounds from device memory written at each call, so a graph
    kept from an earlier call applies the bounds of the current one."""
    torch, vlbm, nn = env
    a = coarse_sim(env, "f32", n=32, seed=6)
    net = _moderate_net(env, 23)
    assert nn.vlbm_step_corrected(a, net, 8, np.full(8, 1e30), 10.0, 1.0) == 0
    assert nn.vlbm_step_corrected(a, net, 8, np.zeros(8), 10.0, 1.0) == 8
    assert nn.vlbm_step_corrected(a, net, 8, np.full(8, 1e30), 10.0, 1.0) == 0
    # a step with the gate closed is the plain step: compare a closed-gate call with
    # the plain sweep from the same populations
    f, par, step = a.vlbm_get_populations()
    b = coarse_sim(env, "f32", n=32, seed=6)
    b.vlbm_set_populations(f, par, step)
    assert nn.vlbm_step_corrected(a, net, 10, np.zeros(8), 10.0, 1.0) == 10
    b.vlbm_step(10)
    assert np.array_equal(a.vlbm_get_populations()[0], b.vlbm_get_populations()[0])


# --- corrected stepping of a 3D lattice (3x3x3 network) --------------------------

SHAPE3 = (32, 16, 8)  # nx, ny, nz


def sim3(env, storage="f64", powell=1, seed=1):
    torch, vlbm, nn = env
    w = synth.workload_slab_3d()
    w["powell"] = powell
    sim = vlbm.Vlbm(gpu_params(vlbm, w, storage, shape=SHAPE3))
    sim.vlbm_init_fields(state3(seed))
    return sim


def state3(seed=1):
    nx, ny, nz = SHAPE3
    return synth.turbulence_3d(n=16, seed=seed, shape=(nz, ny, nx))[:8]


def test_3d_zero_weights_corrected_run_is_the_plain_run(env):
    """Zero network: every step is accepted and adds nothing, so the corrected run
    (two eager steps, captured pairs, a last eager step) is bitwise the plain run."""
    torch, vlbm, nn = env
    a, b = sim3(env), sim3(env)
    net = nn.Net(8, 32, 4, stream=torch.cuda.current_stream().cuda_stream, dim=3)
    assert nn.vlbm_step_corrected(a, net, 9, np.full(8, 1e30), 0.1) == 0
    b.vlbm_step(9)
    assert np.array_equal(a.vlbm_get_populations()[0], b.vlbm_get_populations()[0])


def test_3d_zero_bound_falls_back_every_step(env):
    torch, vlbm, nn = env
    rng = np.random.default_rng(40)
    a, b = sim3(env, "f32"), sim3(env, "f32")
    net = make_net(env, 4, rand_params(rng, 4, dim=3), dim=3)
    assert nn.vlbm_step_corrected(a, net, 7, np.zeros(8), 0.1) == 7
    b.vlbm_step(7)
    assert np.array_equal(a.vlbm_get_populations()[0], b.vlbm_get_populations()[0])


def test_3d_uniform_correction_matches_oracle_emulation(env):
    """Only the last biases nonzero: a uniform correction c, so the corrected run is
    the plain D3Q7 run with f_{k,i} += w_i c_k after every step (oracle, w_0 = 1/4,
    w_i = 1/8), and the totals grow by N c_k per step."""
    torch, vlbm, nn = env
    steps = 8
    c = np.array([1e-4, 2e-5, -1e-5, 3e-5, 2e-4, 1e-5, -2e-5, 1e-5])  # uniform: div B unchanged
    params = [(np.zeros(Ws), np.zeros(bs)) for Ws, bs in C.Net.shapes(8, 32, 4, dim=3)]
    params[3] = (params[3][0], c.astype(np.float32).astype(np.float64))
    net = make_net(env, 4, params, dim=3)
    sim = sim3(env, "f64", powell=0)
    assert nn.vlbm_step_corrected(sim, net, steps, np.full(8, 1.0), 0.1, project_totals=False) == 0
    Qg, tg = sim.vlbm_moments()
    w = synth.workload_slab_3d()
    op = oracle.make_params(dim=3, shape=SHAPE3, tau=w["tau"], s=w["s"], powell=0)
    f = oracle.init(op, state3())
    wts = np.array([1 / 4] + [1 / 8] * 6)
    cf = c.astype(np.float32).astype(np.float64)
    for _ in range(steps):
        oracle.run(op, f, 1)
        f += (cf[:, None] * wts[None, :])[:, :, None]
    Qo, _, to = oracle.moments(op, f)
    assert np.abs(Qg - Qo).max() <= 1e-10
    _, _, t0 = oracle.moments(op, oracle.init(op, state3()))
    N = int(np.prod(SHAPE3))
    assert np.allclose(tg[:8] - t0[:8], steps * N * cf, rtol=1e-6, atol=1e-9)


def test_3d_projection_removes_a_uniform_correction(env):
    """Projected onto zero lattice totals (one 3D lattice), a uniform correction
    vanishes exactly: the run is bitwise the plain run."""
    torch, vlbm, nn = env
    c = np.array([1e-4, 2e-5, -1e-5, 3e-5, 2e-4, 1e-5, -2e-5, 1e-5])
    params = [(np.zeros(Ws), np.zeros(bs)) for Ws, bs in C.Net.shapes(8, 32, 4, dim=3)]
    params[3] = (params[3][0], c.astype(np.float32).astype(np.float64))
    net = make_net(env, 4, params, dim=3)
    a, b = sim3(env, "f32"), sim3(env, "f32")
    assert nn.vlbm_step_corrected(a, net, 6, np.full(8, 1.0), 0.1) == 0
    b.vlbm_step(6)
    assert np.array_equal(a.vlbm_get_populations()[0], b.vlbm_get_populations()[0])


def test_3d_gate_sees_the_z_divergence(env):
    """A one-layer network whose only taps map B_z to dB_z = a (B_z(z+1) - B_z(z-1)):
    it changes div B only through d/dz.  The oracle gate rejects it in 3D and would
    accept it if only the in-plane divergence were checked; the GPU gate falls back."""
    torch, vlbm, nn = env
    a = 0.25
    W = np.zeros((8, 8, 3, 3, 3))
    W[7, 7, 0, 1, 1], W[7, 7, 2, 1, 1] = -a, a
    params = [(W, np.zeros(8))]
    Q = state3()
    dQ = C.Net(params, layers=1, quantize=True, dim=3).forward(Q[None])[0]
    big = np.full(8, 1e30)
    assert not C.gate(Q, dQ, big, 0.1, dim=3)
    assert C.gate(Q, dQ, big, 0.1, dim=2)
    net = make_net(env, 1, params, dim=3)
    sim = sim3(env, "f64")
    assert nn.vlbm_step_corrected(sim, net, 1, big, 0.1) == 1
    # with the divergence allowance raised far enough the same correction is accepted
    sim2 = sim3(env, "f64")
    assert nn.vlbm_step_corrected(sim2, net, 1, big, 0.1, bound_divb_abs=1e3) == 0


def test_3d_corrected_step_refusals(env):
    """On a lattice with faces the corrected step refuses the projection onto zero
    totals (faces change the totals); the bounce-back body (solid cells) is refused by
    the corrected step and by vlbm_inject; a 3D context refuses a 2D network."""
    torch, vlbm, nn = env
    w = synth.workload_slab_3d()
    Q = state3()
    Qin = Q[:, 0, 0, 0].astype(np.float64)
    opened = vlbm.Vlbm(vlbm.make_params(lattice="D3Q7", shape=SHAPE3, model="ideal", storage="f32", gamma=w["gamma"],
                                        flux_scale=w["s"], tau=w["tau"], bc=(1, 2, 0, 0, 0, 0), inflow_Q=Qin,
                                        stream=torch.cuda.current_stream().cuda_stream))
    opened.vlbm_init_fields(Q)
    net3 = nn.Net(8, 32, 1, stream=torch.cuda.current_stream().cuda_stream, dim=3)
    with pytest.raises(vlbm.VlbmError):
        nn.vlbm_step_corrected(opened, net3, 1, np.full(8, 1e30), 0.1, project_totals=True)
    bb = open_sim(env, "f32", mode=1)
    with pytest.raises(vlbm.VlbmError):
        nn.vlbm_step_corrected(bb, nn.Net(8, 32, 1, stream=torch.cuda.current_stream().cuda_stream, dim=3), 1,
                               np.full(8, 1e30), 0.1, project_totals=False)
    with pytest.raises(vlbm.VlbmError):
        nn.vlbm_inject(bb, torch.zeros((8, int(np.prod(OPEN_SHAPE))), dtype=torch.float32, device="cuda"))
    net2 = nn.Net(8, 32, 1, stream=torch.cuda.current_stream().cuda_stream)
    with pytest.raises(vlbm.VlbmError):
        nn.vlbm_step_corrected(sim3(env, "f32"), net2, 1, np.full(8, 1e30), 0.1)


# --- corrected stepping of an open 3D lattice (faces, homogenized body) -----------

OPEN_SHAPE = (32, 32, 16)  # nx, ny, nz
OPEN_BC = (1, 2, 2, 2, 2, 2)


def open_case(mode=2):
    """Inflow at x-, zero gradient elsewhere, a moving rough magnetised body (mode 2
    homogenized, 1 bounce-back) in a perturbed Mach-0.8 inflow state."""
    Qin, _ = synth.inflow_state(mach=0.8, alfven_mach=4.0)
    Q0 = np.broadcast_to(Qin[:, None, None, None], (8,) + OPEN_SHAPE[::-1]).copy()
    Q0 += 0.3 * synth.smooth_box_state(OPEN_SHAPE[::-1], seed=13, amp=0.05, rho=0.0, p=0.0, B0=0.0)
    body = synth.rough_body((12.3, 15.1, 7.7), (0.06, 0.03, 0.0), 5.0, m=(3.0, -2.0, 1.5), rough=0.12, seed=5)
    body["mode"] = mode
    return Q0, Qin, body


def open_sim(env, storage, mode=2):
    torch, vlbm, nn = env
    Q0, Qin, body = open_case(mode)
    sim = vlbm.Vlbm(vlbm.make_params(lattice="D3Q7", shape=OPEN_SHAPE, model="ideal", storage=storage, flux_scale=0.1,
                                     tau=0.7, bc=OPEN_BC, inflow_Q=Qin, body=body,
                                     stream=torch.cuda.current_stream().cuda_stream))
    sim.vlbm_init_fields(Q0)
    return sim


def test_open_zero_weights_corrected_run_is_the_plain_run(env):
    """Zero network on the open lattice: every correction is zero and accepted, and the
    corrected run (injection, moments pass, plain step) is bitwise the plain run."""
    torch, vlbm, nn = env
    a, b = open_sim(env, "f32"), open_sim(env, "f32")
    net = nn.Net(8, 32, 4, stream=torch.cuda.current_stream().cuda_stream, dim=3)
    assert nn.vlbm_step_corrected(a, net, 9, np.full(8, 1e30), 10.0, 1.0, project_totals=False) == 0
    b.vlbm_step(9)
    assert np.array_equal(a.vlbm_get_populations()[0], b.vlbm_get_populations()[0])


def test_open_zero_bound_falls_back_every_step(env):
    torch, vlbm, nn = env
    rng = np.random.default_rng(31)
    a, b = open_sim(env, "f32"), open_sim(env, "f32")
    net = make_net(env, 4, rand_params(rng, 4, dim=3), dim=3)
    assert nn.vlbm_step_corrected(a, net, 7, np.zeros(8), 10.0, 1.0, project_totals=False) == 7
    b.vlbm_step(7)
    assert np.array_equal(a.vlbm_get_populations()[0], b.vlbm_get_populations()[0])


def test_open_gate_rejects_an_unphysical_correction(env):
    """Without the projection the gate also holds the corrected state physical: a
    network whose only nonzero parameter is the last layer's bias in E applies a
    uniform change of the energy; lowering E by 1.5 times the smallest internal-energy
    margin of the state the correction is added to -- the state after the plain step
    (E - |rho u|^2 / (2 rho) - |B|^2 / 2, its minimum over the cells) -- leaves cells with
    a negative pressure and falls back, by half of it is accepted; the oracle's gate
    (conv_ref.physical) decides the same."""
    torch, vlbm, nn = env
    sim = open_sim(env, "f64")
    sim.vlbm_step(1)  # the gate judges the state after the plain step
    Q = sim.vlbm_moments()[0].reshape((8,) + OPEN_SHAPE[::-1])
    margin = float((Q[4] - 0.5 * (Q[1] ** 2 + Q[2] ** 2 + Q[3] ** 2) / Q[0]
                    - 0.5 * (Q[5] ** 2 + Q[6] ** 2 + Q[7] ** 2)).min())
    assert margin > 0
    big = np.full(8, 1e30)
    for frac, want in ((1.5, 1), (0.5, 0)):
        params = [(np.zeros(Ws), np.zeros(bs)) for Ws, bs in C.Net.shapes(8, 32, 4, dim=3)]
        params[-1][1][4] = -frac * margin
        net = make_net(env, 4, params, dim=3)
        net.vlbm_nn_set_norm(np.zeros(8), np.ones(8), np.zeros(8), np.ones(8))
        dQ = np.zeros_like(Q)
        dQ[4] = np.float32(-frac * margin)
        assert C.gate(Q, dQ, big, 10.0, 1.0, dim=3, gamma=5.0 / 3.0) == (want == 0)
        a = open_sim(env, "f64")
        assert nn.vlbm_step_corrected(a, net, 1, big, 10.0, 1.0, project_totals=False) == want, frac


def _oracle_corrected_open(op, f, net_o, steps, t0, bounds, norm):
    """The open-lattice corrected run from the oracle's parts: per step X = the moments
    of the populations, dQ = out_mean + out_std * Net((X - in_mean) / in_std) (no
    projection), one step with the faces and the body (run_bc at time t0 + j), the gate
    on (X', dQ) with X' the moments after that step and the positivity condition, then
    f_{k,i} += w_i dQ_k if the gate accepted.  Returns the applied corrections and the
    decisions."""
    in_mean, in_std, out_mean, out_std = (np.asarray(a, np.float64)[:, None, None, None] for a in norm)
    wts = np.array([op.w0] + [(1.0 - op.w0) / 6.0] * 6)
    applied, decisions = [], []
    for j in range(steps):
        X = oracle.moments(op, f)[0].reshape(8, op.nz, op.ny, op.nx)
        dQ = out_mean + out_std * net_o.forward(((X - in_mean) / in_std)[None])[0]
        oracle.run_bc(op, f, 1, t0 + j)
        Xp = oracle.moments(op, f)[0].reshape(8, op.nz, op.ny, op.nx)
        ok = C.gate(Xp, dQ, bounds[0], bounds[1], bounds[2], dim=3, gamma=5.0 / 3.0)
        if ok:
            f += wts[None, :, None] * dQ.reshape(8, 1, -1)
        applied.append(dQ if ok else np.zeros_like(dQ))
        decisions.append(ok)
    return applied, decisions


def test_open_random_network_corrected_steps_match_oracle(env):
    """A random 4-layer 3x3x3 network drives the corrected step on the open lattice
    (FP64 populations): against the oracle's composition with its own face and body
    step, the first applied correction agrees per channel to the network's BF16
    precision (rel-L2 <= 1e-2); after three steps the departure from the plain run
    agrees per channel to 1e-2, and the state to 1e-2 of that departure (the network's
    BF16 rounding is the only difference; near the body the random network's
    corrections reach about 2 % of the state, so the bound scales with them rather
    than with the state); a step whose correction exceeds its bound is bitwise the
    plain step."""
    torch, vlbm, nn = env
    rng = np.random.default_rng(75)
    params = rand_params(rng, 4, dim=3)
    net = make_net(env, 4, params, dim=3)
    Q0, Qin, body = open_case(2)
    in_mean = Q0.reshape(8, -1).mean(axis=1)
    in_std = Q0.reshape(8, -1).std(axis=1) + 1e-3
    norm = (in_mean, in_std, np.zeros(8), np.full(8, 5e-5))
    net.vlbm_nn_set_norm(*norm)
    net_o = C.Net(params, layers=4, quantize=True, dim=3)

    def oracle_state():
        op = oracle.make_params(dim=3, shape=OPEN_SHAPE, s=0.1, tau=0.7)
        oracle.set_boundaries(op, bc=OPEN_BC, inflow_Q=Qin, body=body, body_mode=2)
        return op, oracle.init(op, Q0)

    a, plain = open_sim(env, "f64"), open_sim(env, "f64")
    op, f = oracle_state()
    opl, fpl = oracle_state()
    big = np.full(8, 1e30)
    applied, ok = _oracle_corrected_open(op, f, net_o, 1, 0, (big, 10.0, 1.0), norm)
    assert ok == [True]
    assert nn.vlbm_step_corrected(a, net, 1, big, 10.0, 1.0, project_totals=False) == 0
    plain.vlbm_step(1)
    oracle.run_bc(opl, fpl, 1, 0)
    shape4 = (8,) + OPEN_SHAPE[::-1]
    Qa, Qp = a.vlbm_moments()[0].reshape(shape4), plain.vlbm_moments()[0].reshape(shape4)
    Qpo = oracle.moments(opl, fpl)[0].reshape(shape4)
    assert np.abs(Qp - Qpo).max() <= 1e-10 * np.abs(Q0).max()
    dq = Qa - Qp
    for k in range(8):
        assert rel_l2(dq[k], applied[0][k]) <= 1e-2, k
    _, ok = _oracle_corrected_open(op, f, net_o, 2, 1, (big, 10.0, 1.0), norm)
    assert ok == [True, True]
    assert nn.vlbm_step_corrected(a, net, 2, big, 10.0, 1.0, project_totals=False) == 0
    plain.vlbm_step(2)
    oracle.run_bc(opl, fpl, 2, 1)
    Qa, Qp = a.vlbm_moments()[0].reshape(shape4), plain.vlbm_moments()[0].reshape(shape4)
    Qo, Qpo = oracle.moments(op, f)[0].reshape(shape4), oracle.moments(opl, fpl)[0].reshape(shape4)
    assert np.abs(Qa - Qo).max() <= 1e-2 * np.abs(Qo - Qpo).max()
    for k in range(8):
        assert rel_l2((Qa - Qp)[k], (Qo - Qpo)[k]) <= 1e-2, k
    # a correction over its bound in E: rejected, the plain step
    probe = f.copy()
    applied, _ = _oracle_corrected_open(op, probe, net_o, 1, 3, (big, 10.0, 1.0), norm)
    e_norm = float(np.sqrt((applied[0][4] ** 2).sum()))
    tight = big.copy()
    tight[4] = 0.5 * e_norm
    _, ok = _oracle_corrected_open(op, f, net_o, 1, 3, (tight, 10.0, 1.0), norm)
    assert ok == [False]
    before, par, step = a.vlbm_get_populations()
    ref = open_sim(env, "f64")
    ref.vlbm_set_populations(before, par, step)
    assert nn.vlbm_step_corrected(a, net, 1, tight, 10.0, 1.0, project_totals=False) == 1
    ref.vlbm_step(1)
    assert np.array_equal(a.vlbm_get_populations()[0], ref.vlbm_get_populations()[0])


@pytest.mark.parametrize("storage", ["f16", "bf16"])
@pytest.mark.parametrize("dim", [2, 3])
def test_low_precision_zero_weights_corrected_run_is_the_plain_run(env, storage, dim):
    """FP16/BF16 deviation storage: a zero network adds nothing (the injecting sweep
    adds zero to the decoded populations; the last injection leaves the stored values
    as they are), so the corrected run is bitwise the plain run."""
    torch, vlbm, nn = env
    if dim == 2:
        a, b = coarse_sim(env, storage, n=32), coarse_sim(env, storage, n=32)
    else:
        a, b = sim3(env, storage), sim3(env, storage)
    net = nn.Net(8, 32, 2, stream=torch.cuda.current_stream().cuda_stream, dim=dim)
    assert nn.vlbm_step_corrected(a, net, 9, np.full(8, 1e30), 0.1) == 0
    b.vlbm_step(9)
    assert np.array_equal(a.vlbm_get_populations()[0], b.vlbm_get_populations()[0])


@pytest.mark.parametrize("storage", ["f16", "bf16"])
def test_low_precision_uniform_correction_moves_the_totals(env, storage):
    """FP16/BF16 storage, a uniform correction c (last biases only): after n steps the
    totals exceed those of the plain run of the same storage by n N c, up to the
    storage's rounding of the populations (2 % here, against 100 % for a missing or
    doubled injection); no step falls back."""
    torch, vlbm, nn = env
    steps = 8
    c = np.full(8, 1e-3)
    params = [(np.zeros(Ws), np.zeros(bs)) for Ws, bs in C.Net.shapes(8, 32, 2, dim=3)]
    params[1] = (params[1][0], c.astype(np.float32).astype(np.float64))
    net = make_net(env, 2, params, dim=3)
    a, b = sim3(env, storage, powell=0), sim3(env, storage, powell=0)
    assert nn.vlbm_step_corrected(a, net, steps, np.full(8, 1.0), 0.1, project_totals=False) == 0
    b.vlbm_step(steps)
    _, ta = a.vlbm_moments()
    _, tb = b.vlbm_moments()
    N = int(np.prod(SHAPE3))
    assert np.allclose(ta[:8] - tb[:8], steps * N * c.astype(np.float32), rtol=2e-2)


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_3d_replayed_steps_equal_single_steps(env, storage):
    """3D lattice: a long call (captured pairs replayed) against the same steps taken
    one call at a time."""
    torch, vlbm, nn = env
    rng = np.random.default_rng(42)
    params = [(W * 0.05, b * 0.01) for W, b in rand_params(rng, 4, dim=3)]
    net = make_net(env, 4, params, dim=3)
    a, b = sim3(env, storage), sim3(env, storage)
    # a bound well above the corrections' norms on the initial state
    q0 = torch.tensor(state3(), dtype=torch.float32, device="cuda").reshape(8, 1, 8, 16, 32)
    out = torch.empty_like(q0)
    net.vlbm_nn_forward(q0, out)
    bound = 4.0 * torch.linalg.vector_norm(out.reshape(8, -1), dim=1).cpu().numpy().astype(np.float64)
    nfa = nn.vlbm_step_corrected(a, net, 13, bound, 10.0, 1.0)
    nfb = sum(nn.vlbm_step_corrected(b, net, 1, bound, 10.0, 1.0) for _ in range(13))
    assert a.vlbm_get_step() == b.vlbm_get_step() == 13
    assert nfa == nfb == 0
    # single calls inject their correction at the end of each call rather than before
    # the next collision: compare the moments, to the storage's rounding
    qa, _ = a.vlbm_moments()
    qb, _ = b.vlbm_moments()
    tol = 1e-5 if storage == "f32" else 2e-3
    assert np.abs(qa - qb).max() <= tol * np.abs(qb).max()


def test_3d_inject_matches_oracle(env):
    """vlbm_inject on a 3D context adds w_i dQ_k to every population."""
    torch, vlbm, nn = env
    rng = np.random.default_rng(41)
    sim = sim3(env, "f64")
    sim.vlbm_step(3)
    Q0, _ = sim.vlbm_moments()
    dQ = rng.normal(0, 1e-3, (8,) + Q0.shape[1:])
    nn.vlbm_inject(sim, torch.tensor(dQ, dtype=torch.float32, device="cuda"))
    Q1, _ = sim.vlbm_moments()
    assert np.abs(Q1 - Q0 - dQ.astype(np.float32)).max() <= 1e-12


# --- a random network's corrected steps against the oracle's composition ---------

def _oracle_corrected(op_list, f_list, net_o, steps, bounds, norm, dim):
    """The corrected coarse run composed from the oracle's parts: per step X = the
    moments of the populations, dQ = P(out_mean + out_std * Net((X - in_mean) /
    in_std)) (the quantised Net rounds its input to BF16; P the projection onto zero
    lattice totals), the gate on (X, dQ) with bounds = (bound_corr, rel, abs), one
    plain VLBM step, then f_{k,i} += w_i dQ_k if the gate accepted.  op_list / f_list:
    one oracle lattice per batch entry (advanced in place).  Returns the applied
    corrections (zero where rejected) and the decisions."""
    in_mean, in_std, out_mean, out_std = (np.asarray(a, np.float64)[:, None, None, None] for a in norm)
    nlat = len(f_list)
    applied, decisions = [], []
    for _ in range(steps):
        X = np.concatenate([oracle.moments(op, f)[0].reshape(8, -1, op.ny, op.nx)
                            for op, f in zip(op_list, f_list)], axis=1)  # [8, nz, ny, nx]
        xs = (X - in_mean) / in_std
        y = np.swapaxes(net_o.forward(np.swapaxes(xs, 0, 1)), 0, 1) if dim == 2 else net_o.forward(xs[None])[0]
        dQ = C.project(out_mean + out_std * y, nlat)
        ok = C.gate(X, dQ, bounds[0], bounds[1], bounds[2], dim=dim)
        per = dQ.shape[1] // nlat
        for j, (op, f) in enumerate(zip(op_list, f_list)):
            oracle.run(op, f, 1)
            if ok:
                NQ = oracle.ndirs(op)
                wts = np.array([op.w0] + [(1.0 - op.w0) / (NQ - 1)] * (NQ - 1))
                f += wts[None, :, None] * dQ[:, j * per:(j + 1) * per].reshape(8, 1, -1)
        applied.append(dQ if ok else np.zeros_like(dQ))
        decisions.append(ok)
    return applied, decisions


@pytest.mark.parametrize("dim", [2, 3])
def test_random_network_corrected_steps_match_oracle(env, dim):
    """A random 4-layer network drives vlbm_step_corrected (FP64 populations, so the
    network is the only low-precision part): one accepted step, two more accepted steps
    in one call, then one step whose correction norm exceeds its bound.  Against the
    oracle's composition (moments -> standardised BF16 input -> quantised Net ->
    de-standardisation -> projection -> gate -> plain step -> injection): the first
    applied correction agrees per channel to the network's BF16 precision (rel-L2 <=
    1e-2, as the forward pass) and has zero lattice totals up to its FP32 rounding; the
    state after three steps agrees to the FP32 bar, 1e-5 of its size (the corrections
    are below 7e-4 of it, their BF16 error below 1e-2 of that), and its departure
    from the plain run to 1e-2; the rejected step is bitwise the plain VLBM step."""
    from test_gpu_parity import oracle_params
    torch, vlbm, nn = env
    rng = np.random.default_rng(70 + dim)
    params = rand_params(rng, 4, dim=dim)
    net = make_net(env, 4, params, dim=dim)
    if dim == 2:
        n, B = 32, 2
        w = synth.workload_fourier_2d(n=n)
        Qs = [synth.fourier_2d(n, seed=60 + j) for j in range(B)]
        shape, lat_shape = (n, n, B), (n, n, 1)
    else:
        w = synth.workload_slab_3d()
        Qs = [state3(seed=3)]
        shape = lat_shape = SHAPE3
    Q0 = np.concatenate(Qs, axis=1)
    nlat = len(Qs)

    def oracle_lattices():
        ops = [oracle_params(w, shape=lat_shape) for _ in Qs]
        return ops, [oracle.init(op, Q) for op, Q in zip(ops, Qs)]

    def oracle_Q(ops, fs):
        return np.concatenate([oracle.moments(op, f)[0].reshape(8, -1, op.ny, op.nx) for op, f in zip(ops, fs)],
                              axis=1)

    in_mean = Q0.reshape(8, -1).mean(axis=1)
    in_std = Q0.reshape(8, -1).std(axis=1) + 1e-3
    norm = (in_mean, in_std, np.zeros(8), np.full(8, 5e-5))
    net.vlbm_nn_set_norm(*norm)
    net_o = C.Net(params, layers=4, quantize=True, dim=dim)

    def fresh():
        sim = vlbm.Vlbm(gpu_params(vlbm, w, "f64", shape=shape))
        sim.vlbm_init_fields(Q0)
        return sim

    a, plain = fresh(), fresh()
    ops, fs = oracle_lattices()
    opl, fpl = oracle_lattices()
    big = np.full(8, 1e30)
    # one step: the applied correction itself
    applied, ok = _oracle_corrected(ops, fs, net_o, 1, (big, 10.0, 1.0), norm, dim)
    assert ok == [True]
    assert nn.vlbm_step_corrected(a, net, 1, big, 10.0, 1.0) == 0
    plain.vlbm_step(1)
    for op, f in zip(opl, fpl):
        oracle.run(op, f, 1)
    Qa, Qp = a.vlbm_moments()[0].reshape(Q0.shape), plain.vlbm_moments()[0].reshape(Q0.shape)
    assert np.abs(Qp - oracle_Q(opl, fpl)).max() <= 1e-10 * np.abs(Q0).max()
    dq = Qa - Qp
    for k in range(8):
        assert rel_l2(dq[k], applied[0][k]) <= 1e-2, k
    per = dq.reshape(8, nlat, -1)
    assert np.abs(per.sum(axis=2)).max() <= 1e-6 * np.abs(per).sum(axis=2).max()
    # two more accepted steps in one call
    _, ok = _oracle_corrected(ops, fs, net_o, 2, (big, 10.0, 1.0), norm, dim)
    assert ok == [True, True]
    assert nn.vlbm_step_corrected(a, net, 2, big, 10.0, 1.0) == 0
    plain.vlbm_step(2)
    for op, f in zip(opl, fpl):
        oracle.run(op, f, 2)
    Qa, Qp = a.vlbm_moments()[0].reshape(Q0.shape), plain.vlbm_moments()[0].reshape(Q0.shape)
    Qo, Qpo = oracle_Q(ops, fs), oracle_Q(opl, fpl)
    assert np.abs(Qa - Qo).max() <= 1e-5 * np.abs(Qo).max()
    for k in range(8):
        assert rel_l2((Qa - Qp)[k], (Qo - Qpo)[k]) <= 1e-2, k
    # a step whose correction is over its bound in E: the oracle's gate rejects it,
    # and the GPU takes the plain step
    probe = [f.copy() for f in fs]
    nxt, _ = _oracle_corrected(ops, probe, net_o, 1, (big, 10.0, 1.0), norm, dim)
    bound = big.copy()
    bound[4] = 0.5 * np.linalg.norm(nxt[0][4])
    _, ok = _oracle_corrected(ops, fs, net_o, 1, (bound, 10.0, 1.0), norm, dim)
    assert ok == [False]
    buf, par, step = a.vlbm_get_populations()
    b = fresh()
    b.vlbm_set_populations(buf, par, step)
    assert nn.vlbm_step_corrected(a, net, 1, bound, 10.0, 1.0) == 1
    b.vlbm_step(1)
    assert np.array_equal(a.vlbm_get_populations()[0], b.vlbm_get_populations()[0])
