"""Pins of the learned-correction oracle (oracle/conv_ref.py), CPU only.

Library routines stand in as independent references: scipy's periodic correlation
and torch's conv2d / conv3d with circular padding for the 3x3 and 3x3x3
convolutions, torch's exact GELU,
torch's bfloat16 rounding and torch's Adam; the gradients are checked by central
finite differences in FP64.  Planted mistakes in a copy of the module source must
make one of the checks fail."""
import importlib.util
import os
import types

import numpy as np
import pytest
import scipy.ndimage as ndi
import torch

import oracle.conv_ref as C

HERE = os.path.dirname(os.path.abspath(__file__))


def rand_params(rng, cin, width, layers, scale=0.3):
    return [(rng.normal(0, scale, Ws), rng.normal(0, 0.1, bs)) for Ws, bs in C.Net.shapes(cin, width, layers)]


def chk_conv_vs_scipy(mod=C):
    rng = np.random.default_rng(0)
    a = rng.normal(size=(2, 3, 7, 6))
    W = rng.normal(size=(4, 3, 3, 3))
    b = rng.normal(size=4)
    z = mod.conv3x3(a, W, b)
    ref = np.zeros_like(z)
    for bb in range(2):
        for o in range(4):
            ref[bb, o] = b[o] + sum(ndi.correlate(a[bb, c], W[o, c], mode="wrap") for c in range(3))
    return np.abs(z - ref).max()


def chk_conv_vs_torch(mod=C):
    rng = np.random.default_rng(1)
    a = rng.normal(size=(2, 5, 8, 9))
    W = rng.normal(size=(3, 5, 3, 3))
    b = rng.normal(size=3)
    z = mod.conv3x3(a, W, b)
    t = torch.nn.functional.pad(torch.tensor(a), (1, 1, 1, 1), mode="circular")
    ref = torch.nn.functional.conv2d(t, torch.tensor(W), torch.tensor(b)).numpy()
    return np.abs(z - ref).max()


def chk_gradients_fd(mod=C):
    """Central finite differences of the MSE loss w.r.t. every parameter of a small
    3-layer net, FP64; returns the worst relative error."""
    rng = np.random.default_rng(2)
    params = rand_params(rng, 3, 4, 3)
    x = rng.normal(size=(2, 3, 5, 6))
    t = rng.normal(size=(2, 3, 5, 6))
    net = mod.Net(params, cin=3, width=4, layers=3)
    _, grads = net.loss_and_grads(x, t)
    worst = 0.0
    h = 1e-5
    gscale = max(np.abs(g).max() for pair in grads for g in pair)
    for l in range(3):
        for j in range(2):
            p = params[l][j]
            g = grads[l][j]
            for idx in [tuple(rng.integers(0, s) for s in p.shape) for _ in range(6)]:
                old = p[idx]
                p[idx] = old + h
                lp, _ = mod.Net(params, cin=3, width=4, layers=3).loss_and_grads(x, t)
                p[idx] = old - h
                lm, _ = mod.Net(params, cin=3, width=4, layers=3).loss_and_grads(x, t)
                p[idx] = old
                fd = (lp - lm) / (2 * h)
                worst = max(worst, abs(fd - g[idx]) / max(abs(fd), 1e-3 * gscale))
    return worst


def chk_conv3_vs_scipy(mod=C):
    rng = np.random.default_rng(10)
    a = rng.normal(size=(2, 3, 5, 4, 6))
    W = rng.normal(size=(2, 3, 3, 3, 3))
    b = rng.normal(size=2)
    z = mod.conv3x3x3(a, W, b)
    ref = np.zeros_like(z)
    for bb in range(2):
        for o in range(2):
            ref[bb, o] = b[o] + sum(ndi.correlate(a[bb, c], W[o, c], mode="wrap") for c in range(3))
    return np.abs(z - ref).max()


def chk_conv3_vs_torch(mod=C):
    rng = np.random.default_rng(11)
    a = rng.normal(size=(2, 4, 3, 5, 7))
    W = rng.normal(size=(3, 4, 3, 3, 3))
    b = rng.normal(size=3)
    z = mod.conv3x3x3(a, W, b)
    t = torch.nn.functional.pad(torch.tensor(a), (1, 1, 1, 1, 1, 1), mode="circular")
    ref = torch.nn.functional.conv3d(t, torch.tensor(W), torch.tensor(b)).numpy()
    return np.abs(z - ref).max()


def chk_gradients3_fd(mod=C):
    """Central finite differences of the MSE loss of a small 2-layer 3D net."""
    rng = np.random.default_rng(12)
    params = [(rng.normal(0, 0.3, Ws), rng.normal(0, 0.1, bs)) for Ws, bs in C.Net.shapes(2, 3, 2, dim=3)]
    x = rng.normal(size=(1, 2, 3, 4, 5))
    t = rng.normal(size=(1, 2, 3, 4, 5))
    _, grads = mod.Net(params, cin=2, width=3, layers=2, dim=3).loss_and_grads(x, t)
    worst = 0.0
    h = 1e-5
    gscale = max(np.abs(g).max() for pair in grads for g in pair)
    for l in range(2):
        for j in range(2):
            p = params[l][j]
            g = grads[l][j]
            for idx in [tuple(rng.integers(0, s) for s in p.shape) for _ in range(8)]:
                old = p[idx]
                p[idx] = old + h
                lp, _ = mod.Net(params, cin=2, width=3, layers=2, dim=3).loss_and_grads(x, t)
                p[idx] = old - h
                lm, _ = mod.Net(params, cin=2, width=3, layers=2, dim=3).loss_and_grads(x, t)
                p[idx] = old
                fd = (lp - lm) / (2 * h)
                worst = max(worst, abs(fd - g[idx]) / max(abs(fd), 1e-3 * gscale))
    return worst


def chk_gelu_vs_torch(mod=C):
    z = np.linspace(-6, 6, 241)
    ref = torch.nn.functional.gelu(torch.tensor(z)).numpy()  # exact (erf) GELU
    zt = torch.tensor(z, requires_grad=True)
    torch.nn.functional.gelu(zt).sum().backward()
    return max(np.abs(mod.gelu(z) - ref).max(), np.abs(mod.gelu_grad(z) - zt.grad.numpy()).max())


def chk_adam_vs_torch(mod=C):
    rng = np.random.default_rng(3)
    params = rand_params(rng, 2, 3, 2)
    tparams = [torch.tensor(p.copy(), requires_grad=True) for pair in params for p in pair]
    opt = torch.optim.Adam(tparams, lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    adam = mod.Adam(params, lr=1e-2)
    cur = params
    for _ in range(5):
        grads = [(rng.normal(size=W.shape), rng.normal(size=b.shape)) for W, b in cur]
        for tp, g in zip(tparams, [g for pair in grads for g in pair]):
            tp.grad = torch.tensor(g)
        opt.step()
        cur = adam.step(cur, grads)
    mine = [p for pair in cur for p in pair]
    return max(np.abs(m - t.detach().numpy()).max() for m, t in zip(mine, tparams))


def test_conv_matches_scipy_periodic_correlation():
    assert chk_conv_vs_scipy() < 1e-12


def test_conv_matches_torch_circular_conv2d():
    assert chk_conv_vs_torch() < 1e-12


def test_identity_kernel():
    rng = np.random.default_rng(4)
    a = rng.normal(size=(1, 4, 6, 5))
    W = np.zeros((4, 4, 3, 3))
    for c in range(4):
        W[c, c, 1, 1] = 1.0
    assert np.array_equal(C.conv3x3(a, W, np.zeros(4)), a)


def test_conv3_matches_scipy_periodic_correlation():
    assert chk_conv3_vs_scipy() < 1e-12


def test_conv3_matches_torch_circular_conv3d():
    assert chk_conv3_vs_torch() < 1e-12


def test_conv3_identity_kernel_and_planar_kernel():
    """The centre tap as identity reproduces the input; a kernel confined to the
    kz = 1 plane acts as the 2D convolution on every z-slice."""
    rng = np.random.default_rng(13)
    a = rng.normal(size=(2, 3, 4, 5, 6))
    W = np.zeros((3, 3, 3, 3, 3))
    for c in range(3):
        W[c, c, 1, 1, 1] = 1.0
    assert np.array_equal(C.conv3x3x3(a, W, np.zeros(3)), a)
    W2 = rng.normal(size=(2, 3, 3, 3))
    b = rng.normal(size=2)
    W3 = np.zeros((2, 3, 3, 3, 3))
    W3[:, :, 1] = W2
    z3 = C.conv3x3x3(a, W3, b)
    for zz in range(4):
        assert np.abs(z3[:, :, zz] - C.conv3x3(a[:, :, zz], W2, b)).max() < 1e-12


def test_conv3_translation_equivariance():
    rng = np.random.default_rng(14)
    a = rng.normal(size=(1, 2, 4, 5, 3))
    W = rng.normal(size=(2, 2, 3, 3, 3))
    b = rng.normal(size=2)
    z = C.conv3x3x3(a, W, b)
    zs = C.conv3x3x3(np.roll(a, (1, 2, -1), axis=(2, 3, 4)), W, b)
    assert np.abs(zs - np.roll(z, (1, 2, -1), axis=(2, 3, 4))).max() < 1e-12


def test_gradients3_finite_differences():
    assert chk_gradients3_fd() < 1e-7


def test_gradients_finite_differences():
    assert chk_gradients_fd() < 1e-7


def test_gelu_matches_torch():
    assert chk_gelu_vs_torch() < 1e-12


def test_adam_matches_torch():
    assert chk_adam_vs_torch() < 1e-12


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(5)
    a = np.concatenate([rng.normal(size=1000) * 10.0 ** rng.integers(-5, 5, 1000), [0.0, -0.0, 1.0]])
    ref = torch.tensor(a, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(C.bf16_round(a), ref)


def test_restriction_conserves_totals_and_constants():
    rng = np.random.default_rng(6)
    Q = rng.normal(size=(8, 1, 16, 12))
    R = C.restrict(Q, 4)
    assert R.shape == (8, 1, 4, 3)
    assert np.allclose(R.sum(axis=(1, 2, 3)) * 16, Q.sum(axis=(1, 2, 3)), rtol=1e-13)
    assert np.allclose(R[:, 0, 1, 2], Q[:, 0, 4:8, 8:12].mean(axis=(1, 2)))
    Q3 = rng.normal(size=(8, 4, 4, 4))
    assert np.allclose(C.restrict(Q3, 2).sum() * 8, Q3.sum())


def test_gate_cases():
    rng = np.random.default_rng(7)
    Q = rng.normal(size=(8, 1, 8, 8))
    dQ = 1e-3 * rng.normal(size=Q.shape)
    big = np.full(8, 1e9)
    assert C.gate(Q, np.zeros_like(Q), big, 0.1)
    assert not C.gate(Q, dQ, np.zeros(8), 0.1)  # bound 0 always falls back
    bad = dQ.copy()
    bad[0, 0, 1, 1] = np.nan
    assert not C.gate(Q, bad, big, 0.1)
    # a correction that only adds divergence is rejected, unless the absolute
    # allowance (a fraction of ||B||) covers it
    div_only = np.zeros_like(Q)
    div_only[5] = 10.0 * np.sin(2 * np.pi * np.arange(8) / 8)[None, None, :]
    assert not C.gate(Q, div_only, big, 0.1)
    assert C.gate(Q, div_only, big, 0.1, bound_divb_abs=100.0)
    assert not C.gate(Q, div_only, big, 0.1, bound_divb_abs=0.01)


def chk_positivity(mod=C):
    """The gate's positivity condition against pressures worked out by hand: rho = 1,
    rho u = (1, 0, 0), B = (0, 1, 0), p = 0.6, gamma = 5/3, so E = 0.9 + 0.5 + 0.5 =
    1.9; lowering E by 1 leaves p = (2/3)(0.9 - 1) < 0 (rejected), by 0.8 leaves
    p = (2/3)(0.1) > 0 (accepted) -- either without the kinetic or without the magnetic
    energy the first would pass; a correction to rho = -0.1 in one cell is rejected;
    without gamma the condition is off.  Returns the number of wrong decisions."""
    Q = np.zeros((8, 1, 4, 4))
    Q[0], Q[1], Q[6], Q[4] = 1.0, 1.0, 1.0, 1.9
    big = np.full(8, 1e9)
    wrong = 0
    for dE, want in ((-1.0, False), (-0.8, True)):
        dQ = np.zeros_like(Q)
        dQ[4, 0, 2, 1] = dE
        wrong += mod.gate(Q, dQ, big, 10.0, 1.0, gamma=5.0 / 3.0) != want
        wrong += mod.gate(Q, dQ, big, 10.0, 1.0) is not True
    dQ = np.zeros_like(Q)
    dQ[0, 0, 1, 3] = -1.1
    wrong += mod.gate(Q, dQ, big, 10.0, 1.0, gamma=5.0 / 3.0) is not False
    return int(wrong)


def test_gate_positivity():
    assert chk_positivity() == 0


def chk_projection(mod=C):
    """The projection onto zero lattice totals, pinned by what defines it rather than
    by its formula: P d has zero total in every channel of every lattice, and d - P d
    is constant over each lattice in each channel (it lies in the orthogonal
    complement of the zero-total fields), which fixes P d uniquely; P is idempotent
    and self-adjoint.  Returns the largest violation, relative to the field's size."""
    rng = np.random.default_rng(17)
    worst = 0.0
    for shape, nlat in (((8, 3, 16, 16), 3), ((8, 4, 8, 16), 1), ((8, 4, 8, 8), 2)):
        d = rng.normal(size=shape) + rng.normal(size=(8, 1, 1, 1))  # nonzero means
        e = rng.normal(size=shape)
        Pd, Pe = mod.project(d, nlat), mod.project(e, nlat)
        per = lambda a: a.reshape(8, nlat, -1)
        scale = np.abs(d).max()
        worst = max(worst,
                    np.abs(per(Pd).sum(axis=2)).max() / (scale * per(Pd).shape[2]),
                    np.ptp(per(d - Pd), axis=2).max() / scale,
                    np.abs(mod.project(Pd, nlat) - Pd).max() / scale,
                    abs((Pd * e).sum() - (d * Pe).sum()) / (np.abs(d).sum() * np.abs(e).max()))
    return worst


def test_projection_onto_zero_lattice_totals():
    assert chk_projection() < 1e-13
    # a uniform correction vanishes; a zero-total one is kept
    u = np.ones((8, 2, 4, 4)) * np.arange(8)[:, None, None, None]
    assert np.abs(C.project(u, 2)).max() < 1e-15
    z = np.zeros((8, 2, 4, 4))
    z[:, :, 0, 0], z[:, :, 1, 1] = 1.0, -1.0
    assert np.array_equal(C.project(z, 2), z)


MUTATIONS = {
    "project_whole_batch": ("per = dQ.reshape(K, nlat, -1)", "per = dQ.reshape(K, 1, -1)"),
    "project_all_channels": ("mean = per.sum(axis=2, keepdims=True) / per.shape[2]",
                             "mean = per.sum(axis=(0, 2), keepdims=True) / (K * per.shape[2])"),
    "project_mean_of_a_slice": ("mean = per.sum(axis=2, keepdims=True) / per.shape[2]",
                                "mean = per.sum(axis=2, keepdims=True) / dQ.shape[-1]"),
    "conv_shift_sign": ("shifted = np.roll(a, shift=(-(ky - 1), -(kx - 1)), axis=(2, 3))  # a[y+ky-1, x+kx-1]",
                        "shifted = np.roll(a, shift=((ky - 1), (kx - 1)), axis=(2, 3))  # a[y+ky-1, x+kx-1]"),
    "backward_scatter_sign": ("da += np.roll(back, shift=(ky - 1, kx - 1), axis=(2, 3))",
                              "da += np.roll(back, shift=(-(ky - 1), -(kx - 1)), axis=(2, 3))"),
    "conv3_shift_sign": ("shifted = np.roll(a, shift=(-(kz - 1), -(ky - 1), -(kx - 1)), axis=(2, 3, 4))",
                         "shifted = np.roll(a, shift=(-(kz - 1), (ky - 1), -(kx - 1)), axis=(2, 3, 4))"),
    "conv3_axes_swapped": ("z += np.einsum(\"oc,bczyx->bozyx\", W[:, :, kz, ky, kx], shifted)",
                           "z += np.einsum(\"oc,bczyx->bozyx\", W[:, :, kx, ky, kz], shifted)"),
    "backward3_scatter_sign": ("da += np.roll(back, shift=off, axis=(2, 3, 4))",
                               "da += np.roll(back, shift=tuple(-o for o in off), axis=(2, 3, 4))"),
    "backward3_weight_transposed": ("back = np.einsum(\"oc,bozyx->bczyx\", W[:, :, kz, ky, kx], dz)",
                                    "back = np.einsum(\"oc,bozyx->bczyx\", W[:, :, 2 - kz, ky, kx], dz)"),
    "gelu_grad_pdf_dropped": ("return cdf + z * pdf", "return cdf"),
    "loss_scale": ("dz = 2.0 * (y - t) / n", "dz = 1.0 * (y - t) / n"),
    "adam_bias_correction": ("new.append(p - self.lr * (m / c1) / (np.sqrt(v / c2) + self.eps))",
                             "new.append(p - self.lr * m / (np.sqrt(v) + self.eps))"),
    "positivity_kinetic_dropped": ("return bool(np.all((gamma - 1.0) * (Q[4] - kinetic - magnetic) >= 0))",
                                   "return bool(np.all((gamma - 1.0) * (Q[4] - magnetic) >= 0))"),
    "positivity_magnetic_dropped": ("return bool(np.all((gamma - 1.0) * (Q[4] - kinetic - magnetic) >= 0))",
                                    "return bool(np.all((gamma - 1.0) * (Q[4] - kinetic) >= 0))"),
    "positivity_rho_ignored": ("    if not np.all(rho > 0):\n        return False\n", ""),
}


def _load_variant(src):
    mod = types.ModuleType("conv_ref_variant")
    exec(compile(src, "conv_ref_variant", "exec"), mod.__dict__)
    return mod


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_conv_pins_catch_planted_mistake(name):
    old, new = MUTATIONS[name]
    src = open(C.__file__).read()
    assert src.count(old) == 1, name
    mod = _load_variant(src.replace(old, new))
    failed = (chk_conv_vs_scipy(mod) > 1e-12 or chk_conv_vs_torch(mod) > 1e-12
              or chk_conv3_vs_scipy(mod) > 1e-12 or chk_conv3_vs_torch(mod) > 1e-12
              or chk_gradients_fd(mod) > 1e-7 or chk_gradients3_fd(mod) > 1e-7
              or chk_gelu_vs_torch(mod) > 1e-12 or chk_adam_vs_torch(mod) > 1e-12
              or chk_projection(mod) > 1e-13 or chk_positivity(mod) > 0)
    assert failed, name
