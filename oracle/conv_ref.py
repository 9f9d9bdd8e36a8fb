"""FP64 CPU oracle of the learned coarse-grid correction -- TEST INFRASTRUCTURE ONLY
(loaded by tests/, the smoke check and the CPU-baseline leg of the benchmark).

The correction network is an extension of the method (it is not in the paper): a
stack of 3x3 (2D lattices) or 3x3x3 (3D lattices) convolutions with periodic
padding on the coarse moment field, GELU between layers, trained by mean-squared
error with Adam.  Everything here is written as plain shifted sums over the 9 or 27
taps -- no blocking or fusion -- so it can be checked by eye:

* conv:   z[b,o,y,x] = bias[o] + sum_{c,ky,kx} W[o,c,ky,kx] a[b,c,(y+ky-1)%H,(x+kx-1)%W]
* conv3:  z[b,o,z,y,x] = bias[o] + sum_{c,kz,ky,kx} W[o,c,kz,ky,kx] a[b,c,z+kz-1,y+ky-1,x+kx-1]
          (every index periodic)
* GELU:   g(z) = z Phi(z) (Phi the standard normal CDF), g'(z) = Phi(z) + z phi(z)
* loss:   L = mean((y - t)^2)
* Adam:   m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
          p -= lr (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps)
* restriction R: r x r block mean of a moment field (conserves totals)
* projection P: from every channel of every lattice of a batch its mean over that
  lattice is removed -- the orthogonal projection onto corrections with zero lattice
  totals (the totals that the fine run, its restriction and the coarse VLBM all keep,
  up to the Powell source)
* gate: the correction is dropped when a per-variable L2 norm exceeds its bound, when
  it raises the central-difference div B norm of the state by more than a relative
  amount plus an absolute amount (a fraction of the field's own L2 norm), when it
  is not finite, or (optionally, gamma given) when it leaves a cell with rho <= 0 or
  a negative pressure.
"""
from __future__ import annotations

import math

import numpy as np

SQRT2 = math.sqrt(2.0)


def _erf(x):
    return np.vectorize(math.erf, otypes=[np.float64])(x)


def gelu(z):
    return z * 0.5 * (1.0 + _erf(z / SQRT2))


def gelu_grad(z):
    cdf = 0.5 * (1.0 + _erf(z / SQRT2))
    pdf = np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)
    return cdf + z * pdf


def bf16_round(a):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    a32 = np.asarray(a, np.float32)
    u = a32.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def conv3x3(a, W, bias):
    """Periodic 3x3 convolution (cross-correlation).  a [B,C,H,W], W [O,C,3,3]."""
    B, C, H, Wd = a.shape
    O = W.shape[0]
    z = np.zeros((B, O, H, Wd))
    for ky in range(3):
        for kx in range(3):
            shifted = np.roll(a, shift=(-(ky - 1), -(kx - 1)), axis=(2, 3))  # a[y+ky-1, x+kx-1]
            z += np.einsum("oc,bcyx->boyx", W[:, :, ky, kx], shifted)
    return z + bias[None, :, None, None]


def conv3x3_backward(a, W, dz):
    """Gradients of conv3x3: returns (da, dW, dbias)."""
    dW = np.zeros_like(W)
    da = np.zeros_like(a)
    for ky in range(3):
        for kx in range(3):
            shifted = np.roll(a, shift=(-(ky - 1), -(kx - 1)), axis=(2, 3))
            dW[:, :, ky, kx] = np.einsum("boyx,bcyx->oc", dz, shifted)
            # z[y] depends on a[y+ky-1]: scatter dz back by the opposite shift
            back = np.einsum("oc,boyx->bcyx", W[:, :, ky, kx], dz)
            da += np.roll(back, shift=(ky - 1, kx - 1), axis=(2, 3))
    return da, dW, dz.sum(axis=(0, 2, 3))


def conv3x3x3(a, W, bias):
    """Periodic 3x3x3 convolution (cross-correlation).  a [B,C,D,H,W], W [O,C,3,3,3]."""
    B, C, D, H, Wd = a.shape
    O = W.shape[0]
    z = np.zeros((B, O, D, H, Wd))
    for kz in range(3):
        for ky in range(3):
            for kx in range(3):
                # a[z+kz-1, y+ky-1, x+kx-1]
                shifted = np.roll(a, shift=(-(kz - 1), -(ky - 1), -(kx - 1)), axis=(2, 3, 4))
                z += np.einsum("oc,bczyx->bozyx", W[:, :, kz, ky, kx], shifted)
    return z + bias[None, :, None, None, None]


def conv3x3x3_backward(a, W, dz):
    """Gradients of conv3x3x3: returns (da, dW, dbias)."""
    dW = np.zeros_like(W)
    da = np.zeros_like(a)
    for kz in range(3):
        for ky in range(3):
            for kx in range(3):
                off = (kz - 1, ky - 1, kx - 1)
                shifted = np.roll(a, shift=tuple(-o for o in off), axis=(2, 3, 4))
                dW[:, :, kz, ky, kx] = np.einsum("bozyx,bczyx->oc", dz, shifted)
                back = np.einsum("oc,bozyx->bczyx", W[:, :, kz, ky, kx], dz)
                da += np.roll(back, shift=off, axis=(2, 3, 4))  # opposite of the forward shift
    return da, dW, dz.sum(axis=(0, 2, 3, 4))


class Net:
    """Layer widths cin -> width -> ... -> cout, `layers` convolutions; dim = 2
    (3x3 kernels, fields [B,C,H,W]) or dim = 3 (3x3x3 kernels, fields [B,C,D,H,W]).

    quantize=True rounds the weights and every stored activation (network input,
    hidden activations) to bfloat16, as the GPU stores them; products and sums stay
    FP64."""

    def __init__(self, params, cin=8, width=32, layers=4, cout=None, quantize=False, dim=2):
        self.cin, self.width, self.layers = cin, width, layers
        self.cout = cin if cout is None else cout
        self.quantize = quantize
        self.dim = dim
        self.conv, self.conv_backward = (conv3x3, conv3x3_backward) if dim == 2 else (conv3x3x3, conv3x3x3_backward)
        self.params = [(np.asarray(W, np.float64), np.asarray(b, np.float64)) for W, b in params]

    @staticmethod
    def shapes(cin=8, width=32, layers=4, cout=None, dim=2):
        cout = cin if cout is None else cout
        dims = [cin] + [width] * (layers - 1) + [cout]
        return [((dims[l + 1], dims[l]) + (3,) * dim, (dims[l + 1],)) for l in range(layers)]

    def _q(self, a):
        return bf16_round(a) if self.quantize else a

    def forward(self, x, keep=False):
        a = self._q(x)
        cache = []
        for l, (W, b) in enumerate(self.params):
            z = self.conv(a, self._q(W), b)
            cache.append((a, z))
            if l < len(self.params) - 1:
                a = self._q(gelu(z))
            else:
                a = z
        return (a, cache) if keep else a

    def loss_and_grads(self, x, t):
        y, cache = self.forward(x, keep=True)
        n = y.size
        loss = float(np.mean((y - t) ** 2))
        dz = 2.0 * (y - t) / n
        grads = [None] * len(self.params)
        for l in range(len(self.params) - 1, -1, -1):
            a, z = cache[l]
            W, _ = self.params[l]
            da, dW, db = self.conv_backward(a, self._q(W), dz)
            grads[l] = (dW, db)
            if l > 0:
                _, zprev = cache[l - 1]
                dz = da * gelu_grad(zprev)
        return loss, grads


class Adam:
    def __init__(self, params, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps
        self.t = 0
        self.m = [[np.zeros_like(W), np.zeros_like(b)] for W, b in params]
        self.v = [[np.zeros_like(W), np.zeros_like(b)] for W, b in params]

    def step(self, params, grads):
        self.t += 1
        c1 = 1.0 - self.b1 ** self.t
        c2 = 1.0 - self.b2 ** self.t
        out = []
        for l, ((W, b), (gW, gb)) in enumerate(zip(params, grads)):
            new = []
            for j, (p, g) in enumerate(((W, gW), (b, gb))):
                m = self.m[l][j] = self.b1 * self.m[l][j] + (1.0 - self.b1) * g
                v = self.v[l][j] = self.b2 * self.v[l][j] + (1.0 - self.b2) * g * g
                new.append(p - self.lr * (m / c1) / (np.sqrt(v / c2) + self.eps))
            out.append(tuple(new))
        return out


def restrict(Q, r):
    """r x r (x r) block mean of a moment field [K, nz, ny, nx] (nz may be 1)."""
    K, nz, ny, nx = Q.shape
    rz = r if nz > 1 else 1
    return Q.reshape(K, nz // rz, rz, ny // r, r, nx // r, r).mean(axis=(2, 4, 6))


def project(dQ, nlat):
    """Projection onto zero lattice totals of a correction dQ [K, nz, ny, nx] whose nz
    slices hold nlat lattices of nz / nlat slices each (a batch of 2D lattices:
    nlat = nz; one 3D lattice: nlat = 1): channel by channel, each lattice loses its
    own mean."""
    K = dQ.shape[0]
    per = dQ.reshape(K, nlat, -1)
    mean = per.sum(axis=2, keepdims=True) / per.shape[2]
    return (per - mean).reshape(dQ.shape)


def b_l2(Q, dim=2):
    """sqrt(sum_x |B_inplane|^2) of a moment field [K, nz, ny, nx]."""
    return float(np.sqrt(sum((Q[5 + a] ** 2).sum() for a in range(dim))))


def central_divb_l2(Q, dim=2):
    """sqrt(sum_x (central div B)^2) of a moment field [K, nz, ny, nx], periodic."""
    div = np.zeros(Q.shape[1:])
    for a in range(dim):
        ax = 2 - a  # component a differentiated along its own axis (x is the last axis)
        div += 0.5 * (np.roll(Q[5 + a], -1, axis=ax) - np.roll(Q[5 + a], 1, axis=ax))
    return float(np.sqrt((div * div).sum()))


def physical(Q, gamma):
    """True if every cell of the ideal-MHD state Q [8, ...] has rho > 0 and
    p = (gamma - 1)(E - |rho u|^2 / (2 rho) - |B|^2 / 2) >= 0."""
    rho = Q[0]
    if not np.all(rho > 0):
        return False
    kinetic = 0.5 * (Q[1] ** 2 + Q[2] ** 2 + Q[3] ** 2) / rho
    magnetic = 0.5 * (Q[5] ** 2 + Q[6] ** 2 + Q[7] ** 2)
    return bool(np.all((gamma - 1.0) * (Q[4] - kinetic - magnetic) >= 0))


def gate(Q, dQ, bound_corr, bound_divb_rel, bound_divb_abs=0.0, dim=2, gamma=None):
    """True if the correction dQ may be applied to state Q: finite, every
    ||dQ_k||_2 <= bound_corr[k], the central div B norm after the correction at
    most (1 + rel) times the one before plus abs times ||B||_2, and (gamma given)
    Q + dQ physical in every cell."""
    if not np.all(np.isfinite(dQ)):
        return False
    K = dQ.shape[0]
    norms = np.sqrt((dQ.reshape(K, -1) ** 2).sum(1))
    if np.any(norms > np.asarray(bound_corr)):
        return False
    before = central_divb_l2(Q, dim)
    after = central_divb_l2(Q + dQ, dim)
    if after > (1.0 + bound_divb_rel) * before + bound_divb_abs * b_l2(Q, dim):
        return False
    return gamma is None or physical(Q + dQ, gamma)
