"""Learned coarse-grid correction for ideal MHD (2D batches and 3D lattices): pair
generation, training and the gain evaluation, driven through the C ABI
(include/vlbm.h, include/vlbm_nn.h).

Every arithmetic step runs in the HIP library: fine and coarse sweeps, moments,
restriction (block mean) and pair targets, network forward/backward/Adam, the gate
and the corrected coarse step.  Python only allocates device buffers (torch),
chooses indices and measures time.  The per-channel normalisation statistics are
computed once on the host from a sample of the training pairs.

Pairs (one coarse step = r fine steps, same flux scale and relaxation time):
  X_n = R(Q_fine(t_n)),  Y_n = R(Q_fine(t_{n+1})) - P(f_n),
where R is the r x r block mean and P one plain coarse VLBM step of a teacher-forced
coarse run: it starts from f^eq(X_0) and after each step takes the true correction,
f_{n+1} = P(f_n) + w_i Y_n, so its moments follow R(Q_fine) while its populations
carry the coarse run's own non-equilibrium part -- the state and the operator the
corrected run applies the network to.
"""
from __future__ import annotations

import time

import numpy as np

from . import nn as N
from . import vlbm as V


def _torch():
    import torch
    return torch


def make_context(shape, batch, storage, workload, stream):
    nx, ny = shape
    return V.Vlbm(V.make_params(lattice="D2Q5", shape=(nx, ny, batch), model="ideal", storage=storage,
                                gamma=workload["gamma"], flux_scale=workload["s"], tau=workload["tau"],
                                powell=workload["powell"], stream=stream))


def initial_batch(seeds, n, kmax, make_state):
    """Stack the seeded initial states [8, 1, n, n] of each seed along z."""
    Q = np.concatenate([make_state(n, seed=s, kmax=kmax) for s in seeds], axis=1)
    return np.ascontiguousarray(Q, dtype=np.float32)


def generate_pairs(seeds, n_fine, r, pairs_per_seed, workload, make_state, kmax=16, storage="f32", stride=1,
                   noise=0.0, seed=0, log=None):
    """Returns (X, Y) device tensors [P, 8, B, nc, nc] (channel-major per pair): every
    `stride`-th pair of a run of pairs_per_seed * stride coarse steps, so that the
    pairs span the horizon the corrected run is used over.  noise > 0: before a
    stored pair's coarse step the teacher-forced state is perturbed by Gaussian noise
    of noise x the initial per-channel spread, and the target still leads to the
    restricted fine state -- the network then also learns to pull a drifted coarse
    state back (the coarse run continues from the true state)."""
    torch = _torch()
    s = torch.cuda.current_stream().cuda_stream
    B, nc = len(seeds), n_fine // r
    fine = make_context((n_fine, n_fine), B, storage, workload, s)
    coarse = make_context((nc, nc), B, storage, workload, s)
    fine.vlbm_init_fields(torch.from_numpy(initial_batch(seeds, n_fine, kmax, make_state)).cuda())
    M = torch.empty((8, B, n_fine, n_fine), dtype=torch.float32, device="cuda")
    Cst = torch.empty((8, B, nc, nc), dtype=torch.float32, device="cuda")
    X = torch.empty((pairs_per_seed, 8, B, nc, nc), dtype=torch.float32, device="cuda")
    Y = torch.empty_like(X)
    cur = torch.empty((8, B, nc, nc), dtype=torch.float32, device="cuda")
    nxt = torch.empty_like(cur)
    tgt = torch.empty_like(cur)
    fine.vlbm_moments(out=M)
    N.vlbm_restrict(M, r, cur, rz=1, stream=s)
    coarse.vlbm_init_fields(cur)
    spread = cur.std(dim=(1, 2, 3), keepdim=True)  # per channel, of the initial state
    gen = torch.Generator(device="cuda").manual_seed(seed)
    eps = torch.empty_like(cur)
    t0 = time.perf_counter()
    for n in range(pairs_per_seed * stride):
        stored = n % stride == 0
        if noise > 0.0 and stored:
            torch.randn(eps.shape, generator=gen, device="cuda", out=eps)
            eps.mul_(spread * noise)
            N.vlbm_inject(coarse, eps)  # the coarse moments become cur + eps
            cur.add_(eps)
        coarse.vlbm_step(1)
        coarse.vlbm_moments(out=Cst)
        fine.vlbm_step(r)
        fine.vlbm_moments(out=M)
        N.vlbm_restrict(M, r, nxt, rz=1, stream=s)
        N.vlbm_restrict(M, r, tgt, rz=1, minus=Cst, stream=s)
        N.vlbm_inject(coarse, tgt)  # teacher forcing: the coarse moments become nxt
        if stored:
            X[n // stride].copy_(cur)
            Y[n // stride].copy_(tgt)
        cur, nxt = nxt, cur
        if log and (n + 1) % (100 * stride) == 0:
            log(f"pairs: {(n + 1) // stride}/{pairs_per_seed} ({n + 1} coarse steps) x {B} seeds, "
                f"{time.perf_counter() - t0:.1f} s")
    torch.cuda.synchronize()
    fine.vlbm_destroy()
    coarse.vlbm_destroy()
    return X, Y


def _divc_l2(F, dim=2):
    """L2 norm of the central-difference divergence of B of a moment batch
    F [8, B, (nz,) ny, nx] (host statistics): the in-plane field in 2D, all three
    components in 3D."""
    d = 0.0
    for a in range(dim):
        ax = -1 - a  # component a along its own axis (x is the last axis)
        d = d + 0.5 * (np.roll(F[5 + a], -1, axis=ax) - np.roll(F[5 + a], 1, axis=ax))
    return float(np.sqrt((d * d).sum()))


def normalisation(X, Y, sample=64, seed=0):
    """Per-channel mean and standard deviation of inputs and targets (host, from up
    to `sample` pairs), the per-lattice RMS L2 norm of each target channel, and the
    RMS div B drift of the true corrections, ||div(B + dB)|| - ||div B||, relative to
    ||B|| (the scale of the gate's absolute div B allowance)."""
    rng = np.random.default_rng(seed)
    P = X.shape[0]
    dim = X.dim() - 3  # X: [P, 8, B, (nz,) ny, nx]
    space = tuple(range(3, 3 + dim))
    idx = np.sort(rng.choice(P, size=min(sample, P), replace=False))
    xs = X[idx].cpu().numpy().astype(np.float64)  # [S, 8, B, (nz,) ny, nx]
    ys = Y[idx].cpu().numpy().astype(np.float64)
    in_mean = xs.mean(axis=(0, 2) + space)
    in_std = xs.std(axis=(0, 2) + space)
    out_mean = np.zeros(8)
    out_std = ys.std(axis=(0, 2) + space)
    in_std = np.where(in_std > 1e-12, in_std, 1.0)
    out_std = np.where(out_std > 1e-20, out_std, 1.0)
    y_l2 = np.sqrt((ys ** 2).sum(axis=space).mean(axis=(0, 2)))  # per channel, one lattice
    drift = []
    for j in range(xs.shape[0]):
        bnorm = np.sqrt(sum((xs[j, 5 + a] ** 2).sum() for a in range(dim)))
        drift.append((_divc_l2(xs[j] + ys[j], dim) - _divc_l2(xs[j], dim)) / max(bnorm, 1e-300))
    drift_rms = float(np.sqrt(np.mean(np.square(drift))))
    return in_mean, in_std, out_mean, out_std, y_l2, drift_rms


def init_weights(layers=4, cin=8, width=32, seed=0, last_scale=0.1, dim=2):
    """He-normal weights, zero biases; the last layer scaled down so training starts
    near the plain coarse VLBM.  dim = 3 gives 3x3x3 kernels."""
    rng = np.random.default_rng(seed)
    dims = [cin] + [width] * (layers - 1) + [cin]
    w = []
    for l in range(layers):
        W = rng.normal(0.0, np.sqrt(2.0 / (3 ** dim * dims[l])), (dims[l + 1], dims[l]) + (3,) * dim)
        if l == layers - 1:
            W *= last_scale
        w += [W.ravel(), np.zeros(dims[l + 1])]
    return np.concatenate(w).astype(np.float32)


def train(net, X, Y, iters, lr, seed=0, log=None, log_every=200):
    """Adam on randomly drawn pairs (each pair is a batch of all its seeds)."""
    rng = np.random.default_rng(seed)
    P = X.shape[0]
    losses = []
    t0 = time.perf_counter()
    for it in range(iters):
        n = int(rng.integers(P))
        want = (it + 1) % log_every == 0 or it == 0
        loss = net.vlbm_nn_train_step(X[n], Y[n], lr, want_loss=want)
        if want:
            losses.append((it + 1, loss))
            if log:
                log(f"train {it + 1}/{iters}: loss {loss:.4e} ({time.perf_counter() - t0:.1f} s)")
    _torch().cuda.synchronize()
    return losses, time.perf_counter() - t0


def field_errors(Q, R):
    """Per-field relative L2 (rho u and B as vectors), Q, R numpy [8, ...]."""
    fam = {"rho": [0], "m": [1, 2, 3], "E": [4], "B": [5, 6, 7]}
    out = {}
    for name, ks in fam.items():
        num = np.sqrt(sum(((Q[k] - R[k]) ** 2).sum() for k in ks))
        den = np.sqrt(sum((R[k] ** 2).sum() for k in ks))
        out[name] = float(num / den)
    return out


def evaluate(net, seeds, n_fine, r, coarse_steps, workload, make_state, bound_corr, bound_divb_rel, bound_divb_abs,
             kmax=16, checkpoints=5, storage="f32", log=None, project=True, fine_storage=None):
    """Coarse plain VLBM vs the corrected coarse run, both scored against the restricted
    fine run (in `fine_storage`, default the coarse runs' storage; "f64" scores both
    against the FP64 fine reference)."""
    torch = _torch()
    s = torch.cuda.current_stream().cuda_stream
    B, nc = len(seeds), n_fine // r
    fine = make_context((n_fine, n_fine), B, fine_storage or storage, workload, s)
    plain = make_context((nc, nc), B, storage, workload, s)
    learned = make_context((nc, nc), B, storage, workload, s)
    fine.vlbm_init_fields(torch.from_numpy(initial_batch(seeds, n_fine, kmax, make_state)).cuda())
    M = torch.empty((8, B, n_fine, n_fine), dtype=torch.float32, device="cuda")
    Rf = torch.empty((8, B, nc, nc), dtype=torch.float32, device="cuda")
    fine.vlbm_moments(out=M)
    N.vlbm_restrict(M, r, Rf, rz=1, stream=s)
    for ctx in (plain, learned):
        ctx.vlbm_init_fields(Rf)
    chunk = coarse_steps // checkpoints
    hist, fallbacks = [], 0
    for c in range(checkpoints):
        fine.vlbm_step(r * chunk)
        plain.vlbm_step(chunk)
        fallbacks += N.vlbm_step_corrected(learned, net, chunk, bound_corr, bound_divb_rel, bound_divb_abs,
                                           project_totals=project)
        fine.vlbm_moments(out=M)
        N.vlbm_restrict(M, r, Rf, rz=1, stream=s)
        ref = Rf.cpu().numpy().astype(np.float64)
        err = {}
        for name, ctx in (("plain", plain), ("learned", learned)):
            q, _ = ctx.vlbm_moments(raise_nonfinite=False)
            err[name] = field_errors(q.reshape(ref.shape), ref)
        hist.append(dict(coarse_step=(c + 1) * chunk, **err))
        if log:
            log(f"eval step {(c + 1) * chunk}: plain {err['plain']} learned {err['learned']} fallbacks {fallbacks}")
    for ctx in (fine, plain, learned):
        ctx.vlbm_destroy()
    return hist, fallbacks


def time_runs(net, n_fine, r, coarse_steps, workload, make_state, bound_corr, bound_divb_rel, bound_divb_abs,
              kmax=16, seed=900, storage="f32", project=True):
    """Wall time of the plain FP32 fine run (r * coarse_steps steps) and of the
    corrected coarse run (coarse_steps steps), one lattice each, inputs resident."""
    torch = _torch()
    s = torch.cuda.current_stream().cuda_stream
    nc = n_fine // r
    fine = make_context((n_fine, n_fine), 1, storage, workload, s)
    learned = make_context((nc, nc), 1, storage, workload, s)
    Q0 = torch.from_numpy(initial_batch([seed], n_fine, kmax, make_state)).cuda()
    fine.vlbm_init_fields(Q0)
    M = torch.empty((8, 1, n_fine, n_fine), dtype=torch.float32, device="cuda")
    Rf = torch.empty((8, 1, nc, nc), dtype=torch.float32, device="cuda")
    fine.vlbm_moments(out=M)
    N.vlbm_restrict(M, r, Rf, rz=1, stream=s)
    learned.vlbm_init_fields(Rf)
    fine.vlbm_step(r * 10)
    N.vlbm_step_corrected(learned, net, 10, bound_corr, bound_divb_rel, bound_divb_abs, project_totals=project)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fine.vlbm_step(r * coarse_steps)
    torch.cuda.synchronize()
    t_fine = time.perf_counter() - t0
    t0 = time.perf_counter()
    nfb = N.vlbm_step_corrected(learned, net, coarse_steps, bound_corr, bound_divb_rel, bound_divb_abs,
                                project_totals=project)
    torch.cuda.synchronize()
    t_learned = time.perf_counter() - t0
    fine.vlbm_destroy()
    learned.vlbm_destroy()
    return t_fine, t_learned, nfb


# flops per output pixel of the 8-32-32-32-8 network with 3x3 kernels
FWD_FLOPS_PER_PIXEL = 2 * 9 * (8 * 32 + 32 * 32 + 32 * 32 + 32 * 8)
# one training step: forward, input gradients of layers 2-4, weight gradients of all
TRAIN_FLOPS_PER_PIXEL = 2 * FWD_FLOPS_PER_PIXEL + 2 * 9 * (32 * 32 + 32 * 32 + 32 * 8)


def time_network(batch=40, n=256, reps=20, seed=0, dim=2, nz=1, ny=None, nx=None):
    """Mean time of the network's forward pass and of one training step (loss,
    gradients, Adam) on a batch of lattices (n x n, or nz x ny x nx for dim = 3), from
    HIP events on the network's stream; returns dict with ms and TFLOP/s (algorithmic
    flops of the 3x3 or 3x3x3 layers)."""
    torch = _torch()
    stream = torch.cuda.current_stream()
    ny = n if ny is None else ny
    nx = n if nx is None else nx
    net = N.Net(8, 32, 4, stream=stream.cuda_stream, dim=dim)
    net.vlbm_nn_set_weights(init_weights(seed=seed, dim=dim))
    net.vlbm_nn_set_norm(np.zeros(8), np.ones(8), np.zeros(8), np.ones(8))
    g = torch.Generator(device="cuda").manual_seed(seed)
    shape = (8, batch, ny, nx) if dim == 2 else (8, batch, nz, ny, nx)
    X = torch.randn(shape, generator=g, device="cuda", dtype=torch.float32)
    T = torch.randn(shape, generator=g, device="cuda", dtype=torch.float32)
    Y = torch.empty_like(X)
    taps = 3 if dim == 3 else 1  # 27 taps = 3 x 9
    npix = batch * (nz if dim == 3 else 1) * ny * nx
    out = {}
    for name, fn, fl in (("forward", lambda: net.vlbm_nn_forward(X, Y), FWD_FLOPS_PER_PIXEL),
                         ("train_step", lambda: net.vlbm_nn_train_step(X, T, 1e-4), TRAIN_FLOPS_PER_PIXEL)):
        fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        out[name] = dict(ms=round(ms, 4), tflops=round(taps * fl * npix / (ms * 1e-3) / 1e12, 2))
    net.vlbm_nn_destroy()
    return out



# --- 3D lattices: one periodic D3Q7 lattice per context -------------------------

def make_context_3d(n, storage, workload, stream):
    return V.Vlbm(V.make_params(lattice="D3Q7", shape=(n, n, n), model="ideal", storage=storage,
                                gamma=workload["gamma"], flux_scale=workload["s"], tau=workload["tau"],
                                powell=workload["powell"], stream=stream))


def _state_3d(make_state, n, seed):
    torch = _torch()
    return torch.from_numpy(np.ascontiguousarray(make_state(n, seed=seed), dtype=np.float32)).cuda()


def generate_pairs_3d(seeds, n_fine, r, pairs_per_seed, workload, make_state, storage="f32", log=None):
    """The pairs of generate_pairs on n^3 lattices, one seed at a time (restriction
    r x r x r): device tensors X, Y [P, 8, 1, nc, nc, nc], P = pairs_per_seed x seeds,
    the pairs of seed j at [j * pairs_per_seed, (j + 1) * pairs_per_seed)."""
    torch = _torch()
    s = torch.cuda.current_stream().cuda_stream
    nc = n_fine // r
    P = pairs_per_seed * len(seeds)
    X = torch.empty((P, 8, 1, nc, nc, nc), dtype=torch.float32, device="cuda")
    Y = torch.empty_like(X)
    M = torch.empty((8, n_fine, n_fine, n_fine), dtype=torch.float32, device="cuda")
    Cst = torch.empty((8, nc, nc, nc), dtype=torch.float32, device="cuda")
    cur = torch.empty_like(Cst)
    nxt = torch.empty_like(Cst)
    tgt = torch.empty_like(Cst)
    t0 = time.perf_counter()
    for j, sd in enumerate(seeds):
        fine = make_context_3d(n_fine, storage, workload, s)
        coarse = make_context_3d(nc, storage, workload, s)
        fine.vlbm_init_fields(_state_3d(make_state, n_fine, sd))
        fine.vlbm_moments(out=M)
        N.vlbm_restrict(M, r, cur, stream=s)
        coarse.vlbm_init_fields(cur)
        for n in range(pairs_per_seed):
            coarse.vlbm_step(1)
            coarse.vlbm_moments(out=Cst)
            fine.vlbm_step(r)
            fine.vlbm_moments(out=M)
            N.vlbm_restrict(M, r, nxt, stream=s)
            N.vlbm_restrict(M, r, tgt, minus=Cst, stream=s)
            N.vlbm_inject(coarse, tgt)  # teacher forcing
            X[j * pairs_per_seed + n, :, 0].copy_(cur)
            Y[j * pairs_per_seed + n, :, 0].copy_(tgt)
            cur, nxt = nxt, cur
        torch.cuda.synchronize()
        fine.vlbm_destroy()
        coarse.vlbm_destroy()
        if log:
            log(f"pairs: seed {sd} done ({(j + 1) * pairs_per_seed}/{P}), {time.perf_counter() - t0:.1f} s")
    return X, Y


def _family_sums(Q, R):
    """Per field family (rho u and B as vectors): (sum (Q - R)^2, sum R^2)."""
    fam = {"rho": [0], "m": [1, 2, 3], "E": [4], "B": [5, 6, 7]}
    return {name: (sum(float(((Q[k] - R[k]) ** 2).sum()) for k in ks), sum(float((R[k] ** 2).sum()) for k in ks))
            for name, ks in fam.items()}


def evaluate_3d(net, seeds, n_fine, r, coarse_steps, workload, make_state, bound_corr, bound_divb_rel,
                bound_divb_abs, checkpoints=5, storage="f32", log=None, project=True, coarse_storage=None):
    """evaluate on 3D lattices: per checkpoint, the per-field relative L2 of the plain
    and of the corrected coarse run (storage form coarse_storage, default storage)
    against the restricted fine run, over all seeds."""
    coarse_storage = coarse_storage or storage
    torch = _torch()
    s = torch.cuda.current_stream().cuda_stream
    nc = n_fine // r
    chunk = coarse_steps // checkpoints
    sums = [{"plain": None, "learned": None} for _ in range(checkpoints)]
    fallbacks = 0
    M = torch.empty((8, n_fine, n_fine, n_fine), dtype=torch.float32, device="cuda")
    Rf = torch.empty((8, nc, nc, nc), dtype=torch.float32, device="cuda")
    for sd in seeds:
        fine = make_context_3d(n_fine, storage, workload, s)
        plain = make_context_3d(nc, coarse_storage, workload, s)
        learned = make_context_3d(nc, coarse_storage, workload, s)
        fine.vlbm_init_fields(_state_3d(make_state, n_fine, sd))
        fine.vlbm_moments(out=M)
        N.vlbm_restrict(M, r, Rf, stream=s)
        for ctx in (plain, learned):
            ctx.vlbm_init_fields(Rf)
        for c in range(checkpoints):
            fine.vlbm_step(r * chunk)
            plain.vlbm_step(chunk)
            fallbacks += N.vlbm_step_corrected(learned, net, chunk, bound_corr, bound_divb_rel, bound_divb_abs,
                                               project_totals=project)
            fine.vlbm_moments(out=M)
            N.vlbm_restrict(M, r, Rf, stream=s)
            ref = Rf.cpu().numpy().astype(np.float64)
            for name, ctx in (("plain", plain), ("learned", learned)):
                q, _ = ctx.vlbm_moments(raise_nonfinite=False)
                fs = _family_sums(q.reshape(ref.shape), ref)
                acc = sums[c][name]
                sums[c][name] = fs if acc is None else {k: (acc[k][0] + fs[k][0], acc[k][1] + fs[k][1]) for k in fs}
        for ctx in (fine, plain, learned):
            ctx.vlbm_destroy()
        if log:
            log(f"eval seed {sd} done, fallbacks so far {fallbacks}")
    hist = []
    for c in range(checkpoints):
        err = {name: {k: float(np.sqrt(a / b)) for k, (a, b) in sums[c][name].items()} for name in ("plain", "learned")}
        hist.append(dict(coarse_step=(c + 1) * chunk, **err))
        if log:
            log(f"eval step {(c + 1) * chunk}: plain {err['plain']} learned {err['learned']}")
    return hist, fallbacks


def time_runs_3d(net, n_fine, r, coarse_steps, workload, make_state, bound_corr, bound_divb_rel, bound_divb_abs,
                 seed=900, storage="f32", project=True, coarse_storage=None):
    """time_runs on 3D lattices: the plain fine run (r * coarse_steps steps, storage
    form storage) and the corrected coarse run (coarse_steps steps, coarse_storage,
    default storage), inputs resident."""
    torch = _torch()
    s = torch.cuda.current_stream().cuda_stream
    nc = n_fine // r
    fine = make_context_3d(n_fine, storage, workload, s)
    learned = make_context_3d(nc, coarse_storage or storage, workload, s)
    fine.vlbm_init_fields(_state_3d(make_state, n_fine, seed))
    M = torch.empty((8, n_fine, n_fine, n_fine), dtype=torch.float32, device="cuda")
    Rf = torch.empty((8, nc, nc, nc), dtype=torch.float32, device="cuda")
    fine.vlbm_moments(out=M)
    N.vlbm_restrict(M, r, Rf, stream=s)
    learned.vlbm_init_fields(Rf)
    fine.vlbm_step(r * 10)
    N.vlbm_step_corrected(learned, net, 10, bound_corr, bound_divb_rel, bound_divb_abs, project_totals=project)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fine.vlbm_step(r * coarse_steps)
    torch.cuda.synchronize()
    t_fine = time.perf_counter() - t0
    t0 = time.perf_counter()
    nfb = N.vlbm_step_corrected(learned, net, coarse_steps, bound_corr, bound_divb_rel, bound_divb_abs,
                                project_totals=project)
    torch.cuda.synchronize()
    t_learned = time.perf_counter() - t0
    fine.vlbm_destroy()
    learned.vlbm_destroy()
    return t_fine, t_learned, nfb
