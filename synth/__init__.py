"""Seeded synthetic inputs for the VLBM MHD workloads.

This module is shared by the oracle tests and the GPU path.  It holds none of the
lattice Boltzmann arithmetic: it only draws random fields and assembles the
conserved state Q = (rho, rho u, e_tot, B [, G, H]) from primitive fields, using
the definition of the total energy (internal + kinetic + magnetic).

Layout of every returned state: float64 array [K, nz, ny, nx], x fastest.
Variable order: 0 rho, 1-3 rho u, 4 e_tot, 5-7 B, 8-16 G (G[3a+b] ~ tau_M d_a B_b),
17-25 H (H[3a+b] ~ tau_H d_a u_b).

Workloads (sizes and statistics follow the workload definitions; no public
dataset is involved):
* ``fourier_2d``: 2D ideal MHD, rho = 1, p = 0.6, u and B sums of random
  Fourier modes with integer wave vectors 1 <= |k| <= kmax, seeded phases, u
  scaled to max |u| = amp, B the discrete central curl of a random vector
  potential scaled to max |B| = amp (so the central divergence of B vanishes).
* ``turbulence_3d``: 3D random solenoidal u and B, complex Gaussian modes with
  1 <= |k| <= kmax, projected perpendicular to k, |u_k| ~ k^-2 (shell energy
  ~ k^-2), normalised to given rms values; G and H set to their relaxed values
  tau_M grad B, tau_H grad u (spectral derivatives).
* ``planar_discontinuity_3d``: a slab with a seeded periodic normal separating
  seeded left/right states, tanh-smoothed over 2 cells.
* ``resistive_2d_state`` / ``brio_wu_2d``: states of the 13-component 2D system
  [13, 1, ny, nx] (rho, rho u_x, rho u_y, e_tot, B_x, B_y, the transported stress
  T_xx, T_xy, T_yy, the transported gradient G_xx, G_xy, G_yx, G_yy): smooth seeded
  Fourier fields with T, G at their relaxed values tau_H mu (grad u + grad u^T),
  tau_M grad B (spectral derivatives); the Brio-Wu left/right states of the paper's
  Sec. 3.1 in a periodic slab.
"""
from __future__ import annotations

import os

import numpy as np
import scipy.fft as sfft


def conserved_from_primitive(rho, u, p, B, gamma):
    """Q = (rho, rho u, e_tot, B) with e_tot = p/(gamma-1) + rho|u|^2/2 + |B|^2/2."""
    rho = np.asarray(rho, np.float64)
    u = np.asarray(u, np.float64)
    B = np.asarray(B, np.float64)
    shape = np.broadcast_shapes(rho.shape, u.shape[1:], np.shape(p), B.shape[1:])
    Q = np.empty((8,) + shape, np.float64)
    Q[0] = rho
    Q[1:4] = rho * u
    Q[4] = np.asarray(p) / (gamma - 1.0) + 0.5 * rho * (u * u).sum(0) + 0.5 * (B * B).sum(0)
    Q[5:8] = B
    return Q


def without_field(Q):
    """The compressible-Euler state [5, ...] of an ideal-MHD state Q [8, ...]: rho,
    rho u, and the total energy without its magnetic part (same p and u)."""
    Q = np.asarray(Q, np.float64)
    E = Q[4] - 0.5 * (Q[5:8] ** 2).sum(0)
    return np.concatenate([Q[:4], E[None]], axis=0)


def _random_mode_field(rng, shape2d, kmax, ncomp):
    """Sum of unit-amplitude Fourier modes cos(2 pi (kx x/nx + ky y/ny) + phase) over
    integer 1 <= |k| <= kmax in the half plane, seeded phases; synthesised with an
    inverse FFT (the same sum, evaluated in O(n^2 log n))."""
    ny, nx = shape2d
    modes = []
    for ky in range(0, kmax + 1):
        for kx in range(-kmax, kmax + 1):
            if ky == 0 and kx <= 0:
                continue
            if 1 <= kx * kx + ky * ky <= kmax * kmax:
                modes.append((kx, ky))
    out = np.zeros((ncomp, ny, nx))
    for c in range(ncomp):
        phases = rng.uniform(0.0, 2.0 * np.pi, size=len(modes))
        F = np.zeros((ny, nx), np.complex128)
        for (kx, ky), ph in zip(modes, phases):
            F[ky % ny, kx % nx] += np.exp(1j * ph)
        out[c] = np.real(np.fft.ifft2(F)) * (nx * ny)
    return out


def _central_curl_2d(A):
    """Discrete central curl of A(x, y) (3 components, d/dz = 0), periodic."""
    def dx(f):
        return 0.5 * (np.roll(f, -1, axis=1) - np.roll(f, 1, axis=1))

    def dy(f):
        return 0.5 * (np.roll(f, -1, axis=0) - np.roll(f, 1, axis=0))

    return np.stack([dy(A[2]), -dx(A[2]), dx(A[1]) - dy(A[0])])


def fourier_2d(n=64, seed=0, kmax=4, amp=0.1, rho0=1.0, p0=0.6, gamma=5.0 / 3.0):
    """2D ideal-MHD state [8, 1, n, n] (random Fourier modes, central div B = 0)."""
    rng = np.random.default_rng(seed)
    u = _random_mode_field(rng, (n, n), kmax, 3)
    u *= amp / np.sqrt((u * u).sum(0)).max()
    A = _random_mode_field(rng, (n, n), kmax, 3)
    B = _central_curl_2d(A)
    B *= amp / np.sqrt((B * B).sum(0)).max()
    rho = np.full((n, n), rho0)
    Q = conserved_from_primitive(rho, u, p0, B, gamma)
    return Q[:, None, :, :].copy()


def _fft_workers():
    return max(1, min(16, len(os.sched_getaffinity(0))))


def _solenoidal_spectral(rng, shape, dx, kmax, rms):
    """Random solenoidal vector field on a periodic box of nz x ny x nx cells of
    size dx, and its gradient grad[a][b] = d_a field_b (spectral)."""
    nz, ny, nx = shape
    kz, ky, kx = np.meshgrid(2 * np.pi * np.fft.fftfreq(nz, d=dx), 2 * np.pi * np.fft.fftfreq(ny, d=dx),
                             2 * np.pi * np.fft.fftfreq(nx, d=dx), indexing="ij")
    kk = np.sqrt(kx * kx + ky * ky + kz * kz)
    mask = (kk >= 1.0 - 1e-9) & (kk <= kmax + 1e-9)
    amp = np.zeros_like(kk)
    amp[mask] = kk[mask] ** -2.0
    vec = (rng.standard_normal((3,) + shape) + 1j * rng.standard_normal((3,) + shape)) * amp
    kvec = np.stack([kx, ky, kz])
    k2 = np.where(kk > 0, kk * kk, 1.0)
    kdotv = (kvec * vec).sum(0)
    vec = vec - kvec * kdotv / k2
    W = _fft_workers()
    field = np.real(sfft.ifftn(vec, axes=(1, 2, 3), workers=W))
    del vec
    field *= rms / np.sqrt((field * field).sum(0).mean())
    fhat = sfft.fftn(field, axes=(1, 2, 3), workers=W)
    grad = np.empty((3, 3) + shape)
    for a, ka in enumerate((kx, ky, kz)):
        for b in range(3):
            grad[a, b] = np.real(sfft.ifftn(1j * ka * fhat[b], workers=W))
    return field, grad


def turbulence_3d(n=256, seed=1, kmax=8, u_rms=0.05, b_rms=0.05, rho0=1.0, p0=0.6,
                  gamma=5.0 / 3.0, tau_M=0.01, tau_H=0.01, dtype=np.float64, shape=None):
    """3D resistive-MHD state [26, nz, ny, nx] with cells of size 2 pi / n (the cube
    [0, 2 pi)^3 when shape is None); random solenoidal u and B."""
    rng = np.random.default_rng(seed)
    shape = (n, n, n) if shape is None else tuple(shape)
    dx = 2.0 * np.pi / n
    u, gu = _solenoidal_spectral(rng, shape, dx, kmax, u_rms)
    B, gB = _solenoidal_spectral(rng, shape, dx, kmax, b_rms)
    Q = np.empty((26,) + shape, dtype)
    Q[:8] = conserved_from_primitive(np.full(shape, rho0), u, p0, B, gamma)
    Q[8:17] = (tau_M * gB).reshape((9,) + shape)
    Q[17:26] = (tau_H * gu).reshape((9,) + shape)
    return Q


def planar_discontinuity_3d(n=512, seed=2, width=2.0, gamma=5.0 / 3.0, dtype=np.float64,
                            shape=None):
    """3D ideal-MHD slab: seeded integer normal k in {-2..2}^3 \\ 0, slab
    frac(k.x/n) in [1/4, 3/4), rho, p ~ U[0.1, 1], |B| ~ U[0, 1] with seeded
    directions on either side, u = 0, tanh profile of the given width."""
    rng = np.random.default_rng(seed)
    while True:
        kvec = rng.integers(-2, 3, size=3)
        if np.any(kvec != 0):
            break
    rhoL, rhoR = rng.uniform(0.1, 1.0, 2)
    pL, pR = rng.uniform(0.1, 1.0, 2)
    bL, bR = rng.uniform(0.0, 1.0, 2)
    dL = rng.standard_normal(3)
    dR = rng.standard_normal(3)
    BL = bL * dL / np.linalg.norm(dL)
    BR = bR * dR / np.linalg.norm(dR)
    nz, ny, nx = (n, n, n) if shape is None else shape
    z = np.arange(nz, dtype=np.float64)[:, None, None]
    y = np.arange(ny, dtype=np.float64)[None, :, None]
    x = np.arange(nx, dtype=np.float64)[None, None, :]
    # phase along the normal in units of one period; the slab is phase in [1/4, 3/4)
    xi = kvec[0] * x / nx + kvec[1] * y / ny + kvec[2] * z / nz
    xi -= np.floor(xi)
    # distance (in cells) to the two interfaces along the normal direction
    period = 1.0 / np.sqrt((kvec[0] / nx) ** 2 + (kvec[1] / ny) ** 2 + (kvec[2] / nz) ** 2)
    w = np.tanh((xi - 0.25) * (period / width))
    w += 1.0
    w *= 1.0 + np.tanh((0.75 - xi) * (period / width))
    w *= 0.25  # 1 inside the slab (right state), 0 outside (left state)
    del xi
    w = w.astype(dtype)
    rho = (rhoL + (rhoR - rhoL) * w).astype(dtype)
    p = (pL + (pR - pL) * w).astype(dtype)
    B = np.stack([(BL[a] + (BR[a] - BL[a]) * w).astype(dtype) for a in range(3)])
    u = np.zeros((3, 1, 1, 1), dtype)
    Q = np.empty((8, nz, ny, nx), dtype)
    Q[0] = rho
    Q[1:4] = 0.0
    Q[4] = p / (gamma - 1.0) + 0.5 * (B * B).sum(0)
    Q[5:8] = B
    info = dict(k=kvec.tolist(), rho=(rhoL, rhoR), p=(pL, pR), BL=BL.tolist(), BR=BR.tolist())
    return Q, info


def uniform_state(shape, rho=1.0, u=(0.0, 0.0, 0.0), p=0.6, B=(0.0, 0.0, 0.0),
                  gamma=5.0 / 3.0, K=8):
    """Spatially uniform state [K, nz, ny, nx] (G = H = 0 for K = 26)."""
    nz, ny, nx = shape
    one = np.ones((nz, ny, nx))
    Q8 = conserved_from_primitive(rho * one, np.array(u)[:, None, None, None] * one, p,
                                  np.array(B)[:, None, None, None] * one, gamma)
    if K == 8:
        return Q8
    Q = np.zeros((K, nz, ny, nx))
    Q[:8] = Q8
    return Q


# ---------------------------------------------------------------------------
# workload parameter sets (the numbers of each synthetic workload; each side maps
# them onto its own parameter structure)
# ---------------------------------------------------------------------------

def elastic_state(shape, seed=0, kmax=3, amp=1e-2, sigma0=(-0.1, -0.1, -0.1, 0.02, 0.0, -0.01)):
    """Linear-elastic state [9, nz, ny, nx] on a periodic box (shape = (nx, ny, nz)):
    momentum density and stress (xx, yy, zz, xy, xz, yz) as sums of seeded Fourier
    modes with integer wavenumbers |k_a| <= kmax (no z-modes when nz = 1), scaled to
    max |.| = amp per component, on a uniform pre-stress sigma0."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = shape

    def wave(kk, n):  # exp(2 pi i k x / n) along one axis
        return np.exp(2j * np.pi * kk * np.arange(n) / n)

    Q = np.zeros((9, nz, ny, nx))
    for k in range(9):
        f = np.zeros((nz, ny, nx))
        for _ in range(4):
            kx, ky = rng.integers(-kmax, kmax + 1, 2)
            kz = rng.integers(-kmax, kmax + 1) if nz > 1 else 0
            ph = rng.uniform(0.0, 2.0 * np.pi)
            # cos(2 pi (kx x / nx + ky y / ny + kz z / nz) + ph) as a product of axis waves
            f += ((np.exp(1j * ph) * wave(kz, nz))[:, None, None] * wave(ky, ny)[None, :, None]
                  * wave(kx, nx)[None, None, :]).real
        f *= amp / max(np.abs(f).max(), 1e-300)
        Q[k] = f + (sigma0[k - 3] if k >= 3 else 0.0)
    return Q


def workload_elastic(dim=2, shape=(64, 64, 1), steps=200):
    """Linear Navier-Cauchy, lambda = mu = rho0 = 1 (P speed sqrt(3), S speed 1), flux
    scale 0.1 (s c_p = 0.17 below c_s^2 = 1/3 or 1/4), tau = 0.6."""
    return dict(dim=dim, shape=shape, model=3, s=0.1, gamma=5.0 / 3.0, tau=0.6, powell=0, divb_mode=0, steps=steps,
                dt=0.0, mu=0.0, eta0=0.0, tau_M=1.0, tau_H=1.0)


def workload_fourier_2d(n=64, steps=200):
    """2D ideal MHD, D2Q5 x 8 variables, periodic, tau = 0.6, flux scale 0.2."""
    return dict(dim=2, shape=(n, n, 1), model=0, s=0.2, gamma=5.0 / 3.0, tau=0.6, powell=1,
                divb_mode=0, steps=steps, dt=0.0, mu=0.0, eta0=0.0, tau_M=1.0, tau_H=1.0)


def workload_resistive_3d(n=256, steps=1000, re=400.0, u_rms=0.05, s=0.2, tau_M=0.01,
                          dt_over_tau_M=None):
    """3D resistive MHD, D3Q7 x 26 variables on [0, 2 pi)^3, Re = Rm = re with
    reference length 1 and velocity u_rms; tau_M = tau_H = 0.01 (physical time), or
    dt / dt_over_tau_M when given (reduced lattices keep the 256^3 ratio 0.49);
    lattice relaxation time 1/2 plus a stabilising diffusion of 5 % of the viscosity."""
    dx = 2.0 * np.pi / n
    dt = s * dx
    if dt_over_tau_M is not None:
        tau_M = dt / dt_over_tau_M
    nu = u_rms * 1.0 / re
    nu_lat = nu * dt / dx ** 2
    cs2 = 0.25
    tau_lb = 0.5 + 0.05 * nu_lat / cs2
    return dict(dim=3, shape=(n, n, n), model=1, s=s, gamma=5.0 / 3.0, tau=tau_lb, powell=1,
                divb_mode=1, steps=steps, dt=dt, mu=nu, eta0=nu, tau_M=tau_M, tau_H=tau_M)


def workload_slab_3d(n=512, steps=2000):
    """3D ideal MHD, D3Q7 x 8 variables, planar discontinuity, tau = 0.6, flux scale
    0.04 (keeps s (|u| + c_fast) below c_s^2 at rho = 0.1, |B| = 1)."""
    return dict(dim=3, shape=(n, n, n), model=0, s=0.04, gamma=5.0 / 3.0, tau=0.6, powell=1,
                divb_mode=0, steps=steps, dt=0.0, mu=0.0, eta0=0.0, tau_M=1.0, tau_H=1.0)


def workload_body_3d(shape=(768, 384, 384), steps=4000, tau=1.5, s=0.05):
    """3D ideal MHD past a moving body, D3Q7 x 8 variables: inflow at x-, zero-gradient
    elsewhere; flux scale 0.05 keeps s (|u| + c_fast) <= c_s^2 at Mach 3; tau = 1.5,
    the smallest tried with which the homogenized body with its dipole field keeps
    every cell physical for 4000 steps at 768 x 384 x 384 (tau = 0.6 and 0.8 lose
    positivity within 500 steps, tau = 1 after about 2200)."""
    return dict(dim=3, shape=tuple(shape), model=0, s=s, gamma=5.0 / 3.0, tau=tau, powell=1, divb_mode=0,
                steps=steps, dt=0.0, mu=0.0, eta0=0.0, tau_M=1.0, tau_H=1.0, bc=(1, 2, 2, 2, 2, 2))


def inflow_state(mach=3.0, alfven_mach=8.0, angle_deg=30.0, rho=1.0, p=0.6, gamma=5.0 / 3.0):
    """Uniform inflow along +x: sound speed sqrt(gamma p / rho) = 1 for the defaults,
    |u| = mach * c, |B| = |u| sqrt(rho) / alfven_mach at `angle_deg` in the x-y plane."""
    c = np.sqrt(gamma * p / rho)
    u = np.array([mach * c, 0.0, 0.0])
    b = u[0] * np.sqrt(rho) / alfven_mach
    a = np.deg2rad(angle_deg)
    B = np.array([b * np.cos(a), b * np.sin(a), 0.0])
    return conserved_from_primitive(rho, u, p, B, gamma), dict(u=u, B=B, rho=rho, p=p)


def body_params(shape=(768, 384, 384), seed=4, R0=48.0, speed=0.02, rough=0.05, dipole_ratio=2.0,
                B_in=0.375, mode=2):
    """Seeded rough sphere: centre at (nx/4, 5 ny/12, nz/2) moving along +y at `speed`
    cells per step; surface radius R0 (1 + delta(n)) with delta a seeded sum of
    degree-1 and degree-2 terms, |delta| <= rough; a dipole along a seeded direction
    whose equatorial surface field is dipole_ratio |B_in|; mode 2 the homogenized
    body, 1 bounce-back."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = shape
    d = rng.standard_normal((4, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    e = rng.standard_normal((4, 3))
    e /= np.linalg.norm(e, axis=1, keepdims=True)
    a = rng.uniform(-1, 1, 4)
    b = rng.uniform(-1, 1, 4)
    # |a.(d.n)| <= |a|, |b ((e.n)^2 - 1/3)| <= 2/3 |b|
    scale = rough / (np.abs(a).sum() + (2.0 / 3.0) * np.abs(b).sum())
    md = rng.standard_normal(3)
    md /= np.linalg.norm(md)
    m = md * dipole_ratio * B_in * R0 ** 3
    return dict(c0=[nx / 4.0, 5.0 * ny / 12.0, nz / 2.0], v=[0.0, speed, 0.0], R0=float(R0),
                a=list(a * scale), d=d.tolist(), b=list(b * scale), e=e.tolist(), m=m.tolist(), mode=int(mode))


def body_initial_state(shape, body, mach=3.0, alfven_mach=8.0, angle_deg=30.0, rho=1.0, p=0.6,
                       gamma=5.0 / 3.0, dtype=np.float64):
    """Inflow state everywhere with the field of a sphere of radius R0 magnetised
    uniformly with the body's moment m superposed on the inflow field (the dipole
    field outside R0, the uniform 2 m / R0^3 inside; divergence free), e_tot from
    that field; [8, nz, ny, nx]."""
    nx, ny, nz = shape
    _, info = inflow_state(mach, alfven_mach, angle_deg, rho, p, gamma)
    z = np.arange(nz, dtype=np.float64)[:, None, None] - body["c0"][2]
    y = np.arange(ny, dtype=np.float64)[None, :, None] - body["c0"][1]
    x = np.arange(nx, dtype=np.float64)[None, None, :] - body["c0"][0]
    R0 = body["R0"]
    r2 = x * x + y * y + z * z
    inside = r2 < R0 * R0
    r2 = np.maximum(r2, R0 * R0)
    m = body["m"]
    mr = m[0] * x + m[1] * y + m[2] * z
    r5 = r2 * r2 * np.sqrt(r2)
    Q = np.empty((8, nz, ny, nx), dtype)
    Bsq = np.zeros((nz, ny, nx))
    for a, ra in enumerate((x, y, z)):
        Ba = info["B"][a] + np.where(inside, 2.0 * m[a] / R0 ** 3, (3.0 * mr * ra - m[a] * r2) / r5)
        Q[5 + a] = Ba
        Bsq = Bsq + Ba * Ba
    u = info["u"]
    Q[0] = rho
    for a in range(3):
        Q[1 + a] = rho * u[a]
    Q[4] = p / (gamma - 1.0) + 0.5 * rho * (u @ u) + 0.5 * Bsq
    return Q


def smooth_box_state(shape, seed, amp=0.1, rho=1.0, p=0.6, B0=0.3, gamma=5.0 / 3.0):
    """Smooth, non-periodic random state [8, nz, ny, nx]: each primitive field is a
    seeded sum of one sine or cosine per axis of the normalised cell coordinates,
    amplitude amp, around rho, u = 0, p and a uniform B0 in every component."""
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz) / nz, np.arange(ny) / ny, np.arange(nx) / nx, indexing="ij")

    def fld():
        a = rng.uniform(-1, 1, 6)
        return a[0] * np.sin(2.1 * x + a[1]) + a[2] * np.cos(1.7 * y + a[3]) + a[4] * np.sin(2.3 * z + a[5])

    r = rho + amp * fld()
    u = amp * np.stack([fld(), fld(), fld()])
    pr = p + amp * fld()
    B = B0 + amp * np.stack([fld(), fld(), fld()])
    return conserved_from_primitive(r, u, pr, B, gamma)


def rough_body(c0, v, R0, m=(0.0, 0.0, 0.0), rough=0.0, seed=1):
    """Body description (the dict the boundary code takes) of a sphere of radius R0
    centred at c0 moving at v, with seeded roughness sum_j |a_j| + |b_j| = rough
    (0: a smooth sphere) and dipole moment m."""
    rng = np.random.default_rng(seed)
    d = rng.standard_normal((4, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    e = rng.standard_normal((4, 3))
    e /= np.linalg.norm(e, axis=1, keepdims=True)
    a = rng.uniform(-1, 1, 4)
    b = rng.uniform(-1, 1, 4)
    if rough > 0:
        scale = rough / (np.abs(a).sum() + np.abs(b).sum())
        a, b = a * scale, b * scale
    else:
        a, b = np.zeros(4), np.zeros(4)
    return dict(c0=[float(c) for c in c0], v=[float(c) for c in v], R0=float(R0), a=list(a), d=d.tolist(),
                b=list(b), e=e.tolist(), m=[float(c) for c in m])


def orszag_tang_2d(n=64, gamma=5.0 / 3.0):
    """Compressible Orszag-Tang vortex (Sec. 3.4) on the periodic unit square with n
    cells per side: rho = 25/(36 pi), p = 5/(12 pi), u = (-sin 2 pi y, sin 2 pi x),
    B = B0 (-sin 2 pi y, sin 4 pi x), B0 = 1/sqrt(4 pi); cell centres at (i + 1/2)/n.
    Returns [8, 1, n, n]."""
    c = (np.arange(n) + 0.5) / n
    y, x = np.meshgrid(c, c, indexing="ij")
    b0 = 1.0 / np.sqrt(4.0 * np.pi)
    u = np.stack([-np.sin(2 * np.pi * y), np.sin(2 * np.pi * x), np.zeros_like(x)])
    B = np.stack([-b0 * np.sin(2 * np.pi * y), b0 * np.sin(4 * np.pi * x), np.zeros_like(x)])
    Q = conserved_from_primitive(25.0 / (36.0 * np.pi) * np.ones_like(x), u, 5.0 / (12.0 * np.pi), B, gamma)
    return Q[:, None]


def workload_orszag_tang_2d(n=4000, tau=None):
    """Lattice parameters of the compressible Orszag-Tang run: acoustic scaling with
    CFL 0.1 (s = 0.1 at sound speed 1); the stabilisation diffusivity 2.5e-5 at
    n = 1000, decreasing linearly with the cell size, is D = c_s^2 (tau - 1/2) dx / s,
    i.e. tau = 1/2 + 2.5e-5 * 1000 * s / c_s^2 = 0.5075 at every n (D2Q5, c_s^2 = 1/3)."""
    s = 0.1
    if tau is None:
        tau = 0.5 + 2.5e-5 * 1000.0 * s / (1.0 / 3.0)
    return dict(dim=2, shape=(n, n, 1), model=0, s=s, gamma=5.0 / 3.0, tau=tau, powell=1, divb_mode=0,
                steps=int(round(0.5 / (s / n))), dt=0.0, mu=0.0, eta0=0.0, tau_M=1.0, tau_H=1.0)



def _spectral_grad_2d(f, dx):
    """d/dx and d/dy of a periodic field f [ny, nx] with cells of size dx."""
    ny, nx = f.shape
    kx = 2 * np.pi * np.fft.fftfreq(nx, d=dx)[None, :]
    ky = 2 * np.pi * np.fft.fftfreq(ny, d=dx)[:, None]
    F = np.fft.fft2(f)
    return np.real(np.fft.ifft2(1j * kx * F)), np.real(np.fft.ifft2(1j * ky * F))


def resistive_2d_state(shape, seed=0, kmax=3, u_amp=0.05, b_amp=0.05, B0=0.3, rho0=1.0, p0=0.6,
                       gamma=5.0 / 3.0, tau_M=0.01, tau_H=0.01, mu=1e-3, dx=None):
    """13-component 2D state [13, 1, ny, nx] on cells of size dx (default 2 pi / nx):
    u and a vector potential A_z sums of seeded Fourier modes 1 <= |k| <= kmax scaled
    to max |u| = u_amp, max |B - B0 x| = b_amp, B = B0 x + (d_y A_z, -d_x A_z); rho and
    p uniform; T = tau_H mu (grad u + grad u^T), G = tau_M grad B (spectral)."""
    ny, nx = shape
    dx = 2.0 * np.pi / nx if dx is None else dx
    rng = np.random.default_rng(seed)
    u = _random_mode_field(rng, (ny, nx), kmax, 2)
    u *= u_amp / np.sqrt((u * u).sum(0)).max()
    A = _random_mode_field(rng, (ny, nx), kmax, 1)[0]
    Ax, Ay = _spectral_grad_2d(A, dx)
    B = np.stack([Ay, -Ax])
    B *= b_amp / np.sqrt((B * B).sum(0)).max()
    B[0] += B0
    rho = np.full((ny, nx), rho0)
    Q = np.zeros((13, 1, ny, nx))
    Q[0, 0] = rho
    Q[1, 0], Q[2, 0] = rho * u[0], rho * u[1]
    Q[3, 0] = p0 / (gamma - 1.0) + 0.5 * rho * (u * u).sum(0) + 0.5 * (B * B).sum(0)
    Q[4, 0], Q[5, 0] = B[0], B[1]
    du = [_spectral_grad_2d(u[b], dx) for b in range(2)]  # du[b][a] = d_a u_b
    dB = [_spectral_grad_2d(B[b], dx) for b in range(2)]
    Q[6, 0] = tau_H * mu * 2.0 * du[0][0]
    Q[7, 0] = tau_H * mu * (du[1][0] + du[0][1])
    Q[8, 0] = tau_H * mu * 2.0 * du[1][1]
    for a in range(2):
        for b in range(2):
            Q[9 + 2 * a + b, 0] = tau_M * dB[b][a]
    return Q


def brio_wu_2d(nx, ny, width=2.0, gamma=2.0, dtype=np.float64):
    """The Brio-Wu shock-tube states of the paper's Sec. 3.1 as a 13-component 2D
    state [13, 1, ny, nx]: (rho, p, u, v, B_x, B_y) = (1, 1, 0, 0, 0.75, 1) in the middle
    half of the periodic x range and (0.125, 0.1, 0, 0, 0.75, -1) outside, blended by
    1/2 (1 + tanh(distance / width)) at both interfaces; T = G = 0."""
    x = np.arange(nx) + 0.5
    d = np.minimum(x - nx / 4.0, 3.0 * nx / 4.0 - x)  # > 0 inside the left-state slab
    wgt = 0.5 * (1.0 + np.tanh(d / width))
    mix = lambda left, right: right + (left - right) * wgt
    rho, p, By = mix(1.0, 0.125), mix(1.0, 0.1), mix(1.0, -1.0)
    Bx = np.full(nx, 0.75)
    Q = np.zeros((13, 1, ny, nx), dtype)
    Q[0, 0] = rho[None, :]
    Q[3, 0] = (p / (gamma - 1.0) + 0.5 * (Bx * Bx + By * By))[None, :]
    Q[4, 0] = Bx[None, :]
    Q[5, 0] = By[None, :]
    return Q


def workload_resistive_2d(n=64, ny=None, s=0.1, tau=0.6, dt_over_tau=0.49, mu=1e-3, eta0=1e-3, j_c=0.5):
    """13-component 2D system on n x ny cells of size 2 pi / n: flux scale s, the
    transported stress and gradient relaxed at dt / tau_M = dt / tau_H = dt_over_tau."""
    dx = 2.0 * np.pi / n
    dt = s * dx
    tau_M = dt / dt_over_tau
    return dict(dim=2, shape=(n, ny or n, 1), model=4, s=s, gamma=5.0 / 3.0, tau=tau, powell=1, divb_mode=1,
                steps=200, dt=dt, mu=mu, eta0=eta0, j_c=j_c, tau_M=tau_M, tau_H=tau_M)


def workload_brio_wu_2d(n=4096, ny=None, s=0.05):
    """The paper's Brio-Wu test (Sec. 3.1) on the 13-component 2D system: [0, 1) in x
    with n cells, gamma = 2 (Brio and Wu's value), ideal (mu = eta = 0) with the
    constant artificial diffusivity 0.75e-4 as the stabilisation of the lattice
    relaxation time, tau = 1/2 + D s / (c_s^2 dx); flux scale s = 0.05 keeps
    s (|u| + c_fast) below c_s^2 = 1/3 (c_fast <= 3.8 in the right state);
    tau_M = tau_H = 0.01 (the paper's tau_M)."""
    dx = 1.0 / n
    tau = 0.5 + 0.75e-4 * s / ((1.0 / 3.0) * dx)
    return dict(dim=2, shape=(n, ny or n, 1), model=4, s=s, gamma=2.0, tau=tau, powell=1, divb_mode=1,
                steps=int(round(0.1 / (s * dx))), dt=s * dx, mu=0.0, eta0=0.0, j_c=0.0, tau_M=0.01, tau_H=0.01)
