"""Pins of the oracle's non-periodic faces and moving body (Sec. 2.4 static
boundaries; the body's bounce-back is a reading, stated in the oracle).

Facts used (none re-calls the oracle's boundary code to produce an expected value):
* with all faces periodic and no body the boundary stepper is the periodic stepper;
* a uniform state equal to the inflow state stays exactly uniform;
* one step at tau = 1 without the Powell source from f = f^eq(Q): every population
  is the equilibrium of its source cell, whose moments are Q -- or, on a
  non-periodic face, the inflow state (inflow faces win at edges) or the moments of
  the nearest cell on no non-periodic face; the expected field is assembled here
  from that definition with numpy indexing;
* a fluid at rest around a static body stays exactly at rest (the anti-bounce-back
  of the momentum populations returns the pressure flux with its sign);
* a uniform flow moving with the body (B = 0) stays exactly uniform, also in the
  cells the body uncovers -- which needs the moving-wall flux corrections of rho
  and e_tot and the refill from fluid neighbours;
* halfway bounce-back conserves mass and energy at a static body (Powell off);
* after one step from rest with B = 0, the field next to a magnetised static body
  is 2 w_i times the textbook dipole field (3 (m.r) r - m r^2) / r^5 at the link
  midpoints, summed over the cut links;
* a smooth body (no roughness) is the set of cell centres strictly inside R0.
Homogenized body (Sec. 2.4 porosity blending):
* a uniform flow moving with an unmagnetised body stays exactly uniform;
* deep inside the body (porosity 0) a uniform state relaxes geometrically,
  rho u - rho u^B and B - B^B shrinking by (1 - 1/tau) per step, with u^B the body's
  velocity and B^B the uniform interior field 2 m / R0^3 of a magnetised sphere;
* one step at tau = 1 without the Powell source: every population is the
  equilibrium of its source cell's homogenized state, assembled here from the
  definition (porosity from the radial signed distance, linear transition of one
  cell; blended u and B; rho and pressure kept).
"""
import numpy as np
import pytest

import oracle
import synth

G53 = 5.0 / 3.0


def _smooth_state(shape, seed, amp=0.1):
    return synth.smooth_box_state(shape, seed, amp)


def _cell_Q(p, f):
    Q, _, _ = oracle.moments(p, f)
    return Q.reshape(8, p.nz, p.ny, p.nx)


def _body(c0, v, R0, m=(0.0, 0.0, 0.0), rough=0.0, seed=1):
    return synth.rough_body(c0, v, R0, m, rough, seed)


# ----------------------------------------------------------------------------
# checks (each returns an error figure)
# ----------------------------------------------------------------------------

def chk_periodic_reduces_to_run(nsteps=6):
    shape = (7, 6, 5)
    p = oracle.make_params(dim=3, shape=shape[::-1], tau=0.7)
    Q = _smooth_state(shape, 3)
    f1 = oracle.init(p, Q)
    f2 = f1.copy()
    oracle.run(p, f1, nsteps)
    oracle.set_boundaries(p, bc=(0,) * 6, inflow_Q=np.zeros(8))
    oracle.run_bc(p, f2, nsteps)
    return float(np.abs(f1 - f2).max())


def chk_uniform_inflow(nsteps=8, bc=(1, 2, 2, 2, 2, 2)):
    shape = (6, 7, 9)
    Qin, _ = synth.inflow_state(mach=1.5, alfven_mach=3.0)
    p = oracle.make_params(dim=3, shape=shape[::-1], tau=0.8)
    oracle.set_boundaries(p, bc=bc, inflow_Q=Qin)
    Q = np.broadcast_to(Qin[:, None, None, None], (8,) + shape).copy()
    f = oracle.init(p, Q)
    oracle.run_bc(p, f, nsteps)
    Qe = _cell_Q(p, f)
    return float(np.abs(Qe - Q).max() / np.abs(Qin).max())


def _expected_one_step(p, Q, bc, Qin):
    """Moments after one tau = 1 step without Powell, from the definition."""
    nz, ny, nx = Q.shape[1:]
    n = (nx, ny, nz)
    Qsrc = Q.copy()
    # face nodes: nearest cell on no non-periodic face, inflow state on inflow faces
    idx = [np.arange(nx), np.arange(ny), np.arange(nz)]
    clamp = []
    for a in range(3):
        if bc[2 * a] != 0:
            clamp.append(np.clip(idx[a], 1, n[a] - 2))
        else:
            clamp.append(idx[a])
    Qnear = Q[:, clamp[2]][:, :, clamp[1]][:, :, :, clamp[0]]
    face = np.zeros((nz, ny, nx), bool)
    inflow = np.zeros((nz, ny, nx), bool)
    for a in range(3):
        for side in range(2):
            kind = bc[2 * a + side]
            if kind == 0:
                continue
            sl = [slice(None)] * 3
            sl[2 - a] = 0 if side == 0 else n[a] - 1
            face[tuple(sl)] = True
            if kind == 1:
                inflow[tuple(sl)] = True
    Qsrc[:, face] = Qnear[:, face]
    Qsrc[:, inflow] = Qin[:, None]
    # equilibria of every source cell (the oracle's f^eq, pinned elsewhere)
    N = nx * ny * nz
    flat = Qsrc.reshape(8, N)
    feq = np.stack([oracle.equilibrium(p, flat[:, c]) for c in range(N)], axis=-1)  # [K, Q, N]
    feq = feq.reshape(8, 7, nz, ny, nx)
    out = feq[:, 0].copy()
    for i in range(1, 7):
        a, sgn = (i - 1) // 2, (1 if i % 2 == 1 else -1)
        out += np.roll(feq[:, i], sgn, axis=3 - a)  # population i arrives from x - e_i
    return out


def chk_face_states_one_step(bc=(1, 2, 2, 2, 2, 2), seed=5):
    shape = (6, 5, 8)
    Q = _smooth_state(shape, seed)
    Qin, _ = synth.inflow_state(mach=1.2, alfven_mach=4.0)
    Qin = Qin * np.array([1.1, 1.0, 1.0, 1.0, 1.05, 0.9, 1.1, 1.0])  # distinct from Q
    p = oracle.make_params(dim=3, shape=shape[::-1], tau=1.0, powell=0)
    oracle.set_boundaries(p, bc=bc, inflow_Q=Qin)
    f = oracle.init(p, Q)
    oracle.run_bc(p, f, 1)
    got = _cell_Q(p, f)
    want = _expected_one_step(p, Q, bc, Qin)
    return float(np.abs(got - want).max() / np.abs(want).max())


def chk_static_body_rest(nsteps=20, rough=0.15):
    shape = (16, 16, 16)
    body = _body((7.6, 8.3, 7.9), (0, 0, 0), 4.5, rough=rough)
    p = oracle.make_params(dim=3, shape=shape[::-1], tau=0.7)
    oracle.set_boundaries(p, bc=(0,) * 6, inflow_Q=np.zeros(8), body=body)
    Q = synth.uniform_state(shape, rho=1.0, p=0.6)
    f = oracle.init(p, Q)
    oracle.run_bc(p, f, nsteps)
    fluid = oracle.solid_mask(p, nsteps) == 0
    Qe = _cell_Q(p, f)
    return float(np.abs(Qe - Q)[:, fluid].max())


def chk_comoving_uniform(nsteps=20):
    shape = (16, 18, 14)
    s = 0.15
    v = (0.06, 0.04, -0.025)  # cells per step; the fluid velocity v / s moves with it
    body = _body((6.2, 7.1, 6.8), v, 3.8, rough=0.1, seed=2)
    p = oracle.make_params(dim=3, shape=shape[::-1], tau=0.8, s=s)
    oracle.set_boundaries(p, bc=(0,) * 6, inflow_Q=synth.uniform_state((1, 1, 1), rho=2.0, p=1.0)[:, 0, 0, 0],
                          body=body)
    Q = synth.uniform_state(shape, rho=1.0, u=tuple(c / s for c in v), p=0.6)
    f = oracle.init(p, Q)
    oracle.run_bc(p, f, nsteps)
    s0, s1 = oracle.solid_mask(p, 0), oracle.solid_mask(p, nsteps)
    assert (s0 & ~s1).sum() > 10, "the body must uncover cells"
    Qe = _cell_Q(p, f)
    return float(np.abs(Qe - Q)[:, s1 == 0].max())


def chk_static_body_conservation(nsteps=15):
    shape = (14, 15, 16)
    body = _body((7.3, 6.9, 7.7), (0, 0, 0), 3.9, m=(0.4, -0.2, 0.3), rough=0.1, seed=3)
    p = oracle.make_params(dim=3, shape=shape[::-1], tau=0.75, powell=0)
    oracle.set_boundaries(p, bc=(0,) * 6, inflow_Q=np.zeros(8), body=body)
    Q = _smooth_state(shape, 7)
    fluid = oracle.solid_mask(p, 0) == 0
    f = oracle.init(p, Q)
    m0 = Q[0][fluid].sum(), Q[4][fluid].sum()
    oracle.run_bc(p, f, nsteps)
    Qe = _cell_Q(p, f)
    m1 = Qe[0][fluid].sum(), Qe[4][fluid].sum()
    return float(max(abs(m1[0] - m0[0]) / m0[0], abs(m1[1] - m0[1]) / m0[1]))


def chk_dipole_wall_field():
    shape = (12, 13, 14)
    c0 = np.array([6.3, 5.8, 6.1])
    m = np.array([0.7, -0.4, 0.5])
    body = _body(c0, (0, 0, 0), 3.2, m=m, rough=0.0)
    p = oracle.make_params(dim=3, shape=shape[::-1], tau=0.7)
    oracle.set_boundaries(p, bc=(0,) * 6, inflow_Q=np.zeros(8), body=body)
    Q = synth.uniform_state(shape, rho=1.0, p=0.6)
    f = oracle.init(p, Q)
    oracle.run_bc(p, f, 1)
    got = _cell_Q(p, f)[5:8]
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    solid = (x - c0[0]) ** 2 + (y - c0[1]) ** 2 + (z - c0[2]) ** 2 < 3.2 ** 2
    wi = 0.75 / 6.0
    want = np.zeros((3,) + shape)
    pos = np.stack([x, y, z]).astype(np.float64)
    for i in range(1, 7):
        a, sgn = (i - 1) // 2, (1 if i % 2 == 1 else -1)
        cut = np.roll(solid, -sgn, axis=2 - a) & ~solid  # neighbour x + e_i solid
        q = pos.copy()
        q[a] += 0.5 * sgn
        r = q - c0[:, None, None, None]
        r2 = (r * r).sum(0)
        mr = (m[:, None, None, None] * r).sum(0)
        Bd = (3.0 * mr * r - m[:, None, None, None] * r2) / r2 ** 2.5
        want += np.where(cut, 2.0 * wi * Bd, 0.0)
    fluid = ~solid
    assert np.abs(want).max() > 1e-3
    return float(np.abs(got - want)[:, fluid].max() / np.abs(want).max())


def chk_smooth_body_geometry():
    shape = (11, 12, 13)
    c0 = (6.2, 5.7, 5.4)
    body = _body(c0, (0.1, 0.0, 0.0), 4.0)
    p = oracle.make_params(dim=3, shape=shape[::-1])
    oracle.set_boundaries(p, body=body)
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    t = 3.0
    want = (x - c0[0] - 0.1 * t) ** 2 + (y - c0[1]) ** 2 + (z - c0[2]) ** 2 < 16.0
    return int((oracle.solid_mask(p, t) != want).sum())


def chk_hlbm_comoving_uniform(nsteps=15):
    shape = (14, 12, 13)
    s = 0.12
    v = (0.05, -0.03, 0.02)
    body = _body((6.1, 5.8, 6.4), v, 3.3, rough=0.1, seed=8)
    p = oracle.make_params(dim=3, shape=shape[::-1], tau=0.7, s=s)
    oracle.set_boundaries(p, bc=(0,) * 6, inflow_Q=np.zeros(8), body=body, body_mode=2)
    Q = synth.uniform_state(shape, rho=1.0, u=tuple(c / s for c in v), p=0.6)
    f = oracle.init(p, Q)
    oracle.run_bc(p, f, nsteps)
    return float(np.abs(_cell_Q(p, f) - Q).max())


def chk_hlbm_interior_relaxation(nsteps=5, tau=0.8):
    shape = (5, 6, 4)
    s = 0.1
    v = np.array([0.02, -0.01, 0.015])
    m = np.array([300.0, -200.0, 500.0])
    R0 = 60.0
    body = _body((2.0, 3.0, 2.5), v, R0, m=m)
    p = oracle.make_params(dim=3, shape=shape[::-1], tau=tau, s=s)
    oracle.set_boundaries(p, bc=(0,) * 6, inflow_Q=np.zeros(8), body=body, body_mode=2)
    u0, B0 = np.array([0.3, 0.1, -0.2]), np.array([0.2, -0.1, 0.3])
    Q = synth.uniform_state(shape, rho=1.3, u=tuple(u0), p=0.7, B=tuple(B0))
    f = oracle.init(p, Q)
    oracle.run_bc(p, f, nsteps)
    Qe = _cell_Q(p, f).reshape(8, -1)
    g = (1.0 - 1.0 / tau) ** nsteps
    mb, Bb = 1.3 * v / s, 2.0 * m / R0 ** 3
    want_m = mb + g * (1.3 * u0 - mb)
    want_B = Bb + g * (B0 - Bb)
    return float(max(np.abs(Qe[1:4] - want_m[:, None]).max(), np.abs(Qe[5:8] - want_B[:, None]).max(),
                     np.abs(Qe[0] - 1.3).max()))


def _hlbm_state(Q, body, s, gamma, t):
    """Homogenized state of every cell, from the definition (numpy)."""
    nz, ny, nx = Q.shape[1:]
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    c = np.array(body["c0"]) + t * np.array(body["v"])
    r = np.stack([x - c[0], y - c[1], z - c[2]]).astype(np.float64)
    rr = np.sqrt((r * r).sum(0))
    n = r / np.where(rr > 0, rr, 1.0)
    dd, ee = np.array(body["d"]), np.array(body["e"])
    delta = sum(body["a"][j] * np.tensordot(dd[j], n, 1) + body["b"][j] * (np.tensordot(ee[j], n, 1) ** 2 - 1 / 3)
                for j in range(4))
    phi = rr - body["R0"] * (1.0 + delta)
    d = np.clip(phi + 0.5, 0.0, 1.0)
    m = np.array(body["m"])[:, None, None, None]
    r2 = rr ** 2
    Bdip = (3.0 * (m * r).sum(0) * r - m * r2) / np.where(r2 > 0, r2, 1.0) ** 2.5
    Bb = np.where(rr < body["R0"], 2.0 * m / body["R0"] ** 3, Bdip)
    ub = (np.array(body["v"]) / s)[:, None, None, None]
    rho = Q[0]
    u = Q[1:4] / rho
    B = Q[5:8]
    pres = (gamma - 1.0) * (Q[4] - 0.5 * rho * (u * u).sum(0) - 0.5 * (B * B).sum(0))
    uh = d * u + (1.0 - d) * ub
    Bh = d * B + (1.0 - d) * Bb
    out = Q.copy()
    out[1:4] = rho * uh
    out[5:8] = Bh
    out[4] = pres / (gamma - 1.0) + 0.5 * rho * (uh * uh).sum(0) + 0.5 * (Bh * Bh).sum(0)
    return np.where(d[None] < 1.0, out, Q), d


def chk_hlbm_one_step_definition():
    shape = (9, 10, 12)
    s = 0.15
    body = _body((5.7, 4.6, 4.2), (0.04, 0.02, -0.03), 3.1, m=(2.0, -1.0, 1.5), rough=0.15, seed=9)
    Q = _smooth_state(shape, 13)
    p = oracle.make_params(dim=3, shape=shape[::-1], tau=1.0, s=s, powell=0)
    oracle.set_boundaries(p, bc=(0,) * 6, inflow_Q=np.zeros(8), body=body, body_mode=2)
    f = oracle.init(p, Q)
    oracle.run_bc(p, f, 1)
    Qh, d = _hlbm_state(Q, body, s, G53, 0.0)
    assert (d == 0).sum() > 20 and ((d > 0) & (d < 1)).sum() > 20
    nz, ny, nx = shape
    N = nx * ny * nz
    flat = Qh.reshape(8, N)
    feq = np.stack([oracle.equilibrium(p, flat[:, c]) for c in range(N)], axis=-1).reshape(8, 7, nz, ny, nx)
    want = feq[:, 0].copy()
    for i in range(1, 7):
        a, sgn = (i - 1) // 2, (1 if i % 2 == 1 else -1)
        want += np.roll(feq[:, i], sgn, axis=3 - a)
    return float(np.abs(_cell_Q(p, f) - want).max() / np.abs(want).max())


# ----------------------------------------------------------------------------
# tests
# ----------------------------------------------------------------------------

def test_all_periodic_is_the_periodic_stepper():
    assert chk_periodic_reduces_to_run() < 1e-15


@pytest.mark.parametrize("bc", [(1, 2, 2, 2, 2, 2), (2, 1, 1, 2, 0, 0), (0, 0, 2, 2, 1, 1)])
def test_uniform_inflow_state_is_steady(bc):
    assert chk_uniform_inflow(bc=bc) < 1e-14


@pytest.mark.parametrize("bc", [(1, 2, 2, 2, 2, 2), (2, 1, 1, 2, 0, 0), (0, 0, 2, 2, 1, 2)])
def test_face_states_follow_their_definition(bc):
    assert chk_face_states_one_step(bc=bc) < 1e-14


def test_fluid_at_rest_around_static_body_stays_at_rest():
    assert chk_static_body_rest() < 1e-14


def test_flow_moving_with_the_body_stays_uniform():
    assert chk_comoving_uniform() < 1e-13


def test_static_body_conserves_mass_and_energy():
    assert chk_static_body_conservation() < 1e-13


def test_wall_field_is_the_dipole_at_link_midpoints():
    assert chk_dipole_wall_field() < 1e-13


def test_hlbm_flow_moving_with_the_body_stays_uniform():
    assert chk_hlbm_comoving_uniform() < 1e-14


def test_hlbm_interior_relaxes_to_body_velocity_and_field():
    assert chk_hlbm_interior_relaxation() < 1e-13


def test_hlbm_one_step_follows_the_definition():
    assert chk_hlbm_one_step_definition() < 1e-14


def test_smooth_body_is_a_sphere():
    assert chk_smooth_body_geometry() == 0


# planted mistakes in the boundary code: each must make a check fail
MUTATIONS = {
    "bb_momentum_sign": ("out = -v + 2.0 * wi * rho * uw[k - 1];", "out = v + 2.0 * wi * rho * uw[k - 1];"),
    "bb_wall_velocity_units": ("p->body_v[1] / p->s, p->body_v[2] / p->s};", "p->body_v[1], p->body_v[2]};"),
    "bb_rho_wall_flux_dropped": ("out = v - 2.0 * wi * ephi_rho / c2;", "out = v;"),
    "bb_energy_wall_flux_dropped": ("out = v - 2.0 * wi * ephi_E / c2;", "out = v;"),
    "bb_field_weight": ("out = -v + 2.0 * wi * Bw[k - 5];", "out = -v + wi * Bw[k - 5];"),
    "bb_midpoint": ("cc[a] + 0.5 * (a < d ? edir(i, a) : 0)", "cc[a] + 1.0 * (a < d ? edir(i, a) : 0)"),
    "bb_slot": ("work[((long)k * NQ + ib) * N + cell] = out;", "work[((long)k * NQ + i) * N + cell] = out;"),
    "face_clamp": ("if (ic[a] < 1) ic[a] = 1;", "if (ic[a] < 2) ic[a] = 2;"),
    "face_inflow_edges": ("if (p->bc[2 * a] == 1) *inflow = 1;", ";"),
    "refill_uses_uncovered": ("if (solid[nb] || solid_next[nb]) continue;", "if (solid_next[nb]) continue;"),
    "solid_roughness_sign": ("delta += p->body_a[j] * dn", "delta -= p->body_a[j] * dn"),
    "hlbm_porosity_offset": ("return phi / eps + 0.5;", "return phi / eps;"),
    "hlbm_blend_swapped": ("const double uh = d * u[a] + (1.0 - d) * p->body_v[a] / p->s;",
                           "const double uh = (1.0 - d) * u[a] + d * p->body_v[a] / p->s;"),
    "hlbm_velocity_units": ("(1.0 - d) * p->body_v[a] / p->s;", "(1.0 - d) * p->body_v[a];"),
    "hlbm_inner_field": ("B[a] = 2.0 * p->body_m[a] / (R0 * R0 * R0);", "B[a] = p->body_m[a] / (R0 * R0 * R0);"),
    "hlbm_energy_kept": ("Q[4] = pres / gm1 + 0.5 * rho * uh2 + 0.5 * Bh2;", "(void)uh2; (void)Bh2;"),
    "hlbm_field_blend": ("const double Bh = d * Q[5 + a] + (1.0 - d) * Bb[a];", "const double Bh = Q[5 + a];"),
}


def _fails(name):
    checks = [
        lambda: chk_uniform_inflow() > 1e-14,
        lambda: chk_face_states_one_step() > 1e-14,
        lambda: chk_face_states_one_step(bc=(2, 1, 1, 2, 0, 0)) > 1e-14,
        lambda: chk_static_body_rest() > 1e-14,
        lambda: chk_comoving_uniform() > 1e-13,
        lambda: chk_static_body_conservation() > 1e-13,
        lambda: chk_dipole_wall_field() > 1e-13,
        lambda: chk_hlbm_comoving_uniform() > 1e-14,
        lambda: chk_hlbm_interior_relaxation() > 1e-13,
        lambda: chk_hlbm_one_step_definition() > 1e-14,
    ]
    if name == "solid_roughness_sign":
        # the roughness enters only the solid test; compare with an independent
        # evaluation of the surface radius
        return _rough_mismatch() > 0
    return any(c() for c in checks)


def _rough_mismatch():
    shape = (12, 12, 12)
    body = _body((5.9, 6.2, 6.1), (0, 0, 0), 4.2, rough=0.2, seed=6)
    p = oracle.make_params(dim=3, shape=shape[::-1])
    oracle.set_boundaries(p, body=body)
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    r = np.stack([x - 5.9, y - 6.2, z - 6.1]).astype(np.float64)
    rr = np.sqrt((r * r).sum(0))
    n = r / np.where(rr > 0, rr, 1.0)
    d, e = np.array(body["d"]), np.array(body["e"])
    delta = sum(body["a"][j] * np.tensordot(d[j], n, 1) + body["b"][j] * (np.tensordot(e[j], n, 1) ** 2 - 1 / 3)
                for j in range(4))
    want = rr < 4.2 * (1 + delta)
    margin = np.abs(rr - 4.2 * (1 + delta)) > 1e-9  # skip cells on the surface within rounding
    return int(((oracle.solid_mask(p, 0) != want) & margin).sum())


def test_rough_body_matches_its_surface_radius():
    assert _rough_mismatch() == 0


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_boundary_pins_catch_planted_mistake(name, tmp_path):
    old, new = MUTATIONS[name]
    src = oracle.source_text()
    assert src.count(old) == 1, f"mutation anchor for {name} not unique/found"
    path = oracle.compile_variant(src.replace(old, new), str(tmp_path / f"mut_{name}.so"))
    with oracle.use_library(path):
        assert _fails(name), f"planted mistake '{name}' was not caught"


# --- loads on the homogenized body (Sec. 5 per-step integrals, Sec. 2.4 body) ----

def _uniform_state(shape, rho=1.0, p=0.6, u=(0.05, 0.0, 0.0), B=(0.3, -0.2, 0.1), gamma=5.0 / 3.0):
    u, B = np.asarray(u, float), np.asarray(B, float)
    Q = np.zeros((8,) + tuple(shape[::-1]))
    Q[0] = rho
    Q[1:4] = rho * u[:, None, None, None]
    Q[5:8] = B[:, None, None, None]
    Q[4] = p / (gamma - 1.0) + 0.5 * rho * (u @ u) + 0.5 * (B @ B)
    return Q


def _smooth_sphere(c, R0, v=(0.0, 0.0, 0.0), m=(0.0, 0.0, 0.0)):
    return dict(c0=c, v=v, R0=R0, a=[0.0] * 4, d=[[1.0, 0.0, 0.0]] * 4, b=[0.0] * 4, e=[[1.0, 0.0, 0.0]] * 4, m=m)


@pytest.mark.parametrize("collision", [0, 1, 2])
def test_body_loads_balance_the_fluid(collision):
    """Periodic domain, Powell off: in one step the fluid's momentum and energy totals
    change by exactly minus the force and energy the loads assign to the body (the
    homogenization is the only non-conservative part of the step), for every
    collision operator; a moving rough magnetised body."""
    shape = (24, 22, 20)
    Qin, _ = synth.inflow_state(mach=0.8, alfven_mach=4.0)
    Q0 = np.broadcast_to(Qin[:, None, None, None], (8,) + shape[::-1]).copy()
    Q0 += 0.3 * synth.smooth_box_state(shape[::-1], seed=12, amp=0.05, rho=0.0, p=0.0, B0=0.0)
    body = synth.rough_body((11.3, 10.1, 9.7), (0.08, 0.04, 0.02), 4.6, m=(3.0, -2.0, 1.5), rough=0.12, seed=5)
    op = oracle.make_params(dim=3, shape=shape, s=0.1, tau=0.7, powell=0, collision=collision)
    oracle.set_boundaries(op, bc=None, inflow_Q=Qin, body=body, body_mode=2)
    f = oracle.init(op, Q0)
    oracle.run_bc(op, f, 3)
    L = oracle.body_loads(op, f, 3)
    Qa, _, _ = oracle.moments(op, f)
    oracle.run_bc(op, f, 1, t0=3)
    Qb, _, _ = oracle.moments(op, f)
    dM = Qb[1:4].sum(1) - Qa[1:4].sum(1)
    dE = Qb[4].sum() - Qa[4].sum()
    assert np.abs(dM + L["force"]).max() <= 1e-11 * np.abs(L["force"]).max(), (dM, L["force"])
    assert abs(dE + L["work"]) <= 1e-11 * abs(L["work"]), (dE, L["work"])
    assert np.abs(L["force"]).max() > 0.1 and abs(L["work"]) > 0.01


@pytest.mark.parametrize("R0,c", [(6.0, (16, 16, 16)), (8.0, (16.3, 16.5, 15.8)), (10.0, (20, 20, 20))])
def test_body_loads_closed_forms(R0, c):
    """A uniform flow u0 x and field B0 around a smooth sphere at rest without a
    moment: every cell of the body pulls the fluid toward rest, so the force is
    omega rho u0 x (the body's porosity volume, sum (1 - d) = 4/3 pi R0^3 to the ramp's
    resolution); the flux of the uniform field through the sphere is pi R0^2 |B0|
    (half the integral of |B0 . n|); a sphere centred on a lattice point takes no
    torque (mirror symmetry of the cells)."""
    n = int(2 * np.ceil(max(c)))
    shape = (n, n, n)
    u0, B0, tau = 0.05, np.array([0.3, -0.2, 0.1]), 0.7
    Q = _uniform_state(shape, u=(u0, 0.0, 0.0), B=B0)
    op = oracle.make_params(dim=3, shape=shape, s=0.1, tau=tau, powell=0)
    oracle.set_boundaries(op, bc=None, inflow_Q=Q[:, 0, 0, 0], body=_smooth_sphere(c, R0), body_mode=2)
    L = oracle.body_loads(op, oracle.init(op, Q), 0)
    vol = 4.0 / 3.0 * np.pi * R0 ** 3
    assert abs(L["force"][0] / (u0 / tau * vol) - 1.0) < 0.01, L
    assert np.abs(L["force"][1:]).max() <= 1e-12 * L["force"][0]
    assert abs(L["flux"] / (np.pi * R0 ** 2 * np.linalg.norm(B0)) - 1.0) < 0.06, L
    if all(float(x).is_integer() for x in c):
        assert np.abs(L["torque"]).max() <= 1e-12 * L["force"][0] * R0, L
