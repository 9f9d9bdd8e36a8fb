"""GPU parity of the non-periodic faces (Sec. 2.4 static boundaries) and of the
moving magnetised body against the oracle, through the C ABI."""
import numpy as np
import pytest

import oracle
import synth
from fieldcheck import rel_l2

pytestmark = pytest.mark.gpu

BCS = [(1, 2, 2, 2, 2, 2), (2, 1, 1, 2, 0, 0), (0, 0, 2, 2, 1, 2)]


@pytest.fixture(scope="module")
def vb():
    import torch
    assert torch.cuda.is_available(), "GPU test on a machine without a GPU"
    torch.cuda.set_device(0)
    from paper_2606_00641_amd import vlbm
    return vlbm


def _stream():
    import torch
    return torch.cuda.current_stream().cuda_stream


def _case(kind, mode=1, nx=None):
    """(shape (nx, ny, nz), Q0, inflow_Q, body, tau, s, steps); mode 1 bounce-back,
    2 homogenized body; nx overrides the body box's x extent."""
    if kind == "faces":
        shape = (20, 12, 10)
        Q0 = synth.smooth_box_state(shape[::-1], seed=11)
        Qin, _ = synth.inflow_state(mach=1.2, alfven_mach=4.0)
        return shape, Q0, Qin, None, 0.7, 0.15, 30
    shape = (nx or 30, 22, 20)
    Qin, _ = synth.inflow_state(mach=0.8, alfven_mach=4.0)
    Q0 = np.broadcast_to(Qin[:, None, None, None], (8,) + shape[::-1]).copy()
    Q0 += 0.3 * (synth.smooth_box_state(shape[::-1], seed=12, amp=0.05, rho=0.0, p=0.0, B0=0.0))
    body = synth.rough_body((9.3, 10.1, 9.7), (0.08, 0.04, 0.02), 4.6, m=(3.0, -2.0, 1.5), rough=0.12, seed=5)
    body["mode"] = mode
    return shape, Q0, Qin, body, 0.7, 0.1, 40


def _run_pair(vb, kind, storage, bc, steps=None, mode=1, nx=None, block_x=0):
    shape, Q0, Qin, body, tau, s, n = _case(kind, mode, nx)
    n = steps or n
    p = vb.make_params(lattice="D3Q7", shape=shape, model="ideal", storage=storage, flux_scale=s, tau=tau,
                       bc=bc, inflow_Q=Qin, body=body, stream=_stream(), block_x=block_x)
    sim = vb.Vlbm(p)
    sim.vlbm_init_fields(Q0)
    sim.vlbm_step(n)
    Qg, tot = sim.vlbm_moments()
    op = oracle.make_params(dim=3, shape=shape, s=s, tau=tau)
    oracle.set_boundaries(op, bc=bc, inflow_Q=Qin, body=body, body_mode=mode)
    f = oracle.init(op, Q0)
    oracle.run_bc(op, f, n)
    Qo, _, _ = oracle.moments(op, f)
    if body and mode == 1:
        fluid = (oracle.solid_mask(op, n) == 0).reshape(-1)
    else:
        fluid = np.ones(np.prod(shape), bool)
    return np.asarray(Qg).reshape(8, -1), Qo, fluid, tot


@pytest.mark.parametrize("bc", BCS)
def test_faces_fp64_parity(vb, bc):
    Qg, Qo, fluid, _ = _run_pair(vb, "faces", "f64", bc)
    err = rel_l2(Qg, Qo, 8)
    assert max(err.values()) < 1e-10, err


def test_faces_fp32_parity(vb):
    Qg, Qo, fluid, _ = _run_pair(vb, "faces", "f32", BCS[0])
    err = rel_l2(Qg, Qo, 8)
    assert max(err.values()) < 1e-5, err


@pytest.mark.parametrize("steps", [39, 40])
def test_body_fp64_parity(vb, steps):
    """Moving rough magnetised body with an inflow face and zero-gradient faces; the
    fluid cells match the oracle, the solid ones report zero moments."""
    Qg, Qo, fluid, tot = _run_pair(vb, "body", "f64", (1, 2, 2, 2, 2, 2), steps=steps)
    err = rel_l2(Qg[:, fluid], Qo[:, fluid], 8)
    assert max(err.values()) < 1e-10, err
    assert np.all(Qg[:, ~fluid] == 0.0)
    assert (~fluid).sum() > 300


def test_body_fp32_parity(vb):
    Qg, Qo, fluid, _ = _run_pair(vb, "body", "f32", (1, 2, 2, 2, 2, 2))
    err = rel_l2(Qg[:, fluid], Qo[:, fluid], 8)
    assert max(err.values()) < 1e-5, err


@pytest.mark.parametrize("storage,tol", [("f16", 2e-3), ("bf16", 2e-2)])
def test_body_low_precision(vb, storage, tol):
    """FP16/BF16 deviation storage with the body: per-field error against the FP64
    oracle after 40 steps, within the storage format's resolution."""
    Qg, Qo, fluid, _ = _run_pair(vb, "body", storage, (1, 2, 2, 2, 2, 2))
    err = rel_l2(Qg[:, fluid], Qo[:, fluid], 8)
    print(storage, err)
    assert max(err.values()) < tol, err


@pytest.mark.parametrize("steps", [39, 40])
def test_homogenized_body_fp64_parity(vb, steps):
    """The paper's homogenized moving body (porosity blending), inflow and
    zero-gradient faces: every cell matches the oracle."""
    Qg, Qo, _, _ = _run_pair(vb, "body", "f64", (1, 2, 2, 2, 2, 2), steps=steps, mode=2)
    err = rel_l2(Qg, Qo, 8)
    assert max(err.values()) < 1e-10, err


def test_homogenized_body_fp32_parity(vb):
    Qg, Qo, _, _ = _run_pair(vb, "body", "f32", (1, 2, 2, 2, 2, 2), mode=2)
    err = rel_l2(Qg, Qo, 8)
    assert max(err.values()) < 1e-5, err


@pytest.mark.parametrize("storage,tol", [("f16", 2e-3), ("bf16", 2e-2)])
def test_homogenized_body_low_precision(vb, storage, tol):
    Qg, Qo, _, _ = _run_pair(vb, "body", storage, (1, 2, 2, 2, 2, 2), mode=2)
    err = rel_l2(Qg, Qo, 8)
    print(storage, err)
    assert max(err.values()) < tol, err


@pytest.mark.parametrize("storage,tol", [("f64", 1e-14), ("f32", 2e-6), ("f16", 2e-3), ("bf16", 2e-2)])
def test_uniform_inflow_stays_uniform_with_faces(vb, storage, tol):
    """The Mach-3 inflow state everywhere stays that state (face nodes re-set to its
    equilibrium, the interior at its fixed point), within the storage's rounding."""
    Qin, _ = synth.inflow_state()
    shape = (17, 9, 8)
    p = vb.make_params(lattice="D3Q7", shape=shape, model="ideal", storage=storage, flux_scale=0.05, tau=1.0,
                       bc=(1, 2, 2, 2, 2, 2), inflow_Q=Qin, stream=_stream())
    sim = vb.Vlbm(p)
    sim.vlbm_init_fields(np.broadcast_to(Qin[:, None, None, None], (8,) + shape[::-1]).copy())
    sim.vlbm_step(9)
    Q, _ = sim.vlbm_moments()
    err = np.abs(np.asarray(Q).reshape(8, -1) - Qin[:, None]).max() / np.abs(Qin).max()
    assert err < tol, err


@pytest.mark.parametrize("mode", [1, 2])
def test_checkpoint_restart_with_body(vb, mode):
    """A restored context continues bit for bit (the bounce-back body recomputes its
    mask for the restored step)."""
    shape, Q0, Qin, body, tau, s, _ = _case("body", mode)
    mk = lambda: vb.Vlbm(vb.make_params(lattice="D3Q7", shape=shape, model="ideal", storage="f32", flux_scale=s,
                                        tau=tau, bc=(1, 2, 2, 2, 2, 2), inflow_Q=Qin, body=body, stream=_stream()))
    a = mk()
    a.vlbm_init_fields(Q0)
    a.vlbm_step(13)
    buf, par, step = a.vlbm_get_populations()
    a.vlbm_step(14)
    b = mk()
    b.vlbm_set_populations(buf, par, step)
    b.vlbm_step(14)
    qa, _ = a.vlbm_moments()
    qb, _ = b.vlbm_moments()
    assert np.array_equal(np.asarray(qa), np.asarray(qb))


@pytest.mark.parametrize("block_x", [64, 128, 256])
def test_homogenized_body_lane_exchange(vb, block_x):
    """x rows of 128 cells: workgroups of 64 (two per row) and 128 (one per row) take
    the parity-1 lane exchange around the body's box, 256 the direct accesses; every
    cell matches the oracle in FP64, and FP32 agrees across the two paths."""
    print("case body lane exchange", block_x, flush=True)
    Qg, Qo, _, _ = _run_pair(vb, "body", "f64", (1, 2, 2, 2, 2, 2), steps=41, mode=2, nx=128, block_x=block_x)
    err = rel_l2(Qg, Qo, 8)
    assert max(err.values()) < 1e-10, err
    a, _, _, _ = _run_pair(vb, "body", "f32", (1, 2, 2, 2, 2, 2), steps=41, mode=2, nx=128, block_x=block_x)
    b, _, _, _ = _run_pair(vb, "body", "f32", (1, 2, 2, 2, 2, 2), steps=41, mode=2, nx=128, block_x=256)
    d = rel_l2(a, b, 8)
    assert max(d.values()) < 1e-6, d


@pytest.mark.parametrize("storage,ulp", [("f16", 2.0 ** -11), ("bf16", 2.0 ** -8)])
@pytest.mark.parametrize("body_x,mode", [(9.3, 2), (127.6, 2), (None, 2), (9.3, 1), (127.6, 1)])
def test_pair_sweep_faces_and_body(vb, storage, ulp, body_x, mode):
    """FP16/BF16 storage sweeps two cells per lane on the open lattice too: x faces in
    the sweep (x = 0 the low cell of its lane, x = nx - 1 the high one) and the
    homogenized body's box left to the box sweep (a lane with one cell in the box stores
    only the other half of its words).  256 x 22 x 20, inflow and zero-gradient faces;
    the body inside the first wavefront (its box x = 3..16 at steps 5-6: both edges
    split a lane), across the boundary at x = 128 between two 64-thread workgroups
    (box 121..135), or no body.  Workgroups of 64 threads (two per row, the end lanes'
    16-bit accesses) and 128 (one per row) take the pair sweep.  After 5 steps, one step
    of each parity from the GPU's own pre-step populations: every population that comes
    from a cell off the faces equals the oracle's boundary step (homogenized body) up to
    one rounding of the stored deviation; every population, the face nodes' outputs
    included (their input is f^eq rounded to the storage, as the oracle does not round
    it), equals to that rounding the one-cell sweep (192-thread workgroups, which the
    pair sweep cannot tile) of the same pre-step populations.  The two pair tilings give
    identical bits.  With the bounce-back body (mode 1) the box -- every solid cell and
    cut link -- goes to the one-cell bounce-back sweep; cells solid after the step are
    left out, and a cell the move uncovers (refilled from the mean of its neighbours'
    stored values, which the full-size test holds to the oracle) is held in its moments
    to the one-cell run, to its own rounding plus its neighbours'."""
    import torch
    shape = (256, 22, 20)
    nx, ny, nz = shape
    Qin, _ = synth.inflow_state(mach=0.8, alfven_mach=4.0)
    Q0 = np.broadcast_to(Qin[:, None, None, None], (8,) + shape[::-1]).copy()
    Q0 += 0.3 * (synth.smooth_box_state(shape[::-1], seed=12, amp=0.05, rho=0.0, p=0.0, B0=0.0))
    body = None
    if body_x is not None:
        body = synth.rough_body((body_x, 10.1, 9.7), (0.08, 0.04, 0.02), 4.6, m=(3.0, -2.0, 1.5), rough=0.12, seed=5)
        body["mode"] = mode
    bc = (1, 2, 2, 2, 2, 2)
    op = oracle.make_params(dim=3, shape=shape, s=0.1, tau=0.7)
    oracle.set_boundaries(op, bc=bc, inflow_Q=Qin, body=body, body_mode=mode)
    cells = np.arange(nx * ny * nz)
    x, y, z = cells % nx, (cells // nx) % ny, cells // (nx * ny)
    face = (x == 0) | (x == nx - 1) | (y == 0) | (y == ny - 1) | (z == 0) | (z == nz - 1)
    # population i of cell c after the step is the output of its upstream cell c - e_i
    from_face = np.empty((len(cells), 7), bool)
    from_face[:, 0] = face
    for i, (dx, dy, dz) in enumerate(((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)), 1):
        from_face[:, i] = face[(x - dx) % nx + nx * ((y - dy) % ny + ny * ((z - dz) % nz))]
    interior = np.broadcast_to(~from_face[:, None, :], (len(cells), 8, 7))
    wts = np.array([0.25] + [0.125] * 6)

    def make(block_x):
        return vb.Vlbm(vb.make_params(lattice="D3Q7", shape=shape, model="ideal", storage=storage, flux_scale=0.1,
                                      tau=0.7, bc=bc, inflow_Q=Qin, body=body, stream=_stream(), block_x=block_x))

    one = make(192)
    one.vlbm_init_fields(Q0)  # the same initial state fixes the same FP16/BF16 codec
    bufs = []
    for block_x in (64, 128):
        print("case pair faces/body", storage, body_x, block_x, flush=True)
        sim = make(block_x)
        sim.vlbm_init_fields(Q0)
        sim.vlbm_step(5)
        rest_Q, sigma = sim.vlbm_get_codec()
        f_rest = oracle.equilibrium(op, rest_Q)
        sc = sigma[:, None] * wts[None, :]
        for _ in range(2):
            t = sim.vlbm_get_step()
            one.vlbm_set_populations(*sim.vlbm_get_populations())
            pre = sim.vlbm_gather_cells(cells)
            f = np.ascontiguousarray(np.transpose(pre, (1, 2, 0)))
            oracle.run_bc(op, f, 1, t)
            sim.vlbm_step(1)
            one.vlbm_step(1)
            torch.cuda.synchronize()
            got = sim.vlbm_gather_cells(cells)
            want = np.transpose(f, (2, 0, 1))
            bound = sc[None] * (2 * ulp * np.abs(want - f_rest[None]) / sc[None] + 2.0 ** -24) \
                + 4e-6 + 2e-6 * np.abs(want)
            keep = np.ones(len(cells), bool)
            refilled = np.zeros(len(cells), bool)
            if body is not None and mode == 1:
                solid0 = (oracle.solid_mask(op, t) != 0).reshape(-1)
                solid1 = (oracle.solid_mask(op, t + 1) != 0).reshape(-1)
                refilled = solid0 & ~solid1
                keep = ~solid1 & ~refilled
            sel = interior & keep[:, None, None]
            err = np.where(sel, np.abs(got - want), 0.0)
            assert np.all(err <= bound), (block_x, t % 2, float((err / bound).max()))
            ref = one.vlbm_gather_cells(cells)
            d = np.where(keep[:, None, None], np.abs(got - ref), 0.0)
            assert np.all(d <= bound), (block_x, t % 2, float((d / bound).max()))
            for c in np.where(refilled)[0]:
                nbs = [c + o for o in (1, -1, nx, -nx, nx * ny, -nx * ny) if 0 <= c + o < len(cells)
                       and not solid1[c + o]]
                allow = bound[c].sum(axis=1) + (np.mean([bound[n].sum(axis=1) for n in nbs], axis=0) if nbs else 0)
                dq = np.abs(got[c].sum(axis=1) - ref[c].sum(axis=1))
                assert np.all(dq <= allow), (block_x, t % 2, int(c), dq, allow)
        bufs.append(sim.vlbm_get_populations()[0])
        sim.vlbm_destroy()
    one.vlbm_destroy()
    assert np.array_equal(bufs[0], bufs[1]), int(np.count_nonzero(bufs[0] != bufs[1]))


@pytest.mark.parametrize("storage,tol,nx,centre", [("f64", 1e-10, 30, (3.5, 10.1, 9.7)),
                                                   ("f32", 1e-5, 30, (3.5, 10.1, 9.7)),
                                                   ("f16", 2e-3, 256, (3.5, 10.1, 9.7)),
                                                   ("f64", 1e-10, 30, (9.3, 2.5, 9.7)),
                                                   ("f64", 1e-10, 30, (9.3, 10.1, 17.0))])
def test_homogenized_body_at_the_faces(vb, storage, tol, nx, centre):
    """A homogenized body whose box reaches the inflow face (centre x = 3.5), or that
    crosses a zero-gradient y or z face: at the x face the box's cells skip the outside
    sweep and the box sweep re-sets no face, so for such steps the face pass takes the x
    faces.  Every cell against the oracle after 40 steps (FP16 on 256-cell rows, where
    the two-cell sweep would otherwise run)."""
    shape = (nx, 22, 20)
    Qin, _ = synth.inflow_state(mach=0.8, alfven_mach=4.0)
    Q0 = np.broadcast_to(Qin[:, None, None, None], (8,) + shape[::-1]).copy()
    Q0 += 0.3 * (synth.smooth_box_state(shape[::-1], seed=12, amp=0.05, rho=0.0, p=0.0, B0=0.0))
    body = synth.rough_body(centre, (0.08, 0.04, 0.02), 4.6, m=(3.0, -2.0, 1.5), rough=0.12, seed=5)
    body["mode"] = 2
    bc = (1, 2, 2, 2, 2, 2)
    print("case homogenized body at the faces", storage, nx, centre, flush=True)
    sim = vb.Vlbm(vb.make_params(lattice="D3Q7", shape=shape, model="ideal", storage=storage, flux_scale=0.1,
                                 tau=0.7, bc=bc, inflow_Q=Qin, body=body, stream=_stream()))
    sim.vlbm_init_fields(Q0)
    sim.vlbm_step(40)
    Qg, _ = sim.vlbm_moments()
    sim.vlbm_destroy()
    op = oracle.make_params(dim=3, shape=shape, s=0.1, tau=0.7)
    oracle.set_boundaries(op, bc=bc, inflow_Q=Qin, body=body, body_mode=2)
    f = oracle.init(op, Q0)
    oracle.run_bc(op, f, 40)
    Qo, _, _ = oracle.moments(op, f)
    err = rel_l2(np.asarray(Qg).reshape(8, -1), Qo, 8)
    assert max(err.values()) < tol, err


@pytest.mark.parametrize("centre", [(9.3, 2.5, 9.7), (9.3, 10.1, 17.0), (3.5, 10.1, 9.7)])
def test_bounce_back_body_at_a_face_is_refused(vb, centre):
    """The body must stay clear of the non-periodic faces; a bounce-back step whose box of
    possibly solid or cut cells reaches one (here a y face, a z face, the inflow face)
    returns VLBM_ERR_STATE instead of stepping."""
    shape = (30, 22, 20)
    Qin, _ = synth.inflow_state(mach=0.8, alfven_mach=4.0)
    Q0 = np.broadcast_to(Qin[:, None, None, None], (8,) + shape[::-1]).copy()
    body = synth.rough_body(centre, (0.08, 0.04, 0.02), 4.6, m=(3.0, -2.0, 1.5), rough=0.12, seed=5)
    body["mode"] = 1
    sim = vb.Vlbm(vb.make_params(lattice="D3Q7", shape=shape, model="ideal", storage="f64", flux_scale=0.1,
                                 tau=0.7, bc=(1, 2, 2, 2, 2, 2), inflow_Q=Qin, body=body, stream=_stream()))
    sim.vlbm_init_fields(Q0)
    with pytest.raises(vb.VlbmError) as ei:
        sim.vlbm_step(1)
    assert ei.value.status == -4 and "non-periodic face" in str(ei.value)
    sim.vlbm_destroy()


@pytest.mark.parametrize("storage,tol", [("f64", 1e-10), ("f32", 1e-5)])
@pytest.mark.parametrize("steps", [13, 14])
def test_body_loads_parity(vb, storage, tol, steps):
    """Loads on the homogenized body (force, torque, energy, flux) after an even and an
    odd number of steps match the oracle's, evaluated on the oracle's own run."""
    shape, Q0, Qin, body, tau, s, _ = _case("body", 2)
    bc = (1, 2, 2, 2, 2, 2)
    p = vb.make_params(lattice="D3Q7", shape=shape, model="ideal", storage=storage, flux_scale=s, tau=tau,
                       bc=bc, inflow_Q=Qin, body=body, stream=_stream())
    sim = vb.Vlbm(p)
    sim.vlbm_init_fields(Q0)
    sim.vlbm_step(steps)
    g = sim.vlbm_body_loads()
    op = oracle.make_params(dim=3, shape=shape, s=s, tau=tau)
    oracle.set_boundaries(op, bc=bc, inflow_Q=Qin, body=body, body_mode=2)
    f = oracle.init(op, Q0)
    oracle.run_bc(op, f, steps)
    o = oracle.body_loads(op, f, steps)
    print(storage, steps, g, o)
    fmax = np.abs(o["force"]).max()
    assert np.abs(g["force"] - o["force"]).max() <= tol * fmax, (g["force"], o["force"])
    # the torque is the moment of the surface forces about the centre: it cancels to a
    # small value, but its rounding is at most the lever arm (the surface-radius bound,
    # R0 (1 + rough) < 1.2 R0) times the forces' rounding
    lever = 1.2 * body["R0"]
    assert np.abs(g["torque"] - o["torque"]).max() <= tol * max(np.abs(o["torque"]).max(), lever * fmax), \
        (g["torque"], o["torque"])
    assert abs(g["energy"] - o["work"]) <= tol * abs(o["work"])
    assert abs(g["flux"] - o["flux"]) <= tol * o["flux"]


def test_body_loads_balance_the_gpu_step(vb):
    """Periodic, Powell off, FP64: the GPU step changes the fluid's momentum and energy
    totals by minus the loads taken before it."""
    shape, Q0, Qin, body, tau, s, _ = _case("body", 2)
    p = vb.make_params(lattice="D3Q7", shape=shape, model="ideal", storage="f64", flux_scale=s, tau=tau,
                       powell=False, body=body, stream=_stream())
    sim = vb.Vlbm(p)
    sim.vlbm_init_fields(Q0)
    sim.vlbm_step(5)
    L = sim.vlbm_body_loads()
    _, t0 = sim.vlbm_moments()
    sim.vlbm_step(1)
    _, t1 = sim.vlbm_moments()
    dM, dE = t1[1:4] - t0[1:4], t1[4] - t0[4]
    assert np.abs(dM + L["force"]).max() <= 1e-10 * np.abs(L["force"]).max(), (dM, L)
    assert abs(dE + L["energy"]) <= 1e-10 * abs(L["energy"]), (dE, L)


def test_body_loads_need_the_homogenized_body(vb):
    shape, Q0, Qin, body, tau, s, _ = _case("body", 1)
    sim = vb.Vlbm(vb.make_params(lattice="D3Q7", shape=shape, model="ideal", storage="f32", flux_scale=s, tau=tau,
                                 bc=(1, 2, 2, 2, 2, 2), inflow_Q=Qin, body=body, stream=_stream()))
    sim.vlbm_init_fields(Q0)
    with pytest.raises(vb.VlbmError):
        sim.vlbm_body_loads()
