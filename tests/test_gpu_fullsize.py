"""Parity at the full workload sizes, in the launch configuration the benchmark
times: the GPU's populations at sampled cells after one sweep of each parity equal
the oracle's collision of the GPU's own pre-sweep populations at the upstream
cells; plus properties that hold at any size (finite, physical totals)."""
import numpy as np
import pytest

import oracle
import synth
from fieldcheck import oracle_one_step
from test_gpu_parity import gpu_params, oracle_params

pytestmark = pytest.mark.gpu

SAMPLES = 3000


@pytest.fixture(scope="module")
def vb():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    from paper_2606_00641_amd import vlbm
    return vlbm


def sampled_one_step(vb, w, Q0, storage, rtol, atol, seed=0, ulp=None):
    import torch
    shape = w["shape"]
    N = int(np.prod(shape))
    print(f"case fullsize {shape} model={w['model']} storage={storage}", flush=True)
    sim = vb.Vlbm(gpu_params(vb, w, storage))
    sim.vlbm_init_fields(Q0)
    op = oracle_params(w)
    rng = np.random.default_rng(seed)
    # corners and faces are included so the periodic wrap is exercised
    cells = np.unique(np.concatenate([rng.integers(0, N, SAMPLES), [0, N - 1, shape[0] - 1,
                                                                    N - shape[0]]]))
    worst = 0.0
    for parity in (0, 1):
        want = oracle_one_step(oracle, op, sim.vlbm_gather_cells, cells, shape, w["dim"])
        sim.vlbm_step(1)
        torch.cuda.synchronize()
        got = sim.vlbm_gather_cells(cells)
        if ulp is None:
            bound = atol + rtol * np.abs(want)
        else:
            rest_Q, sigma = sim.vlbm_get_codec()
            f_rest = oracle.equilibrium(op, rest_Q)
            wts = np.array([0.25] + [0.125] * 6)
            sc = sigma[:, None] * wts[None, :]
            bound = sc[None] * (2 * ulp * np.abs(want - f_rest[None]) / sc[None] + 2.0 ** -24) \
                + atol + rtol * np.abs(want)
        err = np.abs(got - want)
        worst = max(worst, float((err / bound).max()))
        assert np.all(err <= bound), (parity, float((err / bound).max()))
    _, tot = sim.vlbm_moments(with_field=False)
    assert np.all(np.isfinite(tot))
    sim.vlbm_destroy()
    return worst


def test_resistive_256cubed_fp32_sampled(vb):
    w = synth.workload_resistive_3d(n=256)
    Q0 = synth.turbulence_3d(n=256, seed=1, dtype=np.float32)
    sampled_one_step(vb, w, Q0, "f32", rtol=2e-6, atol=1e-6)


@pytest.mark.parametrize("storage", ["f32", "f16", "bf16"])
def test_slab_512cubed_sampled(vb, storage):
    w = synth.workload_slab_3d(n=512)
    Q0, _ = synth.planar_discontinuity_3d(n=512, seed=2, dtype=np.float32)
    ulp = {"f32": None, "f16": 2.0 ** -11, "bf16": 2.0 ** -8}[storage]
    sampled_one_step(vb, w, Q0, storage, rtol=2e-6, atol=1e-6 if ulp is None else 4e-6, ulp=ulp)


@pytest.mark.parametrize("storage", ["f16", "f32"])
def test_body_768x384x384_sampled(vb, storage):
    """The flow past the homogenized magnetised body at its full size (768 x 384 x 384,
    inflow / zero-gradient faces), in the benchmark's launch configuration: after one
    sweep of each parity the GPU's populations at sampled cells -- random interior
    cells and cells on and around the body's surface -- equal the oracle's
    (homogenized) collision of the GPU's own pre-sweep populations.  Cells within two
    cells of a face are left out (their upstream values are re-set at the start of the
    step, after the gather)."""
    import torch
    from fieldcheck import oracle_one_step_at
    shape = (768, 384, 384)
    nx, ny, nz = shape
    w = synth.workload_body_3d(shape=shape)
    Qin, info = synth.inflow_state()
    body = synth.body_params(shape=shape, B_in=float(np.linalg.norm(info["B"])))
    print(f"case fullsize body {shape} storage={storage}", flush=True)
    sim = vb.Vlbm(vb.make_params(lattice="D3Q7", shape=shape, model="ideal", storage=storage, gamma=w["gamma"],
                                 flux_scale=w["s"], tau=w["tau"], powell=w["powell"], bc=w["bc"], inflow_Q=Qin,
                                 body=body, stream=torch.cuda.current_stream().cuda_stream))
    sim.vlbm_init_fields(synth.body_initial_state(shape, body, dtype=np.float32))
    op = oracle.make_params(dim=3, shape=shape, s=w["s"], tau=w["tau"], gamma=w["gamma"], powell=w["powell"])
    oracle.set_boundaries(op, bc=w["bc"], inflow_Q=Qin, body=body, body_mode=2)
    rng = np.random.default_rng(3)
    interior = np.stack([rng.integers(2, n - 2, SAMPLES) for n in shape], axis=1)
    c0 = np.array(body["c0"])
    dirs = rng.standard_normal((SAMPLES, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    radii = body["R0"] + rng.uniform(-3.0, 3.0, SAMPLES)
    surf = np.rint(c0[None] + radii[:, None] * dirs).astype(np.int64)
    xyz = np.concatenate([interior, surf])
    cells = np.unique(xyz[:, 0] + nx * (xyz[:, 1] + ny * xyz[:, 2]))
    ulp = {"f32": None, "f16": 2.0 ** -11}[storage]
    for parity in (0, 1):
        t = sim.vlbm_get_step()
        want = oracle_one_step_at(oracle, op, sim.vlbm_gather_cells, cells, shape, 3, t)
        sim.vlbm_step(1)
        torch.cuda.synchronize()
        got = sim.vlbm_gather_cells(cells)
        if ulp is None:
            bound = 1e-6 + 2e-6 * np.abs(want)
        else:
            rest_Q, sigma = sim.vlbm_get_codec()
            f_rest = oracle.equilibrium(op, rest_Q)
            wts = np.array([0.25] + [0.125] * 6)
            sc = sigma[:, None] * wts[None, :]
            bound = sc[None] * (2 * ulp * np.abs(want - f_rest[None]) / sc[None] + 2.0 ** -24) \
                + 4e-6 + 2e-6 * np.abs(want)
        err = np.abs(got - want)
        assert np.all(err <= bound), (parity, float((err / bound).max()))
    sim.vlbm_destroy()


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_bounce_back_body_768x384x384_sub_box(vb, storage):
    """The configured body treatment at full size: link-wise bounce-back with the
    moving-wall correction, the dipole field on the wall, and the refill of cells the
    body uncovers (768 x 384 x 384, inflow / zero-gradient faces, tau = 1.0).  One
    step of each parity: the GPU's populations on a box enclosing the body with a
    margin are handed to the oracle, which steps the box with the same body (shifted
    into the box, periodic box faces); every fluid cell of the box but its outer layer
    (whose upstream neighbours lie outside the box) must equal the GPU's after its own
    step, as must random cells away from the body and the faces (plain collision).  In
    FP16 a cell the body uncovers is held in its moments to its own rounding plus the
    mean rounding of the neighbours its refill averages (the GPU averages their stored
    values, the oracle their exact ones)."""
    import torch
    shape = (768, 384, 384)
    nx, ny, nz = shape
    w = synth.workload_body_3d(shape=shape, tau=1.0)
    Qin, info = synth.inflow_state()
    body = synth.body_params(shape=shape, B_in=float(np.linalg.norm(info["B"])), mode=1)
    print(f"case fullsize bounce-back body {shape} storage={storage}", flush=True)
    sim = vb.Vlbm(vb.make_params(lattice="D3Q7", shape=shape, model="ideal", storage=storage, gamma=w["gamma"],
                                 flux_scale=w["s"], tau=w["tau"], powell=w["powell"], bc=w["bc"], inflow_Q=Qin,
                                 body=body, stream=torch.cuda.current_stream().cuda_stream))
    sim.vlbm_init_fields(synth.body_initial_state(shape, body, dtype=np.float32))
    # the box: the body's extent (surface radius <= R0 (1 + rough)) plus 5 cells
    c0 = np.array(body["c0"])
    half = int(np.ceil(body["R0"] * 1.05)) + 5
    lo = np.floor(c0).astype(int) - half
    size = 2 * half + 2
    bx = by = bz = size
    zz, yy, xx = np.meshgrid(np.arange(bz) + lo[2], np.arange(by) + lo[1], np.arange(bx) + lo[0], indexing="ij")
    box_cells = (xx + nx * (yy + ny * zz)).reshape(-1)
    inner = np.zeros((bz, by, bx), bool)
    inner[1:-1, 1:-1, 1:-1] = True
    inner = inner.reshape(-1)
    sub_body = dict(body)
    sub_body["c0"] = list(c0 - lo)
    op = oracle.make_params(dim=3, shape=(bx, by, bz), s=w["s"], tau=w["tau"], gamma=w["gamma"], powell=w["powell"])
    oracle.set_boundaries(op, bc=(0, 0, 0, 0, 0, 0), inflow_Q=Qin, body=sub_body, body_mode=1)
    # random cells away from the body's box and the faces: the plain collision
    from fieldcheck import oracle_one_step
    opf = oracle.make_params(dim=3, shape=shape, s=w["s"], tau=w["tau"], gamma=w["gamma"], powell=w["powell"])
    rng = np.random.default_rng(5)
    far = np.stack([rng.integers(2, n - 2, SAMPLES) for n in shape], axis=1)
    far = far[np.any((far < lo[None] - 2) | (far >= lo[None] + size + 2), axis=1)]
    far_cells = np.unique(far[:, 0] + nx * (far[:, 1] + ny * far[:, 2]))
    ulp = {"f32": None, "f16": 2.0 ** -11}[storage]

    def bound_of(wv):
        """One rounding of the stored deviation (FP16) or FP32 arithmetic, per population."""
        if ulp is None:
            return 1e-6 + 2e-6 * np.abs(wv)
        rest_Q, sigma = sim.vlbm_get_codec()
        f_rest = oracle.equilibrium(opf, rest_Q)
        wts = np.array([0.25] + [0.125] * 6)
        sc = sigma[:, None] * wts[None, :]
        return sc[None] * (2 * ulp * np.abs(wv - f_rest[None]) / sc[None] + 2.0 ** -24) + 4e-6 + 2e-6 * np.abs(wv)

    cube = (bz, by, bx)
    for parity in (0, 1):
        t = sim.vlbm_get_step()
        pre = sim.vlbm_gather_cells(box_cells)  # [n, 8, 7]
        f = np.ascontiguousarray(np.transpose(pre, (1, 2, 0)))  # [8, 7, n]
        oracle.run_bc(op, f, 1, t)
        want_far = oracle_one_step(oracle, opf, sim.vlbm_gather_cells, far_cells, shape, 3)
        sim.vlbm_step(1)
        torch.cuda.synchronize()
        solid0 = (oracle.solid_mask(op, t) != 0).reshape(-1)
        solid1 = (oracle.solid_mask(op, t + 1) != 0).reshape(-1)
        got_all = sim.vlbm_gather_cells(box_cells)
        want_all = np.transpose(f, (2, 0, 1))
        bound_all = bound_of(want_all)
        # cells the body uncovered take f^eq of the mean moments of their neighbours that
        # are fluid before and after the move; in FP16 those neighbours' populations are
        # the stored (rounded) ones, so a refilled cell is held, in its moments, to its own
        # rounding plus the mean of those neighbours' roundings
        refilled = solid0 & ~solid1 & inner
        plain = ~solid1 & inner & (~refilled if ulp is not None else True)
        err = np.abs(got_all[plain] - want_all[plain])
        assert np.all(err <= bound_all[plain]), (parity, float((err / bound_all[plain]).max()))
        if ulp is not None and refilled.any():
            both = (~solid0 & ~solid1).reshape(cube)
            for c in np.where(refilled)[0]:
                z, y, x = np.unravel_index(c, cube)
                nbs = [np.ravel_multi_index((z + dz, y + dy, x + dx), cube)
                       for dx, dy, dz in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1))
                       if both[z + dz, y + dy, x + dx]]
                own = bound_all[c].sum(axis=1)
                nbb = np.mean([bound_all[n].sum(axis=1) for n in nbs], axis=0) if nbs else 0.0
                dq = np.abs(got_all[c].sum(axis=1) - want_all[c].sum(axis=1))
                assert np.all(dq <= own + nbb), (parity, c, dq, own + nbb)
        got_far = sim.vlbm_gather_cells(far_cells)
        err = np.abs(got_far - want_far)
        bf = bound_of(want_far)
        assert np.all(err <= bf), (parity, float((err / bf).max()))
    _, tot = sim.vlbm_moments(with_field=False)
    assert np.all(np.isfinite(tot))
    sim.vlbm_destroy()
