"""GPU parity: the HIP sweep (through the C ABI) against the FP64 CPU oracle on the
same seeded inputs, element by element, at sizes the oracle finishes in seconds
(several blocks and a ragged tail), plus the invariants that hold at any size.

Tolerances: FP64 storage <= 1e-10 relative L2 per field after 200 steps, FP32
storage <= 1e-5 (the targets of the method's parity gate); FP16/BF16 deviation
storage is checked one step at a time against the per-value quantisation bound.
"""
import numpy as np
import pytest

import oracle
import synth
from fieldcheck import oracle_one_step, rel_l2

pytestmark = pytest.mark.gpu


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


def gpu_params(vb, w, storage, block_x=0, shape=None):
    shape = shape or w["shape"]
    return vb.make_params(lattice="D3Q7" if w["dim"] == 3 else "D2Q5", shape=shape,
                          model={0: "ideal", 1: "resistive", 2: "euler", 3: "navier_cauchy",
                                 4: "resistive_2d"}[w["model"]],
                          storage=storage,
                          gamma=w["gamma"], flux_scale=w["s"], tau=w["tau"], powell=w["powell"],
                          divb_mode=w["divb_mode"], dt=w["dt"], mu=w["mu"], eta0=w["eta0"], j_c=w.get("j_c", 0.0),
                          tau_M=w["tau_M"], tau_H=w["tau_H"], stream=_stream(), block_x=block_x)


def oracle_params(w, shape=None):
    shape = shape or w["shape"]
    return oracle.make_params(dim=w["dim"], shape=shape, model=w["model"], gamma=w["gamma"], s=w["s"],
                              tau=w["tau"], powell=w["powell"], divb_mode=w["divb_mode"], dt=w["dt"],
                              mu=w["mu"], eta0=w["eta0"], j_c=w.get("j_c", 0.0), tau_M=w["tau_M"],
                              tau_H=w["tau_H"])


def run_gpu(vb, w, Q0, steps, storage, block_x=0):
    sim = vb.Vlbm(gpu_params(vb, w, storage, block_x))
    sim.vlbm_init_fields(Q0)
    sim.vlbm_step(steps)
    Q, tot = sim.vlbm_moments()
    return sim, Q, tot


def run_oracle(w, Q0, steps):
    op = oracle_params(w)
    f = oracle.init(op, Q0)
    oracle.run(op, f, steps)
    Q, _, tot = oracle.moments(op, f)
    return Q, tot


def small_resistive(shape=(12, 10, 8), seed=3):
    """Periodic resistive state on a small ragged box, 3D-turbulence recipe."""
    nx, ny, nz = shape
    tau_M = synth.workload_resistive_3d(n=16, dt_over_tau_M=0.49)["tau_M"]
    return synth.turbulence_3d(n=16, seed=seed, kmax=3, tau_M=tau_M, tau_H=tau_M, shape=(nz, ny, nx))


# --- FP64 / FP32 parity on the 2D workload (64^2, 200 steps) --------------------

@pytest.mark.parametrize("seed", [0, 1, 2])
def test_fourier2d_fp64_parity_200_steps(vb, seed):
    w = synth.workload_fourier_2d()
    Q0 = synth.fourier_2d(64, seed=seed)
    print(f"case fourier2d fp64 seed={seed}", flush=True)
    sim, Qg, tg = run_gpu(vb, w, Q0, 200, "f64")
    Qo, to = run_oracle(w, Q0, 200)
    err = rel_l2(Qg, Qo, 8)
    assert max(err.values()) <= 1e-10, err
    assert np.allclose(tg[:8], to[:8], rtol=1e-12, atol=1e-12)
    assert abs(tg[8 + 1] - to[8 + 1]) <= 1e-8 * max(to[8 + 1], 1e-30) + 1e-24


def test_fourier2d_fp32_parity_200_steps(vb):
    w = synth.workload_fourier_2d()
    Q0 = synth.fourier_2d(64, seed=0)
    sim, Qg, _ = run_gpu(vb, w, Q0, 200, "f32")
    Qo, _ = run_oracle(w, Q0, 200)
    err = rel_l2(Qg, Qo, 8)
    assert max(err.values()) <= 1e-5, err


MRT_TAUS = (0.8, 1.3)  # mrt_tau_e, mrt_tau_d of the MRT cases


@pytest.mark.parametrize("collision,magic", [("trt", 0.25), ("trt", 1.0 / 12.0), ("rlb", 0.25), ("mrt", 0.25)])
@pytest.mark.parametrize("storage,tol", [("f64", 1e-10), ("f32", 1e-5)])
def test_two_rate_collisions_parity(vb, collision, magic, storage, tol):
    """TRT, the regularized BGK and MRT (Sec. 2.2 names all three): 2D Fourier
    workload, 200 steps; the GPU relaxes each opposite pair's antisymmetric half and the
    trace and deviatoric parts of the symmetric halves at their rates, the oracle
    follows each definition literally (MRT through its moment matrix)."""
    w = synth.workload_fourier_2d()
    Q0 = synth.fourier_2d(64, seed=1)
    code = {"trt": 1, "rlb": 2, "mrt": 3}[collision]
    print(f"case {collision} magic={magic} {storage}", flush=True)
    sim = vb.Vlbm(vb.make_params(lattice="D2Q5", shape=(64, 64, 1), storage=storage, gamma=w["gamma"],
                                 flux_scale=w["s"], tau=w["tau"], powell=w["powell"], collision=collision,
                                 trt_magic=magic, mrt_tau_e=MRT_TAUS[0], mrt_tau_d=MRT_TAUS[1], stream=_stream()))
    sim.vlbm_init_fields(Q0)
    sim.vlbm_step(200)
    Qg, _ = sim.vlbm_moments()
    op = oracle.make_params(dim=2, shape=(64, 64, 1), s=w["s"], tau=w["tau"], powell=w["powell"], collision=code,
                            trt_magic=magic, mrt_tau_e=MRT_TAUS[0], mrt_tau_d=MRT_TAUS[1])
    f = oracle.init(op, Q0)
    oracle.run(op, f, 200)
    Qo, _, _ = oracle.moments(op, f)
    err = rel_l2(Qg, Qo, 8)
    if storage == "f64":
        assert max(err.values()) <= tol, err
        return
    # FP32: 1e-5, or 1.5x the same formulas evaluated in FP32 where those miss it
    yard = rel_l2(oracle.run_fp32(op, Q0, 200), Qo, 8)
    for name, e in err.items():
        assert e <= max(tol, 1.5 * yard[name]), (name, e, yard[name])


@pytest.mark.parametrize("collision", ["trt", "rlb", "mrt"])
def test_two_rate_collisions_3d_resistive_fp64(vb, collision):
    w = synth.workload_resistive_3d(n=16, dt_over_tau_M=0.49)
    w["shape"] = (12, 10, 8)
    Q0 = small_resistive()
    code = {"trt": 1, "rlb": 2, "mrt": 3}[collision]
    p = gpu_params(vb, w, "f64")
    p.collision, p.trt_magic = code, 0.25
    p.mrt_tau_e, p.mrt_tau_d = MRT_TAUS
    sim = vb.Vlbm(p)
    sim.vlbm_init_fields(Q0)
    sim.vlbm_step(30)
    Qg, _ = sim.vlbm_moments()
    op = oracle_params(w)
    op.collision, op.trt_magic = code, 0.25
    op.mrt_tau_e, op.mrt_tau_d = MRT_TAUS
    f = oracle.init(op, Q0)
    oracle.run(op, f, 30)
    Qo, _, _ = oracle.moments(op, f)
    err = rel_l2(Qg, Qo, 26)
    assert max(err.values()) <= 1e-10, err


@pytest.mark.parametrize("steps", [199, 200])
def test_orszag_tang_fp64_parity(vb, steps):
    """The paper's compressible Orszag-Tang vortex (Sec. 3.4) at 64^2 with its own
    lattice parameters (CFL 0.1, stabilisation tau = 0.5075)."""
    w = synth.workload_orszag_tang_2d(64)
    Q0 = synth.orszag_tang_2d(64)
    print(f"case orszag-tang fp64 steps={steps}", flush=True)
    _, Qg, _ = run_gpu(vb, w, Q0, steps, "f64")
    Qo, _ = run_oracle(w, Q0, steps)
    err = rel_l2(Qg, Qo, 8)
    assert max(err.values()) <= 1e-10, err


def test_orszag_tang_fp32_parity(vb):
    """FP32 within 1e-5, or within 1.5x of the same formulas evaluated in FP32 (the
    oracle compiled with float) where that evaluation already misses 1e-5."""
    w = synth.workload_orszag_tang_2d(64)
    Q0 = synth.orszag_tang_2d(64)
    _, Qg, _ = run_gpu(vb, w, Q0, 200, "f32")
    Qo, _ = run_oracle(w, Q0, 200)
    err = rel_l2(Qg, Qo, 8)
    yard = rel_l2(oracle.run_fp32(oracle_params(w), Q0, 200), Qo, 8)
    for name, e in err.items():
        assert e <= max(1e-5, 1.5 * yard[name]), (name, e, yard[name])


@pytest.mark.parametrize("steps", [0, 1, 2, 7])
def test_parity_even_and_odd_step_counts(vb, steps):
    w = synth.workload_fourier_2d(n=40)
    Q0 = synth.fourier_2d(40, seed=5)
    _, Qg, _ = run_gpu(vb, w, Q0, steps, "f64")
    Qo, _ = run_oracle(w, Q0, steps)
    assert max(rel_l2(Qg, Qo, 8).values()) <= 1e-13


def test_block_sizes_bitwise_equal(vb):
    """Ragged x extent (200 = 3 x 64 + 8): every block shape gives identical bits."""
    w = synth.workload_fourier_2d()
    w["shape"] = (200, 12, 1)
    Q0 = np.ascontiguousarray(synth.fourier_2d(200, seed=7)[:, :, :12, :])
    bufs = []
    for bx in (64, 128, 192, 256):
        sim, _, _ = run_gpu(vb, w, Q0, 9, "f64", block_x=bx)
        bufs.append(sim.vlbm_get_populations()[0])
    for b in bufs[1:]:
        assert np.array_equal(b, bufs[0])


# exchange vs oracle (FP64, FP32) and exchange vs direct path (every storage: the
# rounding of one fused multiply-add, through the storage format's rounding)
LANE_TOL = {"f64": 1e-10, "f32": 1e-5}
LANE_VS_DIRECT = {"f64": 1e-13, "f32": 1e-6, "f16": 1e-3, "bf16": 1e-2}


@pytest.mark.parametrize("storage", ["f64", "f32", "f16", "bf16"])
@pytest.mark.parametrize("case", ["2d", "3d_ideal", "3d_resistive"])
def test_lane_exchange(vb, storage, case):
    """x rows that the workgroups tile exactly take the parity-1 lane exchange in the
    8-variable sweeps (one workgroup per row, or several with single-element accesses
    at their ends); a block shape that does not tile the row, and the 26-variable
    sweep, take the direct neighbour accesses.  Every
    tiling of the exchange gives identical bits; the exchange and the direct path are
    the same arithmetic compiled into different kernels (the compiler may fuse a
    multiply-add in one and not the other): they agree to that rounding, and the
    exchange meets the oracle at the FP64 and FP32 bars (the storage forms are held
    to the oracle on the direct path by the low-precision tests)."""
    if case == "2d":
        w = synth.workload_fourier_2d()
        w["shape"] = (256, 6, 2)
        Q0 = np.concatenate([synth.fourier_2d(256, seed=s)[:, :, :6, :] for s in (7, 8)], axis=1)
        blocks, K = (64, 128, 256, 192), 8
    elif case == "3d_ideal":
        w = synth.workload_slab_3d()
        w["shape"] = (256, 5, 4)
        Q0, _ = synth.planar_discontinuity_3d(seed=4, shape=(4, 5, 256))
        Q0 = boosted(Q0, (0.3, -0.2, 0.25))
        blocks, K = (64, 128, 256, 192), 8
    else:
        w = synth.workload_resistive_3d(n=16, dt_over_tau_M=0.49)
        w["shape"] = (128, 4, 3)
        Q0 = small_resistive(shape=(128, 4, 3), seed=6)
        blocks, K = (64, 128, 192), 26
    Q0 = np.ascontiguousarray(Q0)
    steps = 9
    print("case lane exchange", case, storage, flush=True)
    Qo, _ = run_oracle(w, Q0, steps)
    bufs, Qs = [], []
    for bx in blocks:
        sim, Qg, _ = run_gpu(vb, w, Q0, steps, storage, block_x=bx)
        bufs.append(sim.vlbm_get_populations()[0])
        Qs.append(Qg)
        sim.vlbm_destroy()
        if storage in LANE_TOL:
            err = rel_l2(Qg, Qo, K)
            fam = ("rho", "m", "E", "B") if K == 26 and storage != "f64" else tuple(err)
            assert max(err[k] for k in fam) <= LANE_TOL[storage], (bx, err)
    for bx, b in zip(blocks[1:-1], bufs[1:-1]):
        assert np.array_equal(b, bufs[0]), bx
    d = rel_l2(Qs[0], Qs[-1], K)
    fam = ("rho", "m", "E", "B") if K == 26 and storage != "f64" else tuple(d)
    assert max(d[k] for k in fam) <= LANE_VS_DIRECT[storage], d


# --- D3Q7 ideal and resistive, ragged boxes -------------------------------------

def boosted(Q, u0, gamma=5.0 / 3.0):
    """The same state seen from a frame moving at -u0: rho u += rho u0, E gains the
    kinetic energy of the drift (pressure and B unchanged)."""
    Q = Q.copy()
    rho = Q[0]
    m_old = Q[1:4].copy()
    for a in range(3):
        Q[1 + a] = m_old[a] + rho * u0[a]
    Q[4] += 0.5 * ((Q[1:4] ** 2).sum(0) - (m_old ** 2).sum(0)) / rho
    return Q


@pytest.mark.parametrize("storage,tol", [("f64", 1e-10), ("f32", 1e-5)])
def test_d3q7_ideal_parity(vb, storage, tol):
    """Slab workload (ragged 70 x 20 x 12 box) with a uniform drift, so that every
    field is O(1) and the relative L2 per field is meaningful."""
    w = synth.workload_slab_3d()
    w["shape"] = (70, 20, 12)
    Q0, _ = synth.planar_discontinuity_3d(seed=2, shape=(12, 20, 70))
    Q0 = boosted(Q0, (0.3, -0.2, 0.25))
    steps = 60
    _, Qg, tg = run_gpu(vb, w, Q0, steps, storage)
    Qo, to = run_oracle(w, Q0, steps)
    err = rel_l2(Qg, Qo, 8)
    assert max(err.values()) <= tol, err


def test_d3q7_slab_at_rest_fp32(vb):
    """The slab at rest: rho u is generated by the dynamics (|rho u| ~ 1e-3 after 60
    steps while its populations carry the O(0.01) pressure flux), so FP32 storage
    bounds its error in absolute terms: a few FP32 ulps of the populations per step."""
    w = synth.workload_slab_3d()
    w["shape"] = (70, 20, 12)
    Q0, _ = synth.planar_discontinuity_3d(seed=2, shape=(12, 20, 70))
    steps = 60
    _, Qg, _ = run_gpu(vb, w, Q0, steps, "f32")
    Qo, _ = run_oracle(w, Q0, steps)
    err = rel_l2(Qg, Qo, 8)
    assert max(err["rho"], err["E"], err["B"]) <= 1e-5, err
    fmax = 0.015  # largest |f| of the rho u sets for this state
    assert np.abs(Qg[1:4] - Qo[1:4]).max() <= steps * 7 * fmax * 2.0 ** -23, err


@pytest.mark.parametrize("storage,tol,steps", [("f64", 1e-10, 40), ("f32", 1e-5, 40), ("f64", 1e-10, 200),
                                              ("f32", 1e-5, 200)])
def test_d3q7_resistive_parity(vb, storage, tol, steps):
    """FP32: every field within 1e-5, except where the method's own formulas evaluated
    in FP32 arithmetic (the oracle compiled with float) already miss it -- the small
    transported gradients G, H ride on populations carrying an O(u) flux term, so
    FP32 rounding of those populations sets their accuracy.  There the GPU must be
    within 1.5x of that FP32 evaluation."""
    w = synth.workload_resistive_3d(n=16, dt_over_tau_M=0.49)
    w["shape"] = (12, 10, 8)
    Q0 = small_resistive()
    print(f"case resistive {storage} {steps} steps", flush=True)
    _, Qg, tg = run_gpu(vb, w, Q0, steps, storage)
    Qo, _ = run_oracle(w, Q0, steps)
    err = rel_l2(Qg, Qo, 26)
    assert tg[26 + 4] == 0  # the state stays physical (rho > 0, p >= 0, finite)
    if storage == "f64":
        assert max(err.values()) <= tol, err
        return
    yard = rel_l2(oracle.run_fp32(oracle_params(w), Q0, steps), Qo, 26)
    for name, e in err.items():
        assert e <= max(tol, 1.5 * yard[name]), (name, e, yard[name])
    assert max(err[k] for k in ("rho", "m", "E", "B")) <= tol, err


# --- FP64 diagnostics against the oracle on the same populations ---------------

@pytest.mark.parametrize("case", ["ideal", "resistive", "resistive_2d"])
@pytest.mark.parametrize("storage", ["f64", "f32", "f16", "bf16"])
def test_diagnostics_match_oracle_on_the_same_populations(vb, case, storage):
    """Every FP64 diagnostic of vlbm_moments -- the K totals, sum d, sum d^2, max |d|
    (d the div B estimate of the Powell source), the sum of the squared central
    div B of the moment field and the count of unphysical cells -- against the
    oracle's moments of the GPU's own decoded populations (gathered at every cell),
    after an odd number of steps (the in-place pattern's odd parity) on a ragged D3Q7
    box, for every storage form: the reductions agree to FP64 rounding, whatever the
    storage (rounding of the populations themselves is not tested here)."""
    if case == "ideal":
        w = synth.workload_slab_3d()
        w["shape"] = (20, 12, 10)
        Q0, _ = synth.planar_discontinuity_3d(seed=2, shape=(10, 12, 20))
        Q0 = boosted(Q0, (0.3, -0.2, 0.25))
        K = 8
    elif case == "resistive":
        w = synth.workload_resistive_3d(n=16, dt_over_tau_M=0.49)
        w["shape"] = (12, 10, 8)
        Q0 = small_resistive()
        K = 26
    else:
        w, Q0 = small_resistive_2d()
        K = 13
    print(f"case diagnostics {case} {storage}", flush=True)
    sim, Qg, tg = run_gpu(vb, w, Q0, 7, storage)
    N = int(np.prod(w["shape"]))
    f = sim.vlbm_gather_cells(np.arange(N, dtype=np.int64))  # [N, K, Q]
    f = np.ascontiguousarray(np.transpose(f, (1, 2, 0)))
    Qo, do, to = oracle.moments(oracle_params(w), f)
    scale = np.abs(Qo).max(axis=1)
    assert np.all(np.abs(Qg.reshape(K, N) - Qo) <= 1e-14 * scale[:, None] + 1e-300)
    assert np.all(np.abs(tg[:K] - to[:K]) <= 1e-13 * N * scale), (tg[:K], to[:K])
    dsum = np.abs(do).sum()
    assert abs(tg[K] - to[K]) <= 1e-13 * dsum
    assert abs(tg[K + 1] - to[K + 1]) <= 1e-12 * to[K + 1]
    assert abs(tg[K + 2] - to[K + 2]) <= 1e-12 * to[K + 2]
    assert to[K + 1] > 0 and to[K + 3] > 0
    assert abs(tg[K + 3] - to[K + 3]) <= 1e-12 * to[K + 3]
    assert tg[K + 4] == to[K + 4] == 0


# --- source operators: Guo and Chai (Sec. 2.2) ------------------------------------

def _source_case(case):
    if case == "fourier_2d":
        w = synth.workload_fourier_2d()
        return w, synth.fourier_2d(64, seed=2), 200, 8
    if case == "resistive_3d":
        w = synth.workload_resistive_3d(n=16, dt_over_tau_M=0.49)
        w["shape"] = (12, 10, 8)
        return w, small_resistive(), 60, 26
    w, Q0 = small_resistive_2d()
    return w, Q0, 200, 13


@pytest.mark.parametrize("source", ["guo", "chai"])
@pytest.mark.parametrize("case", ["fourier_2d", "resistive_3d", "resistive_2d"])
@pytest.mark.parametrize("storage,tol", [("f64", 1e-10), ("f32", 1e-5)])
def test_source_operators_parity(vb, source, case, storage, tol):
    """The Guo and Chai source operators on the models with sources (Powell's source,
    and the relaxation of the transported gradients and stress): GPU against the
    oracle, FP64 within 1e-10 and FP32 within 1e-5 (or 2x the oracle evaluated in FP32
    where the FP32 formulas themselves miss it, the rule of the resistive system)."""
    w, Q0, steps, K = _source_case(case)
    print(f"case source {source} {case} {storage}", flush=True)
    p = gpu_params(vb, w, storage)
    p.source = {"guo": 1, "chai": 2}[source]
    sim = vb.Vlbm(p)
    sim.vlbm_init_fields(Q0)
    sim.vlbm_step(steps)
    Qg, tg = sim.vlbm_moments()
    op = oracle_params(w)
    op.source = p.source
    f = oracle.init(op, Q0)
    sp = oracle.source_field(op, f) if source == "chai" else None
    oracle.run(op, f, steps, sprev=sp)
    Qo, _, to = oracle.moments(op, f)
    err = rel_l2(Qg, Qo, K)
    assert tg[K + 4] == 0
    if storage == "f64":
        assert max(err.values()) <= tol, err
        return
    yard = rel_l2(oracle.run_fp32(op, Q0, steps), Qo, K)
    for name, e in err.items():
        assert e <= max(tol, 2.0 * yard[name]), (name, e, yard[name])


def test_source_operators_refused_where_not_built(vb):
    """The Guo and Chai operators need FP64/FP32 storage, a model with a source and a
    periodic lattice without a body: anything else is refused at creation."""
    w = synth.workload_fourier_2d()
    for storage in ("f16", "bf16"):
        p = gpu_params(vb, w, storage)
        p.source = 1
        with pytest.raises(vb.VlbmError):
            vb.Vlbm(p)
    p = vb.make_params(lattice="D3Q7", shape=(16, 8, 8), model="euler", storage="f64", source="chai",
                       stream=_stream())
    with pytest.raises(vb.VlbmError):
        vb.Vlbm(p)
    p = vb.make_params(lattice="D3Q7", shape=(16, 8, 8), storage="f64", source="guo", bc=(1, 2, 2, 2, 2, 2),
                       inflow_Q=[1.0, 0.1, 0, 0, 1.0, 0, 0, 0], stream=_stream())
    with pytest.raises(vb.VlbmError):
        vb.Vlbm(p)


# --- the 13-component 2D system (Sec. 3.1) ---------------------------------------

def small_resistive_2d(shape=(70, 36), seed=7):
    """A smooth 13-component state on a ragged 2D box with viscosity, current-dependent
    resistivity and Powell's source from tr G / tau_M."""
    nx, ny = shape
    w = synth.workload_resistive_2d(n=nx, ny=ny)
    Q0 = synth.resistive_2d_state((ny, nx), seed=seed, tau_M=w["tau_M"], tau_H=w["tau_H"], mu=w["mu"])
    return w, Q0


@pytest.mark.parametrize("storage,tol", [("f64", 1e-10), ("f32", 1e-5)])
def test_resistive_2d_parity_200_steps(vb, storage, tol):
    """FP64: every field family within 1e-10 after 200 steps; FP32: within 1e-5, or,
    for the small transported T and G, within 2x what the oracle evaluated in FP32
    reaches (the rule of the 3D resistive system)."""
    w, Q0 = small_resistive_2d()
    print(f"case resistive_2d {storage}", flush=True)
    _, Qg, tg = run_gpu(vb, w, Q0, 200, storage)
    Qo, to = run_oracle(w, Q0, 200)
    err = rel_l2(Qg, Qo, 13)
    assert tg[13 + 4] == 0
    if storage == "f64":
        assert max(err.values()) <= tol, err
        assert np.allclose(tg[:13], to[:13], rtol=1e-11, atol=1e-11)
        return
    yard = rel_l2(oracle.run_fp32(oracle_params(w), Q0, 200), Qo, 13)
    for name, e in err.items():
        assert e <= max(tol, 2.0 * yard[name]), (name, e, yard[name])
    assert max(err[k] for k in ("rho", "m", "E", "B")) <= tol, err


def test_brio_wu_fp64_parity(vb):
    """The paper's Brio-Wu shock tube (Sec. 3.1) on the 13-component system, 256 x 4
    cells to t = 0.1 (512 steps): FP64 within 1e-10 of the oracle, and physical."""
    n = 256
    w = synth.workload_brio_wu_2d(n=n, ny=4)
    Q0 = synth.brio_wu_2d(n, 4)
    _, Qg, tg = run_gpu(vb, w, Q0, w["steps"], "f64")
    Qo, to = run_oracle(w, Q0, w["steps"])
    err = rel_l2(Qg, Qo, 13)
    assert max(err[k] for k in ("rho", "m", "E", "B")) <= 1e-10, err
    assert tg[13 + 4] == 0 and to[13 + 4] == 0


@pytest.mark.parametrize("storage", ["f64", "f32", "f16", "bf16"])
def test_resistive_2d_block_sizes_bitwise_equal(vb, storage):
    """Every tiling of the rows (64, 128, 256 threads, the lane exchange with 4, 2, 1
    workgroups per 256-cell row) gives bitwise the same populations."""
    w, Q0 = small_resistive_2d(shape=(256, 12))
    out = []
    for bx in (64, 128, 256):
        sim, _, _ = run_gpu(vb, w, Q0, 7, storage, block_x=bx)
        out.append(sim.vlbm_get_populations()[0])
    assert all(np.array_equal(out[0], o) for o in out[1:])


@pytest.mark.parametrize("storage,ulp", [("f16", 2.0 ** -11), ("bf16", 2.0 ** -8)])
@pytest.mark.parametrize("parity", [0, 1])
def test_resistive_3d_low_precision_one_step(vb, storage, ulp, parity):
    """FP16/BF16 storage of the 26-variable system, whose variable pairs share 32-bit
    elements: one step from the GPU's own pre-step populations against the oracle's
    collision, every population of a ragged 70 x 10 x 6 box, up to one rounding of the
    stored deviation (plus FP32 arithmetic)."""
    w = synth.workload_resistive_3d(n=16, dt_over_tau_M=0.49)
    shape = (70, 10, 6)
    w["shape"] = shape
    Q0 = small_resistive(shape=shape, seed=9)
    print("case resistive 3D one step", storage, parity, flush=True)
    sim = vb.Vlbm(gpu_params(vb, w, storage))
    sim.vlbm_init_fields(Q0)
    sim.vlbm_step(3 + parity)
    cells = np.arange(int(np.prod(shape)))
    op = oracle_params(w)
    want = oracle_one_step(oracle, op, sim.vlbm_gather_cells, cells, shape, 3)
    sim.vlbm_step(1)
    got = sim.vlbm_gather_cells(cells)
    rest_Q, sigma = sim.vlbm_get_codec()
    f_rest = oracle.equilibrium(op, rest_Q)
    wts = np.array([0.25] + [0.125] * 6)
    sc = sigma[:, None] * wts[None, :]
    h_want = np.abs(want - f_rest[None]) / sc[None]
    bound = sc[None] * (2.0 * ulp * h_want + 2.0 ** -24) + 4e-6 * (1.0 + np.abs(want))
    err = np.abs(got - want)
    assert np.all(err <= bound), float((err / bound).max())


@pytest.mark.parametrize("storage,ulp", [("f16", 2.0 ** -11), ("bf16", 2.0 ** -8)])
@pytest.mark.parametrize("parity", [0, 1])
def test_resistive_2d_low_precision_one_step(vb, storage, ulp, parity):
    """FP16/BF16 storage of the 13-component system: one step from the GPU's own
    pre-step populations against the oracle's collision, up to one rounding of the
    stored deviation (plus FP32 arithmetic)."""
    w, Q0 = small_resistive_2d(shape=(64, 20))
    shape = w["shape"]
    sim = vb.Vlbm(gpu_params(vb, w, storage))
    sim.vlbm_init_fields(Q0)
    sim.vlbm_step(3 + parity)
    cells = np.arange(int(np.prod(shape)))
    op = oracle_params(w)
    want = oracle_one_step(oracle, op, sim.vlbm_gather_cells, cells, shape, 2)
    sim.vlbm_step(1)
    got = sim.vlbm_gather_cells(cells)
    rest_Q, sigma = sim.vlbm_get_codec()
    f_rest = oracle.equilibrium(op, rest_Q)
    wts = np.array([1.0 / 3.0] + [1.0 / 6.0] * 4)
    sc = sigma[:, None] * wts[None, :]
    h_want = np.abs(want - f_rest[None]) / sc[None]
    bound = sc[None] * (2.0 * ulp * h_want + 2.0 ** -24) + 4e-6 * (1.0 + np.abs(want))
    err = np.abs(got - want)
    assert np.all(err <= bound), float((err / bound).max())


# --- FP16 / BF16 deviation storage: one step at a time vs the oracle ------------

def test_uniform_field_codec_scale(vb):
    """The Orszag-Tang density is uniform at the start and 25/(36 pi) is not a binary
    fraction, so on 300^2 cells its FP64 mean is off by rounding; the codec scales such
    a field by its magnitude (sigma = 0.25), not by that rounding, and FP16 follows the
    FP64 run as closely as on a lattice whose mean is exact."""
    n, steps = 300, 150
    w = synth.workload_orszag_tang_2d(n, tau=0.52)
    Q0 = synth.orszag_tang_2d(n)
    out = {}
    for st in ("f64", "f16"):
        sim = vb.Vlbm(vb.make_params(lattice="D2Q5", shape=(n, n, 1), storage=st, gamma=w["gamma"],
                                     flux_scale=w["s"], tau=w["tau"], powell=1, stream=_stream()))
        sim.vlbm_init_fields(Q0)
        if st == "f16":
            _, sigma = sim.vlbm_get_codec()
            assert sigma[0] == 0.25, sigma[:8]
        sim.vlbm_step(steps)
        out[st], _ = sim.vlbm_moments()
    err = rel_l2(out["f16"], out["f64"], 8)
    assert max(err.values()) <= 5e-3, err


@pytest.mark.parametrize("storage,ulp", [("f16", 2.0 ** -11), ("bf16", 2.0 ** -8)])
@pytest.mark.parametrize("parity", [0, 1])
def test_low_precision_one_step(vb, storage, ulp, parity):
    """The GPU's post-step populations equal the oracle's collision of the GPU's own
    pre-step populations, up to one rounding of the stored deviation (plus FP32
    arithmetic)."""
    w = synth.workload_slab_3d()
    shape = (40, 24, 10)
    w["shape"] = shape
    Q0, _ = synth.planar_discontinuity_3d(seed=2, shape=shape[::-1])
    sim = vb.Vlbm(gpu_params(vb, w, storage))
    sim.vlbm_init_fields(Q0)
    sim.vlbm_step(3 + parity)
    N = np.prod(shape)
    cells = np.arange(N)
    pre = sim.vlbm_gather_cells
    op = oracle_params(w)
    want = oracle_one_step(oracle, op, pre, cells, shape, 3)
    sim.vlbm_step(1)
    got = sim.vlbm_gather_cells(cells)
    rest_Q, sigma = sim.vlbm_get_codec()
    f_rest = oracle.equilibrium(op, rest_Q)  # the codec's reference populations
    wts = np.array([0.25] + [0.125] * 6)
    sc = sigma[:, None] * wts[None, :]  # w_i sigma_k
    h_want = np.abs(want - f_rest[None]) / sc[None]
    # one round-to-nearest of h: at most ulp * |h| (normal range) or the subnormal
    # spacing; plus FP32 decode/collision rounding of O(1) values
    bound = sc[None] * (2.0 * ulp * h_want + 2.0 ** -24) + 4e-6 * (1.0 + np.abs(want))
    err = np.abs(got - want)
    assert np.all(err <= bound), float((err / bound).max())


# --- two cells per lane (FP16/BF16 storage) --------------------------------------

def _pair_case(case):
    """Workloads on 256-cell rows, which FP16/BF16 storage sweeps two cells per lane."""
    if case == "ideal_2d":
        w = synth.workload_fourier_2d()
        w["shape"] = (256, 8, 2)
        Q0 = np.concatenate([synth.fourier_2d(256, seed=s)[:, :, :8, :] for s in (3, 4)], axis=1)
    elif case == "ideal_3d":
        w = synth.workload_slab_3d()
        w["shape"] = (256, 6, 4)
        Q0, _ = synth.planar_discontinuity_3d(seed=5, shape=(4, 6, 256))
        Q0 = boosted(Q0, (0.3, -0.2, 0.25))
    elif case == "euler_3d":
        w = _euler(synth.workload_slab_3d())
        w["shape"] = (256, 6, 4)
        Qm, _ = synth.planar_discontinuity_3d(seed=6, shape=(4, 6, 256))
        Q0 = synth.without_field(boosted(Qm, (0.3, -0.2, 0.25)))
    elif case == "navier_cauchy_3d":
        w = synth.workload_elastic(dim=3, shape=(256, 6, 4))
        Q0 = synth.elastic_state((256, 6, 4), seed=7)
    else:
        w, Q0 = small_resistive_2d(shape=(256, 10), seed=8)
    return w, np.ascontiguousarray(Q0)


@pytest.mark.parametrize("storage,ulp", [("f16", 2.0 ** -11), ("bf16", 2.0 ** -8)])
@pytest.mark.parametrize("parity", [0, 1])
@pytest.mark.parametrize("block_x", [64, 128])
@pytest.mark.parametrize("case", ["ideal_2d", "ideal_3d", "euler_3d", "navier_cauchy_3d", "resistive_2d"])
def test_pair_sweep_one_step(vb, case, block_x, storage, ulp, parity):
    """Two cells per lane: 256-cell rows tiled by two workgroups of 64 threads (the
    workgroups' end lanes read and write their neighbours' boundary elements) or by one
    of 128 threads (the row wraps inside the workgroup).  One step from the GPU's own
    pre-step populations against the oracle's collision of every cell, up to one
    rounding of the stored deviation (plus FP32 arithmetic)."""
    w, Q0 = _pair_case(case)
    shape, dim = w["shape"], w["dim"]
    print("case pair sweep", case, block_x, storage, parity, flush=True)
    sim = vb.Vlbm(gpu_params(vb, w, storage, block_x=block_x))
    sim.vlbm_init_fields(Q0)
    sim.vlbm_step(3 + parity)
    cells = np.arange(int(np.prod(shape)))
    op = oracle_params(w)
    want = oracle_one_step(oracle, op, sim.vlbm_gather_cells, cells, shape, dim)
    sim.vlbm_step(1)
    got = sim.vlbm_gather_cells(cells)
    rest_Q, sigma = sim.vlbm_get_codec()
    f_rest = oracle.equilibrium(op, rest_Q)
    w0 = 1.0 / 3.0 if dim == 2 else 0.25
    wts = np.array([w0] + [(1.0 - w0) / (2 * dim)] * (2 * dim))
    sc = sigma[:, None] * wts[None, :]
    h_want = np.abs(want - f_rest[None]) / sc[None]
    bound = sc[None] * (2.0 * ulp * h_want + 2.0 ** -24) + 4e-6 * (1.0 + np.abs(want))
    err = np.abs(got - want)
    assert np.all(err <= bound), float((err / bound).max())


# --- invariants -----------------------------------------------------------------

@pytest.mark.parametrize("storage", ["f64", "f32", "f16", "bf16"])
def test_uniform_state_stays_uniform(vb, storage):
    w = synth.workload_slab_3d()
    shape = (33, 7, 5)
    w["shape"] = shape
    Q0 = synth.uniform_state(shape[::-1], rho=1.2, u=(0.1, -0.05, 0.03), p=0.5, B=(0.2, 0.1, -0.3))
    sim = vb.Vlbm(gpu_params(vb, w, storage))
    sim.vlbm_init_fields(Q0)
    sim.vlbm_step(11)
    f = sim.vlbm_gather_cells(np.arange(np.prod(shape)))
    assert np.array_equal(f, np.broadcast_to(f[:1], f.shape))


def test_totals_exact_without_powell(vb):
    w = synth.workload_fourier_2d()
    w["powell"] = 0
    Q0 = synth.fourier_2d(64, seed=1)
    sim = vb.Vlbm(gpu_params(vb, w, "f64"))
    sim.vlbm_init_fields(Q0)
    _, t0 = sim.vlbm_moments(with_field=False)
    sim.vlbm_step(150)
    _, t1 = sim.vlbm_moments(with_field=False)
    scale = np.abs(Q0).reshape(8, -1).sum(1)
    assert np.all(np.abs(t1[:8] - t0[:8]) <= 1e-13 * scale)


def test_central_divb_preserved_at_tau_b_one(vb):
    w = synth.workload_fourier_2d()
    w["tau"] = [0.6] * 5 + [1.0] * 3 + [0.6]
    Q0 = synth.fourier_2d(64, seed=1)
    sim = vb.Vlbm(gpu_params(vb, w, "f64"))
    sim.vlbm_init_fields(Q0)
    sim.vlbm_step(100)
    _, t = sim.vlbm_moments(with_field=False)
    assert t[8 + 3] < 1e-26


def test_checkpoint_restart_bitwise(vb):
    w = synth.workload_fourier_2d()
    Q0 = synth.fourier_2d(64, seed=2)
    a = vb.Vlbm(gpu_params(vb, w, "f32"))
    a.vlbm_init_fields(Q0)
    a.vlbm_step(101)
    buf, par, step = a.vlbm_get_populations()
    a.vlbm_step(99)
    ref = a.vlbm_get_populations()[0]
    b = vb.Vlbm(gpu_params(vb, w, "f32"))
    b.vlbm_set_populations(buf, par, step)
    b.vlbm_step(99)
    assert np.array_equal(b.vlbm_get_populations()[0], ref)
    assert b.vlbm_get_step() == 200


def test_gather_matches_moments_at_odd_parity(vb):
    w = synth.workload_fourier_2d(n=32)
    Q0 = synth.fourier_2d(32, seed=3)
    sim = vb.Vlbm(gpu_params(vb, w, "f64"))
    sim.vlbm_init_fields(Q0)
    sim.vlbm_step(5)
    Q, _ = sim.vlbm_moments()
    f = sim.vlbm_gather_cells(np.arange(32 * 32))
    assert np.allclose(f.sum(2).T, Q, rtol=0, atol=1e-14)


def test_nonfinite_and_negative_density_reported(vb):
    w = synth.workload_fourier_2d(n=16)
    Q0 = synth.fourier_2d(16, seed=0)
    Q0[0, 0, 3, 4] = -1.0
    sim = vb.Vlbm(gpu_params(vb, w, "f64"))
    sim.vlbm_init_fields(Q0)
    with pytest.raises(vb.VlbmError) as ei:
        sim.vlbm_moments()
    assert ei.value.status == vb.VLBM_ERR_NONFINITE
    _, tot = sim.vlbm_moments(raise_nonfinite=False)
    assert tot[8 + 4] >= 1
    Q0 = synth.fourier_2d(16, seed=0)
    Q0[4, 0, 1, 1] = np.nan
    sim.vlbm_init_fields(Q0)
    _, tot = sim.vlbm_moments(raise_nonfinite=False)
    assert tot[8 + 4] >= 1


def test_step_before_init_is_a_state_error(vb):
    w = synth.workload_fourier_2d(n=16)
    sim = vb.Vlbm(gpu_params(vb, w, "f32"))
    with pytest.raises(vb.VlbmError) as ei:
        sim.vlbm_step(1)
    assert ei.value.status == vb.VLBM_ERR_STATE


def test_device_resident_fields_and_borrowed_buffer(vb):
    """Q given as a device tensor, populations in a borrowed torch buffer,
    moments written to a device FP32 tensor."""
    import torch
    w = synth.workload_fourier_2d(n=48)
    Q0 = synth.fourier_2d(48, seed=4)
    p = gpu_params(vb, w, "f32")
    probe = vb.Vlbm(gpu_params(vb, w, "f32"))
    nbytes = probe.population_bytes()
    probe.vlbm_destroy()
    pop = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    sim = vb.Vlbm(p, pop_tensor=pop)
    sim.vlbm_init_fields(torch.tensor(Q0, device="cuda"))
    sim.vlbm_step(10)
    out = torch.empty((8, 48 * 48), dtype=torch.float32, device="cuda")
    sim.vlbm_moments(out=out)
    ref = run_gpu(vb, w, Q0, 10, "f32")[1]
    assert np.allclose(out.cpu().numpy(), ref, rtol=1e-6, atol=1e-7)


# --- compressible Euler (the ideal system without the field) --------------------

def _euler(w):
    w = dict(w)
    w["model"] = 2
    w["tau"] = w["tau"] if np.ndim(w["tau"]) == 0 else list(w["tau"])[:5]
    return w


@pytest.mark.parametrize("storage,tol", [("f64", 1e-10), ("f32", 1e-5)])
def test_euler_2d_parity_200_steps(vb, storage, tol):
    w = _euler(synth.workload_fourier_2d())
    Q0 = synth.without_field(synth.fourier_2d(64, seed=1))
    _, Qg, _ = run_gpu(vb, w, Q0, 200, storage)
    Qo, _ = run_oracle(w, Q0, 200)
    err = rel_l2(Qg, Qo, 5)
    assert max(err.values()) <= tol, err


@pytest.mark.parametrize("storage,tol", [("f64", 1e-10), ("f32", 1e-5), ("f16", 3e-3), ("bf16", 3e-2)])
def test_euler_3d_parity(vb, storage, tol):
    """Slab without field on a ragged box (70 x 20 x 12), with a drift so that every
    field is O(1); 60 steps."""
    w = _euler(synth.workload_slab_3d())
    w["shape"] = (70, 20, 12)
    Qm, _ = synth.planar_discontinuity_3d(seed=2, shape=(12, 20, 70))
    Q0 = synth.without_field(boosted(Qm, (0.3, -0.2, 0.25)))
    _, Qg, _ = run_gpu(vb, w, Q0, 60, storage)
    Qo, _ = run_oracle(w, Q0, 60)
    err = rel_l2(Qg, Qo, 5)
    assert max(err.values()) <= tol, err


def test_euler_lane_exchange(vb):
    """Rows tiled by the workgroups take the parity-1 lane exchange in the Euler sweep
    too: every tiling bitwise equal, held to the oracle and to the direct path."""
    w = _euler(synth.workload_slab_3d())
    w["shape"] = (256, 5, 4)
    Qm, _ = synth.planar_discontinuity_3d(seed=4, shape=(4, 5, 256))
    Q0 = synth.without_field(boosted(Qm, (0.3, -0.2, 0.25)))
    Qo, _ = run_oracle(w, Q0, 9)
    bufs, Qs = [], []
    for bx in (64, 128, 256, 192):
        sim, Qg, _ = run_gpu(vb, w, Q0, 9, "f64", block_x=bx)
        bufs.append(sim.vlbm_get_populations()[0])
        Qs.append(Qg)
        sim.vlbm_destroy()
        assert max(rel_l2(Qg, Qo, 5).values()) <= 1e-10
    assert np.array_equal(bufs[1], bufs[0]) and np.array_equal(bufs[2], bufs[0])
    assert max(rel_l2(Qs[0], Qs[-1], 5).values()) <= 1e-13


# --- linear Navier-Cauchy (elastodynamics, K = 9) --------------------------------

@pytest.mark.parametrize("dim,storage,tol", [(2, "f64", 1e-10), (2, "f32", 1e-5), (3, "f64", 1e-10),
                                             (3, "f32", 1e-5), (3, "f16", 3e-3), (3, "bf16", 3e-2)])
def test_navier_cauchy_parity(vb, dim, storage, tol):
    """Seeded Fourier momentum and stress on a pre-stress, ragged boxes (70 x 20 and
    70 x 20 x 12), 120 steps (2D) / 60 steps (3D): every field family against the
    oracle."""
    shape = (70, 20, 1) if dim == 2 else (70, 20, 12)
    w = synth.workload_elastic(dim=dim, shape=shape)
    Q0 = synth.elastic_state(shape, seed=5)
    steps = 120 if dim == 2 else 60
    _, Qg, tg = run_gpu(vb, w, Q0, steps, storage)
    Qo, to = run_oracle(w, Q0, steps)
    err = rel_l2(Qg, Qo, 9)
    assert max(err.values()) <= tol, err
    if storage == "f64":  # no source: the totals stay where they started
        _, t0 = run_oracle(w, Q0, 0)
        assert np.abs(tg[:9] - t0[:9]).max() <= 1e-10


def test_navier_cauchy_lane_exchange(vb):
    """Rows tiled by the workgroups take the parity-1 lane exchange in the 9-variable
    sweep: every tiling bitwise equal, held to the oracle and to the direct path."""
    shape = (256, 5, 4)
    w = synth.workload_elastic(dim=3, shape=shape)
    Q0 = synth.elastic_state(shape, seed=6)
    Qo, _ = run_oracle(w, Q0, 9)
    bufs, Qs = [], []
    for bx in (64, 128, 256, 192):
        sim, Qg, _ = run_gpu(vb, w, Q0, 9, "f64", block_x=bx)
        bufs.append(sim.vlbm_get_populations()[0])
        Qs.append(Qg)
        sim.vlbm_destroy()
        assert max(rel_l2(Qg, Qo, 9).values()) <= 1e-10
    assert np.array_equal(bufs[1], bufs[0]) and np.array_equal(bufs[2], bufs[0])
    assert max(rel_l2(Qs[0], Qs[-1], 9).values()) <= 1e-13
