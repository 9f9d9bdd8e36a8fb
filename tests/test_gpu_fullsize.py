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
