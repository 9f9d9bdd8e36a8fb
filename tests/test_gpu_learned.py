"""The learned coarse correction, end to end at a reduced size: pairs from batched
fine runs (128^2 -> 32^2, r = 4) with a teacher-forced coarse run, training on the
GPU, and a held-out comparison against the restricted fine run, where the corrected
coarse run must beat the plain coarse VLBM."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def test_learned_correction_beats_plain_coarse():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    from paper_2606_00641_amd import learned as Lr
    from paper_2606_00641_amd import nn as N

    w = synth.workload_fourier_2d()
    print("case learned pipeline 128^2 -> 32^2", flush=True)
    X, Y = Lr.generate_pairs(list(range(100, 108)), 128, 4, 80, w, synth.fourier_2d, kmax=4, stride=3)
    in_mean, in_std, out_mean, out_std, y_l2, drift = Lr.normalisation(X, Y)
    net = N.Net(8, 32, 4, stream=torch.cuda.current_stream().cuda_stream)
    net.vlbm_nn_set_weights(Lr.init_weights(seed=0))
    net.vlbm_nn_set_norm(in_mean, in_std, out_mean, out_std)
    losses, _ = Lr.train(net, X, Y, 600, 1e-3, seed=0)
    assert losses[-1][1] < losses[0][1]
    eval_seeds = [900, 901, 902, 903]
    bound = 5.0 * y_l2 * np.sqrt(len(eval_seeds))
    hist, nfb = Lr.evaluate(net, eval_seeds, 128, 4, 200, w, synth.fourier_2d, bound, 0.1, 5.0 * drift, kmax=4,
                            checkpoints=2)
    print("plain", hist[-1]["plain"], "learned", hist[-1]["learned"], "fallbacks", nfb, flush=True)
    for fam in ("rho", "m", "E", "B"):  # every field family, not only the sum
        assert hist[-1]["learned"][fam] < hist[-1]["plain"][fam], fam


def test_learned_correction_3d_beats_plain_coarse():
    """3D, the 3D study's training at a shorter horizon: teacher-forced pairs from periodic
    turbulence on 128^3 fine lattices restricted 2x to 64^3 (8 seeds x 250 pairs), the
    3x3x3 network trained on the GPU (3000 Adam iterations), then a held-out seed: after
    300 corrected coarse steps every field family is closer to the restricted fine run
    than the plain coarse run.  (With 4 x 150 pairs and 1500 iterations the density
    error was not reduced: the gain in rho needs the full training.)"""
    import torch
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    from paper_2606_00641_amd import learned as Lr
    from paper_2606_00641_amd import nn as N
    from paper_2606_00641_amd import study_learned_3d as S3

    w = S3.workload()

    def make_state(n, seed):
        return synth.turbulence_3d(n=n, seed=seed)[:8]

    print("case learned pipeline 128^3 -> 64^3", flush=True)
    X, Y = Lr.generate_pairs_3d(list(range(100, 108)), 128, 2, 250, w, make_state)
    in_mean, in_std, out_mean, out_std, y_l2, drift = Lr.normalisation(X, Y)
    net = N.Net(8, 32, 4, stream=torch.cuda.current_stream().cuda_stream, dim=3)
    net.vlbm_nn_set_weights(Lr.init_weights(seed=0, dim=3))
    net.vlbm_nn_set_norm(in_mean, in_std, out_mean, out_std)
    losses, _ = Lr.train(net, X, Y, 3000, 1e-3, seed=0)
    assert losses[-1][1] < losses[0][1]
    del X, Y
    torch.cuda.empty_cache()
    hist, nfb = Lr.evaluate_3d(net, [900], 128, 2, 300, w, make_state, 5.0 * y_l2, 0.1, 5.0 * drift, checkpoints=1)
    print("plain", hist[-1]["plain"], "learned", hist[-1]["learned"], "fallbacks", nfb, flush=True)
    for fam in ("rho", "m", "E", "B"):
        assert hist[-1]["learned"][fam] < hist[-1]["plain"][fam], fam


def test_teacher_forced_pairs_follow_the_fine_run():
    """The teacher-forced coarse run of the pair generation has the restricted fine
    moments after every step: injecting the target Y_n into P(f_n) gives X_{n+1}."""
    import torch
    torch.cuda.set_device(0)
    from paper_2606_00641_amd import learned as Lr
    from paper_2606_00641_amd import nn as N

    w = synth.workload_fourier_2d()
    s = torch.cuda.current_stream().cuda_stream
    seeds, n_fine, r, P = [7, 8], 64, 4, 6
    X, Y = Lr.generate_pairs(seeds, n_fine, r, P, w, synth.fourier_2d, kmax=4)
    coarse = Lr.make_context((16, 16), 2, "f32", w, s)
    coarse.vlbm_init_fields(X[0])
    Q = torch.empty_like(X[0])
    for n in range(P - 1):
        coarse.vlbm_step(1)
        N.vlbm_inject(coarse, Y[n])
        coarse.vlbm_moments(out=Q)
        err = float(((Q - X[n + 1]).abs().max() / X[n + 1].abs().max()).item())
        assert err < 1e-6, (n, err)

