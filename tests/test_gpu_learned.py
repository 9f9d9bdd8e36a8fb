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
    plain = sum(hist[-1]["plain"].values())
    learned = sum(hist[-1]["learned"].values())
    print("plain", hist[-1]["plain"], "learned", hist[-1]["learned"], "fallbacks", nfb, flush=True)
    assert learned < plain


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

