"""The learned coarse correction, end to end at a reduced size: pairs from batched
fine runs (128^2 -> 32^2, r = 4), training on the GPU (one round of pairs taken on
the corrected run's own states), and a held-out comparison against the restricted
fine run, where the corrected coarse run must beat the plain coarse VLBM and its own
base operator."""
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
    X, Y = Lr.generate_pairs(list(range(100, 108)), 128, 4, 80, w, synth.fourier_2d, kmax=4)
    in_mean, in_std, out_mean, out_std, y_l2, drift = Lr.normalisation(X, Y)
    net = N.Net(8, 32, 4, stream=torch.cuda.current_stream().cuda_stream)
    net.vlbm_nn_set_weights(Lr.init_weights(seed=0))
    net.vlbm_nn_set_norm(in_mean, in_std, out_mean, out_std)
    losses, _ = Lr.train(net, X, Y, 600, 1e-3, seed=0)
    assert losses[-1][1] < losses[0][1]
    # one round of pairs on the corrected run's own states
    Xr, Yr = Lr.rollout_pairs(net, X, 4, w, 5.0 * y_l2 * np.sqrt(8), 0.1, 5.0 * drift, stride=2)
    Lr.train(net, torch.cat([X, Xr]), torch.cat([Y, Yr]), 600, 5e-4, seed=1)
    eval_seeds = [900, 901, 902, 903]
    bound = 5.0 * y_l2 * np.sqrt(len(eval_seeds))
    hist, nfb = Lr.evaluate(net, eval_seeds, 128, 4, 200, w, synth.fourier_2d, bound, 0.1, 5.0 * drift, kmax=4,
                            checkpoints=2)
    plain = sum(hist[-1]["plain"].values())
    learned = sum(hist[-1]["learned"].values())
    print("plain", hist[-1]["plain"], "learned", hist[-1]["learned"], "base", hist[-1]["base"], "fallbacks", nfb,
          flush=True)
    base = sum(hist[-1]["base"].values())
    assert learned < plain and learned < base


def test_zero_network_is_the_plain_restart_step():
    """With all weights zero (and zero output mean) the correction is exactly zero, so a
    corrected step is the plain coarse step from the equilibrium of the current moments --
    the operator the training targets are taken against: equal to init + one step (up to
    FP32 rounding of the two launch paths), step after step, and no fallbacks."""
    import torch
    torch.cuda.set_device(0)
    from paper_2606_00641_amd import learned as Lr
    from paper_2606_00641_amd import nn as N

    w = synth.workload_fourier_2d()
    s = torch.cuda.current_stream().cuda_stream
    X0 = torch.from_numpy(Lr.initial_batch([3, 4], 32, 4, synth.fourier_2d)).cuda()
    net = N.Net(8, 32, 4, stream=s)
    net.vlbm_nn_set_weights(np.zeros(net.vlbm_nn_num_params(), np.float32))
    net.vlbm_nn_set_norm(np.zeros(8), np.ones(8), np.zeros(8), np.ones(8))
    a = Lr.make_context((32, 32), 2, "f32", w, s)
    b = Lr.make_context((32, 32), 2, "f32", w, s)
    a.vlbm_init_fields(X0)
    Q = X0.clone()
    for step in range(3):
        nfb = N.vlbm_step_corrected(a, net, 1, np.full(8, 1e30), 1e30, 1e30)
        assert nfb == 0
        b.vlbm_init_fields(Q)
        b.vlbm_step(1)
        b.vlbm_moments(out=Q)
        qa = torch.empty_like(Q)
        a.vlbm_moments(out=qa)
        err = float(((qa - Q).abs().max() / Q.abs().max()).item())
        assert err < 1e-6, (step, err)
