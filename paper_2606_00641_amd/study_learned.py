"""Learned coarse correction on the 2D workload at full size: fine 1024^2 runs of 40
seeds restricted 4x to 256^2 give 20k training pairs; a 4-layer 3x3 network with 32
channels is trained on the GPU and the corrected 256^2 run is scored against the
restricted fine run over 5000 coarse steps on 10 held-out seeds, next to the plain
coarse run; the wall time of the plain FP32 fine run is compared with that of the
corrected coarse run.

Usage: python -m paper_2606_00641_amd.study_learned [--out FILE] [--iters N] [--quick]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def log(*a):
    print("[learned]", *a, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(ROOT, "gpurun_out", "learned_coarse_2d.json"))
    ap.add_argument("--iters", type=int, default=3000)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--quick", action="store_true", help="small sizes (smoke)")
    ap.add_argument("--noise", type=float, default=0.0, help="relative noise on the stored pairs' inputs")
    ap.add_argument("--stride", type=int, default=1, help="store every stride-th pair of the teacher-forced run")
    ap.add_argument("--no-project", action="store_true", help="do not project the correction to zero lattice totals")
    ap.add_argument("--seed", type=int, default=0, help="seed of the initial weights and of the training order")
    ap.add_argument("--bound-factor", type=float, default=5.0,
                    help="gate: fall back when a channel's correction norm exceeds this many times the RMS "
                         "norm of the training targets")
    args = ap.parse_args()
    import torch
    import synth
    from paper_2606_00641_amd import learned as Lr
    from paper_2606_00641_amd import nn as N

    torch.cuda.set_device(0)
    if args.quick:
        n_fine, seeds, pairs, eval_seeds, steps, kmax = 256, list(range(100, 108)), 100, [900, 901], 500, 4
    else:
        n_fine, seeds, pairs, eval_seeds, steps, kmax = 1024, list(range(100, 140)), 500, list(range(900, 910)), 5000, 16
    stride = args.stride
    r = 4
    w = synth.workload_fourier_2d()
    t0 = time.perf_counter()
    X, Y = Lr.generate_pairs(seeds, n_fine, r, pairs, w, synth.fourier_2d, kmax=kmax, stride=stride,
                             noise=args.noise, log=log)
    t_pairs = time.perf_counter() - t0
    log(f"{pairs * len(seeds)} pairs in {t_pairs:.1f} s")
    in_mean, in_std, out_mean, out_std, y_l2, drift = Lr.normalisation(X, Y)
    b_abs = 5.0 * drift
    net = N.Net(8, 32, 4, stream=torch.cuda.current_stream().cuda_stream)
    net.vlbm_nn_set_weights(Lr.init_weights(seed=args.seed))
    net.vlbm_nn_set_norm(in_mean, in_std, out_mean, out_std)
    losses, t_train = Lr.train(net, X, Y, args.iters, args.lr, seed=args.seed, log=log)
    del X, Y
    torch.cuda.empty_cache()
    bound = args.bound_factor * y_l2 * np.sqrt(len(eval_seeds))
    hist, nfb = Lr.evaluate(net, eval_seeds, n_fine, r, steps, w, synth.fourier_2d, bound, 0.1, b_abs, kmax=kmax,
                            checkpoints=10, log=log, project=not args.no_project)
    t_fine, t_learned, nfb_t = Lr.time_runs(net, n_fine, r, steps, w, synth.fourier_2d, y_l2 * args.bound_factor, 0.1, b_abs,
                                            kmax=kmax, project=not args.no_project)
    res = dict(
        workload=f"2D ideal MHD D2Q5 x 8, fine {n_fine}^2 -> coarse {n_fine // r}^2 (r = {r}), Fourier modes k <= {kmax}, "
                 f"tau = {w['tau']}, s = {w['s']}, FP32 storage",
        train_seeds=[seeds[0], seeds[-1]], pairs=pairs * len(seeds), pair_stride=stride, pair_noise=args.noise, seed=args.seed,
        projected=not args.no_project,
        eval_seeds=eval_seeds,
        coarse_steps=steps,
        network="4 x conv3x3, 8-32-32-32-8, GELU, BF16 MFMA / FP32 accumulate, Adam lr %g, %d iterations (batch %d lattices)"
                % (args.lr, args.iters, len(seeds)),
        time_pairs_s=round(t_pairs, 2), time_train_s=round(t_train, 2), losses=losses,
        bound_factor=args.bound_factor, bound_corr=list(map(float, bound)), bound_divb_rel=0.1, bound_divb_abs=b_abs, history=hist, fallbacks=nfb,
        wall_fine_s=round(t_fine, 4), wall_learned_coarse_s=round(t_learned, 4),
        speedup_vs_fine=round(t_fine / t_learned, 2), fallbacks_timed_run=nfb_t)
    log(json.dumps({k: res[k] for k in ("speedup_vs_fine", "fallbacks", "wall_fine_s", "wall_learned_coarse_s")}))
    log("final errors", json.dumps(hist[-1]))
    os.makedirs(os.path.dirname(args.out), exist_ok=True)
    with open(args.out, "w") as fh:
        json.dump(res, fh, indent=1)


if __name__ == "__main__":
    main()
