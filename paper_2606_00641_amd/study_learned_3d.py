"""Learned coarse correction on 3D lattices: periodic ideal-MHD turbulence on fine
128^3 lattices (D3Q7 x 8, FP32), restricted 2x to 64^3, gives the teacher-forced
training pairs of a 4-layer 3x3x3 network with 32 channels; the corrected 64^3 run
is scored against the restricted fine run on held-out seeds next to the plain coarse
run, and the wall time of the plain FP32 fine run is compared with that of the
corrected coarse run.  --coarse-storage f16 / bf16 runs the plain and corrected coarse
lattices with FP16/BF16 deviation storage (the network is trained on FP32 pairs).

Usage: python -m paper_2606_00641_amd.study_learned_3d [--out FILE] [--iters N] [--quick]
       [--coarse-storage f32|f16|bf16]
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
    print("[learned3d]", *a, flush=True)


def workload(s=0.1, tau=0.55):
    """Periodic 3D ideal MHD: flux scale 0.1 keeps s (|u| + c_fast) near 0.13 below
    c_s^2 = 1/4 for u_rms = B_rms = 0.05 at rho = 1, p = 0.6."""
    return dict(dim=3, model=0, s=s, gamma=5.0 / 3.0, tau=tau, powell=1)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(ROOT, "gpurun_out", "learned_coarse_3d.json"))
    ap.add_argument("--iters", type=int, default=3000)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--quick", action="store_true", help="small sizes (smoke)")
    ap.add_argument("--seed", type=int, default=0, help="seed of the initial weights and of the training order")
    ap.add_argument("--tau", type=float, default=0.55)
    ap.add_argument("--coarse-storage", default="f32", choices=["f64", "f32", "f16", "bf16"],
                    help="storage form of the plain and corrected coarse runs (pairs, training and the "
                         "fine reference stay FP32)")
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
        n_fine, seeds, pairs, eval_seeds, steps = 64, list(range(100, 102)), 50, [900], 200
    else:
        n_fine, seeds, pairs, eval_seeds, steps = 128, list(range(100, 108)), 250, [900, 901], 2000
    r = 2
    w = workload(tau=args.tau)

    def make_state(n, seed):
        return synth.turbulence_3d(n=n, seed=seed)[:8]

    t0 = time.perf_counter()
    X, Y = Lr.generate_pairs_3d(seeds, n_fine, r, pairs, w, make_state, log=log)
    t_pairs = time.perf_counter() - t0
    log(f"{pairs * len(seeds)} pairs in {t_pairs:.1f} s")
    in_mean, in_std, out_mean, out_std, y_l2, drift = Lr.normalisation(X, Y)
    b_abs = 5.0 * drift
    net = N.Net(8, 32, 4, stream=torch.cuda.current_stream().cuda_stream, dim=3)
    net.vlbm_nn_set_weights(Lr.init_weights(seed=args.seed, dim=3))
    net.vlbm_nn_set_norm(in_mean, in_std, out_mean, out_std)
    losses, t_train = Lr.train(net, X, Y, args.iters, args.lr, seed=args.seed, log=log)
    del X, Y
    torch.cuda.empty_cache()
    bound = args.bound_factor * y_l2  # one lattice per context
    cst = args.coarse_storage
    hist, nfb = Lr.evaluate_3d(net, eval_seeds, n_fine, r, steps, w, make_state, bound, 0.1, b_abs, checkpoints=10,
                               log=log, coarse_storage=cst)
    t_fine, t_learned, nfb_t = Lr.time_runs_3d(net, n_fine, r, steps, w, make_state, bound, 0.1, b_abs,
                                               coarse_storage=cst)
    nc = n_fine // r
    res = dict(
        workload=f"3D ideal MHD D3Q7 x 8, periodic turbulence (u_rms = B_rms = 0.05, modes 1 <= |k| <= 8), "
                 f"fine {n_fine}^3 -> coarse {nc}^3 (r = {r}), tau = {w['tau']}, s = {w['s']}, fine run FP32 "
                 f"storage, coarse runs {cst.upper()} storage",
        coarse_storage=cst,
        train_seeds=[seeds[0], seeds[-1]], pairs=pairs * len(seeds), seed=args.seed, projected=True,
        eval_seeds=eval_seeds, coarse_steps=steps,
        network="4 x conv3x3x3, 8-32-32-32-8, GELU, BF16 MFMA / FP32 accumulate, Adam lr %g, %d iterations "
                "(batch 1 lattice)" % (args.lr, args.iters),
        time_pairs_s=round(t_pairs, 2), time_train_s=round(t_train, 2), losses=losses,
        bound_factor=args.bound_factor, bound_corr=list(map(float, bound)), bound_divb_rel=0.1,
        bound_divb_abs=b_abs, history=hist, fallbacks=nfb,
        wall_fine_s=round(t_fine, 4), wall_learned_coarse_s=round(t_learned, 4),
        speedup_vs_fine=round(t_fine / t_learned, 2), fallbacks_timed_run=nfb_t)
    log(json.dumps({k: res[k] for k in ("speedup_vs_fine", "fallbacks", "wall_fine_s", "wall_learned_coarse_s")}))
    log("final errors", json.dumps(hist[-1]))
    os.makedirs(os.path.dirname(args.out), exist_ok=True)
    with open(args.out, "w") as fh:
        json.dump(res, fh, indent=1)


if __name__ == "__main__":
    main()
