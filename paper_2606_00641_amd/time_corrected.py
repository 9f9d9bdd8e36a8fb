"""Wall time of the corrected coarse step on one lattice (2D 256^2 or 3D 64^3, FP32),
with the network at its initial weights and the gate wide open -- the kernel mix the
learned studies time, for profiling.

Usage: python -m paper_2606_00641_amd.time_corrected [--dim 2|3] [--warm N] [--steps N]
"""
import argparse
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--dim", type=int, default=2, choices=(2, 3))
    ap.add_argument("--warm", type=int, default=100)
    ap.add_argument("--steps", type=int, default=400)
    args = ap.parse_args()
    import torch
    import synth
    from paper_2606_00641_amd import learned as Lr
    from paper_2606_00641_amd import nn as N
    from paper_2606_00641_amd import study_learned_3d as S3

    torch.cuda.set_device(0)
    s = torch.cuda.current_stream().cuda_stream
    net = N.Net(8, 32, 4, stream=s, dim=args.dim)
    net.vlbm_nn_set_weights(Lr.init_weights(seed=0, dim=args.dim))
    if args.dim == 2:
        sim = Lr.make_context((256, 256), 1, "f32", synth.workload_fourier_2d(), s)
        sim.vlbm_init_fields(torch.from_numpy(Lr.initial_batch([900], 256, 16, synth.fourier_2d)).cuda())
        what = "2D 256^2"
    else:
        sim = Lr.make_context_3d(64, "f32", S3.workload(), s)
        sim.vlbm_init_fields(Lr._state_3d(lambda n, seed: synth.turbulence_3d(n=n, seed=seed)[:8], 64, 900))
        what = "3D 64^3"
    wide = np.full(8, 1e30)
    N.vlbm_step_corrected(sim, net, args.warm, wide, 10.0, 1.0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    N.vlbm_step_corrected(sim, net, args.steps, wide, 10.0, 1.0)
    torch.cuda.synchronize()
    print(f"corrected {what} step: {(time.perf_counter() - t0) / args.steps * 1e6:.1f} us", flush=True)


if __name__ == "__main__":
    main()
