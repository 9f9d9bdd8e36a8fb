"""Stability record of the resistive 3D turbulence workload at its full size: the
256^3 periodic lattice (D3Q7 x 26 variables, FP32 storage, Re = Rm = 400, tau_LB =
1/2 + 5 % of the viscous diffusion) run for its configured 1000 steps, with the
library's FP64 diagnostics every `--every` steps: the count of unphysical cells
(rho <= 0, p < 0 or a non-finite moment), the totals of rho, rho u, E and B, the
L2 norm of the central div B, and (from the moment field) the smallest density and
pressure, the largest speed, and the kinetic and magnetic energies.

Usage: python -m paper_2606_00641_amd.study_stability [--n 256] [--steps 1000] [--every 100]
       [--out profiles/stability_resistive_256.json]
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--every", type=int, default=100)
    ap.add_argument("--out", default=None)
    args = ap.parse_args()
    import torch
    import synth
    from paper_2606_00641_amd import vlbm as V

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    w = synth.workload_resistive_3d(n=args.n, steps=args.steps)
    n = args.n
    p = V.make_params(lattice="D3Q7", shape=(n, n, n), model="resistive", storage="f32", gamma=w["gamma"],
                      flux_scale=w["s"], tau=w["tau"], powell=w["powell"], divb_mode=w["divb_mode"], dt=w["dt"],
                      mu=w["mu"], eta0=w["eta0"], tau_M=w["tau_M"], tau_H=w["tau_H"], stream=stream.cuda_stream)
    sim = V.Vlbm(p)
    sim.vlbm_init_fields(torch.from_numpy(synth.turbulence_3d(n=n, seed=1, dtype=np.float32)).cuda())
    K, N = sim.K, sim.N
    Q = torch.empty((K, n, n, n), dtype=torch.float32, device="cuda")
    gm1 = w["gamma"] - 1.0
    rec = []

    def checkpoint(step):
        _, t = sim.vlbm_moments(out=Q, raise_nonfinite=False)
        rho, m, E, B = Q[0].double(), Q[1:4].double(), Q[4].double(), Q[5:8].double()
        ke = 0.5 * (m * m).sum(0) / rho
        me = 0.5 * (B * B).sum(0)
        pres = gm1 * (E - ke - me)
        r = dict(step=step, nbad=float(t[K + 4]), finite=bool(torch.isfinite(Q[:8]).all()),
                 rho_min=float(rho.min()), p_min=float(pres.min()),
                 u_max=float(((m * m).sum(0).sqrt() / rho).max()),
                 kinetic=float(ke.sum()) / N, magnetic=float(me.sum()) / N,
                 totals=[float(v) for v in t[:8]], divb_central_l2=float(t[K + 3]) ** 0.5)
        rec.append(r)
        print("[stability]", json.dumps(r), flush=True)

    checkpoint(0)
    t0 = time.time()
    done = 0
    while done < args.steps:
        k = min(args.every, args.steps - done)
        sim.vlbm_step(k)
        done += k
        checkpoint(done)
    out = dict(command="python -m paper_2606_00641_amd.study_stability --n %d --steps %d --every %d"
               % (n, args.steps, args.every),
               workload="resistive 3D turbulence, %d^3, D3Q7 x 26, FP32 storage, seed 1" % n,
               tau_lb=w["tau"], s=w["s"], dt=w["dt"], mu=w["mu"], eta0=w["eta0"], tau_M=w["tau_M"],
               wall_s=time.time() - t0, checkpoints=rec)
    if args.out:
        with open(args.out, "w") as fh:
            json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
