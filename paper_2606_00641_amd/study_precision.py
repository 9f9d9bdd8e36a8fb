"""Precision study of the storage forms on the GPU: the same workload advanced in
lockstep with FP64, FP32, FP16-deviation and BF16-deviation storage; at checkpoints
the per-field relative L2 error of each form against the FP64 run, and each form's
throughput.

Cases:
  slab  3D ideal MHD, 512^3 periodic planar discontinuity, D3Q7 x 8, 2000 steps,
        checkpoints 500 / 1000 / 2000;
  ot    the paper's compressible Orszag-Tang vortex (Sec. 3.4), 4000^2, D2Q5 x 8,
        CFL 0.1 and tau = 0.5075, to t = 0.5 (20000 steps), checkpoints at t = 0.125,
        0.25, 0.5.

Usage: python -m paper_2606_00641_amd.study_precision --case slab|ot [--n N] [--collision bgk|trt|rlb]
       [--tau TAU] [--out FILE]
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

FAMILIES = {"rho": [0], "m": [1, 2, 3], "E": [4], "B": [5, 6, 7]}
FORMS = ("f64", "f32", "f16", "bf16")


def log(*a):
    print("[precision]", *a, flush=True)


def rel_errors(torch, Q, R):
    """Per field family ||Q - R|| / ||R|| (vectors as vectors); Q, R device [8, ...]."""
    out = {}
    for name, ks in FAMILIES.items():
        num = sum(float(((Q[k].double() - R[k]) ** 2).sum()) for k in ks)
        den = sum(float((R[k] ** 2).sum()) for k in ks)
        out[name] = float(np.sqrt(num / den))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--case", choices=("slab", "ot"), default="slab")
    ap.add_argument("--n", type=int, default=None)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--out", default=None)
    ap.add_argument("--collision", choices=("bgk", "trt", "rlb"), default="bgk")
    ap.add_argument("--tau", type=float, default=None)
    args = ap.parse_args()
    import torch
    import synth
    from paper_2606_00641_amd import vlbm as V

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    if args.case == "slab":
        n = args.n or 512
        w = synth.workload_slab_3d(n=n)
        steps = args.steps or 2000
        marks = [steps // 4, steps // 2, steps]
        Q0 = synth.planar_discontinuity_3d(n=n, seed=2, dtype=np.float64)[0]
        lattice, shape = "D3Q7", (n, n, n)
        desc = f"3D ideal MHD slab (planar discontinuity, seed 2), {n}^3 periodic, D3Q7 x 8, s = {w['s']}, tau = {w['tau']}"
    else:
        n = args.n or 4000
        w = synth.workload_orszag_tang_2d(n, tau=args.tau)
        steps = args.steps or w["steps"]
        marks = [steps // 4, steps // 2, steps]
        Q0 = synth.orszag_tang_2d(n)
        lattice, shape = "D2Q5", (n, n, 1)
        desc = (f"compressible Orszag-Tang vortex, {n}^2 periodic, D2Q5 x 8, s = {w['s']}, tau = {w['tau']}, "
                f"{args.collision.upper()} collision")
    log(desc)
    Qd = torch.from_numpy(np.ascontiguousarray(Q0)).cuda()
    del Q0
    sims = {}
    for st in FORMS:
        p = V.make_params(lattice=lattice, shape=shape, model="ideal", storage=st, gamma=w["gamma"], flux_scale=w["s"],
                          tau=w["tau"], powell=w["powell"], collision=args.collision, stream=stream.cuda_stream)
        sims[st] = V.Vlbm(p)
        sims[st].vlbm_init_fields(Qd)
    del Qd
    torch.cuda.empty_cache()
    N = int(np.prod(shape))
    ref = torch.empty((8, N), dtype=torch.float64, device="cuda")
    tmp = torch.empty((8, N), dtype=torch.float32, device="cuda")
    timing = {st: 0.0 for st in FORMS}
    hist = []
    done = 0
    for mark in marks:
        chunk = mark - done
        for st in FORMS:
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            sims[st].vlbm_step(chunk)
            e1.record(stream)
            torch.cuda.synchronize()
            timing[st] += e0.elapsed_time(e1) / 1e3
        done = mark
        _, tref = sims["f64"].vlbm_moments(out=ref, raise_nonfinite=False)
        rec = dict(step=mark, nbad_f64=float(tref[-1]))
        for st in FORMS[1:]:
            _, t = sims[st].vlbm_moments(out=tmp, raise_nonfinite=False)
            rec[st] = rel_errors(torch, tmp, ref)
            rec[st]["nbad"] = float(t[-1])
        hist.append(rec)
        log(json.dumps(rec))
    perf = {}
    esize = {"f64": 8, "f32": 4, "f16": 2, "bf16": 2}
    Qn = 7 if lattice == "D3Q7" else 5
    for st in FORMS:
        mlups = N * steps / timing[st] / 1e6
        perf[st] = dict(mlups=round(mlups, 1), GBps=round(mlups * 1e6 * 2 * 8 * Qn * esize[st] / 1e9, 1))
    log(json.dumps(perf))
    res = dict(case=args.case, workload=desc, steps=steps, checkpoints=hist, throughput=perf,
               note="errors are per-field relative L2 against the FP64 GPU run of the same workload")
    out = args.out or os.path.join(ROOT, "gpurun_out", f"precision_{args.case}_{args.collision}.json")
    os.makedirs(os.path.dirname(out), exist_ok=True)
    with open(out, "w") as fh:
        json.dump(res, fh, indent=1)


if __name__ == "__main__":
    main()
