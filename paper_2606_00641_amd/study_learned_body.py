"""Learned coarse correction of the flow past the moving magnetised body: 3D ideal MHD
with an inflow face at x-, zero-gradient faces elsewhere and the homogenized rough body
of Sec. 2.4 (D3Q7 x 8, FP32), fine 768 x 384 x 384 restricted 2x to 384 x 192 x 192.

Training pairs come from fine runs past bodies of other seeds (other roughness and
dipole direction) -- or, with --train-seeds set to the evaluation seed, from the early
part of the evaluated run itself -- with the teacher-forced coarse run of the periodic
studies; the
coarse lattice carries the same body scaled by 1/2 (centre and radius halved, dipole
moment / 8 so that its field at the surface is unchanged, the same speed in cells per
step since one coarse step is two fine steps).  Faces and the body change the lattice
totals, so the correction is not projected onto zero totals.  The corrected and the
plain 384 x 192 x 192 runs past the benchmark's body are scored per field against the
restricted FP32 fine run, and the wall time of the corrected coarse run is compared
with that of the plain fine run over the same physical time.

Usage: python -m paper_2606_00641_amd.study_learned_body [--out FILE] [--quick]
       [--train-seeds 5,6,7] [--pairs N] [--pair-every K] [--iters N] [--eval-steps N]
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
    print("[learned-body]", *a, flush=True)


def coarse_body(body, r):
    """The body on the lattice restricted r times: same shape relative to its radius,
    the field at the same relative position unchanged (dipole moment / r^3), the same
    speed in cells per step (one coarse step is r fine steps of 1/r the cell size)."""
    b = dict(body)
    b["c0"] = [c / r for c in body["c0"]]
    b["R0"] = body["R0"] / r
    b["m"] = [m / r ** 3 for m in body["m"]]
    return b


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(ROOT, "gpurun_out", "learned_coarse_body.json"))
    ap.add_argument("--quick", action="store_true", help="192 x 96 x 96 fine lattice (smoke)")
    ap.add_argument("--pairs", type=int, default=480, help="teacher-forced coarse steps of each training run")
    ap.add_argument("--pair-every", type=int, default=8, help="keep every K-th pair")
    ap.add_argument("--iters", type=int, default=1500)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--eval-steps", type=int, default=1500,
                    help="coarse steps (the fine run takes twice as many; its FP32 run past the benchmark's body "
                         "keeps every cell physical to 3000 fine steps, not to 4000)")
    ap.add_argument("--checkpoints", type=int, default=10)
    ap.add_argument("--train-seeds", default="5,6,7", help="body seeds of the training runs")
    ap.add_argument("--eval-seed", type=int, default=4, help="body seed of the evaluation (the benchmark's body)")
    ap.add_argument("--bound-factor", type=float, default=5.0)
    args = ap.parse_args()
    import torch
    import synth
    from paper_2606_00641_amd import learned as Lr
    from paper_2606_00641_amd import nn as N
    from paper_2606_00641_amd import vlbm as V

    torch.cuda.set_device(0)
    s = torch.cuda.current_stream().cuda_stream
    r = 2
    fshape = (192, 96, 96) if args.quick else (768, 384, 384)
    cshape = tuple(n // r for n in fshape)
    if args.quick:
        args.pairs, args.pair_every, args.iters, args.eval_steps = 64, 4, 200, 200
    train_seeds = [int(x) for x in args.train_seeds.split(",")]
    w = synth.workload_body_3d(shape=fshape)
    Qin, info = synth.inflow_state()
    B_in = float(np.linalg.norm(info["B"]))
    R0 = 48.0 * fshape[0] / 768.0

    def body_of(seed):
        return synth.body_params(shape=fshape, seed=seed, R0=R0, B_in=B_in, mode=2)

    def ctx(shape, body, storage="f32"):
        return V.Vlbm(V.make_params(lattice="D3Q7", shape=shape, model="ideal", storage=storage, gamma=w["gamma"],
                                    flux_scale=w["s"], tau=w["tau"], powell=w["powell"], bc=w["bc"], inflow_Q=Qin,
                                    body=body, stream=s))

    Mf = torch.empty((8,) + fshape[::-1], dtype=torch.float32, device="cuda")
    cur = torch.empty((8,) + cshape[::-1], dtype=torch.float32, device="cuda")
    nxt, tgt, Cst = torch.empty_like(cur), torch.empty_like(cur), torch.empty_like(cur)

    # --- teacher-forced pairs past the training bodies
    t0 = time.perf_counter()
    per_seed = args.pairs // args.pair_every
    keep = per_seed * len(train_seeds)
    X = torch.empty((keep, 8, 1) + cshape[::-1], dtype=torch.float32, device="cuda")
    Y = torch.empty_like(X)
    j = 0
    for sd in train_seeds:
        bt = body_of(sd)
        fine = ctx(fshape, bt)
        fine.vlbm_init_fields(torch.from_numpy(synth.body_initial_state(fshape, bt, dtype=np.float32)).cuda())
        coarse = ctx(cshape, coarse_body(bt, r))
        fine.vlbm_moments(out=Mf, raise_nonfinite=False)
        N.vlbm_restrict(Mf, r, cur, stream=s)
        coarse.vlbm_init_fields(cur)
        for n in range(args.pairs):
            coarse.vlbm_step(1)
            coarse.vlbm_moments(out=Cst, raise_nonfinite=False)
            fine.vlbm_step(r)
            fine.vlbm_moments(out=Mf, raise_nonfinite=False)
            N.vlbm_restrict(Mf, r, nxt, stream=s)
            N.vlbm_restrict(Mf, r, tgt, minus=Cst, stream=s)
            N.vlbm_inject(coarse, tgt)
            if n % args.pair_every == args.pair_every - 1:
                X[j, :, 0].copy_(cur)
                Y[j, :, 0].copy_(tgt)
                j += 1
            cur, nxt = nxt, cur
        torch.cuda.synchronize()
        fine.vlbm_destroy()
        coarse.vlbm_destroy()
    t_pairs = time.perf_counter() - t0
    log(f"{keep} pairs (every {args.pair_every} of {args.pairs} coarse steps past bodies {train_seeds}) "
        f"in {t_pairs:.1f} s")

    in_mean, in_std, out_mean, out_std, y_l2, drift = Lr.normalisation(X, Y, sample=min(16, keep))
    net = N.Net(8, 32, 4, stream=s, dim=3)
    net.vlbm_nn_set_weights(Lr.init_weights(seed=0, dim=3))
    net.vlbm_nn_set_norm(in_mean, in_std, out_mean, out_std)
    losses, t_train = Lr.train(net, X, Y, args.iters, args.lr, seed=0, log=log)
    del X, Y
    torch.cuda.empty_cache()
    bound = args.bound_factor * y_l2
    b_abs = 5.0 * drift

    # --- evaluation past the benchmark's body
    be = body_of(args.eval_seed)
    Q0 = torch.from_numpy(synth.body_initial_state(fshape, be, dtype=np.float32)).cuda()
    fine = ctx(fshape, be)
    plain = ctx(cshape, coarse_body(be, r))
    learned = ctx(cshape, coarse_body(be, r))
    fine.vlbm_init_fields(Q0)
    fine.vlbm_moments(out=Mf, raise_nonfinite=False)
    N.vlbm_restrict(Mf, r, cur, stream=s)
    plain.vlbm_init_fields(cur)
    learned.vlbm_init_fields(cur)
    chunk = args.eval_steps // args.checkpoints
    hist, nfb, bad = [], 0, {}
    for c in range(args.checkpoints):
        fine.vlbm_step(r * chunk)
        plain.vlbm_step(chunk)
        nfb += N.vlbm_step_corrected(learned, net, chunk, bound, 0.1, b_abs, project_totals=False)
        fine.vlbm_moments(out=Mf, raise_nonfinite=False)
        N.vlbm_restrict(Mf, r, cur, stream=s)
        ref = cur.cpu().numpy().astype(np.float64)
        err = {}
        for name, cx in (("plain", plain), ("learned", learned)):
            q, tot = cx.vlbm_moments(raise_nonfinite=False)
            fs = Lr._family_sums(q.reshape(ref.shape), ref)
            err[name] = {k: float(np.sqrt(a / b)) for k, (a, b) in fs.items()}
            bad[name] = int(tot[-1])
        _, tf = fine.vlbm_moments(with_field=False, raise_nonfinite=False)
        bad["fine"] = int(tf[-1])
        hist.append(dict(coarse_step=(c + 1) * chunk, **err, unphysical_cells=dict(bad), fallbacks=nfb))
        log(f"step {(c + 1) * chunk}: plain {err['plain']} learned {err['learned']} fallbacks {nfb} "
            f"unphysical {bad}")
    for cx in (fine, plain, learned):
        cx.vlbm_destroy()
    del Q0
    torch.cuda.empty_cache()

    # --- wall time: plain fine run against the corrected coarse run, same physical time
    steps_t = min(args.eval_steps, 400)
    fine = ctx(fshape, be)
    learned = ctx(cshape, coarse_body(be, r))
    fine.vlbm_init_fields(torch.from_numpy(synth.body_initial_state(fshape, be, dtype=np.float32)).cuda())
    fine.vlbm_moments(out=Mf, raise_nonfinite=False)
    N.vlbm_restrict(Mf, r, cur, stream=s)
    learned.vlbm_init_fields(cur)
    fine.vlbm_step(2 * r)
    N.vlbm_step_corrected(learned, net, 2, bound, 0.1, b_abs, project_totals=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fine.vlbm_step(r * steps_t)
    torch.cuda.synchronize()
    t_fine = time.perf_counter() - t0
    t0 = time.perf_counter()
    nfb_t = N.vlbm_step_corrected(learned, net, steps_t, bound, 0.1, b_abs, project_totals=False)
    torch.cuda.synchronize()
    t_learned = time.perf_counter() - t0
    fine.vlbm_destroy()
    learned.vlbm_destroy()

    res = dict(
        workload=f"3D ideal MHD past the moving magnetised homogenized body (Mach 3 inflow at x-, zero-gradient "
                 f"faces), D3Q7 x 8, fine {fshape[0]}x{fshape[1]}x{fshape[2]} -> coarse {cshape[0]}x{cshape[1]}x"
                 f"{cshape[2]} (r = 2), tau = {w['tau']}, s = {w['s']}, FP32 storage; training body seeds "
                 f"{train_seeds}, evaluation body seed {args.eval_seed} (the benchmark's)",
        pairs=dict(coarse_steps=args.pairs, kept_every=args.pair_every, kept=keep), projected=False,
        network="4 x conv3x3x3, 8-32-32-32-8, GELU, BF16 MFMA / FP32 accumulate, Adam lr %g, %d iterations "
                "(batch 1 lattice)" % (args.lr, args.iters),
        time_pairs_s=round(t_pairs, 2), time_train_s=round(t_train, 2), losses=losses,
        gate="norms, div B drift, positivity of the corrected state (rho > 0, p >= 0)",
        bound_factor=args.bound_factor, bound_corr=list(map(float, bound)), bound_divb_rel=0.1,
        bound_divb_abs=float(b_abs), eval_coarse_steps=args.eval_steps, history=hist, fallbacks=nfb,
        timing=dict(coarse_steps=steps_t, wall_fine_fp32_s=round(t_fine, 4), wall_learned_coarse_s=round(t_learned, 4),
                    speedup_vs_fine_fp32=round(t_fine / t_learned, 2), fallbacks=nfb_t))
    log("final", json.dumps(hist[-1]), "speedup", res["timing"]["speedup_vs_fine_fp32"])
    os.makedirs(os.path.dirname(args.out), exist_ok=True)
    with open(args.out, "w") as fh:
        json.dump(res, fh, indent=1)


if __name__ == "__main__":
    main()
