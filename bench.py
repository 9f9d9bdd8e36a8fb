#!/usr/bin/env python3
"""Benchmark of the VLBM MHD sweep on one MI355X.

One step = one full collide-and-stream sweep of the lattice (gather, decode,
moments, equation of state, fluxes, div B estimate, Powell source, BGK with
direct injection, encode, scatter).  The default workload is the 3D resistive
MHD lattice: 256^3 cells, D3Q7 population sets for 26 variables, FP32 storage and
arithmetic, periodic.  Inputs are synthetic (seeded random solenoidal fields) and
resident in HBM before timing starts.

Prints ONE JSON line on stdout: throughput in million lattice updates per second
(MLUPS), the HBM roofline of the sweep kernel (algorithmic bytes per cell update
/ measured kernel time vs 8 TB/s), the same sweep in FP16/BF16 deviation storage
on the 512^3 ideal-MHD slab workload next to FP32, and the FP64 CPU oracle's
throughput on a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
BF16_PEAK_TFLOPS = 2500.0  # dense BF16 matrix-core peak
CSRC = os.path.join(ROOT, "paper_2606_00641_amd", "csrc")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_counters.json")

from paper_2606_00641_amd.pmc_traffic import kernel_source_hash  # noqa: E402


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


MODEL_NAMES = {0: "ideal", 1: "resistive", 2: "euler", 3: "navier_cauchy", 4: "resistive_2d"}
MODEL_K = {0: 8, 1: 26, 2: 5, 3: 9, 4: 13}


def params_for(vlbm, w, storage, stream):
    return vlbm.make_params(lattice="D3Q7" if w["dim"] == 3 else "D2Q5", shape=w["shape"],
                            model=MODEL_NAMES[w["model"]], storage=storage,
                            gamma=w["gamma"], flux_scale=w["s"], tau=w["tau"], powell=w["powell"],
                            divb_mode=w["divb_mode"], dt=w["dt"], mu=w["mu"], eta0=w["eta0"], j_c=w.get("j_c", 0.0),
                            tau_M=w["tau_M"], tau_H=w["tau_H"], bc=w.get("bc"), inflow_Q=w.get("inflow_Q"),
                            body=w.get("body"), stream=stream)


def time_sweep(vlbm, torch, w, Q_dev, storage, steps, warmup, segments=10):
    """Returns dict(wall_s, kernel_ms, kernel_ms_std, ncell, bytes_per_cell, finite):
    the timed steps run as `segments` equal segments bracketed by HIP events on the
    library's stream (kernel_ms: mean per step; kernel_ms_std: spread of the segment
    means), the wall clock around all of them."""
    stream = torch.cuda.current_stream()
    sim = vlbm.Vlbm(params_for(vlbm, w, storage, stream.cuda_stream))
    sim.vlbm_init_fields(Q_dev)
    sim.vlbm_step(warmup)
    torch.cuda.synchronize()
    segments = max(1, min(segments, steps))
    bounds = [round(steps * j / segments) for j in range(segments + 1)]
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(segments + 1)]
    t0 = time.perf_counter()
    ev[0].record(stream)
    for j in range(segments):
        sim.vlbm_step(bounds[j + 1] - bounds[j])
        ev[j + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    seg_ms = [ev[j].elapsed_time(ev[j + 1]) / (bounds[j + 1] - bounds[j]) for j in range(segments)]
    kernel_ms = ev[0].elapsed_time(ev[-1]) / steps
    _, tot = sim.vlbm_moments(with_field=False, raise_nonfinite=False)
    ncell = int(np.prod(w["shape"]))
    K = MODEL_K[w["model"]]
    Qd = 2 * w["dim"] + 1
    esize = {"f64": 8, "f32": 4, "f16": 2, "bf16": 2}[storage]
    sim.vlbm_destroy()
    return dict(wall_s=wall, kernel_ms=kernel_ms, kernel_ms_std=float(np.std(seg_ms)), ncell=ncell,
                bytes_per_cell=2 * K * Qd * esize, finite=bool(np.all(np.isfinite(tot)) and tot[K + 4] == 0))


def copy_bandwidth(vlbm, torch, nbytes=4 << 30, reps=10):
    """GB/s (read + write) of the library's streaming copy kernel on nbytes."""
    src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    stream = torch.cuda.current_stream()
    vlbm.vlbm_copy_kernel(dst, src, stream.cuda_stream)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        vlbm.vlbm_copy_kernel(dst, src, stream.cuda_stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    torch.cuda.empty_cache()
    return 2.0 * nbytes / (ms * 1e-3) / 1e9


def copy_ceiling(vlbm, torch, reps=10):
    """The practical HBM ceiling from several copies: the library's streaming copy
    kernel (16 bytes per lane) at 1, 4 and 16 GiB, and the runtime's device-to-device
    copy (torch copy_, a hipMemcpyAsync) at 4 and 16 GiB; GB/s counting read + write."""
    out = {}
    for gib in (1, 4, 16):
        out[f"library_copy_kernel_{gib}GiB"] = round(copy_bandwidth(vlbm, torch, gib << 30, reps), 1)
    stream = torch.cuda.current_stream()
    for gib in (4, 16):
        src = torch.empty((gib << 30) // 4, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            dst.copy_(src)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        out[f"device_to_device_memcpy_{gib}GiB"] = round(2.0 * (gib << 30) / (ms * 1e-3) / 1e9, 1)
        del src, dst
        torch.cuda.empty_cache()
    out["max"] = max(out.values())
    return out


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def _oracle_rate(oracle, op, Q0, ncell, target_s, max_steps=None):
    """MLUPS of the oracle on one workload: one step to size the run, then as many
    steps as fit in target_s (at least 2)."""
    f = oracle.init(op, Q0)
    t0 = time.perf_counter()
    oracle.run(op, f, 1)
    per = time.perf_counter() - t0
    steps = max(2, int(target_s / max(per, 1e-6)))
    if max_steps:
        steps = min(steps, max_steps)
    t0 = time.perf_counter()
    oracle.run(op, f, steps)
    el = time.perf_counter() - t0
    return dict(mlups=round(ncell * steps / el / 1e6, 4), steps=steps, seconds=round(el, 2))


def cpu_baseline(target_s=10.0):
    """The FP64 oracle (as it stands, OpenMP) timed on the host: the resistive D3Q7 x 26
    recipe on a 48^3 lattice (a bounded sample of the benchmark's workload) on all the
    threads the oracle runs with and on one; the 2D ideal-MHD workload (64^2, D2Q5 x 8,
    200 steps) in full; a 128^3 slice of the slab workload (D3Q7 x 8)."""
    import oracle
    import synth
    threads = oracle.num_threads()
    n = 48
    # the same lattice parameters as the 256^3 workload (dt / tau_M = 0.49)
    w = synth.workload_resistive_3d(n=n, dt_over_tau_M=0.49)
    Q0 = synth.turbulence_3d(n=n, seed=1, kmax=8, tau_M=w["tau_M"], tau_H=w["tau_H"])
    op = oracle.make_params(dim=3, shape=w["shape"], model=1, gamma=w["gamma"], s=w["s"], tau=w["tau"],
                            powell=w["powell"], divb_mode=w["divb_mode"], dt=w["dt"], mu=w["mu"],
                            eta0=w["eta0"], tau_M=w["tau_M"], tau_H=w["tau_H"])
    res_all = _oracle_rate(oracle, op, Q0, n ** 3, target_s)
    w0 = synth.workload_fourier_2d()
    Q2 = synth.fourier_2d(64, seed=0)
    op2 = oracle.make_params(dim=2, shape=(64, 64, 1), tau=w0["tau"], s=w0["s"])
    ws = synth.workload_slab_3d()
    Qs, _ = synth.planar_discontinuity_3d(n=128, seed=2)
    ops = oracle.make_params(dim=3, shape=(128, 128, 128), tau=ws["tau"], s=ws["s"])
    samples = {}
    try:
        for label, nt in (("all_threads", threads), ("one_thread", 1)):
            oracle.set_threads(nt)
            res = res_all if nt == threads else _oracle_rate(oracle, op, Q0, n ** 3, target_s / 2)
            c0 = _oracle_rate(oracle, op2, Q2, 64 * 64, 1e9, max_steps=200)  # config 0 in full: 200 steps
            sl = _oracle_rate(oracle, ops, Qs, 128 ** 3, 1e9, max_steps=10 if nt > 1 else 2)
            samples[label] = {"threads": nt, "resistive_48_d3q7x26": res, "fourier_64_d2q5x8_200_steps": c0,
                              "slab_128_d3q7x8": sl}
    finally:
        oracle.set_threads(threads)
    return dict(value=res_all["mlups"], unit="MLUPS", cores=threads, kind="oracle",
                sample=f"FP64 oracle, resistive MHD D3Q7 x 26 variables, {n}^3 lattice (same recipe and lattice "
                       f"parameters scaled to {n}^3), {res_all['steps']} steps, {res_all['seconds']:.1f} s, "
                       f"{threads} threads",
                cpu_model=_cpu_model(), host_cpus=len(os.sched_getaffinity(0)), samples=samples)


def traffic_for(workload_key, storage):
    """HBM bytes per sweep launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel sources; else None."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("kernel_hash") != kernel_source_hash():
        return None
    rec = t.get("records", {}).get(f"{workload_key}/{storage}")
    if not rec:
        return None
    return rec["bytes_per_launch"]


def run_slab(vlbm, torch, synth, form_steps, only=False):
    """512^3 ideal-MHD slab in FP32, FP16 and BF16 storage."""
    forms = {}
    ws = synth.workload_slab_3d(n=512)
    log("generating the 512^3 slab workload")
    Qs = torch.from_numpy(synth.planar_discontinuity_3d(n=512, seed=2, dtype=np.float32)[0]).cuda()
    for st in ("f32", "f16", "bf16"):
        rr = time_sweep(vlbm, torch, ws, Qs, st, form_steps, 5)
        m = rr["ncell"] * form_steps / rr["wall_s"] / 1e6
        gb = rr["bytes_per_cell"] * rr["ncell"] / (rr["kernel_ms"] * 1e-3) / 1e9
        forms[st] = dict(mlups=round(m, 1), kernel_ms=round(rr["kernel_ms"], 4),
                         bytes_per_cell=rr["bytes_per_cell"], achieved_GBps=round(gb, 1),
                         frac_of_peak=round(gb / HBM_PEAK_GBPS, 4), finite=rr["finite"])
        log(f"slab 512^3 {st}: {m:.1f} MLUPS, {gb:.0f} GB/s")
    del Qs
    torch.cuda.empty_cache()
    for st in ("f16", "bf16"):
        forms[st]["speedup_vs_f32"] = round(forms[st]["mlups"] / forms["f32"]["mlups"], 3)
    if only:  # alone, the form also times the copy kernel (the reference of the HBM counters)
        forms["measured_copy_GBps"] = round(copy_bandwidth(vlbm, torch), 1)
    return forms


RESISTIVE_FAMILIES = {"rho": [0], "m": [1, 2, 3], "E": [4], "B": [5, 6, 7], "G": list(range(8, 17)),
                      "H": list(range(17, 26))}


def run_resistive_storage(vlbm, torch, w, Q, r32, form_steps, err_steps=200):
    """The benchmark's own workload (resistive 256^3, D3Q7 x 26) in FP16 and BF16 deviation
    storage: the sweep's MLUPS and GB/s against the FP32 form timed just before (r32), and
    the error of each field family after err_steps steps against the same run in FP64
    storage (the GPU's FP64 path, held to the oracle at 1e-10): ||Q - Q_64|| / ||Q_64|| per
    family (vector families as vectors), FP64 norms on the host of the FP32 moment fields."""
    stream = torch.cuda.current_stream()

    def moments_after(storage):
        sim = vlbm.Vlbm(params_for(vlbm, w, storage, stream.cuda_stream))
        sim.vlbm_init_fields(Q)
        sim.vlbm_step(err_steps)
        q, tot = sim.vlbm_moments(f32=True, raise_nonfinite=False)
        sim.vlbm_destroy()
        torch.cuda.empty_cache()
        return q, tot

    log(f"resistive 256^3: FP64 reference run of {err_steps} steps")
    ref, _ = moments_after("f64")
    den = {f: float(np.sqrt(sum(np.sum(ref[k].astype(np.float64) ** 2) for k in ks)))
           for f, ks in RESISTIVE_FAMILIES.items()}
    out = {"error_steps": err_steps}
    for st in ("f32", "f16", "bf16"):
        q, tot = moments_after(st)
        err = {}
        for f, ks in RESISTIVE_FAMILIES.items():
            num = np.sqrt(sum(np.sum((q[k].astype(np.float64) - ref[k]) ** 2) for k in ks))
            err[f] = float(num / den[f]) if den[f] > 0 else float(num)
        del q
        entry = {"rel_l2_vs_fp64": err, "finite": bool(np.all(np.isfinite(tot)) and tot[26 + 4] == 0)}
        if st != "f32":
            rr = time_sweep(vlbm, torch, w, Q, st, form_steps, 5)
            m = rr["ncell"] * form_steps / rr["wall_s"] / 1e6
            gb = rr["bytes_per_cell"] * rr["ncell"] / (rr["kernel_ms"] * 1e-3) / 1e9
            entry.update(mlups=round(m, 1), kernel_ms=round(rr["kernel_ms"], 4), bytes_per_cell=rr["bytes_per_cell"],
                         achieved_GBps=round(gb, 1), frac_of_peak=round(gb / HBM_PEAK_GBPS, 4),
                         speedup_vs_f32=round(r32["kernel_ms"] / rr["kernel_ms"], 3))
            log(f"resistive 256^3 {st}: {m:.1f} MLUPS, {gb:.0f} GB/s, error vs FP64 {err}")
        else:
            log(f"resistive 256^3 f32: error vs FP64 {err}")
        out[st] = entry
    del ref
    return out


def run_models(vlbm, torch, synth, form_steps):
    """The other PDEs through the same sweep, 256^3 periodic, FP32: compressible Euler
    (K = 5, the resistive workload's state without its field) and linear Navier-Cauchy
    elastodynamics (K = 9, seeded Fourier momentum and stress on a pre-stress)."""
    out = {}
    n = 256
    Qe = synth.without_field(synth.turbulence_3d(n=n, seed=1)[:8]).astype(np.float32)
    we = dict(dim=3, shape=(n, n, n), model=2, s=0.1, gamma=5.0 / 3.0, tau=0.6, powell=0, divb_mode=0,
              dt=0.0, mu=0.0, eta0=0.0, tau_M=1.0, tau_H=1.0)
    wn = synth.workload_elastic(dim=3, shape=(n, n, n))
    log("generating the 256^3 Euler and Navier-Cauchy states")
    Qn = synth.elastic_state((n, n, n), seed=5).astype(np.float32)
    for name, w, Qh in (("euler_256", we, Qe), ("navier_cauchy_256", wn, Qn)):
        Qd = torch.from_numpy(Qh).cuda()
        rr = time_sweep(vlbm, torch, w, Qd, "f32", form_steps, 5)
        del Qd
        torch.cuda.empty_cache()
        m = rr["ncell"] * form_steps / rr["wall_s"] / 1e6
        gb = rr["bytes_per_cell"] * rr["ncell"] / (rr["kernel_ms"] * 1e-3) / 1e9
        out[name] = dict(mlups=round(m, 1), kernel_ms=round(rr["kernel_ms"], 4), bytes_per_cell=rr["bytes_per_cell"],
                         achieved_GBps=round(gb, 1), frac_of_peak=round(gb / HBM_PEAK_GBPS, 4), finite=rr["finite"])
        log(f"{name} f32: {m:.1f} MLUPS, {gb:.0f} GB/s")
    return out


def run_body(vlbm, torch, synth, form_steps, only=False):
    """Flow past the moving magnetised body: 768 x 384 x 384, inflow / zero-gradient
    faces, homogenized body (the paper's method) and link-wise bounce-back, FP16
    deviation storage next to FP32."""
    body_forms = {}
    shape = (768, 384, 384)
    wb = synth.workload_body_3d(shape=shape)
    Qin, info = synth.inflow_state()
    wb["inflow_Q"] = Qin
    wb["body"] = synth.body_params(shape=shape, B_in=float(np.linalg.norm(info["B"])))
    log("generating the 768 x 384 x 384 body workload")
    Qb = torch.from_numpy(synth.body_initial_state(shape, wb["body"], dtype=np.float32)).cuda()
    for st in ("f16", "f32"):
        rr = time_sweep(vlbm, torch, wb, Qb, st, form_steps, 5)
        m = rr["ncell"] * form_steps / rr["wall_s"] / 1e6
        gb = rr["bytes_per_cell"] * rr["ncell"] / (rr["kernel_ms"] * 1e-3) / 1e9
        body_forms[st] = dict(mlups=round(m, 1), step_ms=round(rr["kernel_ms"], 4),
                              bytes_per_cell=rr["bytes_per_cell"], achieved_GBps=round(gb, 1),
                              frac_of_peak=round(gb / HBM_PEAK_GBPS, 4), finite=rr["finite"])
        log(f"body 768x384x384 {st}: {m:.1f} MLUPS, {gb:.0f} GB/s")
    body_forms["f16"]["speedup_vs_f32"] = round(body_forms["f16"]["mlups"] / body_forms["f32"]["mlups"], 3)
    del Qb
    torch.cuda.empty_cache()
    # the configured body treatment: link-wise bounce-back with the moving-wall correction
    # and the refill of uncovered cells (tau = 1.0, at which it stays physical)
    wbb = synth.workload_body_3d(shape=shape, tau=1.0)
    wbb["inflow_Q"] = Qin
    wbb["body"] = synth.body_params(shape=shape, B_in=float(np.linalg.norm(info["B"])), mode=1)
    Qb = torch.from_numpy(synth.body_initial_state(shape, wbb["body"], dtype=np.float32)).cuda()
    for st in ("f16", "f32"):
        rr = time_sweep(vlbm, torch, wbb, Qb, st, form_steps, 5)
        m = rr["ncell"] * form_steps / rr["wall_s"] / 1e6
        gb = rr["bytes_per_cell"] * rr["ncell"] / (rr["kernel_ms"] * 1e-3) / 1e9
        body_forms["bounce_back_" + st] = dict(mlups=round(m, 1), step_ms=round(rr["kernel_ms"], 4),
                                               bytes_per_cell=rr["bytes_per_cell"], achieved_GBps=round(gb, 1),
                                               frac_of_peak=round(gb / HBM_PEAK_GBPS, 4), finite=rr["finite"])
        log(f"bounce-back body 768x384x384 {st}: {m:.1f} MLUPS, {gb:.0f} GB/s")
    del Qb
    torch.cuda.empty_cache()
    if only:  # alone, the form also times the copy kernel (the reference of the HBM counters)
        body_forms["measured_copy_GBps"] = round(copy_bandwidth(vlbm, torch), 1)
    return body_forms


# The paper's own figures for its 13-component 2D kernel (Sec. 4 table), context only:
# another GPU, kernel and code generator.
PAPER_2D_KERNEL = {"mlups": 1077, "bytes_per_cell": 624, "frac_of_measured_bandwidth": 0.989,
                   "hardware": "NVIDIA RTX A5000, 680 GB/s measured (BabelStream)", "precision": "FP32 (inferred)"}


def run_resistive_2d(vlbm, torch, synth, form_steps):
    """The paper's 13-component 2D system (its Brio-Wu test, Sec. 3.1, and the 2D kernel
    of its Sec. 4 table) on a 4096^2 periodic Brio-Wu slab, FP32 / FP16 / BF16 storage;
    bytes per cell update 13 x 5 populations read and written."""
    out = {}
    n = 4096
    w = synth.workload_brio_wu_2d(n=n)
    log("generating the 4096^2 Brio-Wu state")
    Q = torch.from_numpy(synth.brio_wu_2d(n, n, dtype=np.float32)).cuda()
    for st in ("f32", "f16", "bf16"):
        rr = time_sweep(vlbm, torch, w, Q, st, form_steps, 5)
        m = rr["ncell"] * form_steps / rr["wall_s"] / 1e6
        gb = rr["bytes_per_cell"] * rr["ncell"] / (rr["kernel_ms"] * 1e-3) / 1e9
        out[st] = dict(mlups=round(m, 1), kernel_ms=round(rr["kernel_ms"], 4),
                       kernel_ms_std=round(rr["kernel_ms_std"], 4), bytes_per_cell=rr["bytes_per_cell"],
                       achieved_GBps=round(gb, 1), frac_of_peak=round(gb / HBM_PEAK_GBPS, 4), finite=rr["finite"])
        log(f"13-component 2D 4096^2 {st}: {m:.1f} MLUPS, {gb:.0f} GB/s")
    for st in ("f16", "bf16"):
        out[st]["speedup_vs_f32"] = round(out[st]["mlups"] / out["f32"]["mlups"], 3)
    out["paper_2d_kernel_context"] = PAPER_2D_KERNEL
    del Q
    torch.cuda.empty_cache()
    return out


def run_learned(synth):
    """The learned coarse correction measured in this run (2D, fine 1024^2 -> coarse
    256^2, r = 4, Fourier modes k <= 16): teacher-forced pairs from 8 training seeds,
    1500 Adam iterations of the 4-layer 3x3 network, then the corrected and the plain
    coarse runs on 2 held-out seeds over 1000 coarse steps, scored against the restricted
    FP64 fine run, and the wall time of the corrected coarse run against the plain FP32
    fine run over the same physical time."""
    import torch
    from paper_2606_00641_amd import learned as Lr
    from paper_2606_00641_amd import nn as N
    n_fine, r, kmax = 1024, 4, 16
    seeds, pairs, eval_seeds, steps, iters = list(range(100, 108)), 250, [900, 901], 1000, 1500
    w = synth.workload_fourier_2d()
    t0 = time.perf_counter()
    X, Y = Lr.generate_pairs(seeds, n_fine, r, pairs, w, synth.fourier_2d, kmax=kmax)
    t_pairs = time.perf_counter() - t0
    in_mean, in_std, out_mean, out_std, y_l2, drift = Lr.normalisation(X, Y)
    net = N.Net(8, 32, 4, stream=torch.cuda.current_stream().cuda_stream)
    net.vlbm_nn_set_weights(Lr.init_weights(seed=0))
    net.vlbm_nn_set_norm(in_mean, in_std, out_mean, out_std)
    losses, t_train = Lr.train(net, X, Y, iters, 1e-3, seed=0)
    del X, Y
    torch.cuda.empty_cache()
    b_abs = 5.0 * drift
    hist, nfb = Lr.evaluate(net, eval_seeds, n_fine, r, steps, w, synth.fourier_2d,
                            5.0 * y_l2 * np.sqrt(len(eval_seeds)), 0.1, b_abs, kmax=kmax, checkpoints=2,
                            fine_storage="f64")
    t_fine, t_learned, nfb_t = Lr.time_runs(net, n_fine, r, steps, w, synth.fourier_2d, 5.0 * y_l2, 0.1, b_abs,
                                            kmax=kmax)
    net.vlbm_nn_destroy()
    last = hist[-1]
    log(f"learned 2D: {t_fine / t_learned:.2f}x the FP32 fine run; errors vs FP64 fine: plain {last['plain']}, "
        f"learned {last['learned']}")
    return {"workload": "2D ideal MHD D2Q5 x 8, fine 1024^2 -> coarse 256^2 (r = 4), Fourier modes k <= 16, "
                        "FP32 coarse runs", "training": f"{pairs * len(seeds)} teacher-forced pairs from seeds "
                        f"{seeds[0]}-{seeds[-1]}, {iters} Adam iterations", "eval_seeds": eval_seeds,
            "coarse_steps": steps, "rel_l2_vs_restricted_fp64_fine": {"plain_coarse": last["plain"],
                                                                      "learned_coarse": last["learned"]},
            "fallbacks": nfb, "wall_fine_fp32_s": round(t_fine, 4), "wall_learned_coarse_s": round(t_learned, 4),
            "speedup_vs_fine_fp32": round(t_fine / t_learned, 3), "time_pairs_s": round(t_pairs, 2),
            "time_train_s": round(t_train, 2)}


def run_network():
    """The learned correction's networks (4 layers, 8-32-32-32-8, BF16 MFMA with FP32
    accumulation): 3x3 on its coarse 2D training batch (40 lattices of 256^2) and
    3x3x3 on the coarse grid of the body flow (384 x 192 x 192)."""
    from paper_2606_00641_amd import learned
    nets = {"2d_3x3_40x256x256": learned.time_network(batch=40, n=256),
            "3d_3x3x3_384x192x192": learned.time_network(batch=1, dim=3, nz=192, ny=192, nx=384, reps=5)}
    for name, network in nets.items():
        for k in network:
            network[k]["frac_of_bf16_peak"] = round(network[k]["tflops"] / BF16_PEAK_TFLOPS, 4)
        log(f"network {name}: forward {network['forward']['tflops']} TFLOP/s, "
            f"train step {network['train_step']['tflops']} TFLOP/s")
    nets["peak_TFLOPs_bf16_dense"] = BF16_PEAK_TFLOPS
    return nets


def recorded_studies():
    """Summaries of the committed study outputs under profiles/ (recorded by
    study_precision.py, study_learned.py and study_learned_3d.py on the same GPU; not
    re-measured here)."""
    out = {}
    try:
        with open(os.path.join(ROOT, "profiles", "precision_slab_512.json")) as fh:
            d = json.load(fh)
        last = d["checkpoints"][-1]
        out["precision_slab_512"] = {
            "source": "profiles/precision_slab_512.json", "steps": last["step"],
            "rel_l2_vs_fp64": {st: {k: v for k, v in last[st].items() if k != "nbad"} for st in ("f32", "f16", "bf16")}}
    except (OSError, ValueError, KeyError):
        pass
    for key in ("learned_coarse_2d", "learned_coarse_3d", "learned_coarse_3d_f16", "learned_coarse_3d_bf16"):
        try:
            with open(os.path.join(ROOT, "profiles", key + ".json")) as fh:
                d = json.load(fh)
            last = d["history"][-1]
            out[key] = {
                "source": f"profiles/{key}.json", "workload": d["workload"], "coarse_steps": d["coarse_steps"],
                "speedup_vs_fine_fp32": d["speedup_vs_fine"], "rel_l2_vs_restricted_fine": {
                    "plain_coarse": last["plain"], "learned_coarse": last["learned"]}, "fallbacks": d["fallbacks"]}
        except (OSError, ValueError, KeyError):
            pass
    return out or None


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true", help="skip the slab and body forms and the network timing")
    ap.add_argument("--form-steps", type=int, default=50)
    ap.add_argument("--only", choices=("slab", "body", "models", "resistive_2d", "learned", "copy", "network"),
                    default=None,
                    help="run one secondary part alone and print its result (for profiling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU slab "
              "decomposition is not part of this build", file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    from paper_2606_00641_amd import vlbm

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.only:
        part = {"slab": lambda: run_slab(vlbm, torch, synth, args.form_steps, only=True),
                "body": lambda: run_body(vlbm, torch, synth, args.form_steps, only=True),
                "models": lambda: run_models(vlbm, torch, synth, args.form_steps),
                "resistive_2d": lambda: run_resistive_2d(vlbm, torch, synth, args.form_steps),
                "learned": lambda: run_learned(synth),
                "copy": lambda: copy_ceiling(vlbm, torch),
                "network": run_network}[args.only]()
        print(json.dumps({args.only: part}), flush=True)
        return

    # --- main workload: 3D resistive MHD, 256^3, D3Q7 x 26, FP32 ------------------
    w = synth.workload_resistive_3d(n=256)
    log("generating the 256^3 resistive workload")
    Q = torch.from_numpy(synth.turbulence_3d(n=256, seed=1, dtype=np.float32)).cuda()
    log("timing", args.steps, "sweeps after", args.warmup, "warmup")
    r = time_sweep(vlbm, torch, w, Q, "f32", args.steps, args.warmup)
    res_forms = run_resistive_storage(vlbm, torch, w, Q, r, args.form_steps) if not args.no_forms else {}
    del Q
    torch.cuda.empty_cache()
    mlups = r["ncell"] * args.steps / r["wall_s"] / 1e6
    achieved = r["bytes_per_cell"] * r["ncell"] / (r["kernel_ms"] * 1e-3) / 1e9
    log(f"resistive 256^3 f32: {mlups:.1f} MLUPS, kernel {r['kernel_ms']:.3f} ms, {achieved:.0f} GB/s")

    copy_gbps = copy_bandwidth(vlbm, torch)
    log(f"copy kernel: {copy_gbps:.0f} GB/s")
    copies = copy_ceiling(vlbm, torch) if not args.no_forms else None
    if copies:
        log(f"copy ceiling: {copies}")

    forms = run_slab(vlbm, torch, synth, args.form_steps) if not args.no_forms else {}
    body_forms = run_body(vlbm, torch, synth, args.form_steps) if not args.no_forms else {}
    models = run_models(vlbm, torch, synth, args.form_steps) if not args.no_forms else {}
    r2d = run_resistive_2d(vlbm, torch, synth, args.form_steps) if not args.no_forms else {}
    network = run_network() if not args.no_forms else None
    learned_run = run_learned(synth) if not args.no_forms else None

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample")
        cpu = cpu_baseline()

    traffic = traffic_for("resistive_256", "f32")
    out = {
        "metric": "MLUPS + % HBM roofline, FP32 plain vs FP16-store/learned-coarse at fixed error",
        "value": round(mlups, 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r["wall_s"] / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "3D resistive incompressible MHD, plain VLBM, 256^3 periodic, D3Q7 x 26 variables "
                        "(rho, rho u, E, B, G, H), FP32 storage and arithmetic, random solenoidal u and B "
                        "with k^-2 spectrum 1<=k<=8, rms Mach 0.05, Re = Rm = 400",
            "lattice": "D3Q7", "cells": r["ncell"], "variables": 26, "storage": "f32",
            "bytes_per_cell_update": r["bytes_per_cell"],
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBPS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBPS, 4),
            "traffic": traffic,
            "kernel_ms": round(r["kernel_ms"], 4),
            "kernel_ms_std": round(r["kernel_ms_std"], 4),
            "measured_copy_GBps": round(copy_gbps, 1),
            "frac_of_copy": round(achieved / copy_gbps, 4),
            "copy_ceiling_GBps": copies,
        },
        "cpu_baseline": cpu,
        "forms_resistive_256": res_forms or None,
        "forms_slab_512": forms or None,
        "forms_body_768x384x384": body_forms or None,
        "forms_other_models_256": models or None,
        "forms_13_component_2d_4096": r2d or None,
        "learned_network": network,
        "learned_coarse_2d_measured": learned_run,
        "recorded_studies": recorded_studies(),
        "finite": r["finite"],
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
