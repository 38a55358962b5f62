#!/usr/bin/env python3
"""Benchmark of the SARA/SDMM hot path on one MI355X.

Workload: 1024 x 1024 synthetic sky (Gaussian blobs + 200 point sources, dynamic range 1e4),
M = 2e7 visibilities on a radial-density uv coverage split into R = 64 uneven contiguous blocks,
Kaiser-Bessel width J = 8 on a 2x oversampled grid, 30 dB input SNR.

A timed step is one SDMM iteration of the blocked problem (3): (cg_iters + 1) Phi + Phi^dagger
pairs, Psi and Psi^dagger, the three fused prox/dual updates with float64 block norms and the
stopping-test reductions.  `value` is the Phi + Phi^dagger visibility rate inside those steps,
(cg_iters + 1) * M per step; every CG product goes through a Phi, Phi^dagger pair here (solver option
toeplitz = 0).  Beside it: HIP-event medians and p10/p90 of the steps, of the solver's default
iteration (two CG steps through the Toeplitz form of Re(Phi_hat^H Phi_hat)) and of bare pairs; the HBM
roofline of the dominant interpolation kernel (HIP events on the library's stream); SDMM time to
tolerance with its convergence record (iterations per pass, objective, KKT residuals, a long fixed
schedule for comparison, feasibility re-checked with the FP64 oracle's operator); the FP64 CPU oracle
timed on the host cores.

Usage: python bench.py [--gpus 1] [--steps 20] [--warmup 5] [--no-cpu] [--no-tol] [--no-batch] [--no-unet]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Φ+Φ† visibilities/s and SDMM time-to-tol at 1024², plain vs warm-start, 1 GPU"
HBM_PEAK_GBS = 8000.0
# MI355X vector FP32 peak (published, packed FMA) and the FMA rate without packed math
# (256 CUs x 4 SIMDs x 16 lanes x 2 flop x 2.4 GHz), which is what this build's kernels can issue
FP32_PEAK_TFLOPS = 157.3
FP32_NONPACKED_TFLOPS = 78.6
BF16_PEAK_TFLOPS = 2500.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def stats(ms):
    """median, p10, p90 (ms) of a list of event times."""
    a = np.asarray(ms, dtype=np.float64)
    return {"median_ms": round(float(np.median(a)), 5), "p10_ms": round(float(np.percentile(a, 10)), 5),
            "p90_ms": round(float(np.percentile(a, 90)), 5), "n": int(a.size)}


def event_times(fn, reps):
    """Runs fn() reps times on the current stream, each bracketed by a pair of HIP events; the times (ms)."""
    import torch
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in ev:
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    return [a.elapsed_time(b) for a, b in ev]


def setup_workload(n=1024, m=20_000_000, R=64, J=8, n_points=200, dr=4.0, snr=30.0, cfg=3):
    from paper_1502_05037_amd import synth
    t0 = time.time()
    uv = synth.sort_by_radius(synth.uv_radial(m, synth.rng(cfg, 0, synth.UV)))
    sizes = synth.block_sizes(m, R, synth.rng(cfg, 0, synth.BLOCKS))
    off = synth.offsets(sizes)
    x_true = synth.sky(n, n_points, dr, synth.rng(cfg, 0, synth.SKY)).astype(np.float32)
    draws = synth.complex_normal(m, synth.rng(cfg, 0, synth.NOISE)).astype(np.complex64)
    log(f"[bench] inputs generated in {time.time() - t0:.1f}s (n={n}, M={m}, R={R}, J={J})")
    return dict(n=n, m=m, R=R, J=J, snr=snr, uv=uv, sizes=sizes, off=off, x_true=x_true, draws=draws)


def measured_traffic(kernel_name):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if taken on this kernel source."""
    import hashlib
    try:
        d = json.load(open(os.path.join(ROOT, "profiles", "grid_kernel_traffic.json")))
        src = open(os.path.join(ROOT, d["source"]), "rb").read()
    except (OSError, ValueError, KeyError):
        return None
    names = {"grid": ("grid_kernel", "grid_mfma_kernel"), "degrid": ("degrid_kernel",)}.get(kernel_name, ())
    if d.get("kernel", "").split("<")[0] not in names or hashlib.sha256(src).hexdigest() != d["source_sha256"]:
        return None
    return d["fetch_bytes_per_launch"] + d["write_bytes_per_launch"]


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(wl, x_tol=None, y_host=None):
    """The FP64 oracle timed on this host's cores (and, with x_tol, its FP64 operator re-checking the
    constraints of the GPU's time-to-tolerance image).

    * single thread: the numpy oracle NUFFT, one Phi + Phi^dagger pair on every 20th visibility (1e6);
    * all threads: the oracle NUFFT with compiled interpolation loops, one pair on all 2e7 visibilities
      (taps computed once beforehand, like the GPU plan) -- `value`;
    * the 64^2 workload (direct DFT, M = 2048): one pair and the whole 300-iteration solve;
    * the 256^2 workload (655 360 visibilities, J = 6): one pair and one SDMM iteration (2 CG steps);
    * the 1024^2 solve extrapolated from one oracle SDMM iteration times the GPU's iteration count."""
    from oracle import measurement, problem, sdmm, wavelets
    from paper_1502_05037_amd import synth
    cores = len(os.sched_getaffinity(0))
    n, J, m = wl["n"], wl["J"], wl["m"]
    out = {"unit": "vis/s", "kind": "oracle", "cores_available": cores, "cpu_model": cpu_model()}
    # single thread, numpy, sample of the workload
    stride = max(1, m // 1_000_000)
    uv = wl["uv"][::stride][:1_000_000]
    op1 = measurement.NUFFT(uv, n, J)
    x = wl["x_true"].astype(np.float64)
    v = wl["draws"][::stride][:1_000_000].astype(np.complex128)
    t0 = time.perf_counter()
    op1.fwd(x)
    op1.adj(v)
    dt1 = time.perf_counter() - t0
    out["single_thread"] = {"value": len(uv) / dt1, "threads": 1, "seconds": round(dt1, 2),
                            "sample": f"numpy FP64 NUFFT pair on {len(uv)} of the {m} visibilities (every {stride}th)"}
    log(f"[bench] oracle single thread: {len(uv) / dt1:.4g} vis/s")
    # all threads, compiled interpolation loops, the whole workload
    t0 = time.perf_counter()
    opc = measurement.NUFFTCompiled(wl["uv"], n, J, threads=cores)
    setup = time.perf_counter() - t0
    t0 = time.perf_counter()
    vis = opc.fwd(x)
    opc.adj(vis)
    dtc = time.perf_counter() - t0
    out.update({"value": m / dtc, "cores": cores,
                "sample": f"one FP64 Phi+Phi^dagger pair over all {m} visibilities, n={n}, J={J}, compiled "
                          f"interpolation loops on {cores} threads: {dtc:.2f} s (taps: {setup:.1f} s once)"})
    log(f"[bench] oracle all threads: {m / dtc:.4g} vis/s ({dtc:.2f} s per pair)")
    if x_tol is not None and y_host is not None:
        # the constraints of (3) for the GPU's time-to-tolerance image, with the FP64 operator
        vx = opc.fwd(np.asarray(x_tol, dtype=np.float64))
        off, eps = wl["off"], wl["eps"]
        r = np.array([np.linalg.norm(y_host[off[i]:off[i + 1]] - vx[off[i]:off[i + 1]]) for i in range(len(eps))])
        out["check_time_to_tol"] = {"max_resid_over_eps_fp64": float(np.max(r / eps)),
                                    "worst_block": int(np.argmax(r / eps))}
        log(f"[bench] oracle FP64 feasibility of the time-to-tol image: {np.max(r / eps):.7f}")
    # an oracle SDMM iteration at 1024^2 (2 CG steps, the solver's default), for the extrapolated solve
    psi = wavelets.SARA(n, 4)
    pb = sdmm.Problem(opc, psi, vis, wl["off"], wl["eps"], 1.0)
    st = sdmm.init_state(pb)
    p = sdmm.Params(gamma=1e-6, nu=1.0, max_iter=1, cg_iters=2)
    t0 = time.perf_counter()
    sdmm.sdmm_pass(pb, None, p, st)
    it3 = time.perf_counter() - t0
    out["config3_iteration_s"] = round(it3, 2)
    del opc, vis
    # 64^2, M = 2048, direct DFT: pair and the 300-iteration solve (one weighted-l1 pass)
    uv1 = synth.sort_by_radius(synth.uv_gaussian(2048, synth.rng(1, 0, synth.UV)))
    x1 = synth.sky(64, 20, 3.0, synth.rng(1, 0, synth.SKY))
    d1 = measurement.DFT(uv1, 64)
    t0 = time.perf_counter()
    c1 = d1.fwd(x1)
    d1.adj(c1)
    pair1 = time.perf_counter() - t0
    sig = problem.noise_sigma(c1, 30.0)
    y1 = problem.add_noise(c1, sig, synth.complex_normal(2048, synth.rng(1, 0, synth.NOISE)))
    eps1 = problem.eps_blocks(sig, [2048])
    psi1 = wavelets.SARA(64, 4)
    t0 = time.perf_counter()
    nu1 = measurement.op_norm(d1, np.ones((64, 64)))
    g1 = sdmm.default_gamma(d1, psi1, y1, nu1)
    sdmm.sara(d1, psi1, y1, [0, 2048], eps1, sdmm.Params(gamma=g1, nu=nu1, max_iter=300, cg_iters=2))
    solve1 = time.perf_counter() - t0
    out["config1"] = {"pair_vis_per_s": 2048 / pair1, "solve_300_iterations_s": round(solve1, 2),
                      "what": "64^2, M=2048, direct-DFT oracle, numpy"}
    # 256^2, 655 360 visibilities, J = 6
    m2 = 655_360
    uv2 = synth.sort_by_radius(synth.uv_gaussian(m2, synth.rng(2, 0, synth.UV)))
    x2 = synth.sky(256, 20, 3.0, synth.rng(2, 0, synth.SKY))
    o2 = measurement.NUFFTCompiled(uv2, 256, 6, threads=cores)
    t0 = time.perf_counter()
    c2 = o2.fwd(x2)
    o2.adj(c2)
    pair2 = time.perf_counter() - t0
    sz2 = synth.block_sizes(m2, 8, synth.rng(2, 0, synth.BLOCKS))
    pb2 = sdmm.Problem(o2, wavelets.SARA(256, 4), c2, synth.offsets(sz2), np.ones(8), 1.0)
    t0 = time.perf_counter()
    sdmm.sdmm_pass(pb2, None, sdmm.Params(gamma=1e-6, nu=1.0, max_iter=1, cg_iters=2), sdmm.init_state(pb2))
    it2 = time.perf_counter() - t0
    out["config2"] = {"pair_vis_per_s": m2 / pair2, "iteration_s": round(it2, 3),
                      "solve_5x300_extrapolated_s": round(1500 * it2, 1),
                      "what": "256^2, M=655360, J=6, compiled oracle NUFFT, all threads; solve extrapolated"}
    log(f"[bench] oracle config1 {out['config1']}, config2 {out['config2']}")
    return out


def warm_measure(sh, op, psi, y, eps, prm, n, dev, x_plain, x_true):
    """Warm-started solve of the same problem (trained U-Net + first weights from its output), timed
    from the call to the return like the plain one.  Empty when no trained weights are present."""
    import torch
    from paper_1502_05037_amd import warmstart
    if not os.path.exists(warmstart.WEIGHTS):
        log("[bench] no trained warm-start weights: warm start not measured")
        return {}
    ws = warmstart.WarmStart.load()
    try:
        xw = torch.empty((1, n, n), device=dev)
        log("[bench] warm-started SDMM to the same tolerance ...")
        info, res, secs = warmstart.warm_solve(ws, op, psi, y, eps, prm, n, dev, xw)
    finally:
        ws.close()
    xw = xw.reshape(n, n)
    wi = info.get("warm_info", info)   # the warm attempt's own record (the same as info unless it fell back)
    return {"warm_seconds": round(secs, 3), "warm_path": info["path"], "warm_attempt_pass_iters": wi["pass_iters"],
            "warm_attempt_converged": wi["converged"],
            "warm_iters": info["iters_total"], "warm_passes": info["passes_done"], "warm_pass_iters": info["pass_iters"],
            "warm_converged_last_pass": info["converged"], "warm_max_resid_over_eps": float(np.max(res / eps)),
            "warm_rel_change_at_exit": info["rel_change"],
            "warm_kkt_primal": info["kkt_primal"], "warm_kkt_dual": info["kkt_dual"],
            "warm_error_vs_true_sky": float(torch.linalg.vector_norm(xw - x_true) / torch.linalg.vector_norm(x_true)),
            "warm_vs_plain_image_rel_diff": float(torch.linalg.vector_norm(xw - x_plain.reshape(n, n))
                                                  / torch.linalg.vector_norm(x_plain))}


def unet_flops(base=32, levels=4, n=256):
    """Algorithmic flop of one U-Net forward on an n x n image (2 per multiply-add).  A layer's level
    follows from its channel count c = base 2^l: side n >> l (input side n >> (l+1) for the
    transposed convolution, whose cin = 2c)."""
    from paper_1502_05037_amd.warmstart import layer_list
    f = 0
    for kind, cin, cout in layer_list(base, levels):
        if kind == "conv3":
            side = n >> ((cout // base).bit_length() - 1)
            f += 2 * 9 * cin * cout * side * side
        elif kind == "tconv":
            side = n >> ((cin // base).bit_length() - 1)
            f += 2 * 4 * cin * cout * side * side
        else:
            f += 2 * cin * cout * n * n
    return f


def unet_bench(sh, dev, reps=20):
    """U-Net forward and training step (BF16 MFMA products) at 256^2 batch 8 and forward at 1024^2."""
    import torch
    from paper_1502_05037_amd.warmstart import he_init
    u = sh.unet_create(32, 4)
    out = {}
    try:
        sh.unet_set_params(u, he_init(32, 4, 0))
        for name, B, n, train in (("fwd_256_b8", 8, 256, False), ("train_256_b8", 8, 256, True),
                                  ("fwd_1024_b1", 1, 1024, False)):
            g = torch.Generator(device="cpu").manual_seed(7)
            x = torch.rand((B, n, n), generator=g).to(dev)
            t = torch.rand((B, n, n), generator=g).to(dev)
            y = torch.empty_like(x)
            step = (lambda: sh.unet_train_step(u, x, t, 1e-4, want_loss=False)) if train else \
                (lambda: sh.unet_forward(u, x, y))
            for _ in range(3):
                step()
            torch.cuda.synchronize()
            st = stats(event_times(step, reps))
            ms = st["median_ms"]
            fl = B * unet_flops(n=n) * (3 if train else 1)
            out[name] = {"ms": ms, "p10_ms": st["p10_ms"], "p90_ms": st["p90_ms"], "gflop": round(fl / 1e9, 1),
                         "tflops": round(fl / ms / 1e9, 1), "frac_of_bf16_mfma_peak": round(fl / ms / 1e9 / BF16_PEAK_TFLOPS, 4)}
            log(f"[bench] unet {name}: {out[name]}")
        sh.unet_set_params(u, he_init(32, 4, 0))   # leave no trained state behind
    finally:
        sh.unet_destroy(u)
    return out


def batched_workload(P=32, n=256, cfg=4):
    """32 independent 256 x 256 problems (frequency channels): M_p log-uniform in [1e5, 1e6], R_p uniform
    in 2..16 uneven blocks, Gaussian-density uv coverage, 20 point sources + blobs each, 30 dB SNR."""
    from paper_1502_05037_amd import synth
    g = synth.rng(cfg, 0, synth.BLOCKS)
    M_p = np.round(10 ** g.uniform(5, 6, P)).astype(np.int64)
    R_p = g.integers(2, 17, P).astype(np.int32)
    uvs, offs, xs, draws, sizes = [], [0], [], [], []
    base = 0
    for p in range(P):
        m = int(M_p[p])
        uvs.append(synth.sort_by_radius(synth.uv_gaussian(m, synth.rng(cfg, p, synth.UV))))
        sz = synth.block_sizes(m, int(R_p[p]), synth.rng(cfg, p, synth.BLOCKS))
        sizes.append(sz)
        offs.extend((base + synth.offsets(sz)[1:]).tolist())
        base += m
        xs.append(synth.sky(n, 20, 3.0, synth.rng(cfg, p, synth.SKY)).astype(np.float32))
        draws.append(synth.complex_normal(m, synth.rng(cfg, p, synth.NOISE)).astype(np.complex64))
    return dict(P=P, n=n, M_p=M_p, R_p=R_p, uv=np.concatenate(uvs), off=np.array(offs, dtype=np.int64),
                x_true=np.stack(xs), draws=np.concatenate(draws), sizes=sizes)


def batched_bench(sh, dev, steps, warmup, with_tol=True, snr=30.0):
    """Many small problems in one plan: autotuned plan, graph-replayed SDMM iterations of all problems
    at once, the same problems iterated one plan at a time, and time to tolerance with 3 passes."""
    import torch
    bw = batched_workload()
    P, n, M_p, R_p = bw["P"], bw["n"], bw["M_p"], bw["R_p"]
    M = int(M_p.sum())
    log(f"[bench] batched: {P} problems of {n}^2, M = {M} ({M_p.min()}..{M_p.max()}), R = {int(R_p.sum())}")
    t0 = time.time()
    op, tune = sh.op_autotune(bw["uv"], M_p, n, 2, 1e-5, bw["off"], R_p, reps=3)
    tune_s = time.time() - t0
    log(f"[bench] autotuned in {tune_s:.1f}s: {tune}")
    psi = sh.psi_create_batched(n, 4, sh.SARA_MASK, P)
    x_true = torch.tensor(bw["x_true"], device=dev)
    clean = torch.empty(M, dtype=torch.complex64, device=dev)
    sh.phi_fwd(op, x_true, clean)
    cn = clean.to(torch.complex128)
    y = torch.empty_like(clean)
    draws = torch.tensor(bw["draws"], device=dev)
    eps = []
    vo = np.concatenate([[0], np.cumsum(M_p)])
    for p in range(P):
        lo, hi = int(vo[p]), int(vo[p + 1])
        sig = float(torch.linalg.vector_norm(cn[lo:hi])) / np.sqrt(hi - lo) * 10 ** (-snr / 20)
        y[lo:hi] = clean[lo:hi] + (sig / np.sqrt(2)) * draws[lo:hi]
        sz = bw["sizes"][p].astype(np.float64)
        eps.append(sig * np.sqrt(sz + 2 * np.sqrt(sz)))
    eps = np.concatenate(eps)
    prm = sh.sdmm_default_params()
    prm.cg_iters = 8
    prm.toeplitz = 0
    sess = sh.sdmm_create(op, psi, y, eps, None, None, prm)
    try:
        sh.sdmm_iterate(sess, warmup)
        st = stats(event_times(lambda: sh.sdmm_iterate(sess, 1), steps))
    finally:
        sh.sdmm_destroy(sess)
    dt = st["median_ms"] * 1e-3
    log(f"[bench] batched SDMM iteration {st} for {P} problems -> {9 * M / dt:.4g} vis/s")
    # the same problems one plan at a time (same tiling and width, graph replay), summed
    seq = 0.0
    for p in range(P):
        lo, hi = int(vo[p]), int(vo[p + 1])
        ob = np.concatenate([[0], np.cumsum(bw["sizes"][p])]).astype(np.int64)
        op1 = sh.op_create_tuned(bw["uv"][lo:hi], n, 2, tune["J"], ob, tile=tune["tile"], chunk=tune["chunk"])
        psi1 = sh.psi_create(n, 4)
        e0 = int(np.sum(R_p[:p]))
        s1 = sh.sdmm_create(op1, psi1, y[lo:hi].contiguous(), eps[e0:e0 + int(R_p[p])], None, None, prm)
        try:
            sh.sdmm_iterate(s1, 2)
            seq += stats(event_times(lambda: sh.sdmm_iterate(s1, 1), max(5, steps // 2)))["median_ms"] * 1e-3
        finally:
            sh.sdmm_destroy(s1)
            sh.psi_destroy(psi1)
            sh.op_destroy(op1)
    log(f"[bench] one plan at a time: {1e3 * seq:.3f} ms per iteration of all {P} problems")
    tol = None
    if with_tol:
        # the solver's stopping test (relative change 1e-4, feasibility slack 1e-4, dual residual 1e-2, checked
        # every 10 iterations); this workload needs a cap of 1000 iterations per pass for every problem to
        # meet it (with 300, two problems end their passes at the cap)
        p2 = sh.sdmm_default_params()
        p2.tol_rel, p2.passes, p2.max_iter = 1e-4, 3, 1000
        x = torch.empty((P, n, n), device=dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        infos, res = sh.sdmm_solve(op, psi, y, eps, None, None, p2, x)
        torch.cuda.synchronize()
        ratio = res / eps
        tol = {"seconds": round(time.perf_counter() - t0, 3), "iters_total": infos[0]["iters_total"],
               "passes": infos[0]["passes_done"], "converged_last_pass": int(sum(i["converged"] for i in infos)),
               "max_resid_over_eps": float(np.max(ratio)), "blocks_over_1e-4": int(np.sum(ratio > 1 + 1e-4)),
               "tol_rel": 1e-4, "tol_dual": p2.tol_dual, "max_iter_per_pass": p2.max_iter,
               "most_iters": max(i["iters_total"] for i in infos), "max_kkt_primal": max(i["kkt_primal"] for i in infos),
               "max_kkt_dual": max(i["kkt_dual"] for i in infos)}
        log(f"[bench] batched time-to-tol {tol}")
    sh.psi_destroy(psi)
    sh.op_destroy(op)
    return {"workload": f"{P} independent {n}x{n} problems, M_p log-uniform in [1e5, 1e6] (total {M}), "
                        f"R_p uniform in 2..16 (total {int(R_p.sum())}), Gaussian uv, 30 dB, one batched plan",
            "tune": tune, "tune_seconds": round(tune_s, 2), "ms_per_iteration": 1e3 * dt, "iteration": st,
            "vis_per_s": 9 * M / dt, "one_plan_at_a_time_ms_per_iteration": 1e3 * seq,
            "batching_speedup": seq / dt, "time_to_tol": tol}


def time_to_tol(sh, op, psi, y, eps, n, dev, x_true, long_iters):
    """Plain SDMM to tolerance (5 passes of at most 300 iterations, tol 1e-4, feasibility slack 1e-4), its
    convergence record, a long fixed schedule for comparison, and the warm start."""
    import torch
    p2 = sh.sdmm_default_params()
    p2.tol_rel, p2.passes, p2.max_iter = 1e-4, 5, 300    # checked every 10 iterations, dual residual 1e-2
    x = torch.empty((n, n), device=dev)
    log("[bench] SDMM to tolerance 1e-4, 5 passes of at most 300 iterations ...")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    info, res = sh.sdmm_solve(op, psi, y, eps, None, None, p2, x)
    torch.cuda.synchronize()
    nx = torch.linalg.vector_norm(x_true)
    tol = {"plain_seconds": round(time.perf_counter() - t0, 3), "plain_iters": info["iters_total"],
           "plain_pass_iters": info["pass_iters"], "passes": info["passes_done"],
           "converged_last_pass": info["converged"], "max_resid_over_eps": float(np.max(res / eps)), "tol_rel": 1e-4,
           "plain_rel_change_at_exit": info["rel_change"], "plain_objective": info["objective"],
           "plain_kkt_primal": info["kkt_primal"], "plain_kkt_dual": info["kkt_dual"], "cg_iters": p2.cg_iters,
           "plain_error_vs_true_sky": float(torch.linalg.vector_norm(x - x_true) / nx),
           "tol_dual": p2.tol_dual, "check_every": p2.check_every,
           "warm_seconds": None, "warm_iters": None}
    log(f"[bench] time-to-tol plain: {tol}")
    # the same without the dual-residual test (relative change and feasibility only)
    p0 = sh.sdmm_default_params()
    p0.tol_rel, p0.passes, p0.max_iter, p0.tol_dual = 1e-4, 5, 300, 0.0
    x0 = torch.empty((n, n), device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    i0, r0 = sh.sdmm_solve(op, psi, y, eps, None, None, p0, x0)
    torch.cuda.synchronize()
    tol["without_dual_test"] = {"seconds": round(time.perf_counter() - t0, 3), "pass_iters": i0["pass_iters"],
                                "kkt_dual": i0["kkt_dual"], "max_resid_over_eps": float(np.max(r0 / eps)),
                                "error_vs_true_sky": float(torch.linalg.vector_norm(x0 - x_true) / nx)}
    # a long fixed schedule (the same 5 passes, long_iters iterations each, no stopping test)
    if long_iters:
        pl = sh.sdmm_default_params()
        pl.tol_rel, pl.passes, pl.max_iter = 0.0, 5, long_iters
        xl = torch.empty((n, n), device=dev)
        t0 = time.perf_counter()
        il, rl = sh.sdmm_solve(op, psi, y, eps, None, None, pl, xl)
        torch.cuda.synchronize()
        tol["long_fixed_schedule"] = {
            "iterations_per_pass": long_iters, "seconds": round(time.perf_counter() - t0, 2),
            "objective": il["objective"], "kkt_primal": il["kkt_primal"], "kkt_dual": il["kkt_dual"],
            "max_resid_over_eps": float(np.max(rl / eps)),
            "error_vs_true_sky": float(torch.linalg.vector_norm(xl - x_true) / nx),
            "time_to_tol_image_rel_diff": float(torch.linalg.vector_norm(x - xl) / torch.linalg.vector_norm(xl)),
            "without_dual_test_image_rel_diff": float(torch.linalg.vector_norm(x0 - xl) / torch.linalg.vector_norm(xl))}
        log(f"[bench] long fixed schedule: {tol['long_fixed_schedule']}")
    # block-subset iterations (a random fraction of the 64 blocks per iteration), same stopping test
    tol["block_subset"] = []
    for frac in (0.5, 0.25):
        pf = sh.sdmm_default_params()
        pf.tol_rel, pf.passes, pf.max_iter, pf.block_fraction, pf.block_seed = 1e-4, 5, 300, frac, 1
        xs = torch.empty((n, n), device=dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        isub, rsub = sh.sdmm_solve(op, psi, y, eps, None, None, pf, xs)
        torch.cuda.synchronize()
        secs = time.perf_counter() - t0
        sess = sh.sdmm_create(op, psi, y, eps, None, None, pf)
        try:
            sh.sdmm_iterate(sess, 3)
            it_ms = stats(event_times(lambda: sh.sdmm_iterate(sess, 1), 20))
        finally:
            sh.sdmm_destroy(sess)
        tol["block_subset"].append({
            "block_fraction": frac, "seconds": round(secs, 3), "pass_iters": isub["pass_iters"],
            "iters": isub["iters_total"], "converged": isub["converged"], "kkt_dual": isub["kkt_dual"],
            "max_resid_over_eps": float(np.max(rsub / eps)), "iteration_ms": it_ms["median_ms"],
            "error_vs_true_sky": float(torch.linalg.vector_norm(xs - x_true) / nx),
            "image_rel_diff_vs_full": float(torch.linalg.vector_norm(xs - x) / torch.linalg.vector_norm(x))})
        log(f"[bench] block-subset SDMM {tol['block_subset'][-1]}")
    tol.update(warm_measure(sh, op, psi, y, eps, p2, n, dev, x, x_true))
    return tol, x


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-tol", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the many-small-problems measurement")
    ap.add_argument("--no-unet", action="store_true", help="skip the U-Net kernel measurement")
    ap.add_argument("--only-unet", action="store_true", help="run the U-Net kernel measurement alone")
    ap.add_argument("--long-iters", type=int, default=1000,
                    help="iterations per pass of the long fixed schedule compared with the time-to-tol run (0: skip)")
    ap.add_argument("--m", type=int, default=20_000_000)
    ap.add_argument("--copy-mb", type=int, default=0,
                    help="also run three plain device copies of this many MiB (HBM counter calibration)")
    a = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if a.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the blocked problem shards by data block; see the design notes).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1502_05037_amd import sarahip as sh

    dev = torch.device("cuda:0")
    if a.only_unet:
        print(json.dumps({"unet": unet_bench(sh, dev)}), flush=True)
        return
    wl = setup_workload(m=a.m)
    n, m, R, J = wl["n"], wl["m"], wl["R"], wl["J"]
    t0 = time.time()
    op = sh.op_create(wl["uv"], n, 2, J, wl["off"])
    plan_s = time.time() - t0
    q = sh.op_query(op)
    psi = sh.psi_create(n, 4)
    log(f"[bench] plan built in {plan_s:.1f}s: {q}")

    # data: y = Phi x_true + noise at 30 dB, eps_i from the chi^2 bound (mean + 2 s.d.)
    x_true = torch.tensor(wl["x_true"], device=dev)
    clean = torch.empty(m, dtype=torch.complex64, device=dev)
    sh.phi_fwd(op, x_true, clean)
    sigma = float(torch.linalg.vector_norm(clean.to(torch.complex128))) / np.sqrt(m) * 10 ** (-wl["snr"] / 20)
    y = clean + (sigma / np.sqrt(2)) * torch.tensor(wl["draws"], device=dev)
    sizes = wl["sizes"].astype(np.float64)
    eps = sigma * np.sqrt(sizes + 2 * np.sqrt(sizes))
    wl["eps"] = eps
    log(f"[bench] sigma={sigma:.4g}")

    # ---- timed SDMM iterations: K steps bracketed by synchronisations, each also between HIP events
    prm = sh.sdmm_default_params()
    prm.cg_iters = 8
    prm.toeplitz = 0          # every CG product through a Phi, Phi^dagger pair: 9 pairs per step
    sess = sh.sdmm_create(op, psi, y, eps, None, None, prm)
    try:
        sh.sdmm_iterate(sess, a.warmup)
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(a.steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for e0, e1 in ev:
            e0.record()
            sh.sdmm_iterate(sess, 1)
            e1.record()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        step_stats = stats([e0.elapsed_time(e1) for e0, e1 in ev])
        resid, rel = sh.sdmm_result(sess, None, R)
    finally:
        sh.sdmm_destroy(sess)
    ms_step = 1e3 * dt / a.steps
    pairs = prm.cg_iters + 1
    value = pairs * m / (dt / a.steps)
    log(f"[bench] SDMM iteration {ms_step:.3f} ms -> {value:.4g} vis/s; events {step_stats}")

    # ---- the solver's default iteration: 2 CG steps through the Toeplitz form of Re(Phi_hat^H Phi_hat)
    pd = sh.sdmm_default_params()
    t0 = time.perf_counter()
    sess = sh.sdmm_create(op, psi, y, eps, None, None, pd)
    create_s = time.perf_counter() - t0
    try:
        sh.sdmm_iterate(sess, a.warmup)
        dst = stats(event_times(lambda: sh.sdmm_iterate(sess, 1), a.steps))
        default_it = {"ms": dst["median_ms"], "p10_ms": dst["p10_ms"], "p90_ms": dst["p90_ms"],
                      "cg_iters": pd.cg_iters, "toeplitz": pd.toeplitz, "session_create_s": round(create_s, 3)}
    finally:
        sh.sdmm_destroy(sess)
    log(f"[bench] default SDMM iteration {default_it}")

    # ---- bare Phi + Phi^dagger pairs (internal and user order) and per-kernel event timing
    xin = torch.rand((n, n), device=dev)
    vis = torch.empty(m, dtype=torch.complex64, device=dev)
    xo = torch.empty((n, n), device=dev)

    def pair_int():
        sh.phi_fwd_internal(op, xin, vis)
        sh.phi_adj_internal(op, vis, xo)

    def pair_user():
        sh.phi_fwd(op, xin, vis)
        sh.phi_adj(op, vis, xo)

    for _ in range(3):
        pair_int()
    pst = stats(event_times(pair_int, a.steps))
    pust = stats(event_times(pair_user, a.steps))
    sh.profile_enable(True)
    for _ in range(a.steps):
        pair_int()
    torch.cuda.synchronize()
    kern = {}
    for name in ("degrid", "grid", "fold", "fft_rows", "fft_cols"):
        cnt, ms = sh.profile_read(name)
        kern[name] = {"launches": cnt, "avg_ms": ms / max(cnt, 1)}
    sh.profile_enable(False)
    # one Toeplitz product (three FFT passes), timed the same way
    nu = sh.op_norm(op, torch.ones((n, n), device=dev), iters=100, tol=1e-6)
    tp = sh.toeplitz_create(op, [1.0 / nu ** 2])
    try:
        for _ in range(2):
            sh.toeplitz_apply(tp, xin, xo)
        sh.profile_enable(True)
        for _ in range(a.steps):
            sh.toeplitz_apply(tp, xin, xo)
        torch.cuda.synchronize()
        cnt, ms = sh.profile_read("toeplitz")
        toep_ms = ms / max(cnt, 1)
        sh.profile_enable(False)
    finally:
        sh.toeplitz_destroy(tp)
    default_it["toeplitz_product_ms"] = round(toep_ms, 4)
    log(f"[bench] pair {pst} (internal), {pust} (user order); "
        + ", ".join(f"{k} {v['avg_ms']:.4f} ms" for k, v in kern.items()))

    # ---- roofline of the dominant interpolation kernel (HBM-bound by its arithmetic intensity).
    # Algorithmic bytes of one launch: packed uv (8 B) + one complex64 visibility (8 B) per visibility and
    # one pass over the complex64 K x K grid.  Algorithmic flop: the separable J x J interpolation,
    # 2J^2 + 2J multiply-adds (4J^2 + 4J flop) per visibility; the Kaiser-Bessel weight evaluation is
    # implementation work and not counted.
    K = q["K"]
    N = n * n
    alg_bytes = 16 * m + 8 * K * K
    mac_flop = (4 * J * J + 4 * J) * m
    ridge = FP32_PEAK_TFLOPS * 1e12 / (HBM_PEAK_GBS * 1e9)
    intensity = mac_flop / alg_bytes
    dom = max(("degrid", "grid"), key=lambda k: kern[k]["avg_ms"])
    t_dom = kern[dom]["avg_ms"] * 1e-3
    achieved = alg_bytes / t_dom / 1e9
    pair_bytes = 32 * m + 32 * K * K + 8 * N
    roof = {"kernel": dom, "bound": "hbm" if intensity < ridge else "alu", "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic(dom), "alg_bytes_per_launch": alg_bytes,
            "avg_launch_ms": round(kern[dom]["avg_ms"], 4),
            "intensity_flop_per_byte": round(intensity, 2), "ridge_flop_per_byte": round(ridge, 2),
            "alu_view": {"flop_per_launch": mac_flop, "achieved_TFLOPs": round(mac_flop / t_dom / 1e12, 2),
                         "frac_of_157.3": round(mac_flop / t_dom / 1e12 / FP32_PEAK_TFLOPS, 4),
                         "frac_of_78.6_nonpacked": round(mac_flop / t_dom / 1e12 / FP32_NONPACKED_TFLOPS, 4)},
            "pair": {"alg_bytes": pair_bytes, "median_ms": pst["median_ms"],
                     "frac": round(pair_bytes / (pst["median_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                     "user_order_frac": round(pair_bytes / (pust["median_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}}
    if dom == "grid":
        roof["fold_avg_ms"] = round(kern["fold"]["avg_ms"], 4)
    log(f"[bench] roofline {roof}")

    # ---- SDMM time to tolerance (plain, long fixed schedule, warm start)
    tol, x_tol = (None, None) if a.no_tol else time_to_tol(sh, op, psi, y, eps, n, dev, x_true, a.long_iters)

    if a.copy_mb:
        src = torch.ones(a.copy_mb << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] calibration copies: 3 x {a.copy_mb} MiB")

    y_host = y.cpu().numpy().astype(np.complex128) if (x_tol is not None and not a.no_cpu) else None
    xt_host = x_tol.cpu().numpy() if y_host is not None else None
    sh.psi_destroy(psi)
    sh.op_destroy(op)
    del y, clean, x_true
    batched = None if a.no_batch else batched_bench(sh, dev, a.steps, a.warmup, with_tol=not a.no_tol)
    unet = None if a.no_unet else unet_bench(sh, dev)
    cpu = None if a.no_cpu else cpu_baseline(wl, xt_host, y_host)
    if cpu is not None and tol is not None:
        ct = cpu.get("check_time_to_tol", {})
        tol["max_resid_over_eps_fp64_oracle"] = ct.get("max_resid_over_eps_fp64")
        tol["oracle_solve_extrapolated_s"] = round(cpu["config3_iteration_s"] * tol["plain_iters"], 1)
    out = {
        "metric": METRIC, "value": value, "unit": "vis/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "SARA/SDMM one SDMM iteration, 1024x1024 sky, M=2e7 radial uv, R=64 uneven "
                               "blocks, KB J=8, alpha=2, 8 CG steps", "n": n, "M": m, "R": R, "J": J,
                   "cg_iters": prm.cg_iters, "global_batch": 1},
        "step_events": step_stats,
        "pair": {"internal_vis_per_s": m / (pst["median_ms"] * 1e-3), "user_order_vis_per_s": m / (pust["median_ms"] * 1e-3),
                 "internal": pst, "user": pust},
        "kernels_ms": {k: round(v["avg_ms"], 4) for k, v in kern.items()},
        "default_iteration": default_it,
        "roofline": roof, "cpu_baseline": cpu, "sdmm_time_to_tol": tol, "plan_seconds": round(plan_s, 2),
        "batched": batched, "unet": unet,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
