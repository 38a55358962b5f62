"""Train the warm-start U-Net on pairs (normalised dirty image, plain SARA solution).

Training problems are 256 x 256 (R = 8 uneven blocks, 30 dB input SNR) of two kinds: the 256^2
configuration (Gaussian blobs + 20 point sources, M = 655 360 Gaussian-density uv points) and 256^2
windows of the 1024^2 configuration's skies under its radial coverage and visibility density (see
KINDS); the plain solver (5 passes of at most 300 iterations, tolerance 1e-4) gives the target.  Problems are
generated and solved 32 at a time through one batched plan.  The network input and target are the
dirty image and the solution, both divided by the dirty image's RMS in PSF-peak units.
Training: Adam, batch 8, mean squared error.  The weights and a JSON record of the run are written
next to each other.

Usage: python -m paper_1502_05037_amd.train_warmstart --pairs 256 --pairs-c3 256 --epochs 400 \
           --train-seconds 240 --out paper_1502_05037_amd/weights/unet_b32_l4.npy
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

from . import sarahip as sh
from . import synth
from .warmstart import he_init

TRAIN_CFG = 5          # seed namespace of the training problems; held-out problems use problem >= 10**6


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# Two kinds of training problem, both 256 x 256:
#  "c2": the 256^2 configuration itself (blobs + 20 point sources, dynamic range 1e3, Gaussian-density
#        coverage, M = 655 360, J = 6);
#  "c3": a 256 x 256 window of a 1024^2 sky from the 1024^2 configuration (blobs sized for 1024^2,
#        200 point sources, dynamic range 1e4) under radial-density coverage with that configuration's
#        visibilities per pixel (2e7 / 1024^2, so M = 1 250 000) and J = 8.  Coverage in radians per pixel
#        gives the same PSF in pixels at both sizes, so these windows show the network what the 1024^2
#        problem looks like locally.
KINDS = {"c2": dict(cfg=TRAIN_CFG, m=655_360, J=6), "c3": dict(cfg=TRAIN_CFG + 1, m=1_250_000, J=8)}


def make_problems(first: int, P: int, kind: str = "c2", n=256, R=8, snr=30.0):
    cfg, m = KINDS[kind]["cfg"], KINDS[kind]["m"]
    uvs, offs, xs, draws, sizes = [], [0], [], [], []
    base = 0
    for k in range(P):
        prob = first + k
        g_uv = synth.rng(cfg, prob, synth.UV)
        uv = synth.uv_gaussian(m, g_uv) if kind == "c2" else synth.uv_radial(m, g_uv)
        uv = synth.sort_by_radius(uv)
        sz = synth.block_sizes(m, R, synth.rng(cfg, prob, synth.BLOCKS))
        uvs.append(uv)
        sizes.append(sz)
        offs.extend((base + synth.offsets(sz)[1:]).tolist())
        base += m
        g_sky = synth.rng(cfg, prob, synth.SKY)
        if kind == "c2":
            x = synth.sky(n, 20, 3.0, g_sky)
        else:
            big = synth.sky(1024, 200, 4.0, g_sky)
            r0, c0 = g_sky.integers(0, 1024 - n + 1, size=2)
            x = big[r0:r0 + n, c0:c0 + n]
            x = x / max(float(x.max()), 1e-12)
        xs.append(x.astype(np.float32))
        draws.append(synth.complex_normal(m, synth.rng(cfg, prob, synth.NOISE)).astype(np.complex64))
    return dict(P=P, n=n, m=m, R=R, snr=snr, J=KINDS[kind]["J"], kind=kind, uv=np.concatenate(uvs),
                off=np.array(offs, dtype=np.int64), x_true=np.stack(xs), draws=np.concatenate(draws), sizes=sizes)


def observe(op, pr, dev):
    """y = Phi x_true + noise at the given SNR (per problem), eps_i from the chi^2 bound."""
    import torch
    P, m = pr["P"], pr["m"]
    clean = torch.empty(P * m, dtype=torch.complex64, device=dev)
    sh.phi_fwd(op, torch.tensor(pr["x_true"], device=dev), clean)
    draws = torch.tensor(pr["draws"], device=dev)
    y = torch.empty_like(clean)
    eps = []
    for p in range(P):
        c = clean[p * m:(p + 1) * m]
        sig = float(torch.linalg.vector_norm(c.to(torch.complex128))) / np.sqrt(m) * 10 ** (-pr["snr"] / 20)
        y[p * m:(p + 1) * m] = c + (sig / np.sqrt(2)) * draws[p * m:(p + 1) * m]
        sz = pr["sizes"][p].astype(np.float64)
        eps.append(sig * np.sqrt(sz + 2 * np.sqrt(sz)))
    return y, np.concatenate(eps)


def solve_params(passes=5, max_iter=300, tol=1e-4):
    p = sh.sdmm_default_params()
    p.tol_rel, p.passes, p.max_iter, p.check_every = tol, passes, max_iter, 10
    return p


def make_pairs(first: int, P: int, dev, kind: str = "c2"):
    """Solve P problems together; returns (inputs, targets) on the device, both P x n x n."""
    import torch
    pr = make_problems(first, P, kind)
    n, m, R, J = pr["n"], pr["m"], pr["R"], pr["J"]
    op = sh.op_create_batched(pr["uv"], [m] * P, n, 2, J, pr["off"], [R] * P)
    psi = sh.psi_create_batched(n, 4, sh.SARA_MASK, P)
    try:
        y, eps = observe(op, pr, dev)
        x = torch.empty((P, n, n), device=dev)
        infos, _ = sh.sdmm_solve(op, psi, y, eps, None, None, solve_params(), x)
        d = torch.empty((P, n, n), device=dev)
        s = torch.empty(P, device=dev)
        sh.dirty_normalised(op, y, d, s)
        sh.scale_images(x, s, invert=True)
        torch.cuda.synchronize()
        return d, x, infos
    finally:
        sh.psi_destroy(psi)
        sh.op_destroy(op)


def train(ws_u, inputs, targets, epochs: int, lr: float, batch: int, seed: int, dev, val_frac=0.1, budget_s=None):
    import torch
    N = inputs.shape[0]
    nval = max(1, int(round(val_frac * N)))
    idx_val = torch.arange(N - nval, N, device=dev)
    g = np.random.Generator(np.random.PCG64(np.random.SeedSequence([1502, 5037, 10, seed])))
    hist = []
    t0 = time.time()
    steps = 0
    for ep in range(epochs):
        perm = g.permutation(N - nval)
        losses = []
        for b in range(0, len(perm) - batch + 1, batch):
            sel = torch.as_tensor(perm[b:b + batch], device=dev)
            xb = inputs.index_select(0, sel).contiguous()
            tb = targets.index_select(0, sel).contiguous()
            losses.append(sh.unet_train_step(ws_u, xb, tb, lr))
            steps += 1
        vl = []
        for b in range(0, nval, batch):
            sel = idx_val[b:b + batch]
            vl.append(sh.unet_loss_grad(ws_u, inputs.index_select(0, sel).contiguous(),
                                        targets.index_select(0, sel).contiguous(), want_grads=False)[0])
        hist.append({"epoch": ep + 1, "train_loss": float(np.mean(losses)), "val_loss": float(np.mean(vl)),
                     "seconds": round(time.time() - t0, 1)})
        log(f"[train] epoch {ep + 1}: train {hist[-1]['train_loss']:.4e} val {hist[-1]['val_loss']:.4e} "
            f"({hist[-1]['seconds']} s, {steps} steps)")
        if budget_s and time.time() - t0 > budget_s:
            break
    return hist, steps


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--pairs", type=int, default=256, help="pairs of the 256^2 configuration")
    ap.add_argument("--pairs-c3", type=int, default=256, help="pairs of 256^2 windows of the 1024^2 configuration")
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--lr", type=float, default=3e-4)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--base", type=int, default=32)
    ap.add_argument("--levels", type=int, default=4)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--train-seconds", type=float, default=240.0)
    ap.add_argument("--out", required=True)
    a = ap.parse_args()
    import torch
    dev = torch.device("cuda:0")
    P = 32
    ins, outs, solve_log = [], [], []
    t0 = time.time()
    for kind, count in (("c2", a.pairs), ("c3", a.pairs_c3)):
        for first in range(0, count, P):
            d, x, infos = make_pairs(first, min(P, count - first), dev, kind)
            ins.append(d)
            outs.append(x)
            solve_log.append({"kind": kind, "first": first, "iters_total": infos[0]["iters_total"],
                              "converged": int(sum(i["converged"] for i in infos))})
            log(f"[train] {kind} pairs {first}..{first + d.shape[0] - 1} solved ({time.time() - t0:.0f} s): "
                f"{solve_log[-1]}")
    inputs, targets = torch.cat(ins), torch.cat(outs)
    # validation pairs: the last 10 %, drawn from both kinds
    perm = torch.as_tensor(np.random.Generator(np.random.PCG64(np.random.SeedSequence([1502, 5037, 11]))).permutation(
        inputs.shape[0]), device=dev)
    inputs, targets = inputs.index_select(0, perm).contiguous(), targets.index_select(0, perm).contiguous()
    gen_s = time.time() - t0
    u = sh.unet_create(a.base, a.levels)
    try:
        sh.unet_set_params(u, he_init(a.base, a.levels, a.seed))
        hist, steps = train(u, inputs, targets, a.epochs, a.lr, a.batch, a.seed, dev, budget_s=a.train_seconds)
        w = sh.unet_get_params(u)
    finally:
        sh.unet_destroy(u)
    os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
    np.save(a.out, w.astype(np.float32), allow_pickle=False)
    total = a.pairs + a.pairs_c3
    meta = {"base": a.base, "levels": a.levels, "pairs": total, "val_pairs": max(1, round(0.1 * total)),
            "train_problems": {"c2": f"synth config {TRAIN_CFG}, problems 0..{a.pairs - 1}, M 655360, J 6, Gaussian uv",
                               "c3": f"synth config {TRAIN_CFG + 1}, problems 0..{a.pairs_c3 - 1}, 256^2 windows of "
                                     "1024^2 skies, M 1250000, J 8, radial uv"},
            "n": 256, "R": 8, "snr_db": 30, "solver": "5 passes x <= 300 iterations, tol_rel 1e-4",
            "lr": a.lr, "batch": a.batch, "epochs_run": len(hist), "steps": steps, "init_seed": a.seed,
            "generation_seconds": round(gen_s, 1), "history": hist, "solves": solve_log,
            "command": "python -m paper_1502_05037_amd.train_warmstart " + " ".join(sys.argv[1:])}
    json.dump(meta, open(os.path.splitext(a.out)[0] + ".json", "w"), indent=1)
    log(f"[train] wrote {a.out}")


if __name__ == "__main__":
    main()
