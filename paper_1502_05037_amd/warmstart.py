"""Learned warm start for SARA/SDMM: a U-Net predicts a first image from the dirty image, SDMM finishes.

The network sees the dirty image Phi^dagger y divided by the PSF peak ((Phi^dagger Phi delta)(centre),
so that a unit point source gives a unit peak) and scaled to unit RMS; it predicts the solution
of the plain solver in the same units.  The prediction x0 then starts SDMM together with the weights
W0 = delta / (delta + |Psi^dagger x0|), delta = std(Psi^dagger x0): the network stands in for the
first weighted-l1 pass, so a warm solve runs one pass fewer; the SDMM duals start from the
optimality conditions at x0.  The constraints and the stopping test of the solve are unchanged, so
the network only changes how many iterations are needed, and the plain solve from zero is the
fallback when the warm-started one does not meet the test.

Every step runs in libsarahip (operator, dictionary, solver, U-Net kernels); this module only
arranges the calls.  Training pairs come from the plain batched solver on synthetic skies.
"""
from __future__ import annotations

import json
import os
import time

import numpy as np

from . import sarahip as sh
from . import synth

WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights", "unet_b32_l4.npy")


def layer_list(base: int, levels: int):
    """[(kind, cin, cout)] in the library's parameter order (see sh_unet_create)."""
    out = []
    for l in range(levels):
        c = base << l
        out += [("conv3", 1 if l == 0 else c // 2, c), ("conv3", c, c)]
    for l in range(levels - 2, -1, -1):
        c = base << l
        out += [("tconv", 2 * c, c), ("conv3", 2 * c, c), ("conv3", c, c)]
    out.append(("head", base, 1))
    return out


def he_init(base: int, levels: int, seed: int) -> np.ndarray:
    """Gaussian weights with variance 2 / fan-in and zero biases in the flat layout, except the head:
    weights at a tenth of that scale and bias 0.05, so that the first predictions are small and
    positive, like the targets."""
    g = np.random.Generator(np.random.PCG64(np.random.SeedSequence([1502, 5037, 9, seed])))
    flat = []
    for kind, cin, cout in layer_list(base, levels):
        if kind == "conv3":
            nw, fan_in = cout * cin * 9, cin * 9
        elif kind == "tconv":
            nw, fan_in = cin * cout * 4, cin * 4
        else:
            nw, fan_in = cin * cout, cin
        if kind == "head":
            flat.append(0.1 * g.standard_normal(nw) * np.sqrt(2.0 / fan_in))
            flat.append(np.full(cout, 0.05))
        else:
            flat.append(g.standard_normal(nw) * np.sqrt(2.0 / fan_in))
            flat.append(np.zeros(cout))
    return np.concatenate(flat).astype(np.float32)


class WarmStart:
    """A U-Net with weights, applied as x0 = s * U(d / s)."""

    def __init__(self, weights=None, base: int = 32, levels: int = 4):
        self.base, self.levels = base, levels
        self.u = sh.unet_create(base, levels)
        if weights is not None:
            sh.unet_set_params(self.u, np.asarray(weights, dtype=np.float32))

    @classmethod
    def load(cls, path: str = WEIGHTS):
        meta = json.load(open(os.path.splitext(path)[0] + ".json"))
        return cls(np.load(path, allow_pickle=False), meta["base"], meta["levels"])

    def close(self):
        if self.u:
            sh.unet_destroy(self.u)
            self.u = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def predict(self, op, y, n: int, P: int, dev):
        """x0 (P x n x n, device) for the visibilities y of a plan with P problems."""
        import torch
        x0 = torch.empty((P, n, n), device=dev)
        sh.warm_start(self.u, op, y, x0)
        return x0


def warm_solve(ws: WarmStart, op, psi, y, eps, params, n: int, dev, x_out, replace_first_pass: bool = True,
               duals: bool = True, fallback: bool = True):
    """SDMM from the network's x0.  With replace_first_pass the first weights come from x0 by the
    reweighting rule and the solve runs one pass fewer than params.passes; otherwise x0 only starts
    the first (unweighted) pass.  With duals the SDMM duals also start from x0 (z_from_x0).

    The plain solve from zero stays the fallback: if the warm-started solve ends without meeting its
    stopping test in its last pass, or with a block outside eps_i (1 + eps_slack), the plain solve with
    `params` runs from zero and its image is returned.  Returns (info, block residuals, seconds including
    the network and any fallback); info["path"] is "warm" or "plain fallback" (info["warm_info"] then
    holds the warm attempt's record)."""
    import torch
    P = sh.op_query(op)["P"]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    x0 = ws.predict(op, y, n, P, dev)
    prm = sh.SdmmParams()
    for f, _ in sh.SdmmParams._fields_:
        setattr(prm, f, getattr(params, f))
    if replace_first_pass:
        prm.passes = max(1, params.passes - 1)
        prm.w_from_x0 = 1
    prm.z_from_x0 = 1 if duals else 0
    info, resid = sh.sdmm_solve(op, psi, y, eps, None, x0, prm, x_out)
    infos = info if isinstance(info, list) else [info]
    ok = all(i["converged"] == 1 for i in infos) and bool(np.all(resid <= np.asarray(eps) * (1.0 + params.eps_slack)))
    if fallback and not ok:
        warm = info
        info, resid = sh.sdmm_solve(op, psi, y, eps, None, None, params, x_out)
        for i in (info if isinstance(info, list) else [info]):
            i["path"] = "plain fallback"
            i["warm_info"] = warm
    else:
        for i in infos:
            i["path"] = "warm"
    torch.cuda.synchronize()
    return info, resid, time.perf_counter() - t0
