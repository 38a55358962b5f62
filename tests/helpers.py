"""Seeded problem builders shared by the GPU parity tests (inputs from synth, expected values from oracle)."""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from oracle import measurement, problem as oproblem
from paper_1502_05037_amd import synth


@dataclass
class Problem:
    n: int
    J: int
    uv: np.ndarray
    offsets: np.ndarray
    sizes: np.ndarray
    x_true: np.ndarray
    y: np.ndarray          # complex128, user order, from the oracle NUFFT (FP64) + noise
    eps: np.ndarray
    sigma: float
    op: object             # oracle NUFFT


def build(cfg: int, n: int, m: int, R: int, J: int, coverage: str = "gaussian", n_points: int = 20,
          dr: float = 3.0, prob: int = 0, snr: float = 30.0, spread: float = 0.6) -> Problem:
    g_uv = synth.rng(cfg, prob, synth.UV)
    uv = synth.uv_gaussian(m, g_uv) if coverage == "gaussian" else synth.uv_radial(m, g_uv)
    uv = synth.sort_by_radius(uv)
    sizes = synth.block_sizes(m, R, synth.rng(cfg, prob, synth.BLOCKS), spread) if R > 1 else np.array([m])
    off = synth.offsets(sizes)
    x = synth.sky(n, n_points, dr, synth.rng(cfg, prob, synth.SKY))
    x = x.astype(np.float32).astype(np.float64)
    op = measurement.NUFFT(uv, n, J)
    clean = op.fwd(x)
    sigma = oproblem.noise_sigma(clean, snr)
    y = oproblem.add_noise(clean, sigma, synth.complex_normal(m, synth.rng(cfg, prob, synth.NOISE)))
    y = y.astype(np.complex64).astype(np.complex128)
    eps = oproblem.eps_blocks(sigma, sizes)
    return Problem(n, J, uv, off, sizes, x, y, eps, sigma, op)


def rel(a, b) -> float:
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))
