"""Seeded synthetic inputs: sky images, uv coverages, block splits, noise draws.

This module only draws random inputs.  It holds none of the imaging method's
arithmetic (no measurement operator, no wavelets, no noise scaling), so both the
FP64 CPU oracle and the GPU path can take their inputs from it.

The inputs mirror the workload family of the paper's problem (3): a positive
sky image, M >> N complex visibilities on a continuous uv plane, and R
contiguous data blocks as in the block split (2).  The paper uses no dataset;
these draws stand in for telescope data.

Every generator takes a ``numpy.random.Generator`` built by :func:`rng`, which
keys a PCG64 stream on (1502, 5037, config, problem, stream).  Stream ids:
0 = sky, 1 = uv, 2 = noise, 3 = block sizes.
"""
from __future__ import annotations

import numpy as np

SKY, UV, NOISE, BLOCKS = 0, 1, 2, 3


def rng(config: int, problem: int, stream: int) -> np.random.Generator:
    """PCG64 generator keyed on (1502, 5037, config, problem, stream)."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([1502, 5037, config, problem, stream])))


def sky(n: int, n_points: int, dynamic_range: float, g: np.random.Generator) -> np.ndarray:
    """Positive n x n sky: 3-6 elliptical Gaussian blobs plus point sources.

    Blob widths are drawn in [2, 8] px at n = 64 and scale with n/64.  Point
    source fluxes are log-uniform in [10**-dynamic_range, 1] times the blob peak.
    The image is normalised to a maximum of 1 and returned as float64 (n, n),
    indexed [row, column].
    """
    img = np.zeros((n, n), dtype=np.float64)
    rr, cc = np.meshgrid(np.arange(n, dtype=np.float64), np.arange(n, dtype=np.float64), indexing="ij")
    n_blobs = int(g.integers(3, 7))
    scale = n / 64.0
    for _ in range(n_blobs):
        r0, c0 = g.uniform(0.15 * n, 0.85 * n, size=2)
        s_maj, s_min = g.uniform(2.0, 8.0, size=2) * scale
        ang = g.uniform(0.0, np.pi)
        peak = g.uniform(0.1, 1.0)
        dr, dc = rr - r0, cc - c0
        a = np.cos(ang) * dr + np.sin(ang) * dc
        b = -np.sin(ang) * dr + np.cos(ang) * dc
        img += peak * np.exp(-0.5 * ((a / s_maj) ** 2 + (b / s_min) ** 2))
    peak_val = img.max()
    pr = g.integers(0, n, size=n_points)
    pc = g.integers(0, n, size=n_points)
    flux = 10.0 ** g.uniform(-dynamic_range, 0.0, size=n_points) * peak_val
    np.add.at(img, (pr, pc), flux)
    img /= img.max()
    return img


def uv_gaussian(m: int, g: np.random.Generator, sigma: float = np.pi / 4) -> np.ndarray:
    """M uv points, i.i.d. N(0, sigma^2) per axis, resampled until inside [-pi, pi)."""
    out = np.empty((m, 2), dtype=np.float64)
    filled = 0
    while filled < m:
        cand = g.normal(0.0, sigma, size=(2 * (m - filled) + 16, 2))
        ok = np.all((cand >= -np.pi) & (cand < np.pi), axis=1)
        cand = cand[ok][: m - filled]
        out[filled: filled + len(cand)] = cand
        filled += len(cand)
    return out


def uv_radial(m: int, g: np.random.Generator, r_max: float = 0.98 * np.pi) -> np.ndarray:
    """M uv points with angle ~ U[0, 2pi) and radius ~ U[0, r_max): planar density ~ 1/r."""
    th = g.uniform(0.0, 2.0 * np.pi, size=m)
    r = g.uniform(0.0, r_max, size=m)
    uv = np.stack([r * np.cos(th), r * np.sin(th)], axis=1)
    # cos/sin can round a point onto +pi; keep the half-open box [-pi, pi).
    return np.clip(uv, -np.pi, np.nextafter(np.pi, 0.0))


def sort_by_radius(uv: np.ndarray) -> np.ndarray:
    """Order uv points by |(u, v)| so that contiguous blocks are uv annuli."""
    return uv[np.argsort(np.hypot(uv[:, 0], uv[:, 1]), kind="stable")]


def block_sizes(m: int, r: int, g: np.random.Generator, spread: float = 0.6) -> np.ndarray:
    """R positive block sizes around M/R (each M/R * (1 + U(-spread, spread))) summing to M.

    The draws are rescaled to sum to M and rounded by the largest-remainder rule.
    """
    raw = (m / r) * (1.0 + g.uniform(-spread, spread, size=r))
    raw *= m / raw.sum()
    base = np.floor(raw).astype(np.int64)
    short = m - int(base.sum())
    order = np.argsort(-(raw - base), kind="stable")
    base[order[:short]] += 1
    base = np.maximum(base, 1)
    # the clamp above can only add; take any excess back from the largest block
    base[np.argmax(base)] -= int(base.sum()) - m
    return base


def offsets(sizes: np.ndarray) -> np.ndarray:
    """Block offsets b_0 = 0 < b_1 < ... < b_R = M from block sizes."""
    return np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)


def complex_normal(m: int, g: np.random.Generator) -> np.ndarray:
    """M draws a + ib with a, b ~ N(0, 1) i.i.d. (unscaled)."""
    a = g.normal(size=m)
    b = g.normal(size=m)
    return a + 1j * b


def gaussian_vector(n: int, g: np.random.Generator) -> np.ndarray:
    """n i.i.d. N(0, 1) draws (test vectors, power-iteration starts)."""
    return g.normal(size=n)
