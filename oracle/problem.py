"""Problem set-up for the blocked problem (3) (FP64, host).

The paper models each data block as y_i = Phi_i x + n_i with eps_i an upper
bound on ||n_i||_2 that "can be accurately estimated" (text around (1)-(3)).
Readings used here:
* complex Gaussian noise at a given input SNR:
  sigma = ||Phi x||_2 / sqrt(M) * 10^(-SNR/20), n_m = sigma/sqrt(2) (a + i b);
* ||n_i||^2 ~ (sigma^2/2) chi^2_{2 M_i}, whose mean + 2 s.d. gives
  eps_i = sigma sqrt(M_i + 2 sqrt(M_i));
* dirty image Phi^dagger y divided by the PSF peak (Phi^dagger Phi delta_0)[centre].
"""
from __future__ import annotations

import numpy as np


def noise_sigma(clean_vis: np.ndarray, snr_db: float) -> float:
    return float(np.linalg.norm(clean_vis) / np.sqrt(len(clean_vis)) * 10.0 ** (-snr_db / 20.0))


def add_noise(clean_vis: np.ndarray, sigma: float, draws: np.ndarray) -> np.ndarray:
    """y = Phi x + sigma/sqrt(2) (a + ib) with `draws` = a + ib, a, b ~ N(0, 1)."""
    return clean_vis + sigma / np.sqrt(2.0) * draws


def eps_blocks(sigma: float, sizes) -> np.ndarray:
    m = np.asarray(sizes, dtype=np.float64)
    return sigma * np.sqrt(m + 2.0 * np.sqrt(m))


def dirty_image(op, y: np.ndarray) -> np.ndarray:
    n = op.n
    delta = np.zeros((n, n))
    delta[n // 2, n // 2] = 1.0
    peak = op.adj(op.fwd(delta))[n // 2, n // 2]
    return op.adj(y) / peak
