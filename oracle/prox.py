"""Proximal maps of the three terms of problem (3) (FP64 closed forms).

Problem (3) minimises the weighted l1 norm of Psi^dagger x subject to one l2-ball
constraint per data block and x in the positive orthant.  SDMM touches each term
only through its proximal map:
* weighted l1:  soft(v, tau) = sign(v) max(|v| - tau, 0), tau = gamma w;
* l2 ball B(c, eps):  c + (t - c) min(1, eps / ||t - c||);
* positive orthant:  max(v, 0).
"""
from __future__ import annotations

import numpy as np


def soft(v: np.ndarray, tau) -> np.ndarray:
    """Soft threshold; |v| == tau maps to 0."""
    return np.sign(v) * np.maximum(np.abs(v) - tau, 0.0)


def ball(t: np.ndarray, c: np.ndarray, eps: float) -> np.ndarray:
    """Projection of t onto {s : ||s - c||_2 <= eps}; the identity inside, boundary included."""
    r = np.linalg.norm(t - c)
    if r <= eps:
        return np.array(t, copy=True)
    return c + (t - c) * (eps / r)


def positive(v: np.ndarray) -> np.ndarray:
    return np.maximum(v, 0.0)
