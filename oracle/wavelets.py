"""The SARA sparsity dictionary Psi (FP64, CPU).

The paper's dictionary is a concatenation of q coherent bases,
Psi = [Psi_1, ..., Psi_q], and the analysis prior uses Psi^dagger (SARA
paragraph).  The bases are Dirac plus Daubechies db1..db8, each with four
decomposition levels, scaled by 1/sqrt(q) so that Psi Psi^dagger = I.

Conventions (the paper fixes none):
* db_p scaling filter h (2p taps) from the spectral factorisation of
  P(y) = sum_{k<p} C(p-1+k, k) y^k with y = sin^2(w/2): for each root y_j the
  pair z + 1/z = 2 - 4 y_j is split keeping |z| < 1, and
  (1 + z)^p prod_j (z - z_j) is expanded; h[k] is the coefficient of
  z^(2p-1-k), scaled so that sum(h) = sqrt(2).  For db2 this puts
  (1 + sqrt 3) / (4 sqrt 2) first.  High-pass g[k] = (-1)^k h[2p-1-k].
* Periodic 1D analysis of length L: a[k] = sum_t h[t] x[(2k+t) mod L],
  d[k] = sum_t g[t] x[(2k+t) mod L], k < L/2; synthesis is the transpose.
* One 2D level filters within rows into [a | d], then within columns into
  [a ; d].  Quadrants: LL top-left, (row-high, column-low) top-right,
  (row-low, column-high) bottom-left, HH bottom-right.  Levels recurse on LL
  (Mallat layout), planes ordered Dirac, db1, ..., db8.
"""
from __future__ import annotations

from functools import lru_cache

import mpmath
import numpy as np
import scipy.sparse

SARA_MASK = 0x1FF  # bit 0 = Dirac, bit b = db_b


@lru_cache(maxsize=None)
def daubechies(p: int) -> np.ndarray:
    """db_p scaling filter (2p taps, FP64), by spectral factorisation in 60-digit arithmetic."""
    if p < 1:
        raise ValueError("p >= 1")
    with mpmath.workdps(60):
        coeffs = [mpmath.binomial(p - 1 + k, k) for k in range(p)]  # P(y), increasing powers
        y_roots = mpmath.polyroots(coeffs[::-1], maxsteps=400, extraprec=200) if p > 1 else []
        if not isinstance(y_roots, (list, tuple)):
            y_roots = [y_roots]
        z_roots = []
        for y in y_roots:
            s = 2 - 4 * y
            disc = mpmath.sqrt(s * s - 4)
            za, zb = (s + disc) / 2, (s - disc) / 2
            z_roots.append(za if abs(za) < 1 else zb)
        poly = [mpmath.mpf(1)]  # increasing powers of z
        factors = [[mpmath.mpf(1), mpmath.mpf(1)]] * p + [[-zr, mpmath.mpf(1)] for zr in z_roots]
        for f in factors:
            nxt = [mpmath.mpc(0)] * (len(poly) + 1)
            for i, a in enumerate(poly):
                nxt[i] += a * f[0]
                nxt[i + 1] += a * f[1]
            poly = nxt
        c = [mpmath.re(a) for a in poly]
        tot = mpmath.fsum(c)
        scale = mpmath.sqrt(2) / tot
        h = [c[2 * p - 1 - k] * scale for k in range(2 * p)]
        return np.array([float(v) for v in h], dtype=np.float64)


def highpass(h: np.ndarray) -> np.ndarray:
    L = len(h)
    return np.array([(-1) ** k * h[L - 1 - k] for k in range(L)], dtype=np.float64)


def analysis_matrix(h: np.ndarray, L: int) -> np.ndarray:
    """Periodic one-level analysis matrix A (L x L): rows 0..L/2-1 low-pass, then high-pass."""
    g = highpass(h)
    A = np.zeros((L, L))
    for k in range(L // 2):
        for t in range(len(h)):
            A[k, (2 * k + t) % L] += h[t]
            A[L // 2 + k, (2 * k + t) % L] += g[t]
    return A


@lru_cache(maxsize=None)
def _sparse_analysis(p: int, L: int):
    return scipy.sparse.csr_matrix(analysis_matrix(daubechies(p), L))


def dwt2(x: np.ndarray, p: int, levels: int) -> np.ndarray:
    """Orthonormal periodic 2D analysis W^T x with db_p, Mallat layout."""
    c = np.array(x, dtype=np.float64, copy=True)
    L = c.shape[0]
    for _ in range(levels):
        A = _sparse_analysis(p, L)
        rows = (A @ c[:L, :L].T).T           # within rows into [a | d]
        c[:L, :L] = A @ rows                 # within columns into [a ; d]
        L //= 2
    return c


def idwt2(c: np.ndarray, p: int, levels: int) -> np.ndarray:
    """Synthesis W c with db_p, the transpose of :func:`dwt2`."""
    x = np.array(c, dtype=np.float64, copy=True)
    n = x.shape[0]
    for lev in reversed(range(levels)):
        L = n >> lev
        A = _sparse_analysis(p, L)
        cols = A.T @ x[:L, :L]               # undo the column step
        x[:L, :L] = (A.T @ cols.T).T         # undo the row step
    return x


class SARA:
    """Psi = (1/sqrt q) [Psi_b for b in mask]; bit 0 = Dirac, bit b = db_b (b = 1..8)."""

    def __init__(self, n: int, levels: int = 4, mask: int = SARA_MASK):
        if n % (1 << levels):
            raise ValueError("n must be divisible by 2**levels")
        self.n, self.levels, self.mask = n, levels, mask
        self.bases = [b for b in range(9) if mask >> b & 1]
        self.q = len(self.bases)
        self.scale = 1.0 / np.sqrt(self.q)

    @property
    def D(self) -> int:
        return self.q * self.n * self.n

    def adj(self, x: np.ndarray) -> np.ndarray:
        """Psi^dagger x: (q, n, n) coefficient planes."""
        out = np.empty((self.q, self.n, self.n))
        for i, b in enumerate(self.bases):
            out[i] = x if b == 0 else dwt2(x, b, self.levels)
        return out * self.scale

    def fwd(self, c: np.ndarray) -> np.ndarray:
        """Psi c: image (n, n) from (q, n, n) coefficient planes."""
        x = np.zeros((self.n, self.n))
        for i, b in enumerate(self.bases):
            x += c[i] if b == 0 else idwt2(c[i], b, self.levels)
        return x * self.scale
