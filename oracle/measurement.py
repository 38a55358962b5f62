"""Measurement operator Phi and its real adjoint (FP64, CPU).

The paper discretises the interferometric measurement as y = Phi x + n with
y in C^M, x in R^N (measurement-model paragraph); the image is real and
non-negative (problem (1)), so the adjoint used by every solver step is the
real-linear one, Phi^dagger v = Re(Phi^H v).

Conventions (the paper fixes none):
* x is n x n, indexed x[r, c]; pixel offsets are n1 = r - n/2, n2 = c - n/2.
* u, v are in radians per pixel, in [-pi, pi); u pairs with rows, v with columns.
* (Phi x)_m = sum_{r,c} x[r, c] exp(-i (u_m n1 + v_m n2))  (natural weighting, no w-term).

Two realisations:
* :class:`DFT` is that definition written out (exact, O(M N)).
* :class:`NUFFT` is the operator the GPU computes: Phi = G F Z S with an
  alpha-times oversampled grid of side K = alpha n, S dividing by the KB
  transform, Z zero-padding with pixel offset n placed at grid index n mod K,
  F the unnormalised forward DFT, and G the J x J Kaiser-Bessel interpolation at
  kappa = u K / (2 pi) over taps j = floor(kappa) - J/2 + 1 + t, t = 0..J-1,
  with grid indices taken mod K.
"""
from __future__ import annotations

import os

import numpy as np
import scipy.fft

from . import kb


def pixel_offsets(n: int) -> np.ndarray:
    """Signed pixel offsets n1 = r - n/2 for r = 0..n-1."""
    return np.arange(n, dtype=np.float64) - n // 2


class DFT:
    """Direct evaluation of the discretised measurement equation."""

    def __init__(self, uv: np.ndarray, n: int):
        self.uv = np.asarray(uv, dtype=np.float64)
        self.n = n
        self.M = len(self.uv)
        off = pixel_offsets(n)
        self.E1 = np.exp(-1j * np.outer(self.uv[:, 0], off))  # (M, n) row factor
        self.E2 = np.exp(-1j * np.outer(self.uv[:, 1], off))  # (M, n) column factor

    def fwd_complex(self, x: np.ndarray) -> np.ndarray:
        """Phi x for a complex image x (n, n)."""
        return np.sum((self.E1 @ x) * self.E2, axis=1)

    def adj_complex(self, v: np.ndarray) -> np.ndarray:
        """Phi^H v as a complex image (n, n)."""
        return self.E1.conj().T @ (v[:, None] * self.E2.conj())

    def fwd(self, x: np.ndarray) -> np.ndarray:
        return self.fwd_complex(np.asarray(x, dtype=np.float64))

    def adj(self, v: np.ndarray) -> np.ndarray:
        """Real adjoint Re(Phi^H v)."""
        return self.adj_complex(np.asarray(v, dtype=np.complex128)).real


class NUFFT:
    """FP64 non-uniform FFT with the KB kernel, as computed on the GPU."""

    def __init__(self, uv: np.ndarray, n: int, J: int, alpha: int = 2, chunk: int = 1 << 20):
        if J % 2:
            raise ValueError("kernel width J must be even")
        self.uv = np.asarray(uv, dtype=np.float64)
        self.n, self.J, self.alpha = n, J, alpha
        self.K = K = alpha * n
        self.M = len(self.uv)
        self.beta = kb.beta(J, alpha)
        self.chunk = chunk
        off = pixel_offsets(n)
        ph = kb.psi_hat(off / K, J, self.beta)
        self.deapod = 1.0 / np.outer(ph, ph)                 # S, (n, n)
        self.grid_idx = np.mod(off.astype(np.int64), K)      # Z, pixel offset -> grid index

    def _taps(self, lo: int, hi: int):
        """Grid indices (mod K) and 1D KB weights for visibilities lo..hi-1, per axis."""
        K, J = self.K, self.J
        kappa = self.uv[lo:hi] * (K / (2.0 * np.pi))       # (m, 2)
        base = np.floor(kappa)
        t = np.arange(J, dtype=np.float64)
        j = base[:, :, None] - J / 2 + 1 + t[None, None, :]  # (m, 2, J)
        w = kb.psi(kappa[:, :, None] - j, J, self.beta)
        return np.mod(j.astype(np.int64), K), w

    def grid_of_image(self, x: np.ndarray) -> np.ndarray:
        """F Z S x: the deapodised image placed on the K x K grid (pixel offset n at index n mod K), then
        the unnormalised forward DFT exp(-2 pi i k n / K)."""
        K = self.K
        grid = np.zeros((K, K), dtype=np.complex128)
        grid[np.ix_(self.grid_idx, self.grid_idx)] = np.asarray(x, dtype=np.float64) * self.deapod
        return self._fft2(grid)

    def image_of_grid(self, G: np.ndarray) -> np.ndarray:
        """Re(S Z^T F^H G): unnormalised inverse DFT exp(+2 pi i k n / K), crop, deapodise, real part."""
        Y = self._ifft2(G) * (self.K * self.K)
        return Y[np.ix_(self.grid_idx, self.grid_idx)].real * self.deapod

    def _fft2(self, a):
        return np.fft.fft2(a)

    def _ifft2(self, a):
        return np.fft.ifft2(a)

    def interp(self, X: np.ndarray) -> np.ndarray:
        """G X: J x J Kaiser-Bessel interpolation of the grid at every visibility."""
        out = np.zeros(self.M, dtype=np.complex128)
        for lo in range(0, self.M, self.chunk):
            hi = min(self.M, lo + self.chunk)
            j, w = self._taps(lo, hi)
            acc = np.zeros(hi - lo, dtype=np.complex128)
            for t1 in range(self.J):
                for t2 in range(self.J):
                    acc += w[:, 0, t1] * w[:, 1, t2] * X[j[:, 0, t1], j[:, 1, t2]]
            out[lo:hi] = acc
        return out

    def spread(self, v: np.ndarray) -> np.ndarray:
        """G^H v: every visibility spread onto its J x J taps of the grid."""
        K = self.K
        v = np.asarray(v, dtype=np.complex128)
        gre = np.zeros(K * K)
        gim = np.zeros(K * K)
        for lo in range(0, self.M, self.chunk):
            hi = min(self.M, lo + self.chunk)
            j, w = self._taps(lo, hi)
            vv = v[lo:hi]
            for t1 in range(self.J):
                for t2 in range(self.J):
                    idx = j[:, 0, t1] * K + j[:, 1, t2]
                    ww = w[:, 0, t1] * w[:, 1, t2]
                    gre += np.bincount(idx, weights=ww * vv.real, minlength=K * K)
                    gim += np.bincount(idx, weights=ww * vv.imag, minlength=K * K)
        return (gre + 1j * gim).reshape(K, K)

    def fwd(self, x: np.ndarray) -> np.ndarray:
        return self.interp(self.grid_of_image(x))

    def adj(self, v: np.ndarray) -> np.ndarray:
        """Real adjoint Re(S Z^T F^H G^H v)."""
        return self.image_of_grid(self.spread(v))


class NUFFTCompiled(NUFFT):
    """The same operator with G and G^H as compiled loops (oracle/nufft_c.c, float64, OpenMP) and the
    FFTs on several threads: fast enough for tens of millions of visibilities.  Its Kaiser-Bessel
    weights come from the Bessel series in C, computed once per operator (16 J bytes per visibility
    are held); it agrees with :class:`NUFFT` to rounding."""

    def __init__(self, uv: np.ndarray, n: int, J: int, alpha: int = 2, threads: int | None = None):
        super().__init__(uv, n, J, alpha)
        from . import cbuild
        self._lib = cbuild.load()
        self.threads = int(threads or len(os.sched_getaffinity(0)))
        self.uv = np.ascontiguousarray(self.uv, dtype=np.float64)
        # visit the visibilities sorted by grid cell (u cell, then v cell) so that consecutive ones touch
        # neighbouring grid rows; taps of every visibility computed once, in that order: first index per
        # axis and J weights per axis
        cell = np.floor(self.uv * (self.K / (2.0 * np.pi))).astype(np.int64)
        self.order = np.ascontiguousarray(np.lexsort((cell[:, 1], cell[:, 0])), dtype=np.int64)
        uv_s = np.ascontiguousarray(self.uv[self.order])
        self.j0 = np.empty((self.M, 2), dtype=np.int64)
        self.w = np.empty((self.M, 2, J), dtype=np.float64)
        self._lib.oracle_taps(self.M, uv_s.ctypes.data, self.K, J, self.beta, self.j0.ctypes.data,
                              self.w.ctypes.data, self.threads)

    def _fft2(self, a):
        return scipy.fft.fft2(a, workers=self.threads)

    def _ifft2(self, a):
        return scipy.fft.ifft2(a, workers=self.threads)

    def interp(self, X: np.ndarray) -> np.ndarray:
        X = np.ascontiguousarray(X, dtype=np.complex128)
        out = np.empty(self.M, dtype=np.complex128)
        self._lib.oracle_interp_fwd(self.M, self.K, self.J, self.j0.ctypes.data, self.w.ctypes.data,
                                    self.order.ctypes.data, X.ctypes.data, out.ctypes.data, self.threads)
        return out

    def spread(self, v: np.ndarray) -> np.ndarray:
        v = np.ascontiguousarray(v, dtype=np.complex128)
        G = np.empty((self.K, self.K), dtype=np.complex128)
        if self._lib.oracle_interp_adj(self.M, self.K, self.J, self.j0.ctypes.data, self.w.ctypes.data,
                                       self.order.ctypes.data, v.ctypes.data, G.ctypes.data, self.threads) != 0:
            raise MemoryError("oracle gridding: private grids do not fit in memory")
        return G

    def subset(self, lo: int, hi: int) -> "NUFFTCompiled":
        """The operator restricted to visibilities lo..hi-1 (one data block)."""
        return NUFFTCompiled(self.uv[lo:hi], self.n, self.J, self.alpha, self.threads)


class Identity:
    """Phi = I on R^N viewed in C^N (used to pin the solver against a closed form)."""

    def __init__(self, n: int):
        self.n = n
        self.M = n * n

    def fwd(self, x):
        return np.asarray(x, dtype=np.float64).ravel().astype(np.complex128)

    def adj(self, v):
        return np.asarray(v).real.reshape(self.n, self.n).astype(np.float64)


def op_norm(op, x0: np.ndarray, max_iter: int = 200, tol: float = 1e-12) -> float:
    """||Phi||_2 of the real-linear map R^N -> C^N: power iteration on Re(Phi^H Phi).

    Starts from x0 (a seeded Gaussian image), stops after max_iter steps or when
    the eigenvalue estimate changes by at most tol relative.
    """
    x = np.asarray(x0, dtype=np.float64)
    x = x / np.linalg.norm(x)
    lam = 0.0
    for _ in range(max_iter):
        y = op.adj(op.fwd(x))
        lam_new = float(np.vdot(x, y).real)
        x = y / np.linalg.norm(y)
        if lam > 0 and abs(lam_new - lam) <= tol * lam_new:
            lam = lam_new
            break
        lam = lam_new
    return float(np.sqrt(lam))


def block_density_weights(uv: np.ndarray, n: int, alpha: int, offsets) -> np.ndarray:
    """Density estimate a_b of 1 / ||Phi_b|| for every block b (weights that normalise the data splits).

    The paper splits the data into blocks (2) and constrains each block separately; scaling block b's
    constraint by any positive number leaves its ball unchanged.  For an n x n image the largest
    eigenvalue of Re(Phi_b^H Phi_b) is close to n^2 times the largest number of the block's uv samples
    in a square of side 2 pi / n (uniform density rho per unit area gives (2 pi)^2 rho).  Counted here
    on the cells floor(u K / (2 pi)) mod K of the K x K grid, K = alpha n (cell side 2 pi / K), as the
    largest sum over alpha x alpha cells at any cell offset, periodic in both axes:
        count_b = max_(r, c) sum_(a, d < alpha) H_b[(r + a) mod K, (c + d) mod K],
        a_b = 1 / (n sqrt(count_b)).
    """
    K = alpha * n
    uv = np.asarray(uv, dtype=np.float64)
    cells = np.mod(np.floor(uv * (float(K) / (2.0 * np.pi))).astype(np.int64), K)
    off = np.asarray(offsets, dtype=np.int64)
    out = np.empty(len(off) - 1)
    for b in range(len(off) - 1):
        H = np.zeros((K, K))
        np.add.at(H, (cells[off[b]:off[b + 1], 0], cells[off[b]:off[b + 1], 1]), 1.0)
        win = np.zeros((K, K))
        for a in range(alpha):
            for d in range(alpha):
                win += np.roll(np.roll(H, -a, axis=0), -d, axis=1)
        out[b] = 1.0 / np.sqrt(float(n) * float(n) * win.max())
    return out


class BlockWeighted:
    """The operator with block b's rows scaled by a_b: (A x)_m = a_b (Phi x)_m for m in block b."""

    def __init__(self, op, offsets, a):
        self.op, self.n = op, op.n
        self.w = np.repeat(np.asarray(a, dtype=np.float64), np.diff(np.asarray(offsets, dtype=np.int64)))

    def fwd(self, x):
        return self.w * self.op.fwd(x)

    def adj(self, v):
        return self.op.adj(self.w * np.asarray(v, dtype=np.complex128))
