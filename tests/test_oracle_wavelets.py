"""Pins for the oracle's SARA dictionary: Daubechies filters, periodic DWT, Psi Psi^dagger = I.

Closed forms: db1 = [1, 1]/sqrt 2 and db2 = [1+s3, 3+s3, 3-s3, 1-s3]/(4 sqrt 2).
Invariants: sum h = sqrt 2, double-shift orthonormality, p vanishing moments of
the high-pass, orthonormal periodic transforms at every length, Parseval.
Layout: a one-level Haar step on a 4 x 4 image written out by its textbook
formula fixes the quadrant convention.
"""
import numpy as np
import pytest

from oracle import wavelets
from paper_1502_05037_amd import synth


def test_db1_db2_closed_forms():
    np.testing.assert_allclose(wavelets.daubechies(1), [2 ** -0.5, 2 ** -0.5], rtol=1e-15)
    s3 = np.sqrt(3.0)
    db2 = np.array([1 + s3, 3 + s3, 3 - s3, 1 - s3]) / (4 * np.sqrt(2.0))
    np.testing.assert_allclose(wavelets.daubechies(2), db2, rtol=1e-14, atol=1e-16)


@pytest.mark.parametrize("p", range(1, 9))
def test_filter_invariants(p):
    h = wavelets.daubechies(p)
    g = wavelets.highpass(h)
    assert len(h) == 2 * p
    assert h.sum() == pytest.approx(np.sqrt(2.0), abs=1e-15)
    for m in range(p):
        acc = np.dot(h[: 2 * p - 2 * m], h[2 * m:])
        assert acc == pytest.approx(1.0 if m == 0 else 0.0, abs=1e-14)
        assert np.dot(g[: 2 * p - 2 * m], g[2 * m:]) == pytest.approx(1.0 if m == 0 else 0.0, abs=1e-14)
    k = np.arange(2 * p, dtype=np.float64)
    for j in range(p):
        mom = np.sum(g * k ** j)
        scale = np.sum(np.abs(g) * k ** j)
        assert abs(mom) <= 1e-14 * scale
    # extremal phase: the energy is front-loaded (the partial energies dominate every other
    # filter with the same |H|), so the first tap is the largest among reversals
    assert p == 1 or abs(h[0]) > abs(h[-1])


@pytest.mark.parametrize("p", range(1, 9))
@pytest.mark.parametrize("L", [2, 4, 8, 16, 64])
def test_periodic_analysis_orthonormal(p, L):
    A = wavelets.analysis_matrix(wavelets.daubechies(p), L)
    np.testing.assert_allclose(A @ A.T, np.eye(L), atol=2e-15)
    np.testing.assert_allclose(A.T @ A, np.eye(L), atol=2e-15)


def test_haar_layout_4x4():
    x = np.arange(16, dtype=np.float64).reshape(4, 4) ** 1.5
    c = wavelets.dwt2(x, 1, 1)
    r = 1 / np.sqrt(2)
    # rows: a[k] = (x[2k] + x[2k+1]) r, d[k] = (x[2k] - x[2k+1]) r  (g = [h1, -h0])
    rows = np.concatenate([(x[:, 0::2] + x[:, 1::2]) * r, (x[:, 0::2] - x[:, 1::2]) * r], axis=1)
    expect = np.concatenate([(rows[0::2] + rows[1::2]) * r, (rows[0::2] - rows[1::2]) * r], axis=0)
    np.testing.assert_allclose(c, expect, rtol=1e-13)
    # top-left is the local mean scaled by 2 (low-low), top-right row differences
    assert c[0, 0] == pytest.approx((x[0, 0] + x[0, 1] + x[1, 0] + x[1, 1]) / 2)
    assert c[0, 2] == pytest.approx((x[0, 0] - x[0, 1] + x[1, 0] - x[1, 1]) / 2)
    assert c[2, 0] == pytest.approx((x[0, 0] + x[0, 1] - x[1, 0] - x[1, 1]) / 2)


def test_db2_one_level_entry_by_definition():
    # one coefficient of each quadrant by the periodic sums written out directly
    n = 8
    x = synth.rng(98, 0, 0).normal(size=(n, n))
    h = wavelets.daubechies(2)
    g = wavelets.highpass(h)
    c = wavelets.dwt2(x, 2, 1)

    def row_step(f, r, k):
        return sum(f[t] * x[r, (2 * k + t) % n] for t in range(4))

    def full(fr, fc, k1, k2):
        return sum(fc[t] * row_step(fr, (2 * k1 + t) % n, k2) for t in range(4))

    assert c[1, 2] == pytest.approx(full(h, h, 1, 2), rel=1e-13)
    assert c[1, 4 + 3] == pytest.approx(full(g, h, 1, 3), rel=1e-13)       # row-high, column-low
    assert c[4 + 2, 0] == pytest.approx(full(h, g, 2, 0), rel=1e-13)       # row-low, column-high
    assert c[4 + 3, 4 + 1] == pytest.approx(full(g, g, 3, 1), rel=1e-13)


@pytest.mark.parametrize("n,levels", [(16, 4), (64, 4), (8, 3)])
def test_sara_parseval_and_identity(n, levels):
    psi = wavelets.SARA(n, levels)
    x = synth.rng(98, n, 0).normal(size=(n, n))
    c = psi.adj(x)
    assert c.shape == (9, n, n)
    assert np.linalg.norm(c) == pytest.approx(np.linalg.norm(x), rel=1e-14)
    np.testing.assert_allclose(psi.fwd(c), x, atol=1e-13)
    # adjointness on a random coefficient set
    cc = synth.rng(98, n, 1).normal(size=(9, n, n))
    assert np.sum(psi.adj(x) * cc) == pytest.approx(np.sum(x * psi.fwd(cc)), rel=1e-12)


@pytest.mark.parametrize("p", range(1, 9))
def test_each_basis_perfect_reconstruction(p):
    n = 32
    x = synth.rng(98, p, 2).normal(size=(n, n))
    c = wavelets.dwt2(x, p, 4)
    np.testing.assert_allclose(wavelets.idwt2(c, p, 4), x, atol=1e-13)
    assert np.linalg.norm(c) == pytest.approx(np.linalg.norm(x), rel=1e-14)


def test_dirac_plane_and_masks():
    n = 16
    x = synth.rng(98, 3, 3).normal(size=(n, n))
    psi = wavelets.SARA(n, 4, mask=0b101)   # Dirac + db2
    c = psi.adj(x)
    np.testing.assert_allclose(c[0], x / np.sqrt(2))
    np.testing.assert_allclose(psi.fwd(c), x, atol=1e-13)
