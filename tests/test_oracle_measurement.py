"""Pins for the oracle's measurement operator (KB kernel, DFT, NUFFT, operator norm).

The DFT is pinned by closed forms (point source, constant image) and adjoint
identities; the NUFFT by the DFT within the NUFFT's own approximation error; the
KB transform by numerical quadrature; the operator norm by a dense eigensolver.
"""
import numpy as np
import pytest
import scipy.integrate
import scipy.special

from oracle import kb, measurement
from paper_1502_05037_amd import synth


def test_beta_values():
    # Beatty et al. 2005 shape parameter, evaluated by hand for alpha = 2
    assert kb.beta(6, 2) == pytest.approx(np.pi * np.sqrt(9 * 2.25 - 0.8), rel=1e-15)
    assert kb.beta(6, 2) == pytest.approx(13.8551, abs=1e-4)
    assert kb.beta(8, 2) == pytest.approx(18.6389, abs=1e-4)


@pytest.mark.parametrize("J", [4, 6, 8])
def test_kb_window_values(J):
    b = kb.beta(J, 2)
    assert kb.psi(0.0, J, b) == pytest.approx(1.0)
    assert kb.psi(J / 2, J, b) == pytest.approx(1.0 / scipy.special.i0(b))
    assert kb.psi(J / 2 + 1e-9, J, b) == 0.0
    t = np.linspace(-J / 2, J / 2, 101)
    np.testing.assert_allclose(kb.psi(t, J, b), kb.psi(-t, J, b))


@pytest.mark.parametrize("J", [6, 8])
@pytest.mark.parametrize("xi", [0.0, 0.05, 0.13, 0.25, 0.5, 0.9, 1.4])
def test_kb_transform_matches_quadrature(J, xi):
    b = kb.beta(J, 2)
    num, _ = scipy.integrate.quad(lambda t: kb.psi(np.array([t]), J, b)[0] * np.cos(2 * np.pi * xi * t),
                                  -J / 2, J / 2, epsabs=1e-14, epsrel=1e-13, limit=200)
    assert kb.psi_hat(np.array([xi]), J, b)[0] == pytest.approx(num, rel=1e-9, abs=1e-12)


def _uv(m, seed):
    return synth.uv_gaussian(m, synth.rng(99, seed, synth.UV))


def test_dft_point_source_closed_form():
    n = 16
    uv = _uv(64, 0)
    op = measurement.DFT(uv, n)
    x = np.zeros((n, n))
    r0, c0 = 3, 12
    x[r0, c0] = 2.5
    n1, n2 = r0 - n // 2, c0 - n // 2
    expect = 2.5 * np.exp(-1j * (uv[:, 0] * n1 + uv[:, 1] * n2))
    np.testing.assert_allclose(op.fwd(x), expect, rtol=1e-13, atol=1e-13)


def test_dft_constant_image_dirichlet():
    n = 16
    uv = _uv(50, 1)
    op = measurement.DFT(uv, n)
    x = np.ones((n, n))

    def dirichlet(w):
        # sum_{k=-n/2}^{n/2-1} exp(-i w k) as a geometric series
        return np.exp(1j * w * n / 2) * (1 - np.exp(-1j * w * n)) / (1 - np.exp(-1j * w))

    np.testing.assert_allclose(op.fwd(x), dirichlet(uv[:, 0]) * dirichlet(uv[:, 1]), rtol=1e-11)


def test_dft_adjoint_identities():
    n, m = 12, 40
    g = synth.rng(99, 2, 0)
    op = measurement.DFT(_uv(m, 2), n)
    x = g.normal(size=(n, n))
    xc = x + 1j * g.normal(size=(n, n))
    v = g.normal(size=m) + 1j * g.normal(size=m)
    # real adjoint: <Phi x, v>_R = Re(v^H Phi x) = <x, Re(Phi^H v)>
    lhs = np.vdot(v, op.fwd(x)).real
    assert lhs == pytest.approx(np.sum(x * op.adj(v)), rel=1e-12)
    # complex adjoint
    assert np.vdot(v, op.fwd_complex(xc)) == pytest.approx(np.vdot(op.adj_complex(v), xc), rel=1e-12)


NUFFTS = [measurement.NUFFT, measurement.NUFFTCompiled]


@pytest.mark.parametrize("cls", NUFFTS)
@pytest.mark.parametrize("n,m,J,bound", [(64, 2048, 6, 2e-5), (64, 2048, 8, 2e-7), (32, 700, 6, 2e-5)])
def test_nufft_matches_dft(n, m, J, bound, cls):
    uv = _uv(m, 3)
    x = synth.sky(n, 20, 3.0, synth.rng(99, 3, synth.SKY))
    dft = measurement.DFT(uv, n)
    nu = cls(uv, n, J)
    a, b = nu.fwd(x), dft.fwd(x)
    assert np.linalg.norm(a - b) / np.linalg.norm(b) <= bound
    v = synth.complex_normal(m, synth.rng(99, 3, synth.NOISE))
    a, b = nu.adj(v), dft.adj(v)
    assert np.linalg.norm(a - b) / np.linalg.norm(b) <= bound


def test_nufft_matches_dft_subset_256():
    # 256^2 image, 4000 Gaussian-density visibilities: J = 6 error near 3.5e-6
    n = 256
    uv = _uv(4000, 4)
    x = synth.sky(n, 20, 3.0, synth.rng(99, 4, synth.SKY))
    a = measurement.NUFFT(uv, n, 6).fwd(x)
    b = measurement.DFT(uv, n).fwd(x)
    assert np.linalg.norm(a - b) / np.linalg.norm(b) <= 2e-5


@pytest.mark.parametrize("cls", NUFFTS)
def test_nufft_radial_wraparound_edges(cls):
    # points on the grid edge (kappa near -K/2 and +K/2) exercise the modulo taps
    n = 32
    uv = np.array([[-np.pi, -np.pi], [np.nextafter(np.pi, 0), 0.3], [0.0, np.nextafter(np.pi, 0)],
                   [-np.pi + 1e-9, 3.1], [0.0, 0.0], [1e-12, -1e-12]])
    x = synth.sky(n, 5, 3.0, synth.rng(99, 5, synth.SKY))
    a = cls(uv, n, 8).fwd(x)
    b = measurement.DFT(uv, n).fwd(x)
    assert np.linalg.norm(a - b) / np.linalg.norm(b) <= 2e-7


@pytest.mark.parametrize("cls", NUFFTS)
def test_nufft_adjoint_dot(cls):
    n, m = 32, 900
    g = synth.rng(99, 6, 0)
    op = cls(_uv(m, 6), n, 6)
    x = g.normal(size=(n, n))
    v = g.normal(size=m) + 1j * g.normal(size=m)
    assert np.vdot(v, op.fwd(x)).real == pytest.approx(np.sum(x * op.adj(v)), rel=1e-12)


def test_compiled_bessel_series_matches_library():
    # the compiled oracle sums I0 from its power series; scipy evaluates it by Chebyshev expansions
    from oracle import cbuild
    lib = cbuild.load()
    xs = np.concatenate([np.linspace(0.0, 40.0, 801), [1e-8, 13.8551, 18.6389]])
    got = np.array([lib.oracle_bessel_i0(float(x)) for x in xs])
    np.testing.assert_allclose(got, scipy.special.i0(xs), rtol=1e-14)
    for J in (6, 8):
        b = kb.beta(J, 2)
        t = np.linspace(-J / 2 - 0.5, J / 2 + 0.5, 97)
        np.testing.assert_allclose([lib.oracle_kb(float(s), J, b) for s in t], kb.psi(t, J, b), rtol=1e-14, atol=1e-300)


@pytest.mark.parametrize("J", [6, 8])
def test_compiled_nufft_equals_numpy_nufft(J):
    # same definition, two implementations: agreement to rounding, with several threads and with one
    n, m = 64, 30000
    uv = synth.uv_radial(m, synth.rng(99, 9, synth.UV))
    x = synth.sky(n, 20, 3.0, synth.rng(99, 9, synth.SKY))
    v = synth.complex_normal(m, synth.rng(99, 9, synth.NOISE))
    ref = measurement.NUFFT(uv, n, J)
    for threads in (None, 1):
        op = measurement.NUFFTCompiled(uv, n, J, threads=threads)
        a, b = op.fwd(x), ref.fwd(x)
        assert np.linalg.norm(a - b) / np.linalg.norm(b) <= 1e-13
        a, b = op.adj(v), ref.adj(v)
        assert np.linalg.norm(a - b) / np.linalg.norm(b) <= 1e-13
        # a block of the operator is the operator of that block's visibilities
        sub = op.subset(1000, 4000)
        full = ref.fwd(x)
        np.testing.assert_allclose(sub.fwd(x), full[1000:4000], rtol=0, atol=1e-12 * np.abs(full).max())


def test_op_norm_matches_eigvalsh():
    n, m = 16, 300
    op = measurement.DFT(_uv(m, 7), n)
    # explicit Re(Phi^H Phi), N x N
    E = np.stack([op.fwd(e.reshape(n, n)) for e in np.eye(n * n)], axis=1)
    A = (E.conj().T @ E).real
    lam = np.linalg.eigvalsh(A)[-1]
    x0 = synth.gaussian_vector(n * n, synth.rng(99, 7, 0)).reshape(n, n)
    nu = measurement.op_norm(op, x0, max_iter=20000, tol=0.0)
    assert nu ** 2 == pytest.approx(lam, rel=1e-10)


@pytest.mark.slow
def test_op_norm_matches_eigvalsh_64():
    n, m = 64, 2048
    op = measurement.NUFFT(_uv(m, 8), n, 6)
    E = np.stack([op.fwd(e.reshape(n, n)) for e in np.eye(n * n)], axis=1)
    A = (E.conj().T @ E).real
    lam = np.linalg.eigvalsh(A)[-1]
    x0 = synth.gaussian_vector(n * n, synth.rng(99, 8, 0)).reshape(n, n)
    nu = measurement.op_norm(op, x0, max_iter=20000, tol=0.0)
    assert nu ** 2 == pytest.approx(lam, rel=1e-10)
