"""Hand-computed pins for the oracle's readings that the paper leaves open.

Each expected value below is written out from the mathematics of a case small
enough to do by hand; none is obtained by calling the oracle's own formula.

* The step gamma = 1e-4 max |Psi^dagger Phi_hat^dagger y_hat| (the SDMM
  paragraph names the solver, not its step) on Phi = I with a Dirac dictionary,
  on two blocks with different normalisations c_b = a_b / nu, and on a
  Dirac + Haar dictionary where the 1/sqrt(q) scale of Psi decides the value.
* The reweighting schedule (SARA paragraph: weights near the inverse of the
  previous solution's coefficients) w = delta / (delta + |c|), delta_1 = the
  population standard deviation after pass 1, delta_{t+1} = delta_t / 2, on the
  problem Phi = Psi = I, R = 1, whose weighted-l1 passes have the closed form
  x_j = max(y_j - lambda w_j, 0) with ||y - x|| = eps.
* Minimum phase of db1..db8: after dividing out the p zeros at z = -1, every
  zero of the scaling filter lies strictly inside the unit circle (the
  extremal-phase choice; a least-asymmetric or reversed filter fails).
"""
import numpy as np
import pytest

from oracle import measurement, sdmm, wavelets

S2 = np.sqrt(2.0)


# ---------------------------------------------------------------------------
# gamma
# ---------------------------------------------------------------------------

def test_gamma_identity_dirac_one_block():
    # Phi = I on a 2 x 2 image, Psi = Dirac (q = 1), nu = 2: Phi_hat^dagger y_hat = Re(y) / 4
    op = measurement.Identity(2)
    psi = wavelets.SARA(2, 1, mask=0b1)
    y = np.array([1 + 2j, -3 + 0.5j, 2.0, -0.5j])
    g = sdmm.default_gamma(op, psi, y, 2.0)
    # Re(y) / 4 = [0.25, -0.75, 0.5, 0]: the largest magnitude is 0.75
    assert g == pytest.approx(1e-4 * 0.75, rel=1e-14)
    assert sdmm.default_gamma(op, psi, y, 2.0, factor=1e-3) == pytest.approx(7.5e-4, rel=1e-14)


def test_gamma_two_blocks_with_block_weights():
    # blocks [0, 2) and [2, 4) with a = (1, 3), nu = 2: c = (0.5, 1.5), c^2 = (0.25, 2.25), and
    # Phi_hat^dagger y_hat = c^2 Re(y) = [0.25, -0.75, 4.5, 0] -> gamma = 1e-4 * 4.5
    op = measurement.Identity(2)
    psi = wavelets.SARA(2, 1, mask=0b1)
    y = np.array([1 + 2j, -3 + 0.5j, 2.0, -0.5j])
    g = sdmm.default_gamma(op, psi, y, 2.0, offsets=[0, 2, 4], block_weights=np.array([1.0, 3.0]))
    assert g == pytest.approx(4.5e-4, rel=1e-14)
    # the normalised problem carries the same c_b: data c_b y_b and bounds c_b eps_b
    pb = sdmm.Problem(op, psi, y, [0, 2, 4], [1.0, 1.0], 2.0, np.array([1.0, 3.0]))
    np.testing.assert_allclose(pb.y_hat, [0.5 + 1j, -1.5 + 0.25j, 3.0, -0.75j], rtol=1e-15)
    np.testing.assert_allclose(pb.eps_hat, [0.5, 1.5], rtol=1e-15)


def test_gamma_dirac_plus_haar_scale():
    # Phi = I, nu = 1, Psi = (1/sqrt 2)[I, W_1] on x = [[1, 2], [3, 4]] with one Haar level:
    # rows -> [(1+2), (1-2); (3+4), (3-4)] / sqrt 2, columns -> LL 5, top-right -1, bottom-left -2, HH 0.
    # max |Psi^dagger x| = 5 / sqrt 2 (the Dirac plane only reaches 4 / sqrt 2).
    op = measurement.Identity(2)
    psi = wavelets.SARA(2, 1, mask=0b11)
    y = np.array([1.0, 2.0, 3.0, 4.0]) + 0.25j
    c = psi.adj(op.adj(y))
    np.testing.assert_allclose(c[1], [[5.0 / S2, -1.0 / S2], [-2.0 / S2, 0.0]], atol=1e-15)
    np.testing.assert_allclose(c[0], np.array([[1.0, 2.0], [3.0, 4.0]]) / S2, atol=1e-15)
    assert sdmm.default_gamma(op, psi, y, 1.0) == pytest.approx(1e-4 * 5.0 / S2, rel=1e-14)


# ---------------------------------------------------------------------------
# reweighting schedule
# ---------------------------------------------------------------------------

def _weighted_closed_form(y, w, eps):
    """min sum_j w_j |x_j| s.t. ||y - x|| <= eps, x >= 0 (y > 0 real): x_j = max(y_j - lam w_j, 0),
    lam by bisection so that ||y - x|| = eps (the KKT conditions of the problem)."""
    lo, hi = 0.0, float(np.max(y / w)) + 1.0
    for _ in range(200):
        lam = 0.5 * (lo + hi)
        r = np.linalg.norm(y - np.maximum(y - lam * w, 0.0))
        lo, hi = (lam, hi) if r < eps else (lo, lam)
    return np.maximum(y - 0.5 * (lo + hi) * w, 0.0)


def test_reweighting_schedule_closed_form():
    # y = [4, 0.8, 0.5, 3] on a 2 x 2 image, eps = 1.7.  Pass 1 (W = 1): lambda = 1 gives
    # x1 = [3, 0, 0, 2] and ||y - x1||^2 = 1 + 0.64 + 0.25 + 1 = 2.89 = eps^2.
    y = np.array([4.0, 0.8, 0.5, 3.0])
    eps = 1.7
    x1 = np.array([3.0, 0.0, 0.0, 2.0])
    # delta_1 = population std of x1: mean 5/4, squared deviations 49/16, 25/16, 25/16, 9/16 -> 27/16
    d1 = 3.0 * np.sqrt(3.0) / 4.0
    W2 = np.array([d1 / (d1 + 3.0), 1.0, 1.0, d1 / (d1 + 2.0)])
    # pass 2 solves the weighted problem in closed form; delta_2 = delta_1 / 2
    x2 = _weighted_closed_form(y, W2, eps)
    d2 = d1 / 2.0
    W3 = d2 / (d2 + np.abs(x2))

    op = measurement.Identity(2)
    psi = wavelets.SARA(2, 1, mask=0b1)
    yc = y.astype(np.complex128)
    common = dict(gamma=0.05, nu=1.0, max_iter=6000, tol_rel=1e-13, eps_slack=1e-12)
    # pass 1 alone reaches the unweighted closed form; its reweighting gives W2
    x, W, infos, _ = sdmm.sara(op, psi, yc, [0, 4], [eps], sdmm.Params(passes=2, **common))
    np.testing.assert_allclose(W.ravel(), W2, rtol=0, atol=2e-7)
    assert infos[0].converged and infos[1].converged
    np.testing.assert_allclose(x.ravel(), x2, rtol=0, atol=1e-6)
    # a third pass uses delta_2 = delta_1 / 2 on the pass-2 image (not a fresh standard deviation)
    x, W, infos, _ = sdmm.sara(op, psi, yc, [0, 4], [eps], sdmm.Params(passes=3, **common))
    np.testing.assert_allclose(W.ravel(), W3, rtol=0, atol=1e-6)
    x3 = _weighted_closed_form(y, W3, eps)
    np.testing.assert_allclose(x.ravel(), x3, rtol=0, atol=1e-6)
    # the hand values differ from the plausible misreadings
    assert abs(np.std(x1, ddof=1) - d1) > 0.1                    # sample, not population, std
    assert np.max(np.abs(W3 - np.std(x2) / (np.std(x2) + x2))) > 1e-2   # delta recomputed each pass


# ---------------------------------------------------------------------------
# Daubechies extremal phase
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("p", range(1, 9))
def test_daubechies_minimum_phase(p):
    h = wavelets.daubechies(p)
    # h[k] is the coefficient of z^(2p-1-k): numpy's highest-power-first order
    q = h.copy()
    for _ in range(p):
        q, rem = np.polydiv(q, [1.0, 1.0])
        assert np.max(np.abs(rem)) <= 1e-12          # a zero at z = -1 (one vanishing moment)
    assert len(q) == p
    if p > 1:
        roots = np.roots(q)
        assert np.max(np.abs(roots)) < 0.9, roots    # every other zero strictly inside the unit circle
        # the time-reversed filter (maximum phase) has the reciprocal zeros, all outside
        qr = h[::-1].copy()
        for _ in range(p):
            qr, _ = np.polydiv(qr, [1.0, 1.0])
        assert np.min(np.abs(np.roots(qr))) > 1.1


# ---------------------------------------------------------------------------
# block-subset iterations
# ---------------------------------------------------------------------------

def test_splitmix64_reference_outputs():
    # the first outputs of SplitMix64 seeded with 0, as published with the generator
    assert [sdmm.splitmix64(0, c) for c in range(3)] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_block_subset_selection_frequency():
    R, K, f = 16, 400, 0.3
    sel = np.array([sdmm.block_selected(5, k, R, f) for k in range(K)])
    n = sel.size
    assert abs(sel.mean() - f) <= 4 * np.sqrt(f * (1 - f) / n)
    # every block is drawn at the same rate, and iterations differ
    assert np.all(np.abs(sel.mean(axis=0) - f) <= 5 * np.sqrt(f * (1 - f) / K))
    assert len({tuple(r) for r in sel}) > K // 2
    assert np.all(sdmm.block_selected(5, 3, R, 1.0)) and not np.any(sdmm.block_selected(5, 3, R, 0.0))
