"""Pins for the per-block normalisation of the data splits.

* The density count, written out by hand for placed samples (periodic windows, alpha = 2 and 4) and by
  brute force over every window of a small grid.
* The estimate against the quantity it stands for: the largest eigenvalue of Re(Phi_b^H Phi_b) of the
  direct DFT, by dense eigendecomposition.
* Weighting the blocks leaves the minimiser of (3) unchanged: SDMM with block weights reaches the
  brute-force objective, and its KKT residuals vanish.
"""
import numpy as np
import pytest

from oracle import measurement, sdmm
from paper_1502_05037_amd import synth
from tests import test_oracle_sdmm as tos


def _at_cells(cells, K):
    """uv at the centres of the given (row, col) cells of the K x K grid, in [-pi, pi)."""
    c = np.asarray(cells, dtype=np.float64)
    u = 2 * np.pi * (c + 0.5) / K
    return np.where(u >= np.pi, u - 2 * np.pi, u)


def test_density_count_written_out():
    n, alpha = 8, 2
    K = alpha * n
    # block 0: 3 samples in (0, 0), 2 in (1, 1), 1 in (15, 15): the 2 x 2 window at (0, 0) holds 5,
    # the one at (15, 15) (wrapping to (0, 0)) holds 4
    b0 = [(0, 0)] * 3 + [(1, 1)] * 2 + [(15, 15)]
    # block 1: samples spread over one row, two per cell: any 2 x 2 window holds at most 4
    b1 = [(5, c) for c in range(K) for _ in range(2)]
    # block 2: four samples in four cells that only the periodic window at (15, 15) joins
    b2 = [(15, 15), (0, 15), (15, 0), (0, 0)]
    uv = _at_cells(b0 + b1 + b2, K)
    off = [0, len(b0), len(b0) + len(b1), len(b0) + len(b1) + len(b2)]
    a = measurement.block_density_weights(uv, n, alpha, off)
    np.testing.assert_array_equal(a, 1.0 / np.sqrt(float(n) * n * np.array([5.0, 4.0, 4.0])))
    # alpha = 4: 4 x 4 windows; a cluster spread over a 4 x 4 square is counted whole
    n4 = 4
    K4 = 4 * n4
    b = [(r, c) for r in range(6, 10) for c in range(2, 6)] + [(0, 0)]
    a4 = measurement.block_density_weights(_at_cells(b, K4), n4, 4, [0, len(b)])
    assert a4[0] == 1.0 / np.sqrt(float(n4) * n4 * 16.0)


def test_density_count_brute_force():
    n, alpha = 6, 2
    K = alpha * n
    g = synth.rng(97, 0, synth.UV)
    uv = g.uniform(-np.pi, np.pi, size=(300, 2))
    off = [0, 120, 300]
    a = measurement.block_density_weights(uv, n, alpha, off)
    for b in range(2):
        pts = uv[off[b]:off[b + 1]]
        cells = [(int(np.floor(u * K / (2 * np.pi))) % K, int(np.floor(v * K / (2 * np.pi))) % K) for u, v in pts]
        best = 0
        for r in range(K):
            for c in range(K):
                win = {((r + i) % K, (c + j) % K) for i in range(alpha) for j in range(alpha)}
                best = max(best, sum(1 for q in cells if q in win))
        assert a[b] == pytest.approx(1.0 / (n * np.sqrt(best)), rel=1e-15)


@pytest.mark.parametrize("cov,seed", [("gaussian", 0), ("radial", 1), ("radial", 2)])
def test_estimate_tracks_the_block_norm(cov, seed):
    """a_b ||Phi_b|| stays within a factor 1.5 of 1 for blocks of very different norms."""
    n, m, R = 32, 6000, 6
    g = synth.rng(97, seed, synth.UV)
    uv = synth.sort_by_radius(synth.uv_gaussian(m, g) if cov == "gaussian" else synth.uv_radial(m, g))
    off = synth.offsets(synth.block_sizes(m, R, synth.rng(97, seed, synth.BLOCKS)))
    a = measurement.block_density_weights(uv, n, 2, off)
    ratios = []
    for b in range(R):
        dft = measurement.DFT(uv[off[b]:off[b + 1]], n)
        # dense Re(Phi_b^H Phi_b) on R^(n n)
        E = np.stack([dft.adj(dft.fwd(e.reshape(n, n))).ravel() for e in np.eye(n * n)], axis=1)
        lam = np.linalg.eigvalsh(0.5 * (E + E.T))[-1]
        ratios.append(a[b] * np.sqrt(lam))
    norms = 1.0 / a
    print(cov, "a_b ||Phi_b||:", np.round(ratios, 3), "norm spread", norms.max() / norms.min())
    assert np.all(np.array(ratios) > 1 / 1.5) and np.all(np.array(ratios) < 1.5)


def _weights(op_uv, n, off):
    return measurement.block_density_weights(op_uv, n, 2, off)


def test_block_weights_keep_the_minimiser():
    """Brute force of a tiny problem (3) against SDMM with block weights (Dirac + db2 + db4)."""
    op, psi, y, off, eps = tos._tiny_problem(R=2, m=96, levels=2, mask=0b10101)
    a = _weights(op.uv, psi.n, off)
    nu = measurement.op_norm(measurement.BlockWeighted(op, off, a), np.ones((psi.n, psi.n)), max_iter=5000, tol=0.0)
    gamma = sdmm.default_gamma(op, psi, y, nu, factor=1e-3, offsets=off, block_weights=a)
    p = sdmm.Params(gamma=gamma, nu=nu, max_iter=20000, tol_rel=1e-11, eps_slack=1e-9, block_weights=a)
    x, _, infos, _ = sdmm.sara(op, psi, y, off, eps, p)
    W = np.ones((psi.q, psi.n, psi.n))
    x_bf, obj_bf = tos._brute_force_slsqp(op, psi, y, off, eps, W)
    assert np.sum(np.abs(psi.adj(x))) == pytest.approx(obj_bf, rel=2e-5)
    assert np.all(infos[0].block_resid <= eps * (1 + 1e-6))
    assert np.linalg.norm(x - x_bf) / np.linalg.norm(x_bf) <= 1e-3
    # the residuals returned are in user units: the oracle operator gives the same
    r = np.array([np.linalg.norm(y[off[i]:off[i + 1]] - op.fwd(x)[off[i]:off[i + 1]]) for i in range(len(eps))])
    np.testing.assert_allclose(infos[0].block_resid, r, rtol=1e-9)


def test_block_weighted_kkt_residuals_vanish():
    op, psi, y, off, eps = tos._tiny_problem(R=2, seed=4)
    a = _weights(op.uv, psi.n, off)
    nu = measurement.op_norm(measurement.BlockWeighted(op, off, a), np.ones((psi.n, psi.n)), max_iter=5000, tol=0.0)
    gamma = sdmm.default_gamma(op, psi, y, nu, factor=1e-3, offsets=off, block_weights=a)
    pb = sdmm.Problem(op, psi, y, off, eps, nu, a)
    p = sdmm.Params(gamma=gamma, nu=nu, max_iter=3000, tol_rel=0.0, block_weights=a)
    st, _ = sdmm.sdmm_pass(pb, None, p, sdmm.init_state(pb))
    prim1, dual1 = sdmm.kkt(pb, st, None, gamma)
    st, _ = sdmm.sdmm_pass(pb, None, p, st)
    prim2, dual2 = sdmm.kkt(pb, st, None, gamma)
    print(f"KKT after 3000 / 6000 iterations: primal {prim1:.2e} / {prim2:.2e}, dual {dual1:.2e} / {dual2:.2e}")
    assert prim2 <= 1e-9 and dual2 <= 1e-5
    assert prim2 <= prim1 / 10 and dual2 <= dual1 / 10


def test_weighted_gamma_and_problem_reduce_to_uniform():
    """a_b = 1 for every block is the single normalisation: same data, bounds, operator and gamma."""
    op, psi, y, off, eps = tos._tiny_problem(R=3, seed=5)
    nu = measurement.op_norm(op, np.ones((psi.n, psi.n)))
    ones = np.ones(3)
    g0 = sdmm.default_gamma(op, psi, y, nu)
    g1 = sdmm.default_gamma(op, psi, y, nu, offsets=off, block_weights=ones)
    assert g1 == pytest.approx(g0, rel=1e-14)
    p1 = sdmm.Problem(op, psi, y, off, eps, nu, ones)
    np.testing.assert_allclose(p1.y_hat, np.asarray(y) / nu, rtol=1e-15)
    np.testing.assert_allclose(p1.eps_hat, np.asarray(eps) / nu, rtol=1e-15)
    # a weight of 2 on one block doubles that block's normalised data and bound only
    w = np.array([1.0, 2.0, 1.0])
    p2 = sdmm.Problem(op, psi, y, off, eps, nu, w)
    lo, hi = off[1], off[2]
    np.testing.assert_allclose(p2.y_hat[lo:hi], 2 * p1.y_hat[lo:hi], rtol=1e-15)
    np.testing.assert_allclose(p2.y_hat[:lo], p1.y_hat[:lo], rtol=1e-15)
    assert p2.eps_hat[1] == pytest.approx(2 * p1.eps_hat[1], rel=1e-15)
