"""The per-iteration metrics ring of a solver session (sh_sdmm_metrics_enable / sh_sdmm_metrics_read).

* Against the FP64 oracle: 40 iterations of the 64^2, 2048-visibility problem, whose recorded history gives the
  relative change and every block's residual over eps after each iteration; the objective of the last row
  equals the session's own KKT objective and the oracle's ||W Psi^dagger x||_1.
* Ring mechanics: a 16-row ring read after 10 and after 40 iterations gives rows 1-10, then 25-40 (the oldest
  overwritten), bitwise equal to the rows of a 64-row ring filled by plain launches instead of the replayed
  graph; the last row agrees with sh_sdmm_result; a checkpoint imported into a fresh session (whose ring then
  starts again at the imported iteration count) records the rows the exporting session records next, bit for
  bit; with the ring switched off a read is refused.  For the analysis prior, block-subset iterations and the
  synthesis prior.
"""
import numpy as np
import pytest

from oracle import measurement, sdmm, wavelets
from tests import helpers

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

EINVAL = -1


@pytest.fixture(scope="module")
def sh():
    from paper_1502_05037_amd import sarahip
    return sarahip


def _params(sh, **kw):
    p = sh.sdmm_default_params()
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def test_metrics_follow_the_oracle_history(sh):
    pb = helpers.build(1, 64, 2048, 1, 6)
    psi_o = wavelets.SARA(pb.n, 4, 0x1FF)
    a = measurement.block_density_weights(pb.uv, pb.n, 2, pb.offsets)
    A = measurement.BlockWeighted(pb.op, pb.offsets, a)
    nu = measurement.op_norm(A, np.ones((pb.n, pb.n)), max_iter=200, tol=1e-12)
    gamma = sdmm.default_gamma(pb.op, psi_o, pb.y, nu, offsets=pb.offsets, block_weights=a)
    iters = 40
    p = sdmm.Params(gamma=gamma, nu=nu, max_iter=iters, cg_iters=8, passes=1, block_weights=a)
    _, _, infos, _ = sdmm.sara(pb.op, psi_o, pb.y, pb.offsets, pb.eps, p, record=True)
    eps_hat = sdmm.Problem(pb.op, psi_o, pb.y, pb.offsets, pb.eps, nu, a).eps_hat
    rel_o = np.array([h[0] for h in infos[0].history])
    res_o = np.array([h[1] / eps_hat for h in infos[0].history])
    R = len(pb.eps)

    op = sh.op_create(pb.uv, pb.n, 2, pb.J, pb.offsets)
    psi = sh.psi_create(pb.n, 4)
    s = sh.sdmm_create(op, psi, torch.tensor(pb.y, dtype=torch.complex64, device="cuda"), pb.eps, None, None,
                       _params(sh, gamma=gamma, nu=nu, cg_iters=8))
    try:
        assert sh.sdmm_metrics_enable(s, 64) == 2 + R
        sh.sdmm_iterate(s, iters)
        m = sh.sdmm_metrics_read(s, 1, R, 100)
        _, _, obj = sh.sdmm_kkt(s)
    finally:
        sh.sdmm_destroy(s)
        sh.psi_destroy(psi)
        sh.op_destroy(op)
    assert m["rows"] == iters and m["first_iter"] == 1
    rel_g, res_g = m["rel_change"][:, 0], m["resid_over_eps"]
    dev_rel = np.abs(rel_g - rel_o) / (rel_o + 1e-3)
    dev_res = np.max(np.abs(res_g - res_o) / np.abs(res_o))
    print(f"relative change: iteration 1 {rel_g[0]:.4g} vs {rel_o[0]:.4g}, iteration {iters} {rel_g[-1]:.4g} vs "
          f"{rel_o[-1]:.4g}, worst deviation {dev_rel.max():.2e}; residual/eps worst relative deviation "
          f"{dev_res:.2e}; objective {m['objective'][-1, 0]:.6g} vs oracle {infos[0].objective:.6g}", flush=True)
    # FP32 iterates: the change between iterates carries their rounding (measured: 4e-6 and 1e-6 worst)
    assert np.all(dev_rel <= 1e-4)
    assert dev_res <= 1e-4
    assert m["objective"][-1, 0] == pytest.approx(obj, rel=1e-12)
    assert m["objective"][-1, 0] == pytest.approx(infos[0].objective, rel=1e-4)


@pytest.mark.parametrize("variant", ["analysis", "block_subset", "synthesis"])
def test_ring_wraps_and_matches_plain_launches(sh, variant):
    pb = helpers.build(80, 64, 3000, 4, 6, prob=2)
    R = len(pb.eps)
    kw = {"analysis": {}, "block_subset": dict(block_fraction=0.5, block_seed=7),
          "synthesis": dict(synthesis=1)}[variant]
    op = sh.op_create(pb.uv, 64, 2, 6, pb.offsets)
    psi = sh.psi_create(64, 4)
    y = torch.tensor(pb.y, dtype=torch.complex64, device="cuda")
    try:
        info, _ = sh.sdmm_solve(op, psi, y, pb.eps, None, None, _params(sh, max_iter=1, passes=1, cg_iters=4, **kw),
                                torch.empty((64, 64), device="cuda"))
        base = dict(nu=info["nu"], gamma=info["gamma"], cg_iters=4, **kw)
        a = sh.sdmm_create(op, psi, y, pb.eps, None, None, _params(sh, **base))
        b = sh.sdmm_create(op, psi, y, pb.eps, None, None, _params(sh, graph=0, **base))
        try:
            sh.sdmm_metrics_enable(a, 16)
            sh.sdmm_iterate(a, 10)
            a1 = sh.sdmm_metrics_read(a, 1, R, 100)
            sh.sdmm_iterate(a, 30)
            a2 = sh.sdmm_metrics_read(a, 1, R, 100)
            a3 = sh.sdmm_metrics_read(a, 1, R, 100)
            sh.sdmm_metrics_enable(b, 64)
            sh.sdmm_iterate(b, 40)
            bb = sh.sdmm_metrics_read(b, 1, R, 100)
            resid, rel = sh.sdmm_result(b, None, R)
            # a checkpoint resumed in a fresh session records the rows the exporting session goes on to record
            state = sh.sdmm_state_export(b)
            sh.sdmm_iterate(b, 5)
            bb2 = sh.sdmm_metrics_read(b, 1, R, 100)
            c = sh.sdmm_create(op, psi, y, pb.eps, None, None, _params(sh, **base))
            try:
                sh.sdmm_metrics_enable(c, 8)
                sh.sdmm_iterate(c, 3)
                sh.sdmm_state_import(c, state)
                sh.sdmm_iterate(c, 5)
                cc = sh.sdmm_metrics_read(c, 1, R, 100)
            finally:
                sh.sdmm_destroy(c)
            sh.sdmm_metrics_enable(a, 0)
            with pytest.raises(sh.SarahipError) as e:
                sh.sdmm_metrics_read(a, 1, R, 100)
            assert e.value.status == EINVAL
        finally:
            sh.sdmm_destroy(a)
            sh.sdmm_destroy(b)
    finally:
        sh.psi_destroy(psi)
        sh.op_destroy(op)
    assert (a1["rows"], a1["first_iter"]) == (10, 1)
    assert (a2["rows"], a2["first_iter"]) == (16, 25)
    assert a3["rows"] == 0
    assert (bb["rows"], bb["first_iter"]) == (40, 1)
    assert (bb2["rows"], bb2["first_iter"]) == (5, 41) and (cc["rows"], cc["first_iter"]) == (5, 41)
    for key in ("rel_change", "objective", "resid_over_eps"):
        np.testing.assert_array_equal(cc[key], bb2[key])
    for key in ("rel_change", "objective", "resid_over_eps"):
        np.testing.assert_array_equal(a1[key], bb[key][:10])
        np.testing.assert_array_equal(a2[key], bb[key][24:])
        assert np.all(np.isfinite(bb[key]))
    assert bb["rel_change"][-1, 0] == pytest.approx(rel, rel=1e-14)
    if variant != "block_subset":   # (there the result evaluates every block; the ring holds the selected ones)
        np.testing.assert_allclose(bb["resid_over_eps"][-1] * pb.eps, resid, rtol=1e-12)
    print(f"{variant}: relative change {bb['rel_change'][0, 0]:.3g} -> {bb['rel_change'][-1, 0]:.3g}, worst "
          f"residual/eps at the end {bb['resid_over_eps'][-1].max():.4f}", flush=True)
