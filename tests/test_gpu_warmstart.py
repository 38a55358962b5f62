"""The learned warm start end to end: the network input and prediction against the oracle, and what
the trained network gains on held-out problems."""
import os

import numpy as np
import pytest

from oracle import measurement, unet as ounet
from tests import helpers

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sh():
    from paper_1502_05037_amd import sarahip
    return sarahip


@pytest.fixture(scope="module")
def ws_mod():
    from paper_1502_05037_amd import warmstart
    if not os.path.exists(warmstart.WEIGHTS):
        pytest.skip("trained weights not present")
    return warmstart


def test_warm_start_prediction_matches_oracle(sh, ws_mod):
    """x0 = s U(d / s) with d = Phi^dagger y / PSF peak and s = RMS(d), on a 64 x 64 problem."""
    pb = helpers.build(60, 64, 6000, 2, 6, prob=1)
    flat = np.load(ws_mod.WEIGHTS, allow_pickle=False)
    op = sh.op_create(pb.uv, 64, 2, 6, pb.offsets)
    u = sh.unet_create(32, 4)
    try:
        sh.unet_set_params(u, flat)
        y = torch.tensor(pb.y.astype(np.complex64), device="cuda")
        x0 = torch.empty((1, 64, 64), device="cuda")
        sh.warm_start(u, op, y, x0)
        d = torch.empty((1, 64, 64), device="cuda")
        s = torch.empty(1, device="cuda")
        sh.dirty_normalised(op, y, d, s)
        torch.cuda.synchronize()
        x0, d, s = x0.cpu().numpy()[0], d.cpu().numpy()[0], float(s.cpu()[0])
    finally:
        sh.unet_destroy(u)
        sh.op_destroy(op)
    # oracle: dirty image in PSF-peak units, unit-RMS scaling, emulated-BF16 network
    delta = np.zeros((64, 64))
    delta[32, 32] = 1.0
    peak = pb.op.adj(pb.op.fwd(delta))[32, 32]
    dref = pb.op.adj(pb.y) / peak
    sref = np.sqrt(np.mean(dref ** 2))
    assert s == pytest.approx(sref, rel=1e-5)
    assert helpers.rel(d, dref / sref) <= 1e-5
    net = ounet.UNet(32, 4, emul=True)
    yref, _ = net.forward(ounet.unflatten(flat.astype(np.float64), 32, 4), (dref / sref)[None, None])
    assert helpers.rel(x0, sref * yref[0, 0]) <= 1e-2


def test_what_the_trained_network_gains_on_held_out_problems(sh, ws_mod):
    """On held-out 256^2 problems of both training kinds: the network's first image is closer to the
    plain solver's solution than the dirty image in PSF-peak units (what the data alone give) and
    than the zero start, and within twice the error of the best multiple of the dirty image (a
    rescaling that needs the solution); the warm-started solve then meets the same stopping test with
    every constraint satisfied (checked with the oracle's FP64 operator).
    Iteration counts and errors against the true sky are printed, not asserted: with the default step
    the plain solve itself stops within a few hundred iterations, and a warm start then saves little
    (see the design notes)."""
    from paper_1502_05037_amd import train_warmstart as tw
    dev = torch.device("cuda:0")
    ws = ws_mod.WarmStart.load()
    try:
        for kind in ("c2", "c3"):
            pr = tw.make_problems(10 ** 6 + 1, 1, kind)
            n, R = pr["n"], pr["R"]
            op = sh.op_create(pr["uv"], n, 2, pr["J"], pr["off"])
            psi = sh.psi_create(n, 4)
            try:
                y, eps = tw.observe(op, pr, dev)
                prm = tw.solve_params()
                prm.eps_slack = 1e-3
                x_plain = torch.empty((1, n, n), device=dev)
                info_p, _ = sh.sdmm_solve(op, psi, y, eps, None, None, prm, x_plain)
                x0 = ws.predict(op, y, n, 1, dev)
                d = torch.empty((1, n, n), device=dev)
                s = torch.empty(1, device=dev)
                sh.dirty_normalised(op, y, d, s)
                xs = x_plain.cpu().numpy()[0].astype(np.float64)
                dd = d.cpu().numpy()[0].astype(np.float64)
                sc = float(s.cpu()[0])
                alpha = float(np.sum(dd * xs) / np.sum(dd * dd))       # best multiple, knowing the solution
                e_net = helpers.rel(x0.cpu().numpy()[0], xs)
                e_psf = helpers.rel(sc * dd, xs)                       # dirty image in PSF-peak units
                e_best = helpers.rel(alpha * dd, xs)
                print(f"{kind}: first image vs plain solution: network {e_net:.3f}, dirty image in PSF units "
                      f"{e_psf:.3f}, best multiple of the dirty image {e_best:.3f}, zero start 1")
                # better than what the data alone give, and of the same quality as the best linear rescaling
                assert e_net < e_psf and e_net < 0.2 and e_net <= 2.0 * e_best
                x_warm = torch.empty((1, n, n), device=dev)
                info_w, res_w, secs = ws_mod.warm_solve(ws, op, psi, y, eps, prm, n, dev, x_warm)
                xt = pr["x_true"][0].astype(np.float64)
                print(f"{kind}: iterations plain {info_p['iters_total']}, warm {info_w['iters_total']}; error vs "
                      f"true sky plain {helpers.rel(xs, xt):.4f}, warm {helpers.rel(x_warm.cpu().numpy()[0], xt):.4f}")
                assert info_w["converged"] == 1
                v = measurement.NUFFT(pr["uv"], n, pr["J"]).fwd(x_warm.cpu().numpy()[0].astype(np.float64))
                yy = y.cpu().numpy().astype(np.complex128)
                for i in range(R):
                    lo, hi = pr["off"][i], pr["off"][i + 1]
                    assert np.linalg.norm(yy[lo:hi] - v[lo:hi]) <= eps[i] * (1 + 1.1e-3)
            finally:
                sh.psi_destroy(psi)
                sh.op_destroy(op)
    finally:
        ws.close()
