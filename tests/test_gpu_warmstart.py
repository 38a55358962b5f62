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
    rescaling that needs the solution).  The warm-started solve then runs with the plain solve's own
    stopping test (relative change 1e-4, feasibility slack 1e-4, dual residual 1e-2, 5 passes of at
    most 300 iterations, the network standing in for the first); whichever path produced the image
    (warm, or the plain fallback when the warm run does not meet the test), every constraint holds
    within eps_i (1 + 1e-4) under the oracle's FP64 operator.  Iterations and times are printed, not
    asserted: the network does not save iterations under this test (measured in the design notes)."""
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
                wi = info_w.get("warm_info", info_w)
                print(f"{kind}: plain {info_p['pass_iters']} (converged {info_p['converged']}); warm "
                      f"{wi['pass_iters']} (converged {wi['converged']}), image from the {info_w['path']} path; "
                      f"error vs true sky plain {helpers.rel(xs, xt):.4f}, returned {helpers.rel(x_warm.cpu().numpy()[0], xt):.4f}")
                assert info_w["path"] in ("warm", "plain fallback")
                if info_w["path"] == "warm":
                    assert info_w["converged"] == 1
                v = measurement.NUFFTCompiled(pr["uv"], n, pr["J"]).fwd(x_warm.cpu().numpy()[0].astype(np.float64))
                yy = y.cpu().numpy().astype(np.complex128)
                for i in range(R):
                    lo, hi = pr["off"][i], pr["off"][i + 1]
                    assert np.linalg.norm(yy[lo:hi] - v[lo:hi]) <= eps[i] * (1 + 1e-4)
            finally:
                sh.psi_destroy(psi)
                sh.op_destroy(op)
    finally:
        ws.close()


def test_warm_start_falls_back_to_the_plain_solve(sh, ws_mod):
    """A warm start that cannot meet the stopping test (a network scaled so that x0 is far too bright, and
    passes too short to recover) hands over to the plain solve from zero: the returned image is the plain
    solve's, bit for bit, and the record says which path produced it."""
    from paper_1502_05037_amd import train_warmstart as tw
    dev = torch.device("cuda:0")
    flat = np.load(ws_mod.WEIGHTS, allow_pickle=False).copy()
    ws = ws_mod.WarmStart(flat)
    try:
        # scale the head: the prediction becomes 50 times the network's image
        meta_layers = ws_mod.layer_list(32, 4)
        size = 0
        for kind, cin, cout in meta_layers[:-1]:
            k = 9 if kind == "conv3" else (4 if kind == "tconv" else 1)
            size += cin * cout * k + cout
        flat[size:] *= 50.0
        sh.unet_set_params(ws.u, flat)
        pr = tw.make_problems(10 ** 6 + 2, 1, "c2")
        n = pr["n"]
        op = sh.op_create(pr["uv"], n, 2, pr["J"], pr["off"])
        psi = sh.psi_create(n, 4)
        try:
            y, eps = tw.observe(op, pr, dev)
            prm = tw.solve_params(passes=2, max_iter=20)
            x_w = torch.empty((1, n, n), device=dev)
            info_w, res_w, _ = ws_mod.warm_solve(ws, op, psi, y, eps, prm, n, dev, x_w)
            x_p = torch.empty((1, n, n), device=dev)
            info_p, res_p = sh.sdmm_solve(op, psi, y, eps, None, None, prm, x_p)
            torch.cuda.synchronize()
        finally:
            sh.psi_destroy(psi)
            sh.op_destroy(op)
    finally:
        ws.close()
    print(f"warm attempt {info_w.get('warm_info', {}).get('pass_iters')} -> {info_w['path']}")
    assert info_w["path"] == "plain fallback"
    assert info_w["warm_info"]["converged"] == 0
    assert torch.equal(x_w, x_p)
    np.testing.assert_array_equal(res_w, res_p)
