"""End-to-end checks of the GPU solver against the FP64 oracle at the full sizes of two workloads.

* 256 x 256 sky, M = 655 360 Gaussian-density visibilities in 8 uneven blocks, J = 6;
* 1024 x 1024 sky (200 point sources, dynamic range 1e4), M = 2e7 radial-density visibilities in 64
  uneven blocks, J = 8 (the benchmark's workload).

The data y = Phi x + n come from the oracle's FP64 NUFFT (its interpolation loops compiled, so that it
handles 2e7 visibilities), rounded to complex64 for the GPU.  Checks, for each workload:

* Phi on the dense sky image, block by block: each block's error <= 1e-5 of the larger of its own
  norm and its share of the whole vector's norm (the float32 floor is absolute, near 1e-7 of the RMS
  visibility, so blocks of visibilities far below the RMS are measured against the RMS level);
* Phi^dagger of the data restricted to each block, block by block (<= 1e-5 each), and of all the data
  pixel by pixel (largest pixel error <= 1e-5 of the largest pixel);
* the run to tolerance with the solver's defaults (relative change 1e-4, feasibility slack 1e-4, relative
  dual residual 1e-2, 5 passes of at most 300 iterations): every block's residual ||y_i - Phi_i x|| re-evaluated with the oracle's FP64 operator
  is <= eps_i (1 + 1e-4), the bound of problem (3) with the stopping test's slack;
* a short fixed schedule (two weighted-l1 passes with one reweighting, CG with two steps, the same
  gamma and nu on both sides, the solver's default normalisation and Toeplitz CG products): the
  image matches the oracle's within 1e-4 norm-wise.
"""
import numpy as np
import pytest

from oracle import measurement, problem, sdmm, wavelets
from paper_1502_05037_amd import synth
from tests import helpers

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

OP_TOL = 1e-5
IMG_TOL = 1e-4
SLACK = 1e-4

WORKLOADS = {
    # name: (config seed, n, M, R, J, coverage, point sources, dynamic range, fixed-schedule iterations per pass)
    "256": (2, 256, 655_360, 8, 6, "gaussian", 20, 3.0, 10),
    "1024": (3, 1024, 20_000_000, 64, 8, "radial", 200, 4.0, 3),
}


@pytest.fixture(scope="module")
def sh():
    from paper_1502_05037_amd import sarahip
    return sarahip


def _say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module", params=list(WORKLOADS))
def wl(request, sh):
    name = request.param
    cfg, n, m, R, J, cov, npts, dr, iters = WORKLOADS[name]
    _say(f"[e2e {name}] inputs: n={n} M={m} R={R} J={J} {cov}")
    g_uv = synth.rng(cfg, 0, synth.UV)
    uv = synth.sort_by_radius(synth.uv_gaussian(m, g_uv) if cov == "gaussian" else synth.uv_radial(m, g_uv))
    sizes = synth.block_sizes(m, R, synth.rng(cfg, 0, synth.BLOCKS))
    off = synth.offsets(sizes)
    x_true = synth.sky(n, npts, dr, synth.rng(cfg, 0, synth.SKY)).astype(np.float32).astype(np.float64)
    _say(f"[e2e {name}] oracle operator (compiled FP64 NUFFT)")
    op_o = measurement.NUFFTCompiled(uv, n, J)
    clean = op_o.fwd(x_true)
    sigma = problem.noise_sigma(clean, 30.0)
    y = problem.add_noise(clean, sigma, synth.complex_normal(m, synth.rng(cfg, 0, synth.NOISE)))
    y = y.astype(np.complex64).astype(np.complex128)
    eps = problem.eps_blocks(sigma, sizes)
    _say(f"[e2e {name}] GPU plan")
    op = sh.op_create(uv, n, 2, J, off)
    psi = sh.psi_create(n, 4)
    d = dict(name=name, n=n, m=m, R=R, J=J, uv=uv, off=off, sizes=sizes, x_true=x_true, op_o=op_o, clean=clean,
             y=y, eps=eps, op=op, psi=psi, iters=iters,
             y_dev=torch.tensor(y, dtype=torch.complex64, device="cuda"))
    yield d
    sh.psi_destroy(psi)
    sh.op_destroy(op)


def _blocks(wl):
    o = wl["off"]
    return [(int(o[i]), int(o[i + 1])) for i in range(len(o) - 1)]


def test_dense_phi_per_block(sh, wl):
    _say(f"[e2e {wl['name']}] Phi of the sky on the GPU")
    vis = torch.empty(wl["m"], dtype=torch.complex64, device="cuda")
    sh.phi_fwd(wl["op"], torch.tensor(wl["x_true"], dtype=torch.float32, device="cuda"), vis)
    got = vis.cpu().numpy().astype(np.complex128)
    ref = wl["clean"]
    # Each block's error against its own norm, and against its share of the whole vector's norm
    # (||Phi x|| sqrt(M_b / M)): float32 rounding in the FFT leaves every grid value, and so every
    # visibility, with an absolute error near 1e-7 of the RMS visibility, so a block whose visibilities
    # are far below the RMS (radial annuli away from the centre) shows a larger error against its own
    # norm.  The bar takes the larger of the two scales: an error confined to one block still has to
    # stay below 1e-5 of what that block would hold at the RMS level.
    m = wl["m"]
    nref = np.linalg.norm(ref)
    own = np.array([helpers.rel(got[lo:hi], ref[lo:hi]) for lo, hi in _blocks(wl)])
    scale = np.array([max(np.linalg.norm(ref[lo:hi]), nref * np.sqrt((hi - lo) / m)) for lo, hi in _blocks(wl)])
    err = np.array([np.linalg.norm(got[lo:hi] - ref[lo:hi]) for lo, hi in _blocks(wl)])
    print(f"[e2e {wl['name']}] Phi per block: error / own norm max {own.max():.2e} (block {own.argmax()}), "
          f"median {np.median(own):.2e}; error / max(own norm, share of the RMS) max {(err / scale).max():.2e}; "
          f"whole vector {helpers.rel(got, ref):.2e}")
    assert helpers.rel(got, ref) <= OP_TOL
    assert np.all(err <= OP_TOL * scale)


def test_dense_phi_adjoint_per_block_and_pixel(sh, wl):
    n = wl["n"]
    out = torch.empty((n, n), dtype=torch.float32, device="cuda")
    errs = []
    for b, (lo, hi) in enumerate(_blocks(wl)):
        vb = torch.zeros(wl["m"], dtype=torch.complex64, device="cuda")
        vb[lo:hi] = wl["y_dev"][lo:hi]
        sh.phi_adj(wl["op"], vb, out)
        got = out.cpu().numpy().astype(np.float64)
        ref = wl["op_o"].subset(lo, hi).adj(wl["y"][lo:hi])
        errs.append(helpers.rel(got, ref))
    errs = np.array(errs)
    _say(f"[e2e {wl['name']}] Phi^dagger of the data on the GPU")
    sh.phi_adj(wl["op"], wl["y_dev"], out)
    got = out.cpu().numpy().astype(np.float64)
    ref = wl["op_o"].adj(wl["y"])
    pix = float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))
    c = n // 2
    centre = helpers.rel(got[c - 32:c + 32, c - 32:c + 32], ref[c - 32:c + 32, c - 32:c + 32])
    print(f"[e2e {wl['name']}] Phi^dagger per-block errors: max {errs.max():.2e} (block {errs.argmax()}); "
          f"all data {helpers.rel(got, ref):.2e}, largest pixel error / largest pixel {pix:.2e}, "
          f"central 64 x 64 {centre:.2e}")
    assert errs.max() <= OP_TOL
    assert helpers.rel(got, ref) <= OP_TOL
    assert pix <= OP_TOL
    assert centre <= OP_TOL


def test_time_to_tol_feasible_under_oracle_operator(sh, wl):
    n = wl["n"]
    prm = sh.sdmm_default_params()
    prm.tol_rel, prm.passes, prm.max_iter = 1e-4, 5, 300    # check every 10 iterations, dual residual 1e-2
    x = torch.empty((n, n), dtype=torch.float32, device="cuda")
    _say(f"[e2e {wl['name']}] solve to tolerance on the GPU")
    info, resid = sh.sdmm_solve(wl["op"], wl["psi"], wl["y_dev"], wl["eps"], None, None, prm, x)
    xh = x.cpu().numpy().astype(np.float64)
    v = wl["op_o"].fwd(xh)
    r = np.array([np.linalg.norm(wl["y"][lo:hi] - v[lo:hi]) for lo, hi in _blocks(wl)])
    ratio = r / wl["eps"]
    print(f"[e2e {wl['name']}] to tolerance: {info['iters_total']} iterations, converged {info['converged']}; "
          f"max ||y_i - Phi_i x|| / eps_i = {ratio.max():.7f} (oracle FP64), "
          f"{np.max(resid / wl['eps']):.7f} (GPU FP32); "
          f"GPU vs oracle residuals {np.max(np.abs(resid - r) / r):.2e}")
    assert info["converged"] == 1
    assert np.all(ratio <= 1 + SLACK), (int(ratio.argmax()), float(ratio.max()))
    assert xh.min() >= -1e-3 * xh.max()


def test_fixed_schedule_image_parity(sh, wl):
    n, iters = wl["n"], wl["iters"]
    psi_o = wavelets.SARA(n, 4)
    _say(f"[e2e {wl['name']}] oracle: block weights, nu, gamma")
    a = measurement.block_density_weights(wl["uv"], n, 2, wl["off"])
    np.testing.assert_array_equal(a, sh.block_weights(wl["op"]))   # the same counts on the same cells
    # two power-iteration steps from the ones image: any nu > 0 normalises (3) without changing its
    # solutions, and both sides are given the same one
    nu = measurement.op_norm(measurement.BlockWeighted(wl["op_o"], wl["off"], a), np.ones((n, n)), max_iter=2, tol=0.0)
    gamma = sdmm.default_gamma(wl["op_o"], psi_o, wl["y"], nu, offsets=wl["off"], block_weights=a)
    _say(f"[e2e {wl['name']}] oracle: 2 passes x {iters} SDMM iterations (nu {nu:.6g}, gamma {gamma:.4g})")
    p = sdmm.Params(gamma=gamma, nu=nu, max_iter=iters, cg_iters=2, passes=2, block_weights=a)
    x_ref, W_ref, infos, _ = sdmm.sara(wl["op_o"], psi_o, wl["y"], wl["off"], wl["eps"], p)
    prm = sh.sdmm_default_params()
    prm.gamma, prm.nu, prm.max_iter, prm.cg_iters, prm.passes = gamma, nu, iters, 2, 2
    x = torch.empty((n, n), dtype=torch.float32, device="cuda")
    _say(f"[e2e {wl['name']}] GPU: the same schedule")
    info, resid = sh.sdmm_solve(wl["op"], wl["psi"], wl["y_dev"], wl["eps"], None, None, prm, x)
    got = x.cpu().numpy().astype(np.float64)
    err = helpers.rel(got, x_ref)
    rerr = float(np.max(np.abs(resid - infos[-1].block_resid) / infos[-1].block_resid))
    print(f"[e2e {wl['name']}] fixed schedule: image error vs oracle {err:.2e}, block residuals {rerr:.2e}, "
          f"objective {info['objective']:.8g} vs {infos[-1].objective:.8g}")
    assert info["iters_total"] == 2 * iters
    assert err <= IMG_TOL
    assert rerr <= 1e-4
    assert info["objective"] == pytest.approx(infos[-1].objective, rel=1e-4)
