"""Parity at the full measured size, in the configuration the benchmark times: a 1024 x 1024 image,
M = 2e7 visibilities of radial density in 64 uneven blocks, J = 8 on the 2048 x 2048 grid, the
default plan (tile 16, default work-item size).

The FP64 oracle cannot transform the whole problem within a test's time, so each map is checked where
the oracle's answer is exact for a part of it:

* Phi: degridding is per visibility, so the oracle NUFFT evaluated at 4096 sampled coordinates gives
  exactly those entries of Phi x; they are compared in user order and, through the plan's permutation,
  in the solver's internal order.
* Phi^dagger: a visibility vector that is zero except at 20 000 sampled positions goes through the
  full plan (every work item, every fold cell); the oracle adjoint of the samples alone is its exact
  image.
* The adjoint identity <Phi x, v> = <x, Phi^dagger v> with x and v dense over all 2e7 visibilities.
* The Toeplitz form of Re(Phi^H Phi) applied to a point source at c: its output at pixel p is
  k(p - c) = sum_m cos(u_m . (p - c)), which the oracle sums directly over all 2e7 visibilities at 24
  sampled pixels (the definition written out).
* The per-block l2-ball projection and dual update over the plan's 64 blocks, element-wise against the
  oracle's closed form, with the float64 block norms.
* The same sampled checks of Phi and Phi^dagger for the batched workload: 32 problems of 256 x 256 with
  1e5..1e6 visibilities each (1.15e7 in all) in one plan with the tuner's choice for it (J = 6, tile 16,
  work items of at most 1024 visibilities).

Bar: norm-wise relative error <= 1e-5 (as at the small sizes).
"""
import numpy as np
import pytest

from oracle import measurement, prox
from paper_1502_05037_amd import synth
from tests import helpers

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-5
N, M, R, J = 1024, 20_000_000, 64, 8
CFG = 3   # the seed stream of the benchmark's workload


@pytest.fixture(scope="module")
def sh():
    from paper_1502_05037_amd import sarahip
    return sarahip


@pytest.fixture(scope="module")
def full(sh):
    print(f"full-size parity: n={N} M={M} R={R} J={J}, building the plan", flush=True)
    uv = synth.sort_by_radius(synth.uv_radial(M, synth.rng(CFG, 0, synth.UV)))
    off = synth.offsets(synth.block_sizes(M, R, synth.rng(CFG, 0, synth.BLOCKS)))
    x = synth.sky(N, 200, 4.0, synth.rng(CFG, 0, synth.SKY)).astype(np.float32)
    op = sh.op_create(uv, N, 2, J, off)
    q = sh.op_query(op)
    assert (q["M"], q["K"], q["J"], q["R"], q["tile"]) == (M, 2 * N, J, R, 16)
    yield dict(uv=uv, off=off, x=x, op=op)
    sh.op_destroy(op)


def test_forward_sampled_entries(sh, full):
    uv, x, op = full["uv"], full["x"], full["op"]
    idx = np.sort(synth.rng(CFG, 1, synth.UV).choice(M, 4096, replace=False))
    vis = torch.empty(M, dtype=torch.complex64, device="cuda")
    sh.phi_fwd(op, torch.tensor(x, device="cuda"), vis)
    vint = torch.empty_like(vis)
    sh.phi_fwd_internal(op, torch.tensor(x, device="cuda"), vint)
    torch.cuda.synchronize()
    ref = measurement.NUFFT(uv[idx], N, J).fwd(x.astype(np.float64))
    got = vis.cpu().numpy()[idx].astype(np.complex128)
    print(f"Phi, user order: rel error {helpers.rel(got, ref):.2e} on {len(idx)} sampled visibilities", flush=True)
    assert helpers.rel(got, ref) <= TOL
    # internal position i holds user visibility perm[i]; the two orders hold the same values
    p = sh.op_permutation(op)
    inv = np.empty(M, dtype=np.int64)
    inv[p] = np.arange(M)
    got_int = vint.cpu().numpy()[inv[idx]].astype(np.complex128)
    assert helpers.rel(got_int, ref) <= TOL


def test_adjoint_of_sampled_visibilities(sh, full):
    uv, op = full["uv"], full["op"]
    idx = np.sort(synth.rng(CFG, 2, synth.UV).choice(M, 20_000, replace=False))
    vs = synth.complex_normal(len(idx), synth.rng(CFG, 2, synth.NOISE)).astype(np.complex64)
    v = np.zeros(M, dtype=np.complex64)
    v[idx] = vs
    xa = torch.empty((N, N), dtype=torch.float32, device="cuda")
    sh.phi_adj(op, torch.tensor(v, device="cuda"), xa)
    torch.cuda.synchronize()
    ref = measurement.NUFFT(uv[idx], N, J).adj(vs.astype(np.complex128))
    err = helpers.rel(xa.cpu().numpy().astype(np.float64), ref)
    print(f"Phi^dagger of {len(idx)} sampled visibilities through the full plan: rel error {err:.2e}", flush=True)
    assert err <= TOL


def test_adjoint_identity_dense(sh, full):
    op = full["op"]
    x = full["x"].astype(np.float64) - 0.5 * float(full["x"].mean())   # signed image
    v = synth.complex_normal(M, synth.rng(CFG, 3, synth.NOISE)).astype(np.complex64)
    vis = torch.empty(M, dtype=torch.complex64, device="cuda")
    sh.phi_fwd(op, torch.tensor(x, dtype=torch.float32, device="cuda"), vis)
    xa = torch.empty((N, N), dtype=torch.float32, device="cuda")
    sh.phi_adj(op, torch.tensor(v, device="cuda"), xa)
    torch.cuda.synchronize()
    fx = vis.cpu().numpy().astype(np.complex128)
    lhs = np.vdot(fx, v.astype(np.complex128)).real
    rhs = float(np.sum(x.astype(np.float32).astype(np.float64) * xa.cpu().numpy().astype(np.float64)))
    scale = np.linalg.norm(v.astype(np.complex128)) * np.linalg.norm(fx)
    print(f"<Phi x, v> = {lhs:.6e}, <x, Phi^dagger v> = {rhs:.6e}, |diff| / (|v| |Phi x|) = "
          f"{abs(lhs - rhs) / scale:.2e}", flush=True)
    assert abs(lhs - rhs) <= 1e-5 * scale


def test_toeplitz_point_source_sampled_pixels(sh, full):
    uv, op = full["uv"], full["op"]
    c = (N // 2 + 37, N // 2 - 101)
    x = np.zeros((N, N), dtype=np.float32)
    x[c] = 1.0
    t = sh.toeplitz_create(op)
    try:
        out = torch.empty((N, N), dtype=torch.float32, device="cuda")
        sh.toeplitz_apply(t, torch.tensor(x, device="cuda"), out)
        torch.cuda.synchronize()
    finally:
        sh.toeplitz_destroy(t)
    got_img = out.cpu().numpy().astype(np.float64)
    # the source pixel, its neighbours, and pixels across the image (offsets up to n - 1 in each axis)
    g = synth.rng(CFG, 5, synth.SKY)
    pix = [c, (c[0] + 1, c[1]), (c[0], c[1] - 1), (c[0] + 3, c[1] + 2)]
    pix += [tuple(int(v) for v in g.integers(0, N, 2)) for _ in range(20)]
    ref = np.empty(len(pix))
    for i, p in enumerate(pix):
        d = np.array([p[0] - c[0], p[1] - c[1]], dtype=np.float64)
        acc = 0.0
        for lo in range(0, M, 1 << 22):
            acc += float(np.sum(np.cos(uv[lo:lo + (1 << 22)] @ d)))
        ref[i] = acc
    got = np.array([got_img[p] for p in pix])
    err = np.max(np.abs(got - ref)) / ref[0]
    print(f"Toeplitz product of a point source: k(0) = {ref[0]:.6e}, max |error| / k(0) over {len(pix)} pixels "
          f"{err:.2e}, norm-wise {helpers.rel(got, ref):.2e}", flush=True)
    assert ref[0] == pytest.approx(M, rel=1e-12)
    assert helpers.rel(got, ref) <= TOL and err <= TOL


def test_ball_projection_all_blocks(sh, full):
    op, off = full["op"], full["off"]
    g = synth.rng(CFG, 4, 0)
    cplx = lambda k: (g.normal(size=k) + 1j * g.normal(size=k)).astype(np.complex64)
    s, z, yh = cplx(M), 0.1 * cplx(M), cplx(M)
    t64 = s.astype(np.complex128) + z.astype(np.complex128)
    y64 = yh.astype(np.complex128)
    # blocks inside, on and outside their balls
    f = np.resize([0.5, 1.0, 2.0, 0.1, 1.5, 0.9, 1e-3], R)
    eps = np.array([np.linalg.norm(t64[off[i]:off[i + 1]] - y64[off[i]:off[i + 1]]) * f[i] for i in range(R)])
    zd = torch.tensor(z, device="cuda")
    vd = torch.empty(M, dtype=torch.complex64, device="cuda")
    resid = torch.empty(R, dtype=torch.float64, device="cuda")
    sh.prox_ball(op, torch.tensor(s, device="cuda"), zd, torch.tensor(yh, device="cuda"),
                 torch.tensor(eps, dtype=torch.float64, device="cuda"), vd, resid)
    torch.cuda.synchronize()
    zg, vg, rg = zd.cpu().numpy(), vd.cpu().numpy(), resid.cpu().numpy()
    s64 = s.astype(np.complex128)
    worst_z = worst_v = 0.0
    for i in range(R):
        lo, hi = off[i], off[i + 1]
        y = prox.ball(t64[lo:hi], y64[lo:hi], eps[i])
        zr = t64[lo:hi] - y
        worst_z = max(worst_z, float(np.max(np.abs(zg[lo:hi] - zr))))
        worst_v = max(worst_v, float(np.max(np.abs(vg[lo:hi] - (y - zr)))))
        assert rg[i] == pytest.approx(np.linalg.norm(s64[lo:hi] - y64[lo:hi]), rel=1e-12)
    print(f"ball projection over {R} blocks of {M} visibilities: max |dz| {worst_z:.2e}, max |dv| {worst_v:.2e}",
          flush=True)
    assert worst_z <= 2e-6 and worst_v <= 4e-6


@pytest.fixture(scope="module")
def batched(sh):
    import bench
    bw = bench.batched_workload()
    print(f"batched full-size parity: {bw['P']} problems of {bw['n']}^2, M = {int(bw['M_p'].sum())}", flush=True)
    op = sh.op_create_batched(bw["uv"], bw["M_p"], bw["n"], 2, 6, bw["off"], bw["R_p"], tile=16, chunk=1024)
    q = sh.op_query(op)
    assert (q["P"], q["J"], q["tile"]) == (bw["P"], 6, 16)
    yield bw, op
    sh.op_destroy(op)


def _problem_of(bw, idx):
    starts = np.concatenate([[0], np.cumsum(bw["M_p"])])
    return np.searchsorted(starts, idx, side="right") - 1, starts


def test_batched_forward_sampled_entries(sh, batched):
    bw, op = batched
    Mt, n = int(bw["M_p"].sum()), bw["n"]
    vis = torch.empty(Mt, dtype=torch.complex64, device="cuda")
    sh.phi_fwd(op, torch.tensor(bw["x_true"], device="cuda"), vis)
    torch.cuda.synchronize()
    idx = np.sort(synth.rng(4, 1, synth.UV).choice(Mt, 4096, replace=False))
    prob, _ = _problem_of(bw, idx)
    got = vis.cpu().numpy()[idx].astype(np.complex128)
    ref = np.empty(len(idx), dtype=np.complex128)
    for p in np.unique(prob):
        sel = prob == p
        ref[sel] = measurement.NUFFT(bw["uv"][idx[sel]], n, 6).fwd(bw["x_true"][p].astype(np.float64))
    err = helpers.rel(got, ref)
    print(f"batched Phi: rel error {err:.2e} on {len(idx)} sampled visibilities", flush=True)
    assert err <= TOL


def test_batched_adjoint_of_sampled_visibilities(sh, batched):
    bw, op = batched
    Mt, n, P = int(bw["M_p"].sum()), bw["n"], bw["P"]
    idx = np.sort(synth.rng(4, 2, synth.UV).choice(Mt, 20_000, replace=False))
    vs = synth.complex_normal(len(idx), synth.rng(4, 2, synth.NOISE)).astype(np.complex64)
    v = np.zeros(Mt, dtype=np.complex64)
    v[idx] = vs
    xa = torch.empty((P, n, n), dtype=torch.float32, device="cuda")
    sh.phi_adj(op, torch.tensor(v, device="cuda"), xa)
    torch.cuda.synchronize()
    got = xa.cpu().numpy().astype(np.float64)
    prob, _ = _problem_of(bw, idx)
    ref = np.zeros((P, n, n))
    for p in np.unique(prob):
        sel = prob == p
        ref[p] = measurement.NUFFT(bw["uv"][idx[sel]], n, 6).adj(vs[sel].astype(np.complex128))
    err = helpers.rel(got, ref)
    print(f"batched Phi^dagger of {len(idx)} sampled visibilities: rel error {err:.2e}", flush=True)
    assert err <= TOL


def test_largest_grid_against_direct_dft(sh):
    """n = 4096, alpha = 2: the largest grid side (8192) and FFT length the library accepts.  Phi at 64
    sampled visibilities and Phi^dagger of those 64 samples against the oracle's direct DFT (exact
    discretised measurement equation; the NUFFT's own error at J = 8 is ~2e-7), and the Toeplitz product
    of a point source against k(d) summed directly."""
    n, m, J = 4096, 20_000, 8
    uv = synth.sort_by_radius(synth.uv_radial(m, synth.rng(CFG, 7, synth.UV)))
    off = synth.offsets(synth.block_sizes(m, 4, synth.rng(CFG, 7, synth.BLOCKS)))
    x = synth.sky(n, 20, 3.0, synth.rng(CFG, 7, synth.SKY)).astype(np.float32)
    idx = np.sort(synth.rng(CFG, 8, synth.UV).choice(m, 64, replace=False))
    vs = synth.complex_normal(len(idx), synth.rng(CFG, 8, synth.NOISE)).astype(np.complex64)
    v = np.zeros(m, dtype=np.complex64)
    v[idx] = vs
    op = sh.op_create(uv, n, 2, J, off)
    try:
        assert sh.op_query(op)["K"] == 8192
        vis = torch.empty(m, dtype=torch.complex64, device="cuda")
        sh.phi_fwd(op, torch.tensor(x, device="cuda"), vis)
        xa = torch.empty((n, n), dtype=torch.float32, device="cuda")
        sh.phi_adj(op, torch.tensor(v, device="cuda"), xa)
        c = (n // 2 - 700, n // 2 + 1234)
        delta = torch.zeros((n, n), dtype=torch.float32, device="cuda")
        delta[c] = 1.0
        t = sh.toeplitz_create(op)
        try:
            tout = torch.empty_like(delta)
            sh.toeplitz_apply(t, delta, tout)
            torch.cuda.synchronize()
        finally:
            sh.toeplitz_destroy(t)
    finally:
        sh.op_destroy(op)
    dft = measurement.DFT(uv[idx], n)
    e_fwd = helpers.rel(vis.cpu().numpy()[idx].astype(np.complex128), dft.fwd(x.astype(np.float64)))
    e_adj = helpers.rel(xa.cpu().numpy().astype(np.float64), dft.adj(vs.astype(np.complex128)))
    pix = [c, (c[0] + 1, c[1] - 1)] + [tuple(int(q) for q in synth.rng(CFG, 9, synth.SKY).integers(0, n, 2))
                                       for _ in range(6)]
    got = np.array([float(tout[p].item()) for p in pix])
    ref = np.array([np.sum(np.cos(uv @ np.array([p[0] - c[0], p[1] - c[1]], dtype=np.float64))) for p in pix])
    e_toep = helpers.rel(got, ref)
    print(f"n = {n}, K = 8192: Phi rel error {e_fwd:.2e}, Phi^dagger {e_adj:.2e}, Toeplitz {e_toep:.2e}", flush=True)
    assert e_fwd <= TOL and e_adj <= TOL and e_toep <= TOL
