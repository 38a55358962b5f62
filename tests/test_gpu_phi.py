"""GPU parity of the measurement operator Phi and its real adjoint against the FP64 oracle NUFFT.

Bar: norm-wise relative error <= 1e-5 for both maps (FP32 operator vs FP64 oracle with the same
J, alpha and Kaiser-Bessel shape), on ragged sizes, several tiles, heavy tiles split into many
work items, grid-edge coordinates, single visibilities and one-visibility blocks.
"""
import numpy as np
import pytest

from oracle import measurement
from paper_1502_05037_amd import synth
from tests import helpers

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-5


@pytest.fixture(scope="module")
def sh():
    from paper_1502_05037_amd import sarahip
    return sarahip


def _dev(a, dtype):
    return torch.tensor(np.asarray(a), dtype=dtype, device="cuda")


def _fwd_adj(sh, uv, n, J, off, x, v):
    op = sh.op_create(uv, n, 2, J, off)
    try:
        vis = torch.empty(len(uv), dtype=torch.complex64, device="cuda")
        sh.phi_fwd(op, _dev(x, torch.float32), vis)
        xa = torch.empty((n, n), dtype=torch.float32, device="cuda")
        sh.phi_adj(op, _dev(v, torch.complex64), xa)
        torch.cuda.synchronize()
        return vis.cpu().numpy().astype(np.complex128), xa.cpu().numpy().astype(np.float64), sh.op_query(op)
    finally:
        sh.op_destroy(op)


def _inputs(n, m, seed):
    x = synth.sky(n, 20, 3.0, synth.rng(11, seed, synth.SKY)).astype(np.float32).astype(np.float64)
    v = synth.complex_normal(m, synth.rng(11, seed, synth.NOISE)).astype(np.complex64).astype(np.complex128)
    return x, v


@pytest.mark.parametrize("n,m,J,R,cov", [
    (64, 2048, 6, 1, "gaussian"),      # config-1 shape
    (64, 3001, 8, 3, "radial"),        # ragged M, J = 8
    (32, 777, 6, 2, "gaussian"),
    (16, 300, 4, 1, "gaussian"),       # smallest image / grid
    (128, 20000, 10, 5, "radial"),
    (256, 65536, 6, 8, "gaussian"),    # config-2 image, 1/10 of its visibilities
])
def test_phi_parity(sh, n, m, J, R, cov):
    print(f"phi parity n={n} m={m} J={J} R={R} {cov}", flush=True)
    g = synth.rng(11, n + m, synth.UV)
    uv = synth.sort_by_radius(synth.uv_gaussian(m, g) if cov == "gaussian" else synth.uv_radial(m, g))
    off = synth.offsets(synth.block_sizes(m, R, synth.rng(11, m, synth.BLOCKS))) if R > 1 else [0, m]
    x, v = _inputs(n, m, n + J)
    ref = measurement.NUFFT(uv, n, J)
    vis, xa, q = _fwd_adj(sh, uv, n, J, off, x, v)
    assert helpers.rel(vis, ref.fwd(x)) <= TOL
    assert helpers.rel(xa, ref.adj(v)) <= TOL


@pytest.mark.parametrize("J", [6, 8])
def test_internal_order_and_permutation(sh, J):
    n, m, R = 64, 5000, 4
    uv = synth.sort_by_radius(synth.uv_radial(m, synth.rng(12, 0, synth.UV)))
    off = synth.offsets(synth.block_sizes(m, R, synth.rng(12, 0, synth.BLOCKS)))
    x, v = _inputs(n, m, 3)
    op = sh.op_create(uv, n, 2, J, off)
    try:
        perm = sh.op_permutation(op)
        assert np.array_equal(np.sort(perm), np.arange(m))
        np.testing.assert_array_equal(sh.op_block_offsets(op), off)
        for b in range(R):   # the permutation stays inside each block
            seg = perm[off[b]:off[b + 1]]
            assert seg.min() >= off[b] and seg.max() < off[b + 1]
        xd = _dev(x, torch.float32)
        vi = torch.empty(m, dtype=torch.complex64, device="cuda")
        vu = torch.empty_like(vi)
        sh.phi_fwd_internal(op, xd, vi)
        sh.phi_fwd(op, xd, vu)
        back = torch.empty_like(vi)
        sh.vis_to_user(op, vi, back)
        fwd_i = torch.empty_like(vi)
        sh.vis_to_internal(op, vu, fwd_i)
        torch.cuda.synchronize()
        vi_h, vu_h = vi.cpu().numpy(), vu.cpu().numpy()
        np.testing.assert_array_equal(vi_h, vu_h[perm])
        np.testing.assert_array_equal(back.cpu().numpy(), vu_h)
        np.testing.assert_array_equal(fwd_i.cpu().numpy(), vi_h)
        # adjoint on internal order equals adjoint of the same values in user order
        vd = _dev(v, torch.complex64)
        vint = torch.empty_like(vd)
        sh.vis_to_internal(op, vd, vint)
        a1 = torch.empty((n, n), dtype=torch.float32, device="cuda")
        a2 = torch.empty_like(a1)
        sh.phi_adj(op, vd, a1)
        sh.phi_adj_internal(op, vint, a2)
        torch.cuda.synchronize()
        np.testing.assert_allclose(a1.cpu().numpy(), a2.cpu().numpy(), rtol=0, atol=1e-4 * float(a1.abs().max()))
    finally:
        sh.op_destroy(op)


def test_edges_heavy_tile_single_and_unit_blocks(sh):
    n, J = 32, 8
    # grid-edge coordinates, exact zero, values just below +pi
    edge = np.array([[-np.pi, -np.pi], [np.nextafter(np.pi, 0), 0.3], [0.0, np.nextafter(np.pi, 0)],
                     [-np.pi + 1e-9, 3.1], [0.0, 0.0], [1e-12, -1e-12]])
    # 20000 visibilities around kappa = 3 (one tile of the 64-cell grid): the tile is split into
    # several work items whose patches the fold sums
    heavy = 0.3 + 0.01 * synth.uv_gaussian(20000, synth.rng(13, 0, synth.UV))
    uv = np.concatenate([edge, heavy])
    m = len(uv)
    off = np.concatenate([np.arange(0, 6), [m]])        # five 1-visibility blocks then one big block
    x, v = _inputs(n, m, 4)
    ref = measurement.NUFFT(uv, n, J)
    vis, xa, q = _fwd_adj(sh, uv, n, J, off, x, v)
    assert q["max_items_per_tile"] >= 4
    assert helpers.rel(vis, ref.fwd(x)) <= TOL
    assert helpers.rel(xa, ref.adj(v)) <= TOL
    # a single visibility
    vis1, xa1, _ = _fwd_adj(sh, uv[:1], n, J, [0, 1], x, v[:1])
    assert helpers.rel(vis1, ref.fwd(x)[:1]) <= TOL
    assert helpers.rel(xa1, measurement.NUFFT(uv[:1], n, J).adj(v[:1])) <= TOL


def test_adjoint_dot_on_gpu(sh):
    n, m, J = 128, 30000, 8
    uv = synth.sort_by_radius(synth.uv_radial(m, synth.rng(14, 0, synth.UV)))
    x, v = _inputs(n, m, 5)
    x = x - 0.5  # signed image
    vis, xa, _ = _fwd_adj(sh, uv, n, J, [0, m], x, v)
    lhs = np.vdot(v, vis).real
    rhs = np.sum(x * xa)
    assert abs(lhs - rhs) <= 1e-5 * np.linalg.norm(v) * np.linalg.norm(vis)


def test_op_norm_matches_oracle(sh):
    n, m, J = 64, 2048, 6
    uv = synth.uv_gaussian(m, synth.rng(15, 0, synth.UV))
    ones = np.ones((n, n))
    ref = measurement.op_norm(measurement.NUFFT(uv, n, J), ones, max_iter=200, tol=1e-12)
    op = sh.op_create(uv, n, 2, J, [0, m])
    try:
        nu = sh.op_norm(op, _dev(ones, torch.float32), iters=200, tol=1e-12)
    finally:
        sh.op_destroy(op)
    assert nu == pytest.approx(ref, rel=1e-5)


@pytest.mark.parametrize("J", [6, 8])
def test_determinism_two_runs(sh, J):
    n, m = 64, 8000
    uv = synth.uv_radial(m, synth.rng(16, 0, synth.UV))
    x, v = _inputs(n, m, 6)
    a = _fwd_adj(sh, uv, n, J, [0, m], x, v)
    b = _fwd_adj(sh, uv, n, J, [0, m], x, v)
    np.testing.assert_array_equal(a[0], b[0])          # degridding: fixed summation order
    np.testing.assert_array_equal(a[1], b[1])          # gridding: atomic-free, fixed summation order


@pytest.mark.parametrize("tile,chunk", [(8, 64), (16, 300), (32, 0), (16, 0)])
def test_phi_parity_tuned_tiling(sh, tile, chunk):
    """Every tiling the autotuner may pick gives the same operator (small chunks force many items)."""
    n, m, J, R = 64, 6000, 8, 3
    uv = synth.sort_by_radius(synth.uv_radial(m, synth.rng(17, tile, synth.UV)))
    off = synth.offsets(synth.block_sizes(m, R, synth.rng(17, tile, synth.BLOCKS)))
    x, v = _inputs(n, m, tile)
    ref = measurement.NUFFT(uv, n, J)
    op = sh.op_create_tuned(uv, n, 2, J, off, tile=tile, chunk=chunk)
    try:
        vis = torch.empty(m, dtype=torch.complex64, device="cuda")
        sh.phi_fwd(op, _dev(x, torch.float32), vis)
        xa = torch.empty((n, n), dtype=torch.float32, device="cuda")
        sh.phi_adj(op, _dev(v, torch.complex64), xa)
        torch.cuda.synchronize()
        assert sh.op_query(op)["tile"] == tile
    finally:
        sh.op_destroy(op)
    assert helpers.rel(vis.cpu().numpy(), ref.fwd(x)) <= TOL
    assert helpers.rel(xa.cpu().numpy(), ref.adj(v)) <= TOL


def _cells_uv(K, cells, frac):
    """uv of visibilities at grid cells: kappa = cell + fraction in [0, K), uv = 2 pi kappa / K in [0, 2 pi)."""
    kappa = np.asarray(cells, dtype=np.float64) + np.asarray(frac)
    return kappa * (2.0 * np.pi / K)


@pytest.mark.parametrize("tile,chunk", [(0, 0), (8, 0), (32, 0), (16, 64)])
def test_gridding_j8_runs_streams_batches(sh, tile, chunk):
    """Gridding with J = 8, whose work items split into independent streams that accumulate runs of one
    cell and add each finished run into their own patch copy: one cell holding 5000 visibilities (a run
    longer than a batch, crossing every stream of its items), a tile with one visibility per cell (runs of
    one), a tile with three visibilities (fewer than a work item has streams), a tile with 257 (one past a
    full batch of every stream), and Gaussian-density visibilities elsewhere (tiles of 16 cells for the
    description; each tiling and a small chunk are run).  The adjoint of random data against the oracle
    pixel by pixel, and the forward map."""
    n, J = 64, 8
    K = 2 * n
    g = synth.rng(18, tile + chunk, synth.UV)
    one = _cells_uv(K, np.tile([[10, 20]], (5000, 1)), g.random((5000, 2)))
    grid16 = np.stack(np.meshgrid(np.arange(16), np.arange(16), indexing="ij"), -1).reshape(-1, 2)
    singles = _cells_uv(K, grid16 + [32, 16], g.random((256, 2)))             # every cell of tile (2, 1)
    three = _cells_uv(K, [[33, 34], [33, 35], [46, 40]], g.random((3, 2)))   # tile (2, 2)
    many = _cells_uv(K, [16, 32] + g.integers(0, 16, (257, 2)), g.random((257, 2)))   # tile (1, 2)
    rest = synth.uv_gaussian(4000, g)
    rc = np.floor(np.mod(rest, 2 * np.pi) * (K / (2 * np.pi))).astype(int) // 16
    keep = ~(((rc[:, 0] == 2) & (rc[:, 1] == 1)) | ((rc[:, 0] == 2) & (rc[:, 1] == 2)) | ((rc[:, 0] == 1) & (rc[:, 1] == 2)))
    uv = np.concatenate([one, singles, three, many, rest[keep]])
    uv = np.where(uv >= np.pi, uv - 2 * np.pi, uv)
    m = len(uv)
    off = [0, 2600, 5600, m]                                                # blocks split the one-cell run
    x, v = _inputs(n, m, 40 + tile)
    ref = measurement.NUFFT(uv, n, J)
    op = sh.op_create_tuned(uv, n, 2, J, off, tile=tile, chunk=chunk)
    try:
        vis = torch.empty(m, dtype=torch.complex64, device="cuda")
        sh.phi_fwd(op, _dev(x, torch.float32), vis)
        xa = torch.empty((n, n), dtype=torch.float32, device="cuda")
        sh.phi_adj(op, _dev(v, torch.complex64), xa)
        torch.cuda.synchronize()
        q = sh.op_query(op)
    finally:
        sh.op_destroy(op)
    got, want = xa.cpu().numpy().astype(np.float64), ref.adj(v)
    pix = float(np.max(np.abs(got - want)) / np.max(np.abs(want)))
    print(f"J=8 gridding tile {q['tile']} chunk {chunk}: {q['n_items']} items, adjoint error {helpers.rel(got, want):.2e}, "
          f"largest pixel error / largest pixel {pix:.2e}", flush=True)
    assert helpers.rel(got, want) <= TOL
    assert pix <= TOL
    assert helpers.rel(vis.cpu().numpy(), ref.fwd(x)) <= TOL
