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

Bar: norm-wise relative error <= 1e-5 (as at the small sizes).
"""
import numpy as np
import pytest

from oracle import measurement
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
