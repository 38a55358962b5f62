"""Checkpoint and resume of a solver session, the device-memory cap and plan creation on a caller's stream.

* 150 iterations, export, a fresh session of the same inputs, import, 150 more: the image and block
  residuals equal those of 300 iterations of one session bitwise (every kernel sums in a fixed order), for
  the analysis prior, block-subset iterations (whose iteration counter and running image are part of the
  state) and the synthesis prior (whose coefficients are).
* An import checks the state's size and header against the session: a truncated state, or one from a
  session with other options, is refused with SH_EINVAL and leaves the session as it was.
* SH_MAX_DEVICE_BYTES caps the device memory the library holds: a plan that would pass the cap fails with
  SH_ENOMEM, the library's live byte count is back where it was, and without the cap the same plan builds.
* A plan built with its uploads on a side stream gives the same operator as one built on the null stream.
"""
import os

import numpy as np
import pytest

from tests import helpers

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

ENOMEM, EINVAL = -2, -1


@pytest.fixture(scope="module")
def sh():
    from paper_1502_05037_amd import sarahip
    return sarahip


def _params(sh, **kw):
    p = sh.sdmm_default_params()
    for k, v in kw.items():
        setattr(p, k, v)
    return p


@pytest.fixture(scope="module")
def problem(sh):
    pb = helpers.build(80, 64, 3000, 4, 6, prob=2)
    op = sh.op_create(pb.uv, 64, 2, 6, pb.offsets)
    psi = sh.psi_create(64, 4)
    y = torch.tensor(pb.y, dtype=torch.complex64, device="cuda")
    yield pb, op, psi, y
    sh.psi_destroy(psi)
    sh.op_destroy(op)


def _run(sh, op, psi, y, eps, p, iters, state=None):
    """A fresh session; optionally imports `state`; `iters` iterations; returns (x, residuals, state)."""
    s = sh.sdmm_create(op, psi, y, eps, None, None, p)
    try:
        if state is not None:
            sh.sdmm_state_import(s, state)
        sh.sdmm_iterate(s, iters)
        x = torch.empty((64, 64), device="cuda")
        r, _ = sh.sdmm_result(s, x, len(eps))
        out = sh.sdmm_state_export(s)
        torch.cuda.synchronize()
        return x.cpu().numpy(), r, out
    finally:
        sh.sdmm_destroy(s)


@pytest.mark.parametrize("variant", ["analysis", "block_subset", "synthesis"])
def test_checkpoint_resume_bitwise(sh, problem, variant):
    pb, op, psi, y = problem
    kw = {"analysis": {}, "block_subset": dict(block_fraction=0.5, block_seed=7), "synthesis": dict(synthesis=1)}[variant]
    p = _params(sh, cg_iters=4, **kw)
    # nu and gamma from one solve, so that every session starts from the same normalisation
    info, _ = sh.sdmm_solve(op, psi, y, pb.eps, None, None, _params(sh, max_iter=1, passes=1, cg_iters=4, **kw),
                            torch.empty((64, 64), device="cuda"))
    p.nu, p.gamma = info["nu"], info["gamma"]
    x300, r300, _ = _run(sh, op, psi, y, pb.eps, p, 300)
    x150, _, st150 = _run(sh, op, psi, y, pb.eps, p, 150)
    xr, rr, _ = _run(sh, op, psi, y, pb.eps, p, 150, state=st150)
    print(f"{variant}: state {st150.nbytes} bytes; resumed vs single run max |dx| {np.max(np.abs(xr - x300)):.3g}; "
          f"150 vs 300 iterations differ by {helpers.rel(x150, x300):.2e}", flush=True)
    assert helpers.rel(x150, x300) > 0          # the second half did something
    np.testing.assert_array_equal(xr, x300)
    np.testing.assert_array_equal(rr, r300)


def test_import_refuses_other_sessions(sh, problem):
    pb, op, psi, y = problem
    p = _params(sh, cg_iters=2)
    info, _ = sh.sdmm_solve(op, psi, y, pb.eps, None, None, _params(sh, max_iter=1, passes=1, cg_iters=2),
                            torch.empty((64, 64), device="cuda"))
    p.nu, p.gamma = info["nu"], info["gamma"]
    _, _, st = _run(sh, op, psi, y, pb.eps, p, 20)
    q = _params(sh, cg_iters=2, block_fraction=0.5, nu=p.nu, gamma=p.gamma)
    s = sh.sdmm_create(op, psi, y, pb.eps, None, None, q)
    try:
        with pytest.raises(sh.SarahipError) as e:      # other options: the state has no counter or running image
            sh.sdmm_state_import(s, st)
        assert e.value.status == EINVAL
    finally:
        sh.sdmm_destroy(s)
    s = sh.sdmm_create(op, psi, y, pb.eps, None, None, p)
    try:
        before = sh.sdmm_state_export(s)
        for bad in (st[:-8], np.concatenate([st, np.zeros(8, np.uint8)])):
            with pytest.raises(sh.SarahipError) as e:
                sh.sdmm_state_import(s, bad)
            assert e.value.status == EINVAL
        corrupt = st.copy()
        corrupt[0] ^= 0xFF                              # the header's tag
        with pytest.raises(sh.SarahipError) as e:
            sh.sdmm_state_import(s, corrupt)
        assert e.value.status == EINVAL
        np.testing.assert_array_equal(sh.sdmm_state_export(s), before)   # refused imports change nothing
    finally:
        sh.sdmm_destroy(s)


def test_device_memory_cap(sh, problem):
    pb = problem[0]
    live0, cap0 = sh.device_bytes()
    assert cap0 == -1
    os.environ["SH_MAX_DEVICE_BYTES"] = str(live0 + 4096)
    try:
        assert sh.device_bytes()[1] == live0 + 4096
        with pytest.raises(sh.SarahipError) as e:
            sh.op_create(pb.uv, 64, 2, 6, pb.offsets)
        assert e.value.status == ENOMEM
        assert "SH_MAX_DEVICE_BYTES" in str(e.value)
    finally:
        del os.environ["SH_MAX_DEVICE_BYTES"]
    assert sh.device_bytes() == (live0, -1)           # the failed plan gave back what it had taken
    op = sh.op_create(pb.uv, 64, 2, 6, pb.offsets)
    try:
        assert sh.device_bytes()[0] > live0
    finally:
        sh.op_destroy(op)
    assert sh.device_bytes()[0] == live0


def test_plan_on_a_side_stream(sh, problem):
    pb, op, _, _ = problem
    side = torch.cuda.Stream()
    x = torch.tensor(helpers.build(80, 64, 3000, 4, 6, prob=2).x_true, dtype=torch.float32, device="cuda")
    with torch.cuda.stream(side):
        op2 = sh.op_create_stream(pb.uv, 64, 2, 6, pb.offsets, stream=side.cuda_stream)
    try:
        v1 = torch.empty(len(pb.uv), dtype=torch.complex64, device="cuda")
        v2 = torch.empty_like(v1)
        sh.phi_fwd(op, x, v1)
        sh.phi_fwd(op2, x, v2)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(v1.cpu().numpy(), v2.cpu().numpy())
    finally:
        sh.op_destroy(op2)
