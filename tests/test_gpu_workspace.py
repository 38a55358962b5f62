"""Solver, dictionary and Toeplitz operator on caller-provided device memory (a torch tensor).

With a workspace of the size the library asks for, every device allocation of the call is carved from
it, and the results are those of the allocating entry points bit for bit: the workspace only changes
where the memory comes from.  A workspace smaller than asked for, or misaligned, is refused before
anything is enqueued.
"""
import numpy as np
import pytest

from tests import helpers

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sh():
    from paper_1502_05037_amd import sarahip
    return sarahip


def _params(sh, **kw):
    p = sh.sdmm_default_params()
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def _ws(nbytes):
    return torch.empty(max(nbytes, 1), dtype=torch.uint8, device="cuda")


@pytest.mark.parametrize("flags", [{}, {"synthesis": 1}, {"block_fraction": 0.5, "block_seed": 3},
                                   {"toeplitz": 0, "block_norm": 0}, {"tol_rel": 1e-4, "max_iter": 200}])
def test_solve_on_a_workspace_equals_the_allocating_solve(sh, flags):
    pb = helpers.build(70, 64, 3000, 3, 6, prob=1)
    op = sh.op_create(pb.uv, pb.n, 2, pb.J, pb.offsets)
    psi = sh.psi_create(pb.n, 4)
    try:
        kw = dict(max_iter=30, passes=2)
        kw.update(flags)
        prm = _params(sh, **kw)
        y = torch.tensor(pb.y, dtype=torch.complex64, device="cuda")
        x1 = torch.empty((pb.n, pb.n), device="cuda")
        i1, r1 = sh.sdmm_solve(op, psi, y, pb.eps, None, None, prm, x1)
        nbytes = sh.workspace_bytes(op, psi, prm)
        ws = _ws(nbytes)
        x2 = torch.empty_like(x1)
        i2, r2 = sh.sdmm_solve_ws(op, psi, y, pb.eps, None, None, prm, x2, ws)
        torch.cuda.synchronize()
        print(f"{flags}: workspace {nbytes / 2**20:.1f} MiB")
        assert torch.equal(x1, x2)
        np.testing.assert_array_equal(r1, r2)
        assert i1["pass_iters"] == i2["pass_iters"] and i1["objective"] == i2["objective"]
        # too small, or misaligned: refused
        with pytest.raises(sh.SarahipError) as e:
            sh.sdmm_solve_ws(op, psi, y, pb.eps, None, None, prm, x2, _ws(nbytes - 256))
        assert e.value.status == -1
        big = _ws(nbytes + 512)
        with pytest.raises(sh.SarahipError):
            sh.sdmm_solve_ws(op, psi, y, pb.eps, None, None, prm, x2, big[1:])
    finally:
        sh.psi_destroy(psi)
        sh.op_destroy(op)


def test_session_on_a_workspace(sh):
    pb = helpers.build(71, 64, 3000, 3, 6, prob=2)
    op = sh.op_create(pb.uv, pb.n, 2, pb.J, pb.offsets)
    psi = sh.psi_create(pb.n, 4)
    try:
        prm = _params(sh)
        y = torch.tensor(pb.y, dtype=torch.complex64, device="cuda")
        ws = _ws(sh.workspace_bytes(op, psi, prm))
        s1 = sh.sdmm_create(op, psi, y, pb.eps, None, None, prm)
        s2 = sh.sdmm_create_ws(op, psi, y, pb.eps, None, None, prm, ws)
        try:
            sh.sdmm_iterate(s1, 25)
            sh.sdmm_iterate(s2, 25)
            x1 = torch.empty((pb.n, pb.n), device="cuda")
            x2 = torch.empty_like(x1)
            r1, _ = sh.sdmm_result(s1, x1, 3)
            r2, _ = sh.sdmm_result(s2, x2, 3)
        finally:
            sh.sdmm_destroy(s2)
            sh.sdmm_destroy(s1)
        assert torch.equal(x1, x2)
        np.testing.assert_array_equal(r1, r2)
    finally:
        sh.psi_destroy(psi)
        sh.op_destroy(op)


def test_dictionary_and_toeplitz_on_workspaces(sh):
    pb = helpers.build(72, 64, 3000, 2, 6, prob=3)
    n = pb.n
    g = torch.Generator(device="cpu").manual_seed(3)
    x = torch.rand((n, n), generator=g).cuda()
    psi1 = sh.psi_create(n, 4)
    wsp = _ws(sh.psi_workspace_bytes(n, 4, sh.SARA_MASK, 1))
    psi2 = sh.psi_create_ws(n, 4, sh.SARA_MASK, 1, wsp)
    op = sh.op_create(pb.uv, n, 2, pb.J, pb.offsets)
    try:
        c1 = torch.empty((9, n, n), device="cuda")
        c2 = torch.empty_like(c1)
        sh.psi_adj(psi1, x, c1)
        sh.psi_adj(psi2, x, c2)
        y1 = torch.empty_like(x)
        y2 = torch.empty_like(x)
        sh.psi_fwd(psi1, c1, y1)
        sh.psi_fwd(psi2, c1, y2)
        torch.cuda.synchronize()
        assert torch.equal(c1, c2) and torch.equal(y1, y2)
        t1 = sh.toeplitz_create(op)
        wst = _ws(sh.toeplitz_workspace_bytes(op))
        t2 = sh.toeplitz_create_ws(op, wst)
        try:
            o1 = torch.empty_like(x)
            o2 = torch.empty_like(x)
            sh.toeplitz_apply(t1, x, o1)
            sh.toeplitz_apply(t2, x, o2)
            torch.cuda.synchronize()
            assert torch.equal(o1, o2)
        finally:
            sh.toeplitz_destroy(t2)
            sh.toeplitz_destroy(t1)
        with pytest.raises(sh.SarahipError):
            sh.toeplitz_create_ws(op, _ws(sh.toeplitz_workspace_bytes(op) - 256))
    finally:
        sh.op_destroy(op)
        sh.psi_destroy(psi2)
        sh.psi_destroy(psi1)
