"""GPU parity of the fused proximal/dual steps and the float64 reductions against the oracle.

Element-wise results: within FP32 rounding of the oracle's closed forms on the same FP32 inputs.
Float64 reductions (block norms, standard deviation): 1e-12 relative on identical FP32 inputs.
"""
import numpy as np
import pytest

from oracle import prox, sdmm
from paper_1502_05037_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sh():
    from paper_1502_05037_amd import sarahip
    return sarahip


def _f32(a):
    return np.asarray(a, dtype=np.float32)


def _dev(a, dtype=torch.float32):
    return torch.tensor(np.asarray(a), dtype=dtype, device="cuda")


@pytest.mark.parametrize("D,weighted", [(1, False), (1000, True), (100003, True), (589824, False),
                                        (9 * 1024 * 1024, True)])   # the 1024^2 SARA coefficient vector
def test_prox_l1(sh, D, weighted):
    g = synth.rng(31, D, 0)
    s, z = _f32(g.normal(size=D)), _f32(0.3 * g.normal(size=D))
    W = _f32(g.uniform(0.01, 1.0, size=D)) if weighted else None
    gamma = np.float32(0.4)
    zd, vd = _dev(z), torch.empty(D, device="cuda")
    sh.prox_l1(_dev(s), zd, _dev(W) if weighted else None, float(gamma), vd)
    t = s.astype(np.float64) + z
    y = prox.soft(t, float(gamma) * (W.astype(np.float64) if weighted else 1.0))
    zr = t - y
    np.testing.assert_allclose(zd.cpu().numpy(), zr, rtol=0, atol=1e-6)
    np.testing.assert_allclose(vd.cpu().numpy(), y - zr, rtol=0, atol=2e-6)


def test_prox_pos(sh):
    N = 70001
    g = synth.rng(32, 0, 0)
    s, z = _f32(g.normal(size=N)), _f32(0.5 * g.normal(size=N))
    zd, vd = _dev(z), torch.empty(N, device="cuda")
    sh.prox_pos(_dev(s), zd, vd)
    t = s.astype(np.float64) + z
    y = prox.positive(t)
    np.testing.assert_allclose(zd.cpu().numpy(), t - y, rtol=0, atol=1e-6)
    np.testing.assert_allclose(vd.cpu().numpy(), 2 * y - t, rtol=0, atol=2e-6)


def test_prox_ball_blocks(sh):
    n, m, R = 32, 50000, 7
    uv = synth.uv_gaussian(m, synth.rng(33, 0, synth.UV))
    off = synth.offsets(synth.block_sizes(m, R, synth.rng(33, 0, synth.BLOCKS)))
    g = synth.rng(33, 0, 0)
    cplx = lambda k: (g.normal(size=k) + 1j * g.normal(size=k)).astype(np.complex64)
    s, z, yh = cplx(m), 0.1 * cplx(m), cplx(m)
    # a mix of blocks inside, on and outside their balls
    eps = np.array([np.linalg.norm((s + z - yh).astype(np.complex128)[off[i]:off[i + 1]]) * f
                    for i, f in enumerate([0.5, 1.0, 2.0, 0.1, 1.5, 0.9, 1e-3])])
    op = sh.op_create(uv, n, 2, 6, off)
    try:
        zd = _dev(z, torch.complex64)
        vd = torch.empty(m, dtype=torch.complex64, device="cuda")
        resid = torch.empty(R, dtype=torch.float64, device="cuda")
        sh.prox_ball(op, _dev(s, torch.complex64), zd, _dev(yh, torch.complex64), _dev(eps, torch.float64), vd, resid)
        torch.cuda.synchronize()
    finally:
        sh.op_destroy(op)
    s64, z64, y64 = (a.astype(np.complex128) for a in (s, z, yh))
    zr = np.empty(m, complex)
    vr = np.empty(m, complex)
    for i in range(R):
        lo, hi = off[i], off[i + 1]
        t = s64[lo:hi] + z64[lo:hi]
        y = prox.ball(t, y64[lo:hi], eps[i])
        zr[lo:hi] = t - y
        vr[lo:hi] = y - zr[lo:hi]
        assert resid[i].item() == pytest.approx(np.linalg.norm(s64[lo:hi] - y64[lo:hi]), rel=1e-12)
    np.testing.assert_allclose(zd.cpu().numpy(), zr, rtol=0, atol=2e-6)
    np.testing.assert_allclose(vd.cpu().numpy(), vr, rtol=0, atol=4e-6)


def test_std_and_reweight(sh):
    D = 589824
    c = _f32(synth.rng(34, 0, 0).standard_t(3, size=D))
    cd = _dev(c)
    sd = sh.std(cd)
    assert sd == pytest.approx(np.std(c.astype(np.float64)), rel=1e-12)
    Wd = torch.empty(D, device="cuda")
    sh.reweight(cd, 0.25, Wd)
    np.testing.assert_allclose(Wd.cpu().numpy(), sdmm.reweight(c.astype(np.float64), 0.25), rtol=1e-6)
    with pytest.raises(sh.SarahipError):
        sh.reweight(cd, 0.0, Wd)
