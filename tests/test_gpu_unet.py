"""GPU parity of the warm-start U-Net (BF16 MFMA products, FP32 accumulation) against the FP64 oracle
with bfloat16 emulated at the same points: forward within 1e-2, norm-wise.  Gradients, per parameter
tensor: within 2e-2 of the emulated oracle or within 0.6 of that tensor's BF16 noise (the distance
between the emulated and the exact FP64 gradient), and no further from the exact gradient than
1.5 times that noise.  Two correct BF16 computations that round in a different order drift apart
through the deep layers, so a fixed 2e-2 cannot hold there.  The Adam step is checked against its
closed form on the GPU's own gradient.
"""
import numpy as np
import pytest

from oracle import unet as ounet
from tests import helpers

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sh():
    from paper_1502_05037_amd import sarahip
    return sarahip


def _init(base, levels, seed):
    g = np.random.default_rng(seed)
    flat = []
    for name, shape in ounet.param_shapes(base, levels):
        if name.endswith(".w"):
            fan_in = shape[0] * 4 if name.endswith("t.w") else int(np.prod(shape[1:]))
            flat.append(g.standard_normal(int(np.prod(shape))) * np.sqrt(2.0 / fan_in))
        else:
            flat.append(0.05 * g.standard_normal(int(np.prod(shape))))
    return np.concatenate(flat).astype(np.float32)


def _data(B, n, seed):
    g = np.random.default_rng(seed)
    x = np.abs(g.standard_normal((B, n, n))).astype(np.float32)
    t = np.abs(g.standard_normal((B, n, n))).astype(np.float32)
    return x, t


# base 16 sends the 16-channel layers through the implicit-im2col product and the others through the direct
# convolution
@pytest.mark.parametrize("base,levels,n,B", [(16, 4, 32, 2), (16, 2, 24, 1), (32, 1, 16, 3), (16, 3, 20, 2)])
def test_forward_and_gradients_match_emulated_oracle(sh, base, levels, n, B):
    flat = _init(base, levels, 1)
    x, t = _data(B, n, 2)
    u = sh.unet_create(base, levels)
    try:
        assert sh.unet_num_params(u) == flat.size
        sh.unet_set_params(u, flat)
        np.testing.assert_array_equal(sh.unet_get_params(u), flat)
        xd, td = torch.tensor(x, device="cuda"), torch.tensor(t, device="cuda")
        y = torch.empty_like(xd)
        sh.unet_forward(u, xd, y)
        loss, grads = sh.unet_loss_grad(u, xd, td)
        torch.cuda.synchronize()
        y = y.cpu().numpy()
    finally:
        sh.unet_destroy(u)
    net = ounet.UNet(base, levels, emul=True)
    params = ounet.unflatten(flat.astype(np.float64), base, levels)
    y_ref, _ = net.forward(params, x[:, None].astype(np.float64))
    err = helpers.rel(y, y_ref[:, 0])
    print(f"forward error {err:.2e}")
    assert err <= 1e-2
    X, T = x[:, None].astype(np.float64), t[:, None].astype(np.float64)
    loss_ref, g_ref = net.loss_and_grads(params, X, T)
    assert loss == pytest.approx(loss_ref, rel=1e-2)
    _, g64 = ounet.UNet(base, levels, emul=False).loss_and_grads(params, X, T)
    gpu = ounet.unflatten(grads.astype(np.float64), base, levels)
    for name, _ in ounet.param_shapes(base, levels):
        if np.linalg.norm(g_ref[name]) == 0:
            continue
        e = helpers.rel(gpu[name], g_ref[name])            # GPU vs BF16-emulated oracle
        noise = helpers.rel(g_ref[name], g64[name])         # BF16 emulation vs exact FP64
        exact = helpers.rel(gpu[name], g64[name])           # GPU vs exact FP64
        print(f"{name:8s} gpu-emul {e:.2e} emul-fp64 {noise:.2e} gpu-fp64 {exact:.2e}")
        # within 2e-2 of the emulation, or well inside the BF16 rounding noise of that tensor
        assert e <= 2e-2 or e <= 0.6 * noise, (name, e, noise)
        # and never less accurate than the BF16 emulation itself
        assert exact <= 1.5 * noise + 1e-3, (name, exact, noise)


@pytest.mark.parametrize("n,B", [(64, 2), (40, 1)])
def test_warm_start_network_shape_matches_oracle(sh, n, B):
    """The warm start's own network (base 32, 4 levels: every 3x3 layer but the first in the direct convolution,
    64-channel tiles, the pooling formed inside the encoder convolutions), at whole and partial 8 x 32 pixel
    tiles.  Forward within 1e-2 of the emulated oracle; every gradient tensor no further from the exact FP64
    gradient than 1.5 times that tensor's BF16 noise (the emulation's own distance from it) + 1e-3, i.e. as
    accurate as a BF16 computation at these rounding points can be.  The distance to the emulation itself is
    printed, not bounded by 0.6 times the noise as in the smaller cases: in this 18-layer network two correct
    BF16 computations that sum in different orders drift apart by up to 0.9 times the noise (measured for the
    implicit-GEMM build as well as the direct-convolution one)."""
    base, levels = 32, 4
    flat = _init(base, levels, 1)
    x, t = _data(B, n, 2)
    u = sh.unet_create(base, levels)
    try:
        sh.unet_set_params(u, flat)
        xd, td = torch.tensor(x, device="cuda"), torch.tensor(t, device="cuda")
        y = torch.empty_like(xd)
        sh.unet_forward(u, xd, y)
        loss, grads = sh.unet_loss_grad(u, xd, td)
        torch.cuda.synchronize()
        y = y.cpu().numpy()
    finally:
        sh.unet_destroy(u)
    net = ounet.UNet(base, levels, emul=True)
    params = ounet.unflatten(flat.astype(np.float64), base, levels)
    y_ref, _ = net.forward(params, x[:, None].astype(np.float64))
    err = helpers.rel(y, y_ref[:, 0])
    print(f"forward error {err:.2e}")
    assert err <= 1e-2
    X, T = x[:, None].astype(np.float64), t[:, None].astype(np.float64)
    loss_ref, g_ref = net.loss_and_grads(params, X, T)
    assert loss == pytest.approx(loss_ref, rel=1e-2)
    _, g64 = ounet.UNet(base, levels, emul=False).loss_and_grads(params, X, T)
    gpu = ounet.unflatten(grads.astype(np.float64), base, levels)
    for name, _ in ounet.param_shapes(base, levels):
        if np.linalg.norm(g_ref[name]) == 0:
            continue
        noise = helpers.rel(g_ref[name], g64[name])
        exact = helpers.rel(gpu[name], g64[name])
        print(f"{name:8s} gpu-emul {helpers.rel(gpu[name], g_ref[name]):.2e} emul-fp64 {noise:.2e} "
              f"gpu-fp64 {exact:.2e}")
        assert exact <= 1.5 * noise + 1e-3, (name, exact, noise)


def test_adam_step_closed_form_and_training_reduces_loss(sh):
    base, levels, n, B = 16, 3, 32, 2
    flat = _init(base, levels, 3)
    x, t = _data(B, n, 4)
    u = sh.unet_create(base, levels)
    try:
        sh.unet_set_params(u, flat)
        xd, td = torch.tensor(x, device="cuda"), torch.tensor(t, device="cuda")
        loss0, g = sh.unet_loss_grad(u, xd, td)
        l_step = sh.unet_train_step(u, xd, td, 1e-3)
        assert l_step == loss0
        p1 = sh.unet_get_params(u).astype(np.float64)
        ref = flat.astype(np.float64) - 1e-3 * g / (np.abs(g) + 1e-8)
        np.testing.assert_allclose(p1, ref, rtol=1e-5, atol=1e-7)
        losses = [sh.unet_train_step(u, xd, td, 1e-3) for _ in range(30)]
        assert losses[-1] < 0.7 * loss0, (loss0, losses[-5:])
    finally:
        sh.unet_destroy(u)


def test_weight_operands_follow_parameter_changes(sh):
    """The bfloat16 weight operands are converted once per set of parameters: a forward pass after set_params or
    after a training step uses the new parameters (bit for bit the output of a fresh handle loaded with them),
    and repeated forward passes with unchanged parameters agree bit for bit."""
    base, levels, n, B = 16, 3, 32, 2
    pa, pb = _init(base, levels, 5), _init(base, levels, 6)
    x, t = _data(B, n, 7)
    xd, td = torch.tensor(x, device="cuda"), torch.tensor(t, device="cuda")
    u, v = sh.unet_create(base, levels), sh.unet_create(base, levels)
    try:
        y = torch.empty_like(xd)
        yref = torch.empty_like(xd)

        def fwd(h, out):
            sh.unet_forward(h, xd, out)
            torch.cuda.synchronize()
            return out.cpu().numpy().copy()

        sh.unet_set_params(u, pa)
        ya = fwd(u, y)
        np.testing.assert_array_equal(fwd(u, y), ya)
        sh.unet_set_params(u, pb)
        sh.unet_set_params(v, pb)
        yb = fwd(u, y)
        np.testing.assert_array_equal(yb, fwd(v, yref))
        assert not np.array_equal(ya, yb)
        sh.unet_train_step(u, xd, td, 1e-3)
        yc = fwd(u, y)
        sh.unet_set_params(v, sh.unet_get_params(u))
        np.testing.assert_array_equal(yc, fwd(v, yref))
        assert not np.array_equal(yb, yc)
    finally:
        sh.unet_destroy(u)
        sh.unet_destroy(v)


def test_unet_argument_errors(sh):
    for base, levels in ((8, 4), (24, 4), (16, 0), (16, 7)):
        with pytest.raises(sh.SarahipError) as e:
            sh.unet_create(base, levels)
        assert e.value.status == -1
    u = sh.unet_create(16, 4)
    try:
        x = torch.ones((1, 20, 20), device="cuda")   # 20 is not divisible by 8
        with pytest.raises(sh.SarahipError):
            sh.unet_forward(u, x, torch.empty_like(x))
        with pytest.raises(sh.SarahipError):
            sh.unet_set_params(u, np.zeros(10, dtype=np.float32))
        bad = np.zeros(sh.unet_num_params(u), dtype=np.float32)
        bad[5] = np.nan
        with pytest.raises(sh.SarahipError) as e:
            sh.unet_set_params(u, bad)
        assert e.value.status == -4
    finally:
        sh.unet_destroy(u)
