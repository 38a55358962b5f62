"""Pins of the U-Net oracle: each layer against an independent definition or library routine, every
parameter gradient against central finite differences, the bfloat16 rounding against hand-computed
ties, and Adam's first step against its closed form."""
import numpy as np
import pytest
from scipy import signal

from oracle import unet


def test_conv3_matches_scipy_correlate2d():
    g = np.random.default_rng(0)
    x = g.standard_normal((2, 3, 7, 9))
    W = g.standard_normal((4, 3, 3, 3))
    b = g.standard_normal(4)
    y = unet.conv3(x, W, b)
    for bi in range(2):
        for o in range(4):
            ref = b[o] + sum(signal.correlate2d(x[bi, c], W[o, c], mode="same", boundary="fill")
                             for c in range(3))
            np.testing.assert_allclose(y[bi, o], ref, rtol=1e-12, atol=1e-12)


def test_tconv_matches_scatter_definition():
    g = np.random.default_rng(1)
    x = g.standard_normal((2, 3, 3, 4))
    W = g.standard_normal((3, 5, 2, 2))
    b = g.standard_normal(5)
    ref = np.zeros((2, 5, 6, 8)) + b[None, :, None, None]
    for bi in range(2):
        for c in range(3):
            for yy in range(3):
                for xx in range(4):
                    for i in range(2):
                        for j in range(2):
                            ref[bi, :, 2 * yy + i, 2 * xx + j] += W[c, :, i, j] * x[bi, c, yy, xx]
    np.testing.assert_allclose(unet.tconv(x, W, b), ref, rtol=1e-12, atol=1e-12)


def test_pool_value_and_first_maximum_on_ties():
    x = np.array([[[[1.0, 3.0, 2.0, 2.0],
                    [3.0, 0.0, 2.0, 2.0],
                    [5.0, 4.0, -1.0, -2.0],
                    [4.0, 5.0, -3.0, -1.0]]]])
    y, idx = unet.pool(x)
    np.testing.assert_array_equal(y[0, 0], [[3.0, 2.0], [5.0, -1.0]])
    np.testing.assert_array_equal(idx[0, 0], [[1, 0], [0, 0]])   # ties: first in row-major order
    g = unet.pool_grad(np.ones((1, 1, 2, 2)), idx)
    np.testing.assert_array_equal(g[0, 0], [[0, 1, 1, 0], [0, 0, 0, 0], [1, 0, 1, 0], [0, 0, 0, 0]])


def test_bf16_rounding_ties_to_even():
    one = 1.0
    assert unet.bf16(one + 2.0 ** -8) == 1.0                           # halfway, 1.0 is even
    assert unet.bf16(one + 3 * 2.0 ** -8) == one + 2.0 ** -6          # halfway, rounds up to even
    assert unet.bf16(one + 2.0 ** -8 + 2.0 ** -20) == one + 2.0 ** -7  # above halfway
    assert unet.bf16(-(one + 3 * 2.0 ** -8)) == -(one + 2.0 ** -6)
    assert unet.bf16(1e-30) > 0                                       # float32 exponent range kept
    v = np.random.default_rng(2).standard_normal(1000)
    r = unet.bf16(v)
    np.testing.assert_array_equal(unet.bf16(r), r)
    assert np.max(np.abs(r - v) / np.abs(v)) <= 2.0 ** -8


def test_param_layout():
    shapes = dict(unet.param_shapes(32, 4))
    assert shapes["enc1a.w"] == (32, 1, 3, 3) and shapes["enc4b.w"] == (256, 256, 3, 3)
    assert shapes["up3t.w"] == (256, 128, 2, 2) and shapes["up3a.w"] == (128, 256, 3, 3)
    assert shapes["head.w"] == (1, 32, 1, 1)
    n = sum(int(np.prod(s)) for _, s in unet.param_shapes(32, 4))
    assert n == 1_925_025    # summed by hand, layer by layer
    flat = np.arange(n, dtype=np.float64)
    np.testing.assert_array_equal(unet.flatten(unet.unflatten(flat, 32, 4), 32, 4), flat)


def _tiny(seed=3, base=2, levels=4, n=16, B=2):
    g = np.random.default_rng(seed)
    params = {}
    for name, shape in unet.param_shapes(base, levels):
        fan_in = int(np.prod(shape[1:])) if not name.startswith("up") or not name.endswith("t.w") else shape[0] * 4
        params[name] = g.standard_normal(shape) * np.sqrt(2.0 / fan_in) if name.endswith(".w") \
            else 0.1 * g.standard_normal(shape)
    x = np.abs(g.standard_normal((B, 1, n, n)))
    t = np.abs(g.standard_normal((B, 1, n, n)))
    return params, x, t


def test_gradients_match_central_differences():
    params, x, t = _tiny()
    net = unet.UNet(2, 4, emul=False)
    loss, grads = net.loss_and_grads(params, x, t)
    y, tape = net.forward(params, x)
    assert loss == pytest.approx(float(np.mean((tape["head_z"] - t) ** 2)), rel=1e-15)
    np.testing.assert_array_equal(y, np.maximum(tape["head_z"], 0.0))
    g = np.random.default_rng(4)
    h = 1e-6
    for name, shape in unet.param_shapes(2, 4):
        flat = params[name].ravel()
        picks = g.choice(flat.size, size=min(flat.size, 6), replace=False)
        fd, an = [], []
        for k in picks:
            p1 = dict(params)
            p2 = dict(params)
            a, b = flat.copy(), flat.copy()
            a[k] += h
            b[k] -= h
            p1[name], p2[name] = a.reshape(shape), b.reshape(shape)
            l1 = float(np.mean((net.forward(p1, x)[1]["head_z"] - t) ** 2))
            l2 = float(np.mean((net.forward(p2, x)[1]["head_z"] - t) ** 2))
            fd.append((l1 - l2) / (2 * h))
            an.append(grads[name].ravel()[k])
        fd, an = np.array(fd), np.array(an)
        assert np.linalg.norm(fd - an) <= 1e-6 * np.linalg.norm(an) + 1e-10, (name, fd, an)


def test_emulated_forward_is_close_to_fp64_and_rounds_activations():
    params, x, t = _tiny(seed=5)
    y64, _ = unet.UNet(2, 4, emul=False).forward(params, x)
    y16, tape = unet.UNet(2, 4, emul=True).forward(params, x)
    assert np.linalg.norm(y16 - y64) <= 3e-2 * np.linalg.norm(y64)
    for k in ("enc1a_out", "enc4b_out", "up1b_out"):
        np.testing.assert_array_equal(unet.bf16(tape[k]), tape[k])


def test_adam_first_step_closed_form():
    g = np.random.default_rng(6)
    p = {"w": g.standard_normal(10)}
    gr = {"w": g.standard_normal(10)}
    opt = unet.Adam(lr=1e-3)
    out = opt.step(p, gr)
    np.testing.assert_allclose(out["w"], p["w"] - 1e-3 * gr["w"] / (np.abs(gr["w"]) + 1e-8), rtol=1e-12)
    # second step with the same gradient: m_hat = g, v_hat = g^2 again
    out2 = opt.step(out, gr)
    np.testing.assert_allclose(out2["w"], out["w"] - 1e-3 * gr["w"] / (np.abs(gr["w"]) + 1e-8), rtol=1e-10)


def test_warm_start_layer_layout_matches_oracle():
    """The flat parameter layout the warm-start module initialises (and the library reads) is the
    oracle's: same layers, kinds and channel counts in the same order."""
    from paper_1502_05037_amd import warmstart
    for base, levels in ((16, 1), (16, 3), (32, 4)):
        ours = warmstart.layer_list(base, levels)
        ref = [(kind, cin, cout) for _, kind, cin, cout in unet.layer_specs(base, levels)]
        assert ours == ref
        n = sum(int(np.prod(s)) for _, s in unet.param_shapes(base, levels))
        assert warmstart.he_init(base, levels, 0).size == n
