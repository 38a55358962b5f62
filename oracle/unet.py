"""FP64 oracle of the learned warm start: a small U-Net that maps a dirty image to a first image estimate.

The paper has no network; this is the warm-start design the hot path adds in front of SDMM.  Its
layers are plain definitions written out in NumPy, NCHW, float64:

* conv3   3x3 cross-correlation with zero padding 1, plus bias;
* relu    max(., 0);
* pool    2x2 max-pool with stride 2; on ties the gradient goes to the first maximum of the window in
          row-major order;
* tconv   2x2 stride-2 transposed convolution: out[o, 2y+a, 2x+b] = bias[o] + sum_c W[c, o, a, b] x[c, y, x];
* concat  channel concatenation [upsampled, skip];
* head    1x1 convolution to one channel; the prediction is relu of it.

Architecture (levels L, base channels c, channels c_l = c 2^(l-1)): encoder level l has two conv3 +
relu (level 1 from 1 input channel); levels 2..L start with a pool; level L is the bottleneck.
Decoder level l = L-1..1: tconv c_{l+1} -> c_l, concat with encoder level l's output, two conv3 +
relu (2 c_l -> c_l -> c_l).  Then the head.  Loss: mean squared error over all pixels between the head
output before its relu and the target (the relu applies to predictions only, so the head cannot stop
passing gradient).  Training: Adam with bias correction.

BF16 emulation (emul=True) rounds, to the nearest bfloat16 with ties to even, exactly the values
that enter a matrix product on the GPU: the network input, the weights (copies of the float64
master), every stored activation, and every gradient with respect to a layer output before it is
contracted.  Biases, the head output, the loss and all accumulations stay in float64.

Test infrastructure only: used by tests/ to check the HIP kernels.
"""
from __future__ import annotations

import numpy as np
from numpy.lib.stride_tricks import sliding_window_view


# ---- layer list (the flat parameter order of the network) -----------------------------------

def layer_specs(base: int, levels: int):
    """[(name, kind, cin, cout)] in parameter order; kind in {conv3, tconv, head}."""
    ch = [base * 2 ** l for l in range(levels)]
    specs = []
    for l in range(levels):
        cin = 1 if l == 0 else ch[l - 1]
        specs.append((f"enc{l + 1}a", "conv3", cin, ch[l]))
        specs.append((f"enc{l + 1}b", "conv3", ch[l], ch[l]))
    for l in range(levels - 2, -1, -1):
        specs.append((f"up{l + 1}t", "tconv", ch[l + 1], ch[l]))
        specs.append((f"up{l + 1}a", "conv3", 2 * ch[l], ch[l]))
        specs.append((f"up{l + 1}b", "conv3", ch[l], ch[l]))
    specs.append(("head", "head", ch[0], 1))
    return specs


def weight_shape(kind: str, cin: int, cout: int):
    return {"conv3": (cout, cin, 3, 3), "tconv": (cin, cout, 2, 2), "head": (cout, cin, 1, 1)}[kind]


def param_shapes(base: int, levels: int):
    """[(name, shape)]: for every layer its weight, then its bias (cout,)."""
    out = []
    for name, kind, cin, cout in layer_specs(base, levels):
        out.append((name + ".w", weight_shape(kind, cin, cout)))
        out.append((name + ".b", (cout,)))
    return out


def unflatten(flat, base: int, levels: int) -> dict:
    flat = np.asarray(flat, dtype=np.float64)
    params, k = {}, 0
    for name, shape in param_shapes(base, levels):
        n = int(np.prod(shape))
        params[name] = flat[k:k + n].reshape(shape)
        k += n
    if k != flat.size:
        raise ValueError(f"{flat.size} values for {k} parameters")
    return params


def flatten(params: dict, base: int, levels: int) -> np.ndarray:
    return np.concatenate([np.asarray(params[name], dtype=np.float64).ravel()
                           for name, _ in param_shapes(base, levels)])


# ---- bfloat16 rounding ------------------------------------------------------------------------

def bf16(a):
    """Nearest bfloat16 (8 significant bits, float32 exponent range), ties to even, via float32."""
    f = np.asarray(a, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


# ---- layers and their gradients ---------------------------------------------------------------

def conv3(x, W, b):
    win = sliding_window_view(np.pad(x, ((0, 0), (0, 0), (1, 1), (1, 1))), (3, 3), axis=(2, 3))
    return np.einsum("bchwij,ocij->bohw", win, W, optimize=True) + b[None, :, None, None]


def conv3_grads(x, W, g):
    """(dx, dW, db) of conv3 for upstream gradient g."""
    win = sliding_window_view(np.pad(x, ((0, 0), (0, 0), (1, 1), (1, 1))), (3, 3), axis=(2, 3))
    dW = np.einsum("bohw,bchwij->ocij", g, win, optimize=True)
    gwin = sliding_window_view(np.pad(g, ((0, 0), (0, 0), (1, 1), (1, 1))), (3, 3), axis=(2, 3))
    dx = np.einsum("bohwij,ocij->bchw", gwin, W[:, :, ::-1, ::-1], optimize=True)
    return dx, dW, g.sum(axis=(0, 2, 3))


def pool(x):
    """2x2 max-pool; also returns the row-major index (0..3) of the first maximum of each window."""
    B, C, H, W = x.shape
    w = x.reshape(B, C, H // 2, 2, W // 2, 2).transpose(0, 1, 2, 4, 3, 5).reshape(B, C, H // 2, W // 2, 4)
    idx = np.argmax(w, axis=-1)
    return np.take_along_axis(w, idx[..., None], axis=-1)[..., 0], idx


def pool_grad(g, idx):
    B, C, h, w = g.shape
    out = np.zeros((B, C, h, w, 4))
    np.put_along_axis(out, idx[..., None], g[..., None], axis=-1)
    return out.reshape(B, C, h, w, 2, 2).transpose(0, 1, 2, 4, 3, 5).reshape(B, C, 2 * h, 2 * w)


def tconv(x, W, b):
    B, C, H, Wd = x.shape
    y = np.einsum("bcyx,coij->boyixj", x, W, optimize=True).reshape(B, W.shape[1], 2 * H, 2 * Wd)
    return y + b[None, :, None, None]


def tconv_grads(x, W, g):
    B, C, H, Wd = x.shape
    g6 = g.reshape(B, g.shape[1], H, 2, Wd, 2)
    dx = np.einsum("boyixj,coij->bcyx", g6, W, optimize=True)
    dW = np.einsum("bcyx,boyixj->coij", x, g6, optimize=True)
    return dx, dW, g.sum(axis=(0, 2, 3))


def head(x, W, b):
    return np.einsum("bchw,oc->bohw", x, W[:, :, 0, 0]) + b[None, :, None, None]


def head_grads(x, W, g):
    dx = np.einsum("bohw,oc->bchw", g, W[:, :, 0, 0])
    dW = np.einsum("bohw,bchw->oc", g, x)[:, :, None, None]
    return dx, dW, g.sum(axis=(0, 2, 3))


# ---- network ------------------------------------------------------------------------------------

class UNet:
    def __init__(self, base: int, levels: int, emul: bool = True):
        if levels < 1:
            raise ValueError("levels >= 1")
        self.base, self.levels, self.emul = base, levels, emul
        self.specs = layer_specs(base, levels)

    def _r(self, a):
        return bf16(a) if self.emul else np.asarray(a, dtype=np.float64)

    def forward(self, params: dict, x):
        """x: (B, 1, H, W) with H, W divisible by 2^(levels-1).  Returns (y, tape)."""
        r, L = self._r, self.levels
        Wr = {k: (r(v) if k.endswith(".w") else np.asarray(v, dtype=np.float64)) for k, v in params.items()}
        tape = {"W": Wr}
        a = r(x)
        skips = []
        for l in range(1, L + 1):
            if l > 1:
                tape[f"pool{l}_in"] = a
                a, tape[f"pool{l}_idx"] = pool(a)
            for s in "ab":
                name = f"enc{l}{s}"
                tape[name + "_in"] = a
                a = r(np.maximum(conv3(a, Wr[name + ".w"], Wr[name + ".b"]), 0.0))
                tape[name + "_out"] = a
            if l < L:
                skips.append(a)
        for l in range(L - 1, 0, -1):
            name = f"up{l}t"
            tape[name + "_in"] = a
            up = r(tconv(a, Wr[name + ".w"], Wr[name + ".b"]))
            a = np.concatenate([up, skips[l - 1]], axis=1)
            for s in "ab":
                name = f"up{l}{s}"
                tape[name + "_in"] = a
                a = r(np.maximum(conv3(a, Wr[name + ".w"], Wr[name + ".b"]), 0.0))
                tape[name + "_out"] = a
        tape["head_in"] = a
        z = head(a, Wr["head.w"], Wr["head.b"])
        tape["head_z"] = z
        return np.maximum(z, 0.0), tape

    def loss_and_grads(self, params: dict, x, target):
        """Loss mean((z - target)^2) over all pixels, z the head output before its relu, and its
        gradient with respect to every parameter."""
        r, L = self._r, self.levels
        _, t = self.forward(params, x)
        W = t["W"]
        z = t["head_z"]
        cnt = z.size
        loss = float(np.mean((z - target) ** 2))
        grads = {}
        g = r(2.0 * (z - target) / cnt)
        ga, grads["head.w"], grads["head.b"] = head_grads(t["head_in"], W["head.w"], g)
        skip_g = {}
        for l in range(1, L):
            for s in "ba":
                name = f"up{l}{s}"
                gm = r(ga * (t[name + "_out"] > 0))
                ga, grads[name + ".w"], grads[name + ".b"] = conv3_grads(t[name + "_in"], W[name + ".w"], gm)
            c = self.base * 2 ** (l - 1)
            gup, skip_g[l] = ga[:, :c], ga[:, c:]
            name = f"up{l}t"
            ga, grads[name + ".w"], grads[name + ".b"] = tconv_grads(t[name + "_in"], W[name + ".w"], r(gup))
        # encoder, bottleneck first; ga now holds the gradient at the bottleneck output
        for l in range(L, 0, -1):
            if l < L:
                ga = ga + skip_g[l]
            for s in "ba":
                name = f"enc{l}{s}"
                gm = r(ga * (t[name + "_out"] > 0))
                ga, grads[name + ".w"], grads[name + ".b"] = conv3_grads(t[name + "_in"], W[name + ".w"], gm)
            if l > 1:
                ga = pool_grad(ga, t[f"pool{l}_idx"])
        return loss, grads


class Adam:
    """theta <- theta - lr m_hat / (sqrt(v_hat) + eps), with bias-corrected moments."""

    def __init__(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, beta1, beta2, eps
        self.t = 0
        self.m, self.v = {}, {}

    def step(self, params: dict, grads: dict) -> dict:
        self.t += 1
        out = {}
        for k, p in params.items():
            g = grads[k]
            m = self.b1 * self.m.get(k, 0.0) + (1 - self.b1) * g
            v = self.b2 * self.v.get(k, 0.0) + (1 - self.b2) * g * g
            self.m[k], self.v[k] = m, v
            mh = m / (1 - self.b1 ** self.t)
            vh = v / (1 - self.b2 ** self.t)
            out[k] = p - self.lr * mh / (np.sqrt(vh) + self.eps)
        return out
