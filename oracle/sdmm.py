"""SDMM on problem (3) and the SARA reweighting loop (FP64, CPU).

Problem (3): minimise ||W Psi^dagger x||_1 over x in R_+^N subject to
||y_i - Phi_i x||_2 <= eps_i for every block i of the split (2).  The paper
solves it with SDMM (the PURIFY paragraph).  Written as a sum of functions of
linear maps,

    f_0(Psi^dagger x) + sum_i iota_{B_i}(Phi_i x) + iota_+(x),

SDMM keeps one primal/dual pair (y_j, z_j) per term and iterates
    x   = Q^{-1} sum_j L_j^T (y_j - z_j),     Q = sum_j L_j^T L_j,
    s_j = L_j x,
    y_j = prox_{gamma g_j}(s_j + z_j),
    z_j = z_j + s_j - y_j.
Here L = {Psi^dagger, Phi_1..Phi_R, I}; Psi Psi^dagger = I, so
Q = 2 I + Re(Phi^H Phi).  Everything runs on normalised splits: block b uses
Phi_hat_b = c_b Phi_b, data c_b y_b and bound c_b eps_b with c_b = a_b / nu, where
a_b are block weights (1, or measurement.block_density_weights) and nu is the
norm of the a-weighted operator.  Any c_b > 0 leaves the solution set of (3)
unchanged; this choice puts the spectrum of Q in [2, 3].

Readings where the paper is silent (each also listed in the design notes):
* Q^{-1} by conjugate gradients warm-started at the previous x, either to a
  relative residual of 1e-12 or for a fixed number of steps.
* gamma = 1e-4 ||Psi^dagger Phi_hat^dagger y_hat||_inf unless given.
* block weights a_b ~ 1 / ||Phi_b|| (density estimate), so that every block's
  constraint acts on x with a comparable force; a_b = 1 gives one
  normalisation for all blocks.
* stop when ||x_n - x_{n-1}|| / ||x_n|| <= tol_rel and every block satisfies
  ||y_i - Phi_i x_n|| <= eps_i (1 + eps_slack), or after max_iter iterations;
  tol_rel = 0 runs the fixed schedule.  Optionally (tol_dual > 0) the relative dual
  residual ||sum_j L_j^T z_j|| / max_j ||L_j^T z_j|| (the stationarity part of the KKT
  conditions, see kkt) must also be <= tol_dual.  The test is evaluated every
  check_every iterations of a pass.
* block-subset iterations (the SDMM paragraph's stochastic variant, a reading):
  in iteration k only the data blocks selected by block_selected update their
  split variables; the x-update uses every block's current (y_i, z_i).
* SARA reweighting (SARA paragraph: weights near the inverse of the previous
  solution's coefficients): w = delta / (delta + |Psi^dagger x|), delta_1 the
  population standard deviation of Psi^dagger x after pass 1 and
  delta_{t+1} = beta delta_t; each pass warm-starts the whole SDMM state.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import prox


@dataclass
class Params:
    gamma: float
    nu: float
    max_iter: int = 300
    tol_rel: float = 0.0
    eps_slack: float = 1e-4
    cg_iters: int | None = None   # None: CG to cg_tol
    cg_tol: float = 1e-12
    passes: int = 1
    rw_beta: float = 0.5
    block_weights: np.ndarray | None = None   # a_b per block; None: 1
    check_every: int = 1          # the stopping test is evaluated every check_every iterations of a pass
    tol_dual: float = 0.0         # > 0: the test also needs the relative dual residual <= tol_dual
    block_fraction: float = 1.0   # < 1: block-subset iterations (see block_selected)
    block_seed: int = 0


@dataclass
class State:
    x: np.ndarray
    y_psi: np.ndarray
    z_psi: np.ndarray
    y_phi: np.ndarray
    z_phi: np.ndarray
    y_pos: np.ndarray
    z_pos: np.ndarray
    k: int = 0                    # SDMM iterations run from this state's start (draws the block subsets)

    def copy(self) -> "State":
        return State(*(np.array(getattr(self, f), copy=True) for f in list(self.__dataclass_fields__)[:-1]), k=self.k)


@dataclass
class Info:
    iters: int = 0
    converged: bool = False
    rel_change: float = np.inf
    block_resid: np.ndarray = field(default_factory=lambda: np.zeros(0))  # ||y_i - Phi_i x||, user units
    objective: float = 0.0
    history: list = field(default_factory=list)


_MASK64 = (1 << 64) - 1


def splitmix64(seed: int, c: int) -> int:
    """The c-th output (counted from 0) of the SplitMix64 sequence seeded with `seed` (Steele, Lea &
    Flood 2014): state_c = seed + (c + 1) * 0x9E3779B97F4A7C15 mod 2^64, then two xor-shift-multiply
    rounds and a final xor-shift."""
    z = (seed + (c + 1) * 0x9E3779B97F4A7C15) & _MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK64
    return z ^ (z >> 31)


def block_selected(seed: int, k: int, R: int, fraction: float) -> np.ndarray:
    """Blocks of iteration k in block-subset SDMM (the SDMM paragraph: iterations that use only a subset of the
    data blocks y_i): block b takes part when u = (top 53 bits of splitmix64(seed, k R + b)) / 2^53 < fraction."""
    return np.array([(splitmix64(seed, k * R + b) >> 11) * 2.0 ** -53 < fraction for b in range(R)], dtype=bool)


def cg(Q, b, x0, iters=None, tol=1e-12, max_iter=500):
    """Conjugate gradients on the SPD map Q from x0: fixed `iters` steps, or to ||r|| <= tol ||b||."""
    x = np.array(x0, dtype=np.float64, copy=True)
    r = b - Q(x)
    p = r.copy()
    rs = float(np.vdot(r, r).real)
    bn = float(np.linalg.norm(b))
    k = 0
    while True:
        if iters is None:
            if np.sqrt(rs) <= tol * bn or k >= max_iter:
                break
        elif k >= iters:
            break
        if rs == 0.0:
            break
        Ap = Q(p)
        alpha = rs / float(np.vdot(p, Ap).real)
        x += alpha * p
        r -= alpha * Ap
        rs_new = float(np.vdot(r, r).real)
        p = r + (rs_new / rs) * p
        rs = rs_new
        k += 1
    return x


class Problem:
    """Normalised problem (3): block b uses c_b Phi_b, c_b y_b, c_b eps_b with c_b = a_b / nu."""

    def __init__(self, op, psi, y, offsets, eps, nu, block_weights=None):
        self.op, self.psi = op, psi
        self.nu = float(nu)
        self.offsets = np.asarray(offsets, dtype=np.int64)
        R = len(self.offsets) - 1
        a = np.ones(R) if block_weights is None else np.asarray(block_weights, dtype=np.float64)
        self.c = a / self.nu                                   # c_b per block
        self.cv = np.repeat(self.c, np.diff(self.offsets))     # c_b per visibility
        self.y_hat = self.cv * np.asarray(y, dtype=np.complex128)
        self.eps_hat = self.c * np.asarray(eps, dtype=np.float64)
        self.n = psi.n

    def fwd(self, x):
        return self.cv * self.op.fwd(x)

    def adj(self, v):
        return self.op.adj(self.cv * np.asarray(v, dtype=np.complex128))

    def Q(self, x):
        return 2.0 * x + self.adj(self.fwd(x))

    def blocks(self):
        o = self.offsets
        return [(int(o[i]), int(o[i + 1])) for i in range(len(o) - 1)]


def default_gamma(op, psi, y, nu, factor: float = 1e-4, offsets=None, block_weights=None) -> float:
    """gamma = factor max |Psi^dagger Phi_hat^dagger y_hat| = factor max |Psi^dagger Phi^dagger (c^2 y)|
    (c_b = a_b / nu; with a = 1: factor max |Psi^dagger Phi^dagger y| / nu^2).

    The minimiser does not depend on gamma, only the path to it does."""
    y = np.asarray(y, dtype=np.complex128)
    if block_weights is not None:
        y = y * np.repeat(np.asarray(block_weights, dtype=np.float64) ** 2, np.diff(np.asarray(offsets)))
    return factor * float(np.max(np.abs(psi.adj(op.adj(y))))) / nu ** 2


def init_state(pb: Problem, x0=None) -> State:
    """Zero start, or the warm start y_psi = Psi^dagger x0, y_i = Phi_hat_i x0, y_+ = x0, z = 0."""
    n, M = pb.n, len(pb.y_hat)
    D = pb.psi.adj(np.zeros((n, n))).shape
    if x0 is None:
        x = np.zeros((n, n))
        return State(x, np.zeros(D), np.zeros(D), np.zeros(M, complex), np.zeros(M, complex),
                     np.zeros((n, n)), np.zeros((n, n)))
    x = np.asarray(x0, dtype=np.float64).copy()
    return State(x, pb.psi.adj(x), np.zeros(D), pb.fwd(x), np.zeros(M, complex), x.copy(), np.zeros((n, n)))


def dual_warm_start(pb: Problem, st: State, W, gamma: float) -> State:
    """Duals for a warm start at x0 = st.x (whose splits hold y_j = L_j x0), from the optimality conditions
    of the weighted problem at x0 (a reading: the paper starts SDMM from zero):
    * l1 split: the soft threshold's own split of c = Psi^dagger x0, y_psi = soft(c, gamma W) and
      z_psi = c - y_psi (the subgradient gamma W sign(c) where |c| exceeds the threshold, c below it);
    * positivity: z_+ = 0 (x0 >= 0);
    * data blocks: y_i = the projection of Phi_hat_i x0 onto ball i and z_i = lambda (y_i - y_hat_i), a
      multiple of the ball's outward normal, with the single lambda >= 0 that minimises the stationarity
      residual ||Psi z_psi + sum_i Phi_hat_i^dagger z_i||, lambda = max(0, -<Psi z_psi, g> / <g, g>),
      g = sum_i Phi_hat_i^dagger (y_i - y_hat_i)."""
    st = st.copy()
    W = np.ones_like(st.y_psi) if W is None else np.asarray(W, dtype=np.float64)
    c = pb.psi.adj(st.x)
    st.y_psi = prox.soft(c, gamma * W)
    st.z_psi = c - st.y_psi
    s_phi = pb.fwd(st.x)
    d = np.empty_like(s_phi)
    for i, (lo, hi) in enumerate(pb.blocks()):
        d[lo:hi] = prox.ball(s_phi[lo:hi], pb.y_hat[lo:hi], pb.eps_hat[i]) - pb.y_hat[lo:hi]
    g = pb.adj(d)
    h = pb.psi.fwd(st.z_psi)
    gg = float(np.sum(g * g))
    lam = max(0.0, -float(np.sum(h * g)) / gg) if gg > 0 else 0.0
    st.y_phi = pb.y_hat + d
    st.z_phi = lam * d
    st.y_pos = np.array(st.x, copy=True)
    st.z_pos = np.zeros_like(st.x)
    return st


def sdmm_pass(pb: Problem, W, p: Params, st: State, record=False):
    """One weighted-l1 solve of (3) by SDMM, continuing from state `st` (modified copy returned)."""
    st = st.copy()
    W = np.ones_like(st.y_psi) if W is None else np.asarray(W, dtype=np.float64)
    info = Info()
    blocks = pb.blocks()
    for it in range(p.max_iter):
        if p.block_fraction < 1.0:
            sel = block_selected(p.block_seed, st.k, len(blocks), p.block_fraction)
        else:
            sel = np.ones(len(blocks), dtype=bool)
        st.k += 1
        b = pb.psi.fwd(st.y_psi - st.z_psi) + pb.adj(st.y_phi - st.z_phi) + (st.y_pos - st.z_pos)
        x_prev = st.x
        x = cg(pb.Q, b, x_prev, iters=p.cg_iters, tol=p.cg_tol)
        s_psi = pb.psi.adj(x)
        s_phi = pb.fwd(x)
        st.y_psi = prox.soft(s_psi + st.z_psi, p.gamma * W)
        st.z_psi = st.z_psi + s_psi - st.y_psi
        resid = np.empty(len(blocks))
        for i, (lo, hi) in enumerate(blocks):
            resid[i] = np.linalg.norm(s_phi[lo:hi] - pb.y_hat[lo:hi])
            if not sel[i]:          # a block left out of this iteration keeps its split variables
                continue
            t = s_phi[lo:hi] + st.z_phi[lo:hi]
            yi = prox.ball(t, pb.y_hat[lo:hi], pb.eps_hat[i])
            st.z_phi[lo:hi] = st.z_phi[lo:hi] + s_phi[lo:hi] - yi
            st.y_phi[lo:hi] = yi
        st.y_pos = prox.positive(x + st.z_pos)
        st.z_pos = st.z_pos + x - st.y_pos
        st.x = x
        dx = float(np.linalg.norm(x - x_prev))
        xn = float(np.linalg.norm(x))
        rel = dx / xn if xn > 0 else (0.0 if dx == 0 else np.inf)
        info.iters = it + 1
        info.rel_change = rel
        info.block_resid = resid / pb.c
        feasible = bool(np.all(resid <= pb.eps_hat * (1.0 + p.eps_slack)))
        if record:
            info.history.append((rel, resid.copy()))
        if p.tol_rel > 0 and (it + 1) % p.check_every == 0 and rel <= p.tol_rel and feasible:
            if p.tol_dual <= 0 or kkt(pb, st, W, p.gamma)[1] <= p.tol_dual:
                info.converged = True
                break
    info.objective = float(np.sum(np.abs(W * pb.psi.adj(st.x))))
    return st, info


def reweight(coeffs: np.ndarray, delta: float) -> np.ndarray:
    """SARA weights w = delta / (delta + |c|), in [0, 1].  Where delta + |c| = 0 (delta = 0 after a pass
    whose image has all analysis coefficients zero, at a zero coefficient) the weight is 1, the rule's
    value at c = 0 for every delta > 0."""
    c = np.abs(np.asarray(coeffs, dtype=np.float64))
    den = delta + c
    return np.where(den > 0, delta / np.where(den > 0, den, 1.0), 1.0)


def sara(op, psi, y, offsets, eps, p: Params, x0=None, W0=None, delta0=None, record=False, duals_from_x0=False):
    """SARA: p.passes weighted-l1 solves of (3), reweighting between passes.

    Returns (x, W_last, infos, state).  With x0 the SDMM state is warm-started
    from x0 (and with duals_from_x0 its duals from :func:`dual_warm_start`); with
    W0 the first pass uses W0 (delta0 its delta), else W = I.
    """
    pb = Problem(op, psi, y, offsets, eps, p.nu, p.block_weights)
    st = init_state(pb, x0)
    if duals_from_x0:
        st = dual_warm_start(pb, st, W0, p.gamma)
    W = W0
    delta = delta0
    infos = []
    for t in range(p.passes):
        st, info = sdmm_pass(pb, W, p, st, record=record)
        infos.append(info)
        if t < p.passes - 1:
            c = psi.adj(st.x)
            delta = float(np.std(c)) if delta is None else p.rw_beta * delta
            W = reweight(c, delta)
    return st.x, W, infos, st


def kkt(pb: Problem, st: State, W, gamma: float):
    """Relative KKT residuals of SDMM's state: primal ||s_j - y_j||, dual ||sum_j L_j^T z_j||."""
    s_psi = pb.psi.adj(st.x)
    s_phi = pb.fwd(st.x)
    prim = np.sqrt(np.sum((s_psi - st.y_psi) ** 2) + np.sum(np.abs(s_phi - st.y_phi) ** 2)
                   + np.sum((st.x - st.y_pos) ** 2))
    scale_p = np.sqrt(np.sum(s_psi ** 2) + np.sum(np.abs(s_phi) ** 2) + np.sum(st.x ** 2))
    parts = [pb.psi.fwd(st.z_psi), pb.adj(st.z_phi), st.z_pos]
    dual = np.linalg.norm(sum(parts))
    scale_d = max(np.linalg.norm(q) for q in parts)
    return prim / scale_p, dual / scale_d if scale_d > 0 else 0.0


# ---------------------------------------------------------------------------------------------------
# Synthesis prior (the SDMM paragraph: the same solver handles other sparsity priors)
# ---------------------------------------------------------------------------------------------------
#
# min ||W alpha||_1 over alpha in R^D subject to ||y_i - Phi_i Psi alpha||_2 <= eps_i for every block and
# Psi alpha >= 0: the image is synthesised from its coefficients, x = Psi alpha.  As a sum of functions of
# linear maps of alpha, f_0(alpha) + sum_i iota_{B_i}(Phi_hat_i Psi alpha) + iota_+(Psi alpha), with
# L = {I, Phi_hat_1 Psi .. Phi_hat_R Psi, Psi} and Q = I + Psi^dagger (I + Re(Phi_hat^H Phi_hat)) Psi (spectrum
# in [1, 3]: Psi Psi^dagger = I, so Psi^dagger A Psi has the eigenvalues of A restricted to range(Psi^dagger)
# and 0).  The splits, proximal maps and dual updates are those of the analysis form.


@dataclass
class SynthState:
    alpha: np.ndarray
    y_l1: np.ndarray
    z_l1: np.ndarray
    y_phi: np.ndarray
    z_phi: np.ndarray
    y_pos: np.ndarray
    z_pos: np.ndarray

    def copy(self) -> "SynthState":
        return SynthState(*(np.array(getattr(self, f), copy=True) for f in self.__dataclass_fields__))


def synth_init_state(pb: Problem, x0=None) -> SynthState:
    """Zero start, or from an image x0: alpha = Psi^dagger x0 (so Psi alpha = x0), y_j = L_j alpha, z = 0."""
    D = pb.psi.adj(np.zeros((pb.n, pb.n))).shape
    M = len(pb.y_hat)
    if x0 is None:
        z = np.zeros(D)
        return SynthState(z, z.copy(), z.copy(), np.zeros(M, complex), np.zeros(M, complex),
                          np.zeros((pb.n, pb.n)), np.zeros((pb.n, pb.n)))
    a = pb.psi.adj(np.asarray(x0, dtype=np.float64))
    x = pb.psi.fwd(a)
    return SynthState(a, a.copy(), np.zeros(D), pb.fwd(x), np.zeros(M, complex), x, np.zeros((pb.n, pb.n)))


def synth_pass(pb: Problem, W, p: Params, st: SynthState, record=False):
    """One weighted-l1 solve of the synthesis problem by SDMM, continuing from `st`."""
    st = st.copy()
    psi = pb.psi
    W = np.ones_like(st.alpha) if W is None else np.asarray(W, dtype=np.float64)
    info = Info()
    blocks = pb.blocks()

    def Q(a):
        xa = psi.fwd(a)
        return a + psi.adj(xa + pb.adj(pb.fwd(xa)))

    x_prev = psi.fwd(st.alpha)
    for it in range(p.max_iter):
        b = (st.y_l1 - st.z_l1) + psi.adj(pb.adj(st.y_phi - st.z_phi) + (st.y_pos - st.z_pos))
        alpha = cg(Q, b, st.alpha, iters=p.cg_iters, tol=p.cg_tol)
        x = psi.fwd(alpha)
        s_phi = pb.fwd(x)
        st.y_l1 = prox.soft(alpha + st.z_l1, p.gamma * W)
        st.z_l1 = st.z_l1 + alpha - st.y_l1
        resid = np.empty(len(blocks))
        for i, (lo, hi) in enumerate(blocks):
            resid[i] = np.linalg.norm(s_phi[lo:hi] - pb.y_hat[lo:hi])
            t = s_phi[lo:hi] + st.z_phi[lo:hi]
            yi = prox.ball(t, pb.y_hat[lo:hi], pb.eps_hat[i])
            st.z_phi[lo:hi] = st.z_phi[lo:hi] + s_phi[lo:hi] - yi
            st.y_phi[lo:hi] = yi
        st.y_pos = prox.positive(x + st.z_pos)
        st.z_pos = st.z_pos + x - st.y_pos
        st.alpha = alpha
        dx = float(np.linalg.norm(x - x_prev))
        xn = float(np.linalg.norm(x))
        rel = dx / xn if xn > 0 else (0.0 if dx == 0 else np.inf)
        x_prev = x
        info.iters = it + 1
        info.rel_change = rel
        info.block_resid = resid / pb.c
        feasible = bool(np.all(resid <= pb.eps_hat * (1.0 + p.eps_slack)))
        if p.tol_rel > 0 and (it + 1) % p.check_every == 0 and rel <= p.tol_rel and feasible:
            if p.tol_dual <= 0 or synth_kkt(pb, st, W, p.gamma)[1] <= p.tol_dual:
                info.converged = True
                break
    info.objective = float(np.sum(np.abs(W * st.alpha)))
    return st, info


def sara_synthesis(op, psi, y, offsets, eps, p: Params, x0=None, W0=None, delta0=None):
    """The SARA loop on the synthesis prior: passes of synth_pass, reweighting w = delta / (delta + |alpha|)
    between them (delta_1 = std(alpha) after pass 1, delta_{t+1} = beta delta_t).  Returns (x = Psi alpha,
    W_last, infos, state)."""
    pb = Problem(op, psi, y, offsets, eps, p.nu, p.block_weights)
    st = synth_init_state(pb, x0)
    W, delta, infos = W0, delta0, []
    for t in range(p.passes):
        st, info = synth_pass(pb, W, p, st)
        infos.append(info)
        if t < p.passes - 1:
            delta = float(np.std(st.alpha)) if delta is None else p.rw_beta * delta
            W = reweight(st.alpha, delta)
    return psi.fwd(st.alpha), W, infos, st


def synth_kkt(pb: Problem, st: SynthState, W, gamma: float):
    """Relative KKT residuals of the synthesis state: primal ||s_j - y_j|| over the splits, dual
    ||z_l1 + Psi^dagger (Phi_hat^dagger z_phi + z_+)|| against the largest of its terms."""
    psi = pb.psi
    x = psi.fwd(st.alpha)
    s_phi = pb.fwd(x)
    prim = np.sqrt(np.sum((st.alpha - st.y_l1) ** 2) + np.sum(np.abs(s_phi - st.y_phi) ** 2)
                   + np.sum((x - st.y_pos) ** 2))
    scale_p = np.sqrt(np.sum(st.alpha ** 2) + np.sum(np.abs(s_phi) ** 2) + np.sum(x ** 2))
    parts = [st.z_l1, psi.adj(pb.adj(st.z_phi)), psi.adj(st.z_pos)]
    dual = np.linalg.norm(sum(parts))
    scale_d = max(np.linalg.norm(q) for q in parts)
    return prim / scale_p, dual / scale_d if scale_d > 0 else 0.0
