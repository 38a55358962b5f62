"""GPU block weights (density estimate of 1 / ||Phi_b||) against the oracle: the counts are integers
taken on the same float64 cells, so the weights agree exactly."""
import numpy as np
import pytest

from oracle import measurement
from paper_1502_05037_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sh():
    from paper_1502_05037_amd import sarahip
    return sarahip


def _coverage(n, m, R, cov, seed):
    g = synth.rng(17, seed, synth.UV)
    uv = synth.sort_by_radius(synth.uv_gaussian(m, g) if cov == "gaussian" else synth.uv_radial(m, g))
    sizes = synth.block_sizes(m, R, synth.rng(17, seed, synth.BLOCKS)) if R > 1 else np.array([m])
    return uv, synth.offsets(sizes)


@pytest.mark.parametrize("n,m,R,J,alpha,cov", [
    (64, 2048, 1, 6, 2, "gaussian"),
    (64, 20000, 16, 6, 2, "radial"),      # blocks of very different density
    (32, 3001, 5, 8, 4, "gaussian"),      # 4 x 4 windows
    (256, 200000, 40, 8, 2, "radial"),    # many blocks, several passes of the counters
])
def test_block_weights_match_oracle(sh, n, m, R, J, alpha, cov):
    print(f"block weights n={n} m={m} R={R} alpha={alpha} {cov}", flush=True)
    uv, off = _coverage(n, m, R, cov, n + R)
    op = sh.op_create(uv, n, alpha, J, off)
    try:
        b = sh.block_weights(op)
    finally:
        sh.op_destroy(op)
    np.testing.assert_array_equal(b, measurement.block_density_weights(uv, n, alpha, off))


def test_block_weights_of_a_batched_plan(sh):
    n, J = 64, 6
    covs = [_coverage(n, m, R, c, 50 + k) for k, (m, R, c) in enumerate([(3000, 3, "radial"), (1500, 1, "gaussian"),
                                                                          (5000, 6, "radial")])]
    uv = np.concatenate([c[0] for c in covs])
    offs, base = [0], 0
    for c in covs:
        offs.extend((base + c[1][1:]).tolist())
        base += int(c[1][-1])
    op = sh.op_create_batched(uv, [int(c[1][-1]) for c in covs], n, 2, J, np.array(offs), [len(c[1]) - 1 for c in covs])
    try:
        b = sh.block_weights(op)
    finally:
        sh.op_destroy(op)
    ref = np.concatenate([measurement.block_density_weights(c[0], n, 2, c[1]) for c in covs])
    np.testing.assert_array_equal(b, ref)
