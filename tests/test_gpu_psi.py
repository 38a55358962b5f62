"""GPU parity of the SARA dictionary Psi (synthesis) and Psi^dagger (analysis) against the FP64 oracle.

Bar: norm-wise relative error <= 1e-5 per coefficient plane and for the image; Psi Psi^dagger = I.
"""
import numpy as np
import pytest

from oracle import wavelets
from paper_1502_05037_amd import synth
from tests import helpers

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sh():
    from paper_1502_05037_amd import sarahip
    return sarahip


@pytest.mark.parametrize("n,levels,mask", [(64, 4, 0x1FF), (256, 4, 0x1FF), (16, 4, 0x1FF), (32, 3, 0b101010101),
                                           (64, 4, 0x1), (128, 2, 0x1FE), (1024, 4, 0x1FF), (48, 4, 0x1FF)])
def test_psi_parity(sh, n, levels, mask):
    print(f"psi parity n={n} levels={levels} mask={mask:#x}", flush=True)
    ref = wavelets.SARA(n, levels, mask)
    x = synth.rng(21, n, 0).normal(size=(n, n)).astype(np.float32).astype(np.float64)
    c = synth.rng(21, n, 1).normal(size=(ref.q, n, n)).astype(np.float32).astype(np.float64)
    psi = sh.psi_create(n, levels, mask)
    try:
        assert sh.psi_planes(psi) == ref.q
        cd = torch.empty((ref.q, n, n), dtype=torch.float32, device="cuda")
        sh.psi_adj(psi, torch.tensor(x, dtype=torch.float32, device="cuda"), cd)
        xd = torch.empty((n, n), dtype=torch.float32, device="cuda")
        sh.psi_fwd(psi, torch.tensor(c, dtype=torch.float32, device="cuda"), xd)
        back = torch.empty_like(xd)
        sh.psi_fwd(psi, cd, back)
        torch.cuda.synchronize()
    finally:
        sh.psi_destroy(psi)
    ca = ref.adj(x)
    got = cd.cpu().numpy().astype(np.float64)
    for i in range(ref.q):
        assert helpers.rel(got[i], ca[i]) <= 1e-5, f"plane {i}"
    assert helpers.rel(xd.cpu().numpy(), ref.fwd(c)) <= 1e-5
    assert helpers.rel(back.cpu().numpy(), x) <= 1e-5
