"""Autotuner: the kernel-width accuracy estimate (CPU), the tuned plan and its cache file (GPU).

The estimate is pinned to the oracle: the FP64 oracle NUFFT of a white image, compared with the
exact sum of the measurement equation (the direct DFT), has the relative error the estimate
predicts, for every width from 2 to 8.
"""
import numpy as np
import pytest

from oracle import measurement
from tests import helpers


@pytest.fixture(scope="module")
def sh():
    from paper_1502_05037_amd import sarahip
    return sarahip


@pytest.mark.parametrize("J", [2, 4, 6, 8])
def test_alias_estimate_predicts_oracle_nufft_error(sh, J):
    g = np.random.default_rng(11)
    n, M = 32, 3000
    uv = g.uniform(-np.pi, np.pi, (M, 2))
    x = g.standard_normal((n, n))
    exact = measurement.DFT(uv, n).fwd(x)
    err = helpers.rel(measurement.NUFFT(uv, n, J).fwd(x), exact)
    est = sh.kb_alias_error(J, 2)
    assert 0.8 <= err / est <= 1.25, (J, err, est)


def test_alias_estimate_decreases_and_rejects_bad_width(sh):
    e = [sh.kb_alias_error(J, 2) for J in range(2, 17, 2)]
    assert all(b < a / 10 for a, b in zip(e, e[1:]))
    assert sh.kb_alias_error(6, 4) < sh.kb_alias_error(6, 2)
    for J in (3, 18):
        with pytest.raises(sh.SarahipError):
            sh.kb_alias_error(J, 2)


def test_autotune_rejects_invalid_targets(sh):
    uv = np.zeros((4, 2))
    for acc in (0.0, 1.5, float("nan"), 1e-20):
        with pytest.raises(sh.SarahipError) as e:
            sh.op_autotune(uv, [4], 16, 2, acc, [0, 4], [1], stream=0)
        assert e.value.status == -1


@pytest.mark.gpu
def test_autotuned_plan_meets_target_and_is_cached(sh):
    import torch
    pbs = [helpers.build(50, 64, m, R, 6, coverage="radial", prob=k) for k, (m, R) in enumerate([(3000, 3), (1200, 2)])]
    uv = np.concatenate([pb.uv for pb in pbs])
    M_p, R_p = [len(pb.uv) for pb in pbs], [len(pb.offsets) - 1 for pb in pbs]
    offs = np.concatenate([[0], pbs[0].offsets[1:], len(pbs[0].uv) + pbs[1].offsets[1:]])
    op, res = sh.op_autotune(uv, M_p, 64, 2, 1e-5, offs, R_p, reps=2)
    try:
        assert res["J"] == 6 and res["alias_error"] <= 1e-5 and res["cached"] == 0
        assert res["candidates"] >= 3 and res["tile"] in (8, 16, 32) and res["ms_pair"] > 0
        q = sh.op_query(op)
        assert q["J"] == 6 and q["tile"] == res["tile"] and q["P"] == 2
        # accuracy against the exact sum of the measurement equation
        g = np.random.default_rng(5)
        xs = g.standard_normal((2, 64, 64)).astype(np.float32)
        v = torch.empty(sum(M_p), dtype=torch.complex64, device="cuda")
        sh.phi_fwd(op, torch.tensor(xs, device="cuda"), v)
        v = v.cpu().numpy()
        base = 0
        for p, pb in enumerate(pbs):
            exact = measurement.DFT(pb.uv, 64).fwd(xs[p].astype(np.float64))
            assert helpers.rel(v[base:base + M_p[p]], exact) <= 2e-5
            base += M_p[p]
    finally:
        sh.op_destroy(op)
    op2, res2 = sh.op_autotune(uv, M_p, 64, 2, 1e-5, offs, R_p, reps=2)
    sh.op_destroy(op2)
    assert res2["cached"] == 1 and res2["candidates"] == 0
    assert (res2["tile"], res2["chunk"], res2["J"]) == (res["tile"], res["chunk"], res["J"])
    op3, res3 = sh.op_autotune(uv, M_p, 64, 2, 1e-7, offs, R_p, reps=1)
    sh.op_destroy(op3)
    assert res3["J"] == 8


@pytest.mark.gpu
def test_tuning_persists_in_the_cache_file(sh, tmp_path, monkeypatch):
    """SH_TUNE_CACHE: the first tuning appends its choice, a process that has not tuned these inputs (here: the
    process cache forgotten) takes it from the file without timing, a later invalid line of the same key is
    skipped, and without the variable nothing is written."""
    pb = helpers.build(52, 64, 2000, 2, 6, coverage="radial")
    M_p, R_p = [len(pb.uv)], [len(pb.offsets) - 1]
    path = tmp_path / "tune.txt"
    monkeypatch.setenv("SH_TUNE_CACHE", str(path))
    sh.tune_cache_clear()
    op, res = sh.op_autotune(pb.uv, M_p, 64, 2, 1e-5, pb.offsets, R_p, reps=1)
    sh.op_destroy(op)
    assert res["cached"] == 0 and res["candidates"] >= 3
    lines = path.read_text().splitlines()
    assert len(lines) == 1
    tag, key, J, tile, chunk, ms = lines[0].split()
    assert tag == "sarahip-tune-1" and key.startswith("sarahip-")
    assert (int(J), int(tile), int(chunk)) == (res["J"], res["tile"], res["chunk"])
    with open(path, "a") as f:   # a later line of the same key with a tiling no plan has: skipped
        f.write(f"{tag} {key} {J} 7 {chunk} {ms}\nnot a cache line\n")
    sh.tune_cache_clear()
    op, res2 = sh.op_autotune(pb.uv, M_p, 64, 2, 1e-5, pb.offsets, R_p, reps=1)
    q = sh.op_query(op)
    sh.op_destroy(op)
    assert res2["cached"] == 2 and res2["candidates"] == 0
    assert (res2["J"], res2["tile"], res2["chunk"]) == (res["J"], res["tile"], res["chunk"])
    assert q["tile"] == res["tile"]
    op, res3 = sh.op_autotune(pb.uv, M_p, 64, 2, 1e-5, pb.offsets, R_p, reps=1)   # now in the process cache
    sh.op_destroy(op)
    assert res3["cached"] == 1
    monkeypatch.delenv("SH_TUNE_CACHE")
    sh.tune_cache_clear()
    before = path.read_text()
    op, res4 = sh.op_autotune(pb.uv, M_p, 64, 2, 1e-5, pb.offsets, R_p, reps=1)
    sh.op_destroy(op)
    assert res4["cached"] == 0 and path.read_text() == before
