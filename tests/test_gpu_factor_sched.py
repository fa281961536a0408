"""IC(0) schedules: the level-launch factor (the default) against the
sync-free factor (one launch per shift attempt) and the oracle."""

import time

import numpy as np
import pytest
import torch

import paper_2412_07127_amd as pkg
from gpu_common import named_matrix, oracle_factor, workload_problem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    torch.cuda.set_device(0)
    return pkg.Context()


@pytest.fixture(scope="module")
def ctx_sync():
    import os
    os.environ["ICPCG_IC0_SYNC_FREE"] = "1"
    try:
        c = pkg.Context()
    finally:
        del os.environ["ICPCG_IC0_SYNC_FREE"]
    yield c
    c.close()


def to_gpu(A):
    return pkg.CSR.from_numpy(*A, device="cuda")


# q1e5s2.0 needs one shifted restart and kershaw nine, so failed attempts
# (abandoned everywhere once a pivot fails) are exercised too.
@pytest.mark.parametrize("key", ["w:q1_8", "q1e5s2.0", "lap7", "tridiag", "kershaw", "w:q1_40"])
def test_sync_free_and_level_schedules_agree_bitwise(ctx, ctx_sync, key):
    A_h = named_matrix(key)
    A = to_gpu(A_h)
    Ls, info_s = ctx_sync.factor(A)
    Ll, info_l = ctx.factor(A)
    assert info_s["alpha"] == info_l["alpha"] and info_s["restarts"] == info_l["restarts"]
    assert info_s["min_pivot"] == info_l["min_pivot"]
    assert torch.equal(Ls.row_ptr, Ll.row_ptr) and torch.equal(Ls.col, Ll.col)
    assert torch.equal(Ls.val.view(torch.int64), Ll.val.view(torch.int64))
    _, L, _, alpha = oracle_factor(key)
    assert info_s["alpha"] == alpha
    g = Ls.val.cpu().numpy()
    assert np.abs(g - L[2]).max() / np.abs(L[2]).max() <= 1e-12


def test_repeated_sync_free_factors_identical(ctx_sync):
    """The pending pattern is restored before every attempt: a second factor
    into fresh buffers, and one after a shifted matrix, give the same bits."""
    A = to_gpu(named_matrix("w:q1_8"))
    L1, _ = ctx_sync.factor(A)
    ctx_sync.factor(to_gpu(named_matrix("q1e5s2.0")))
    L2, _ = ctx_sync.factor(A)
    assert torch.equal(L1.val.view(torch.int64), L2.val.view(torch.int64))


def test_factor_schedules_time(ctx, ctx_sync):
    """P-time of both schedules on the 40^3 workload, as measured."""
    prob, _ = workload_problem("q1_40")
    A = to_gpu((prob.row_ptr, prob.col, prob.val))
    out = {}
    for name, c in (("sync_free", ctx_sync), ("levels", ctx)):
        c.factor(A)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, info = c.factor(A)
        torch.cuda.synchronize()
        out[name] = dict(s=round(time.perf_counter() - t0, 4), alpha=info["alpha"], restarts=info["restarts"],
                         levels=info["nlevels"])
    print("IC(0) schedules at 40^3:", out)
    assert out["sync_free"]["alpha"] == out["levels"]["alpha"]


def test_factor_wait_limit_reports_device_error(ctx, ctx_sync, monkeypatch):
    """Forced from the host: a context whose dependency waits may not wait at
    all. A sync-free factor that meets a pending value then gives up, every
    wave exits, and the call reports ICPCG_E_DEVICE (or, if no wave ever had to
    wait, the factor is complete and correct). The normal context still
    factors afterwards."""
    prob, _ = workload_problem("q1_40")
    A = to_gpu((prob.row_ptr, prob.col, prob.val))
    monkeypatch.setenv("ICPCG_WAIT_LIMIT_US", "0")
    monkeypatch.setenv("ICPCG_IC0_SYNC_FREE", "1")
    ctx0 = pkg.Context()
    monkeypatch.delenv("ICPCG_WAIT_LIMIT_US")
    monkeypatch.delenv("ICPCG_IC0_SYNC_FREE")
    Lref, _ = ctx.factor(A)
    try:
        L0, _ = ctx0.factor(A)
        print("no wave had to wait")
        assert torch.equal(L0.val.view(torch.int64), Lref.val.view(torch.int64))
    except pkg.IcpcgError as e:
        # the level analysis before the factor waits the same way
        assert e.status == pkg._lib.E_DEVICE and "time" in str(e)
    L1, _ = ctx.factor(A)
    assert torch.equal(L1.val.view(torch.int64), Lref.val.view(torch.int64))
    ctx0.close()
