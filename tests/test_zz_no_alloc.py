"""The entry point that allocates nothing (icpcg_apply_rz_noalloc) against
icpcg_apply_rz, through the C ABI: same kernels and launch shapes, so Y, Z
and r^T z must be bit-identical. Two calls in a row share the static partials
array, the second on a smaller input (fewer rows and fewer columns), so a
stale partial left by the first would show up in the second's r^T z."""

import ctypes

import numpy as np
import pytest
import torch

import paper_2412_07127_amd as pkg
from gpu_common import oracle_factor

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    torch.cuda.set_device(0)
    return pkg.Context()


def _call(ctx, P, Rh):
    Rt = torch.from_numpy(Rh).cuda()
    Y, Z, rz = P.apply_rz(Rt)
    Y2, Z2, rz2 = torch.full_like(Y, 7.0), torch.full_like(Z, 7.0), torch.full_like(rz, 7.0)
    P.apply_rz_noalloc(Rt, Y2, Z2, rz2)
    torch.cuda.synchronize()
    return (Y, Z, rz), (Y2, Z2, rz2)


@pytest.mark.parametrize("dt", ["f64", "f32", "bf16"])
def test_noalloc_matches_apply_rz_two_calls(ctx, dt):
    # first call: 40^3 workload (201,720 rows) at 16 columns; second: 8^3 (1,944 rows) at 4 columns
    for key, R, seed in (("w:q1_40", 16, 11), ("w:q1_8", 4, 12), ("w:q1_8", 1, 13)):
        _, L, _, _ = oracle_factor(key)
        n = L[0].shape[0] - 1
        P = ctx.prec(pkg.CSR.from_numpy(*L, device="cuda"), dt)
        Rh = np.random.default_rng(seed).standard_normal((n, R)) if R > 1 else \
            np.random.default_rng(seed).standard_normal(n)
        ref, got = _call(ctx, P, Rh)
        for a, b in zip(ref, got):
            assert torch.equal(a, b), (key, R, dt)
        assert bool(torch.isfinite(got[2]).all()) and bool((got[2] > 0).all())


def test_noalloc_rejects_bad_width(ctx):
    _, L, _, _ = oracle_factor("w:q1_8")
    n = L[0].shape[0] - 1
    P = ctx.prec(pkg.CSR.from_numpy(*L, device="cuda"), "f32")
    lib = ctx.lib
    R = torch.zeros(n * 3, dtype=torch.float64, device="cuda")
    Y = torch.zeros(n * 3, dtype=torch.float32, device="cuda")
    Z = torch.zeros_like(Y)
    rz = torch.zeros(3, dtype=torch.float64, device="cuda")
    st = lib.icpcg_apply_rz_noalloc(ctx.h, P.h, ctypes.c_void_p(R.data_ptr()), ctypes.c_void_p(Y.data_ptr()),
                                    ctypes.c_void_p(Z.data_ptr()), ctypes.c_void_p(rz.data_ptr()), 3)
    assert st == pkg._lib.E_INVALID
