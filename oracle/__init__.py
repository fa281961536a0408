"""ctypes shim over the plain-C FP64 oracle (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg import
this package. It shares no code with the GPU library and never calls it.
Arrays are numpy: CSR row pointers int64, column indices int32, values float64.
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

OK, INVALID, PIVOT, BREAKDOWN, MAXITER, NONFINITE, TRUE_RESIDUAL = 0, 1, 2, 3, 4, 5, 8

_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_build.LIB) or os.path.getmtime(_build.LIB) < os.path.getmtime(_build.SRC):
        _build.build()
    lib = C.CDLL(_build.LIB)
    P = C.c_void_p
    i64 = C.c_int64
    lib.orc_spmv.argtypes = [i64, P, P, P, P, P]
    lib.orc_dot.argtypes = [i64, P, P]
    lib.orc_dot.restype = C.c_double
    lib.orc_check_csr.argtypes = [i64, P, P]
    lib.orc_tril_nnz.argtypes = [i64, P, P]
    lib.orc_tril_nnz.restype = i64
    lib.orc_tril.argtypes = [i64, P, P, P, P, P, P]
    lib.orc_transpose.argtypes = [i64, P, P, P, P, P, P]
    lib.orc_ic0.argtypes = [i64, P, P, P, C.c_double, P, P]
    lib.orc_ic0_shifted.argtypes = [i64, P, P, P, P, P, P, C.c_int, P, P, P]
    lib.orc_levels_lower.argtypes = [i64, P, P, P]
    lib.orc_levels_lower.restype = i64
    lib.orc_levels_upper.argtypes = [i64, P, P, P]
    lib.orc_levels_upper.restype = i64
    lib.orc_level_sort.argtypes = [i64, P, i64, P, P]
    lib.orc_trsv_lower.argtypes = [i64, P, P, P, P, P]
    lib.orc_trsv_upper.argtypes = [i64, P, P, P, P, P]
    lib.orc_round_bf16.argtypes = [C.c_float]
    lib.orc_round_bf16.restype = C.c_float
    lib.orc_cast_values.argtypes = [i64, P, C.c_int, P]
    lib.orc_apply_f32.argtypes = [i64, P, P, P, P, P, P, P, P, P, P]
    lib.orc_pcg_simple.argtypes = [i64, P, P, P, C.c_int, P, P, C.c_double, i64, C.c_int, P, P, P, P, P]
    lib.orc_pcg.argtypes = [i64, P, P, P, P, P, P, P, P, P, P, P, C.c_double, i64, C.c_int,
                            C.c_int, P, P, P, P, P, i64, i64, i64, P, P]
    lib.orc_apply.argtypes = [i64, P, P, P, P, P, P, P, P, P]
    lib.orc_apply_adjoint.argtypes = [i64, P, P, P, P, P, P, i64, P, P, P, P, P, P, P]
    lib.orc_set_threads.argtypes = [C.c_int]
    lib.orc_max_threads.restype = C.c_int
    _lib = lib
    return lib


def set_threads(t: int) -> int:
    """Threads of the row-parallel loops (SpMV rows, vector updates); returns
    the count now in effect. Results do not depend on it."""
    lib = _load()
    lib.orc_set_threads(int(t))
    return lib.orc_max_threads()


def _p(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _csr(rp, ci, v=None):
    rp = np.ascontiguousarray(rp, dtype=np.int64)
    ci = np.ascontiguousarray(ci, dtype=np.int32)
    v = None if v is None else np.ascontiguousarray(v, dtype=np.float64)
    return rp, ci, v


def spmv(rp, ci, v, x):
    rp, ci, v = _csr(rp, ci, v)
    x = np.ascontiguousarray(x, dtype=np.float64)
    w = np.empty(rp.shape[0] - 1)
    _load().orc_spmv(w.shape[0], _p(rp), _p(ci), _p(v), _p(x), _p(w))
    return w


def dot(a, b):
    a = np.ascontiguousarray(a, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    return _load().orc_dot(a.shape[0], _p(a), _p(b))


def check_csr(rp, ci):
    rp, ci, _ = _csr(rp, ci)
    return _load().orc_check_csr(rp.shape[0] - 1, _p(rp), _p(ci))


def tril(rp, ci, v):
    rp, ci, v = _csr(rp, ci, v)
    n = rp.shape[0] - 1
    lib = _load()
    m = lib.orc_tril_nnz(n, _p(rp), _p(ci))
    lrp = np.empty(n + 1, np.int64)
    lci = np.empty(m, np.int32)
    lv = np.empty(m)
    lib.orc_tril(n, _p(rp), _p(ci), _p(v), _p(lrp), _p(lci), _p(lv))
    return lrp, lci, lv


def transpose(lrp, lci, lv):
    lrp, lci, lv = _csr(lrp, lci, lv)
    n = lrp.shape[0] - 1
    urp = np.empty(n + 1, np.int64)
    uci = np.empty(lci.shape[0], np.int32)
    uv = np.empty(lci.shape[0])
    _load().orc_transpose(n, _p(lrp), _p(lci), _p(lv), _p(urp), _p(uci), _p(uv))
    return urp, uci, uv


def ic0(lrp, lci, lv_tril, alpha=0.0):
    """IC(0) on the given lower pattern with fixed shift alpha.
    Returns (status, L values, failing row, min squared pivot)."""
    lrp, lci, lv = _csr(lrp, lci, lv_tril)
    lv = lv.copy()
    fr = C.c_int64(-1)
    mp = C.c_double(0)
    st = _load().orc_ic0(lrp.shape[0] - 1, _p(lrp), _p(lci), _p(lv), alpha, C.byref(fr), C.byref(mp))
    return st, lv, fr.value, mp.value


def ic0_shifted(rp, ci, v, max_restarts=30):
    """IC(0) of tril(A) with the global shift rule. Returns
    (status, (lrp, lci, lv), alpha, restarts, min squared pivot)."""
    rp, ci, v = _csr(rp, ci, v)
    n = rp.shape[0] - 1
    lib = _load()
    m = lib.orc_tril_nnz(n, _p(rp), _p(ci))
    lrp = np.empty(n + 1, np.int64)
    lci = np.empty(m, np.int32)
    lv = np.empty(m)
    a = C.c_double(0)
    r = C.c_int(0)
    mp = C.c_double(0)
    st = lib.orc_ic0_shifted(n, _p(rp), _p(ci), _p(v), _p(lrp), _p(lci), _p(lv), max_restarts,
                             C.byref(a), C.byref(r), C.byref(mp))
    return st, (lrp, lci, lv), a.value, r.value, mp.value


def levels_lower(lrp, lci):
    lrp, lci, _ = _csr(lrp, lci)
    n = lrp.shape[0] - 1
    lev = np.empty(n, np.int32)
    nl = _load().orc_levels_lower(n, _p(lrp), _p(lci), _p(lev))
    return lev, nl


def levels_upper(lrp, lci):
    lrp, lci, _ = _csr(lrp, lci)
    n = lrp.shape[0] - 1
    lev = np.empty(n, np.int32)
    nl = _load().orc_levels_upper(n, _p(lrp), _p(lci), _p(lev))
    return lev, nl


def level_sort(level, nlev):
    level = np.ascontiguousarray(level, dtype=np.int32)
    perm = np.empty(level.shape[0], np.int32)
    lp = np.empty(nlev + 1, np.int32)
    _load().orc_level_sort(level.shape[0], _p(level), nlev, _p(perm), _p(lp))
    return perm, lp


def trsv_lower(lrp, lci, lv, r):
    lrp, lci, lv = _csr(lrp, lci, lv)
    r = np.ascontiguousarray(r, dtype=np.float64)
    y = np.empty_like(r)
    _load().orc_trsv_lower(r.shape[0], _p(lrp), _p(lci), _p(lv), _p(r), _p(y))
    return y


def trsv_upper(urp, uci, uv, y):
    urp, uci, uv = _csr(urp, uci, uv)
    y = np.ascontiguousarray(y, dtype=np.float64)
    z = np.empty_like(y)
    _load().orc_trsv_upper(y.shape[0], _p(urp), _p(uci), _p(uv), _p(y), _p(z))
    return z


def round_bf16(x: float) -> float:
    return _load().orc_round_bf16(x)


def cast_values(v, prec):
    v = np.ascontiguousarray(v, dtype=np.float64)
    out = np.empty(v.shape[0], np.float32)
    _load().orc_cast_values(v.shape[0], _p(v), prec, _p(out))
    return out


def apply(L, U, r):
    (lrp, lci, lv), (urp, uci, uv) = _csr(*L), _csr(*U)
    r = np.ascontiguousarray(r, dtype=np.float64)
    y = np.empty_like(r)
    z = np.empty_like(r)
    _load().orc_apply(r.shape[0], _p(lrp), _p(lci), _p(lv), _p(urp), _p(uci), _p(uv),
                      _p(r), _p(y), _p(z))
    return y, z


def apply_f32(L, U, r, prec=1):
    """Preconditioner solve with the factor rounded to float (prec 1) or
    bfloat16 (prec 2) and float arithmetic; returns z as float64."""
    (lrp, lci, lv), (urp, uci, uv) = _csr(*L), _csr(*U)
    l32 = cast_values(lv, prec)
    u32 = cast_values(uv, prec)
    r = np.ascontiguousarray(r, dtype=np.float64)
    n = r.shape[0]
    z = np.empty(n)
    y32 = np.empty(n, np.float32)
    z32 = np.empty(n, np.float32)
    _load().orc_apply_f32(n, _p(lrp), _p(lci), _p(l32), _p(urp), _p(uci), _p(u32), _p(r), _p(z),
                          _p(y32), _p(z32))
    return z


def pcg(A, L, U, b, x0=None, rtol=1e-8, max_iter=None, max_replace=3, prec=0, history=False, snap=None):
    """PCG of supplementary Algorithm 1 (readings in icpcg_oracle.c). Returns a
    dict: x, status, iters, replacements, relres, true_relres (and hist).
    snap = (idx, k_from, k_to): also x[idx] after every step k_from..k_to
    (inclusive) as "x_snap", a (k_to - k_from + 1, len(idx)) array (rows of
    steps not reached stay NaN)."""
    rp, ci, v = _csr(*A)
    (lrp, lci, lv), (urp, uci, uv) = _csr(*L), _csr(*U)
    b = np.ascontiguousarray(b, dtype=np.float64)
    n = b.shape[0]
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    if max_iter is None:
        max_iter = default_max_iter(n)
    it = C.c_int64(0)
    rep = C.c_int(0)
    rr = C.c_double(0)
    tr = C.c_double(0)
    hist = np.zeros(max_iter + 1) if history else None
    sidx, sfrom, scount, sout = None, 0, 0, None
    if snap is not None:
        sidx = np.ascontiguousarray(snap[0], dtype=np.int64)
        sfrom, scount = int(snap[1]), int(snap[2]) - int(snap[1]) + 1
        sout = np.full((scount, sidx.shape[0]), np.nan)
    st = _load().orc_pcg(n, _p(rp), _p(ci), _p(v), _p(lrp), _p(lci), _p(lv), _p(urp), _p(uci),
                         _p(uv), _p(b), _p(x), rtol, max_iter, max_replace, prec, C.byref(it),
                         C.byref(rep), C.byref(rr), C.byref(tr), _p(hist), sfrom, scount,
                         0 if sidx is None else sidx.shape[0], _p(sidx), _p(sout))
    out = dict(x=x, status=st, iters=it.value, replacements=rep.value, relres=rr.value,
               true_relres=tr.value)
    if history:
        out["hist"] = hist[:it.value + 1]
    if snap is not None:
        out["x_snap"] = sout
    return out


def pcg_simple(A, b, kind, x0=None, rtol=1e-8, max_iter=None, max_replace=3, history=False):
    """The PCG of `pcg` with Table 1's baselines: kind "jacobi" (z_i = r_i / a_ii)
    or "none" (plain CG). Same result dict."""
    k = {"jacobi": 1, "none": 2}[kind]
    rp, ci, v = _csr(*A)
    b = np.ascontiguousarray(b, dtype=np.float64)
    n = b.shape[0]
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    if max_iter is None:
        max_iter = default_max_iter(n)
    it = C.c_int64(0)
    rep = C.c_int(0)
    rr = C.c_double(0)
    tr = C.c_double(0)
    hist = np.zeros(max_iter + 1) if history else None
    st = _load().orc_pcg_simple(n, _p(rp), _p(ci), _p(v), k, _p(b), _p(x), rtol, max_iter, max_replace,
                                C.byref(it), C.byref(rep), C.byref(rr), C.byref(tr), _p(hist))
    out = dict(x=x, status=st, iters=it.value, replacements=rep.value, relres=rr.value,
               true_relres=tr.value)
    if history:
        out["hist"] = hist[:it.value + 1]
    return out


def default_max_iter(n: int) -> int:
    """10 sqrt(n), at least 10, at most n (stated reading; the paper sets no cap)."""
    import math
    return int(min(max(n, 1), max(10, int(10 * math.sqrt(n)))))


def apply_adjoint(L, U, R, G):
    """Reference gradient of Z = L^-T L^-1 R. R, G: (n, m) arrays. Returns
    dict Y, Z, Ybar, Rbar, dL (dL on L's stored entries)."""
    (lrp, lci, lv), (urp, uci, uv) = _csr(*L), _csr(*U)
    R = np.ascontiguousarray(R, dtype=np.float64)
    G = np.ascontiguousarray(G, dtype=np.float64)
    if R.ndim == 1:
        R = R[:, None]
        G = G[:, None]
    n, m = R.shape
    Y = np.empty_like(R); Z = np.empty_like(R); Yb = np.empty_like(R); Rb = np.empty_like(R)
    dL = np.empty(lci.shape[0])
    _load().orc_apply_adjoint(n, _p(lrp), _p(lci), _p(lv), _p(urp), _p(uci), _p(uv), m, _p(R),
                              _p(G), _p(Y), _p(Z), _p(Yb), _p(Rb), _p(dL))
    return dict(Y=Y, Z=Z, Ybar=Yb, Rbar=Rb, dL=dL)


def dropout(L, eps):
    """Fill-in dropout of Eq. 10 on a lower CSR factor: an off-diagonal entry
    with |l_ij| <= eps becomes a structural zero (removed); the diagonal is
    kept. Returns the new CSR triple (row_ptr int64, col int32, val float64)."""
    rp, ci, v = (np.asarray(a) for a in L)
    n = len(rp) - 1
    rows = np.repeat(np.arange(n), np.diff(rp))
    keep = (ci == rows) | (np.abs(v) > eps)
    new_rp = np.zeros(n + 1, np.int64)
    np.add.at(new_rp, rows[keep] + 1, 1)
    return np.cumsum(new_rp), ci[keep].astype(np.int32), v[keep].astype(np.float64)
