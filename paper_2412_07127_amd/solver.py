"""Python binding over the C ABI (include/icpcg.h) with torch tensors as device
memory and torch's current stream as the HIP stream. Argument marshalling
only: every numerical step runs in libicpcg.so's kernels.
"""

from __future__ import annotations

import ctypes as C
import dataclasses

import numpy as np
import torch

from . import _lib as L

DTYPES = {"f64": L.F64, "f32": L.F32, "bf16": L.BF16}


class IcpcgError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{L.STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _block_width(X: torch.Tensor, n: int, dtype=None) -> int:
    """Checks an n x R row-major block (or an n-vector) and returns R."""
    if not X.is_cuda or not X.is_contiguous():
        raise ValueError("blocks must be contiguous CUDA tensors")
    if dtype is not None and X.dtype != dtype:
        raise ValueError(f"expected {dtype}, got {X.dtype}")
    if X.dim() == 1:
        R = 1
    elif X.dim() == 2:
        R = X.shape[1]
    else:
        raise ValueError("blocks are 1-D or 2-D")
    if X.shape[0] != n:
        raise ValueError(f"block has {X.shape[0]} rows, expected {n}")
    return R


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


@dataclasses.dataclass
class CSR:
    """Square CSR matrix on the GPU: row_ptr int64, col int32, val float64."""
    row_ptr: torch.Tensor
    col: torch.Tensor
    val: torch.Tensor

    @property
    def n(self) -> int:
        return self.row_ptr.numel() - 1

    @property
    def nnz(self) -> int:
        return self.col.numel()

    @classmethod
    def from_numpy(cls, row_ptr, col, val, device="cuda"):
        return cls(torch.as_tensor(np.asarray(row_ptr, np.int64)).to(device),
                   torch.as_tensor(np.asarray(col, np.int32)).to(device),
                   torch.as_tensor(np.asarray(val, np.float64)).to(device))

    def numpy(self):
        return (self.row_ptr.cpu().numpy(), self.col.cpu().numpy(), self.val.cpu().numpy())

    def check(self):
        for t, dt in ((self.row_ptr, torch.int64), (self.col, torch.int32), (self.val, torch.float64)):
            if t.dtype != dt or not t.is_cuda or not t.is_contiguous():
                raise ValueError(f"CSR arrays must be contiguous CUDA tensors of {dt}")
        if self.val.numel() != self.col.numel():
            raise ValueError("val and col lengths differ")

    def cstruct(self) -> L.Csr:
        self.check()
        return L.Csr(self.n, self.nnz, self.row_ptr.data_ptr(), self.col.data_ptr(), self.val.data_ptr())


class Matrix:
    """A CSR matrix analyzed once for repeated products (row groups of
    identical column lists). Keeps a reference to the CSR tensors."""

    def __init__(self, ctx: "Context", A: CSR):
        self.ctx, self.A = ctx, A
        ctx._bind()
        h = C.c_void_p()
        a = A.cstruct()
        ctx._check(ctx.lib.icpcg_mat_create(ctx.h, C.byref(a), C.byref(h)))
        self.h = h

    @property
    def n(self):
        return self.A.n

    def close(self):
        if getattr(self, "h", None):
            self.ctx.lib.icpcg_mat_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def spmv(self, X: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        self.ctx._bind()
        R = _block_width(X, self.n, torch.float64)
        W = torch.empty_like(X) if out is None else out
        _block_width(W, self.n, torch.float64)
        self.ctx._check(self.ctx.lib.icpcg_mat_spmv(self.ctx.h, self.h, _ptr(X), _ptr(W), R))
        return W


class Context:
    """An icpcg context bound to the current device; every call runs on
    torch's current stream."""

    def __init__(self):
        self.lib = L.load()
        h = C.c_void_p()
        self._check(self.lib.icpcg_create(C.byref(h), _stream()), ctx=None)
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.icpcg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st, ctx="self"):
        if st != 0:
            msg = ""
            if ctx == "self" and getattr(self, "h", None):
                msg = (self.lib.icpcg_last_error(self.h) or b"").decode()
            raise IcpcgError(st, msg or self.lib.icpcg_status_string(st).decode())

    def _bind(self):
        self.lib.icpcg_set_stream(self.h, _stream())

    # ------------------------------------------------------------- factor
    def tril_nnz(self, A: CSR) -> int:
        self._bind()
        out = C.c_int64()
        a = A.cstruct()
        self._check(self.lib.icpcg_tril_nnz(self.h, C.byref(a), C.byref(out)))
        return out.value

    def factor(self, A: CSR, max_restarts: int = -1, alpha_min: float = 0.0, raise_on_pivot=True):
        """IC(0) of tril(A) on the GPU. Returns (L, info dict)."""
        m = self.tril_nnz(A)
        dev = A.val.device
        Lr = torch.empty(A.n + 1, dtype=torch.int64, device=dev)
        Lc = torch.empty(m, dtype=torch.int32, device=dev)
        Lv = torch.empty(m, dtype=torch.float64, device=dev)
        a = A.cstruct()
        opts = L.FactorOpts(max_restarts, alpha_min)
        info = L.FactorInfo()
        st = self.lib.icpcg_factor(self.h, C.byref(a), _ptr(Lr), _ptr(Lc), _ptr(Lv), C.byref(opts), C.byref(info))
        if st != 0 and (raise_on_pivot or st != L.E_PIVOT):
            self._check(st)
        return CSR(Lr, Lc, Lv), dict(alpha=info.alpha, restarts=info.restarts, min_pivot=info.min_pivot,
                                     nlevels=info.nlevels, status=st)

    # ---------------------------------------------------- preconditioner
    def prec(self, Lf: CSR, dtype: str = "f64") -> "Preconditioner":
        self._bind()
        h = C.c_void_p()
        l = Lf.cstruct()
        self._check(self.lib.icpcg_prec_create(self.h, C.byref(l), DTYPES[dtype], C.byref(h)))
        return Preconditioner(self, h, Lf, dtype)

    def dropout(self, Lf: CSR, eps: float) -> CSR:
        """Fill-in dropout (Eq. 10): off-diagonal entries with |l| <= eps removed."""
        self._bind()
        dev = Lf.val.device
        rp = torch.empty(Lf.n + 1, dtype=torch.int64, device=dev)
        ci = torch.empty(Lf.nnz, dtype=torch.int32, device=dev)
        v = torch.empty(Lf.nnz, dtype=torch.float64, device=dev)
        cnt = C.c_int64()
        l = Lf.cstruct()
        self._check(self.lib.icpcg_dropout(self.h, C.byref(l), float(eps), _ptr(rp), _ptr(ci), _ptr(v),
                                           C.byref(cnt)))
        k = cnt.value
        return CSR(rp, ci[:k].clone(), v[:k].clone())

    def color_order(self, A: CSR, seed: int = 0):
        """Multicolour node order: (perm int32 tensor, new row -> old row; colour count)."""
        self._bind()
        perm = torch.empty(A.n, dtype=torch.int32, device=A.val.device)
        nc = C.c_int32()
        a = A.cstruct()
        self._check(self.lib.icpcg_color_order(self.h, C.byref(a), C.c_uint64(seed), _ptr(perm), C.byref(nc)))
        return perm, nc.value

    def block_color_order(self, A: CSR, block: torch.Tensor, nblocks: int = 0):
        """Block multicolour order of a row partition (block: int32 tensor, block
        id per row): (perm int32 tensor, new row -> old row; colour count)."""
        self._bind()
        b = block.to(device=A.val.device, dtype=torch.int32).contiguous()
        nb = int(nblocks) if nblocks else (int(b.max().item()) + 1 if b.numel() else 1)
        perm = torch.empty(A.n, dtype=torch.int32, device=A.val.device)
        nc = C.c_int32()
        a = A.cstruct()
        self._check(self.lib.icpcg_block_color_order(self.h, C.byref(a), _ptr(b), nb, _ptr(perm), C.byref(nc)))
        return perm, nc.value

    def permute(self, A: CSR, perm: torch.Tensor) -> CSR:
        """P A P^T."""
        self._bind()
        dev = A.val.device
        out = CSR(torch.empty(A.n + 1, dtype=torch.int64, device=dev), torch.empty(A.nnz, dtype=torch.int32, device=dev),
                  torch.empty(A.nnz, dtype=torch.float64, device=dev))
        a = A.cstruct()
        self._check(self.lib.icpcg_permute_matrix(self.h, C.byref(a), _ptr(perm), _ptr(out.row_ptr), _ptr(out.col),
                                                  _ptr(out.val)))
        return out

    def permute_rows(self, perm: torch.Tensor, X: torch.Tensor, inverse: bool = False) -> torch.Tensor:
        """Y[i] = X[perm[i]] (or the inverse scatter) for an n-vector or n x R block."""
        self._bind()
        Xc = X.contiguous()
        R = _block_width(Xc, perm.numel(), torch.float64)
        Y = torch.empty_like(Xc)
        self._check(self.lib.icpcg_permute_rows(self.h, _ptr(perm), perm.numel(), R, _ptr(Xc), _ptr(Y),
                                                int(bool(inverse))))
        return Y

    def prec_simple(self, A: CSR, kind: str) -> "Preconditioner":
        """Table 1's baselines: kind "jacobi" (z_i = r_i / a_ii) or "none" (plain CG)."""
        self._bind()
        k = {"jacobi": L.PREC_JACOBI, "none": L.PREC_NONE}[kind]
        h = C.c_void_p()
        a = A.cstruct()
        self._check(self.lib.icpcg_prec_create_simple(self.h, C.byref(a), k, C.byref(h)))
        P = Preconditioner(self, h, None, "f64")
        P.kind, P._n = kind, A.n
        return P

    # ------------------------------------------------------------ kernels
    def spmv(self, A: CSR, X: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        self._bind()
        R = _block_width(X, A.n, torch.float64)
        W = torch.empty_like(X) if out is None else out
        _block_width(W, A.n, torch.float64)
        a = A.cstruct()
        self._check(self.lib.icpcg_spmv(self.h, C.byref(a), _ptr(X.contiguous()), _ptr(W), R))
        return W

    def matrix(self, A: CSR) -> Matrix:
        return Matrix(self, A)

    def solve(self, A, P: "Preconditioner", B: torch.Tensor, X0: torch.Tensor | None = None,
              rtol: float = 1e-8, max_iter: int = 0, max_replace: int = 3, block_width: int = 0,
              check_every: int = 8, use_graph: bool = False, raise_on_error: bool = False):
        """PCG (supplementary Algorithm 1) for the columns of B. Returns (X, infos).

        block_width 0 takes the autotuner's width (see autotune); use_graph
        replays the steps between two convergence polls as a captured hipGraph."""
        self._bind()
        R = _block_width(B, A.n, torch.float64)
        if P.n != A.n:
            raise ValueError("preconditioner and matrix sizes differ")
        X = torch.zeros_like(B) if X0 is None else X0.clone().contiguous()
        if X.shape != B.shape:
            raise ValueError("X0 and B shapes differ")
        opts = L.SolveOpts(rtol, max_iter, max_replace, block_width, check_every, int(bool(use_graph)))
        infos = (L.ColInfo * R)()
        if isinstance(A, Matrix):
            st = self.lib.icpcg_solve_mat(self.h, A.h, P.h, _ptr(B), _ptr(X), R, C.byref(opts), infos)
        else:
            a = A.cstruct()
            st = self.lib.icpcg_solve(self.h, C.byref(a), P.h, _ptr(B), _ptr(X), R, C.byref(opts), infos)
        if st in (L.E_INVALID, L.E_DEVICE, L.E_NOMEM) or (st != 0 and raise_on_error):
            self._check(st)
        out = [dict(iters=i.iters, replacements=i.replacements, status=i.status, relres=i.relres,
                    true_relres=i.true_relres) for i in infos]
        return X, out

    def autotune(self, M: "Matrix", P: "Preconditioner", nrhs: int) -> dict:
        """Block width for nrhs columns (timed on the operands, cached in the context)."""
        self._bind()
        info = L.TuneInfo()
        self._check(self.lib.icpcg_autotune(self.h, M.h, P.h, int(nrhs), C.byref(info)))
        return dict(block_width=info.block_width, ms_per_rhs=info.ms_per_rhs,
                    ms_per_step={w: info.ms_per_step[i] for i, w in enumerate((1, 2, 4, 8, 16))
                                 if info.ms_per_step[i] > 0})

    STEP_PHASES = ("trsv_L", "trsv_U", "update_p", "spmv", "pw", "update_xr")

    def step_timing(self, enable: bool = True):
        """Record the phase durations of the next eager PCG steps (up to 64)."""
        self._bind()
        self._check(self.lib.icpcg_step_timing(self.h, int(bool(enable))))

    def step_timing_get(self) -> dict:
        """Mean ms per phase over the recorded steps, and their count."""
        self._bind()
        ms = (C.c_double * len(self.STEP_PHASES))()
        steps = C.c_int64(0)
        self._check(self.lib.icpcg_step_timing_get(self.h, ms, C.byref(steps)))
        out = {k: ms[i] for i, k in enumerate(self.STEP_PHASES)}
        out["steps"] = steps.value
        return out

    def sync(self):
        self._check(self.lib.icpcg_sync(self.h))


class Preconditioner:
    """P = L L^T with cached L^T, supernode schedules and reduced-precision copies."""

    def __init__(self, ctx: Context, h, Lf: CSR, dtype: str):
        self.ctx, self.h, self.L, self.dtype = ctx, h, Lf, dtype
        self.kind = "factor"
        self._n = Lf.n if Lf is not None else 0
        self.version = 0  # bumped by every update_values call

    def close(self):
        if getattr(self, "h", None):
            self.ctx.lib.icpcg_prec_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def n(self):
        return self._n

    def vec_dtype(self):
        return torch.float64 if self.dtype == "f64" else torch.float32

    def info(self) -> dict:
        self.ctx._bind()
        i = L.PrecInfo()
        self.ctx._check(self.ctx.lib.icpcg_prec_get_info(self.ctx.h, self.h, C.byref(i)))
        return {k: getattr(i, k) for k, _ in L.PrecInfo._fields_}

    def update_values(self, val: torch.Tensor):
        self.ctx._bind()
        v = val.to(torch.float64).contiguous()
        self.ctx._check(self.ctx.lib.icpcg_prec_update_values(self.ctx.h, self.h, _ptr(v)))
        self.L = CSR(self.L.row_ptr, self.L.col, v)
        self.version += 1

    def levels(self) -> dict:
        info = self.info()
        dev = self.L.val.device
        n = self.n
        mk = lambda m: torch.empty(m, dtype=torch.int32, device=dev)
        out = dict(level_L=mk(n), perm_L=mk(n), level_ptr_L=mk(info["nlevels_L"] + 1),
                   level_U=mk(n), perm_U=mk(n), level_ptr_U=mk(info["nlevels_U"] + 1))
        self.ctx._bind()
        self.ctx._check(self.ctx.lib.icpcg_prec_levels(
            self.ctx.h, self.h, *[_ptr(out[k]) for k in ("level_L", "perm_L", "level_ptr_L",
                                                          "level_U", "perm_U", "level_ptr_U")]))
        return out

    def transpose(self) -> CSR:
        dev = self.L.val.device
        U = CSR(torch.empty(self.n + 1, dtype=torch.int64, device=dev),
                torch.empty(self.L.nnz, dtype=torch.int32, device=dev),
                torch.empty(self.L.nnz, dtype=torch.float64, device=dev))
        self.ctx._bind()
        self.ctx._check(self.ctx.lib.icpcg_prec_transpose(self.ctx.h, self.h, _ptr(U.row_ptr), _ptr(U.col),
                                                          _ptr(U.val)))
        return U

    def _width(self, X):
        return _block_width(X, self.n)

    def trsv(self, Rhs: torch.Tensor, transpose: bool = False) -> torch.Tensor:
        self.ctx._bind()
        r64 = Rhs.dtype == torch.float64
        if self.dtype == "f64" and not r64:
            raise ValueError("an f64 preconditioner takes float64 blocks")
        if self.dtype != "f64" and not r64 and Rhs.dtype != torch.float32:
            raise ValueError("blocks must be float32 or float64")
        if transpose and self.dtype != "f64" and r64:
            raise ValueError("the backward solve of a reduced-precision preconditioner takes float32 blocks")
        Y = torch.empty(Rhs.shape, dtype=self.vec_dtype(), device=Rhs.device)
        Rc = Rhs.contiguous()
        self._width(Rc)
        self.ctx._check(self.ctx.lib.icpcg_trsv(self.ctx.h, self.h, int(transpose), _ptr(Rc), int(r64), _ptr(Y),
                                                self._width(Rhs)))
        return Y

    def apply(self, Rhs: torch.Tensor):
        """Y = L^-1 R, Z = L^-T Y. Returns (Y, Z)."""
        self.ctx._bind()
        r64 = Rhs.dtype == torch.float64
        if self.dtype == "f64" and not r64:
            raise ValueError("an f64 preconditioner takes float64 blocks")
        Y = torch.empty(Rhs.shape, dtype=self.vec_dtype(), device=Rhs.device)
        Z = torch.empty_like(Y)
        Rc = Rhs.contiguous()
        self._width(Rc)
        self.ctx._check(self.ctx.lib.icpcg_apply(self.ctx.h, self.h, _ptr(Rc), int(r64), _ptr(Y), _ptr(Z),
                                                 self._width(Rhs)))
        return Y, Z

    def apply_rz(self, Rhs: torch.Tensor):
        """The preconditioner solve of a PCG step: Y = L^-1 R, Z = L^-T Y for an
        FP64 block R, and r^T z per column (FP64). Returns (Y, Z, rz)."""
        self.ctx._bind()
        if Rhs.dtype != torch.float64:
            raise ValueError("apply_rz takes a float64 block")
        Rc = Rhs.contiguous()
        R = self._width(Rc)
        Y = torch.empty(Rc.shape, dtype=self.vec_dtype(), device=Rc.device)
        Z = torch.empty_like(Y)
        rz = torch.empty(R, dtype=torch.float64, device=Rc.device)
        self.ctx._check(self.ctx.lib.icpcg_apply_rz(self.ctx.h, self.h, _ptr(Rc), _ptr(Y), _ptr(Z), _ptr(rz), R))
        return Y, Z, rz

    def trsv_rz(self, Y: torch.Tensor, Rhs: torch.Tensor, Z: torch.Tensor = None, rz: torch.Tensor = None):
        """Backward solve Z = L^-T Y with r^T z per column, as a PCG step
        launches it (fused for FP32 / BF16 factors on 2-16 columns). Y: the
        factor's block dtype; R: FP64 of Y's shape. Returns (Z, rz)."""
        self.ctx._bind()
        if Rhs.dtype != torch.float64 or not Rhs.is_contiguous():
            raise ValueError("trsv_rz takes a contiguous float64 R")
        if Y.shape != Rhs.shape or Y.dtype != self.vec_dtype() or not Y.is_contiguous():
            raise ValueError("Y must be contiguous, R's shape and the factor's block dtype")
        R = self._width(Rhs)
        Z = torch.empty_like(Y) if Z is None else Z
        rz = torch.empty(R, dtype=torch.float64, device=Y.device) if rz is None else rz
        self.ctx._check(self.ctx.lib.icpcg_trsv_rz(self.ctx.h, self.h, _ptr(Y), _ptr(Rhs), _ptr(Z), _ptr(rz), R))
        return Z, rz

    def apply_rz_noalloc(self, Rhs: torch.Tensor, Y: torch.Tensor, Z: torch.Tensor, rz: torch.Tensor):
        """apply_rz into caller-made outputs through the entry point that
        allocates nothing (its partials live in the library's static device
        array). Y and Z: the factor's block dtype, R's shape; rz: nrhs FP64."""
        self.ctx._bind()
        if Rhs.dtype != torch.float64 or not Rhs.is_contiguous():
            raise ValueError("apply_rz_noalloc takes a contiguous float64 block")
        R = self._width(Rhs)
        for T in (Y, Z):
            if T.shape != Rhs.shape or T.dtype != self.vec_dtype() or not T.is_contiguous():
                raise ValueError("Y, Z must be contiguous, R's shape and the factor's block dtype")
        if rz.dtype != torch.float64 or rz.numel() != R:
            raise ValueError("rz must hold nrhs float64 values")
        self.ctx._check(self.ctx.lib.icpcg_apply_rz_noalloc(self.ctx.h, self.h, _ptr(Rhs), _ptr(Y), _ptr(Z),
                                                            _ptr(rz), R))
        return Y, Z, rz

    def apply_backward(self, G: torch.Tensor, Y: torch.Tensor, Z: torch.Tensor):
        """Gradients of Z = L^-T L^-1 R given G = dl/dZ. Returns (dR, dL_val)."""
        self.ctx._bind()
        dt = self.vec_dtype()
        G = G.to(dt).contiguous()
        for T in (Y, Z):
            if T.shape != G.shape or T.dtype != dt:
                raise ValueError("Y, Z must match G's shape and the preconditioner's block dtype")
        Ybar = torch.empty_like(G)
        dR = torch.empty_like(G)
        dL = torch.empty(self.L.nnz, dtype=dt, device=G.device)
        self.ctx._check(self.ctx.lib.icpcg_apply_backward(self.ctx.h, self.h, _ptr(G), _ptr(Y.contiguous()),
                                                          _ptr(Z.contiguous()), _ptr(Ybar), _ptr(dR), _ptr(dL),
                                                          self._width(G)))
        return dR, dL
