"""Learned correction of the IC(0) factor, L_pred = L_IC + GNN(A) (Eq. 2):
binding of the icpcg_gnn_* calls and a trainer that sequences them.

The network, its loss (Eq. 5, one Rademacher probe per step) and its
gradient, and the Adam update all run in libicpcg.so; this module draws the
probes, keeps the learning-rate schedule and orders the calls.
"""

from __future__ import annotations

import ctypes as C
import math

import numpy as np
import torch

from . import _lib as L
from .solver import CSR, Context, Preconditioner, _ptr


def num_params() -> int:
    return int(L.load().icpcg_gnn_num_params())


def init_params(seed: int, zero_output: bool = True, device="cuda") -> torch.Tensor:
    """Seeded starting parameters: normalization alpha = gamma = 1, beta = 0;
    weights uniform in +-1/sqrt(fan in), biases 0; with zero_output the last
    edge layer is zero, so the corrected factor starts at L_IC exactly."""
    rng = np.random.default_rng(seed)
    parts = [np.ones(9), np.ones(9), np.zeros(9)]
    for b in range(3):
        din = (1 if b == 0 else 2) + 18
        w2 = rng.uniform(-1, 1, 8) / math.sqrt(8)
        W1 = rng.uniform(-1, 1, (8, din)) / math.sqrt(din)
        if zero_output and b == 2:
            w2 = np.zeros(8)
        parts += [W1.ravel(), np.zeros(8), w2, np.zeros(1)]
        if b < 2:
            parts += [(rng.uniform(-1, 1, (8, 11)) / math.sqrt(11)).ravel(), np.zeros(8),
                      (rng.uniform(-1, 1, (9, 8)) / math.sqrt(8)).ravel(), np.zeros(9)]
    th = np.concatenate(parts)
    assert th.size == num_params()
    return torch.from_numpy(th).to(device)


class GNNGraph:
    """A matrix prepared for the network: A (full CSR) with the FP64
    preconditioner P holding its IC(0) factor (pattern = tril(A))."""

    def __init__(self, ctx: Context, A: CSR, P: Preconditioner):
        if P.dtype != "f64":
            raise ValueError("the learned correction starts from an FP64 IC(0) preconditioner")
        self.ctx, self.A, self.P = ctx, A, P
        ctx._bind()
        h = C.c_void_p()
        a = A.cstruct()
        ctx._check(ctx.lib.icpcg_gnn_create(ctx.h, C.byref(a), P.h, C.byref(h)))
        self.h = h
        self.n, self.nnz = A.n, P.L.nnz

    def close(self):
        if getattr(self, "h", None):
            self.ctx.lib.icpcg_gnn_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def inputs(self):
        """(node features n x 9, edge inputs, scale s)."""
        self.ctx._bind()
        x = torch.empty(self.n, 9, dtype=torch.float64, device="cuda")
        e = torch.empty(self.nnz, dtype=torch.float64, device="cuda")
        s = C.c_double()
        self.ctx._check(self.ctx.lib.icpcg_gnn_inputs(self.ctx.h, self.h, _ptr(x), _ptr(e), C.byref(s)))
        return x, e, s.value

    def forward(self, theta: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """L_pred values on the factor's pattern."""
        self.ctx._bind()
        _check_theta(theta)
        out = torch.empty(self.nnz, dtype=torch.float64, device="cuda") if out is None else out
        self.ctx._check(self.ctx.lib.icpcg_gnn_forward(self.ctx.h, self.h, _ptr(theta), _ptr(out)))
        return out

    def factor(self, theta: torch.Tensor) -> CSR:
        """The corrected factor as a CSR matrix (L's pattern, L_pred values)."""
        Lf = self.P.L
        return CSR(Lf.row_ptr, Lf.col, self.forward(theta))

    def loss_grad(self, theta, z, loss, grad, accumulate=False):
        """Eq. 5 loss for probe z and its gradient (device outputs)."""
        self.ctx._bind()
        _check_theta(theta)
        if z.dtype != torch.float64 or z.numel() != self.n or not z.is_cuda:
            raise ValueError("z must be a CUDA float64 vector of length n")
        self.ctx._check(self.ctx.lib.icpcg_gnn_loss_grad(self.ctx.h, self.h, _ptr(theta), _ptr(z), _ptr(loss),
                                                         _ptr(grad), int(bool(accumulate))))


def _check_theta(theta):
    if theta.dtype != torch.float64 or not theta.is_cuda or theta.numel() != num_params() or \
            not theta.is_contiguous():
        raise ValueError(f"theta must be a contiguous CUDA float64 vector of {num_params()} values")


def adam_step(ctx: Context, theta, grad, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    ctx._bind()
    ctx._check(ctx.lib.icpcg_adam_step(ctx.h, _ptr(theta), _ptr(grad), _ptr(m), _ptr(v), theta.numel(), int(t),
                                       float(lr), float(beta1), float(beta2), float(eps)))


def rademacher(n: int, gen: torch.Generator, device="cuda") -> torch.Tensor:
    """A probe of +-1 entries from a seeded CPU generator."""
    z = torch.randint(0, 2, (n,), generator=gen, dtype=torch.int64)
    return (2.0 * z.to(torch.float64) - 1.0).to(device)


class Trainer:
    """Adam on the Eq. 5 loss over a set of prepared matrices, with a linear
    learning-rate warm-up (Training and Inference section: Adam, initial rate
    0.005, warm-up). One step sums the loss and gradient of `batch` matrices,
    each with `probes` fresh probes (Adam's step does not depend on the
    gradient's overall scale, so the sum serves as the mean)."""

    def __init__(self, ctx: Context, theta: torch.Tensor, lr=0.005, warmup=20, batch=1, probes=1, seed=0):
        self.ctx, self.theta = ctx, theta
        self.lr, self.warmup, self.batch, self.probes = lr, warmup, batch, probes
        self.m = torch.zeros_like(theta)
        self.v = torch.zeros_like(theta)
        self.grad = torch.zeros_like(theta)
        self.loss = torch.zeros(1, dtype=torch.float64, device=theta.device)
        self.t = 0
        self.gen = torch.Generator().manual_seed(seed)

    def step(self, graphs):
        first = True
        for g in graphs:
            for _ in range(self.probes):
                z = rademacher(g.n, self.gen, self.theta.device)
                g.loss_grad(self.theta, z, self.loss, self.grad, accumulate=not first)
                first = False
        self.t += 1
        lr = self.lr * min(1.0, self.t / max(1, self.warmup))
        adam_step(self.ctx, self.theta, self.grad, self.m, self.v, self.t, lr)
        return self.loss  # device scalar: sum over the batch and probes (before the update)

    def epoch(self, graphs):
        """One pass over the graphs in a seeded order; returns the mean loss."""
        order = torch.randperm(len(graphs), generator=self.gen).tolist()
        total = 0.0
        for i in range(0, len(order), self.batch):
            batch = [graphs[j] for j in order[i:i + self.batch]]
            total += float(self.step(batch).item())
        return total / (len(graphs) * self.probes)


def mean_loss(graphs, theta, probes=8, seed=123):
    """Average Eq. 5 loss over a few seeded probes per matrix (evaluation)."""
    gen = torch.Generator().manual_seed(seed)
    loss = torch.zeros(1, dtype=torch.float64, device=theta.device)
    grad = torch.zeros_like(theta)
    tot = 0.0
    for g in graphs:
        for p in range(probes):
            z = rademacher(g.n, gen, theta.device)
            g.loss_grad(theta, z, loss, grad, accumulate=False)
            tot += float(loss.item())
    return tot / (probes * len(graphs))
