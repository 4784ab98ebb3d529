"""torch.autograd over the pcad kernels: one Function per combinator.

    reduce(op, x0, x1=None)                 -> y
    scan(op, x0, x1=None, mode="auto")      -> y            (linrec: y, or (y, A))
    scan_linrec(a, b, mode, return_A=False) / scan_mat2(M, mode)
    reduce_by_index(op, idx, v, m, return_argk=False) -> hist (, argk)
    scan_matd(M) / reduce_matd(M)           3x3 or 5x5 matrix products (..., n, d, d)
    vscan(op, x) / vreduce(op, x) / vreduce_by_index(op, idx, v, m)
                                            vectorised operators, x (..., n, d)

Each forward runs the HIP forward kernel and keeps what the adjoint kernel
needs; each backward runs the adjoint kernel (the rules of Sections 3 to 5,
adjoints written, not accumulated, since autograd sums them itself).

What a scan keeps between the passes comes in the two forms the paper weighs
(a tape of intermediates against redundant execution, Section 2):
  recompute   the exclusive prefix of every tile (n / 8192 values per row);
              the adjoint kernel recomputes the forward prefixes inside each
              tile;
  checkpoint  the forward output itself (n values, plus A for a linear
              recurrence whose A output is differentiated); the adjoint kernel
              reads the prefixes from it and never reads the offsets b.
mode="auto" takes checkpoint when that tape fits CHECKPOINT_BUDGET_BYTES.
Reductions and reduce-by-index keep their lifted side results (zero counts
and products of the non-zeros, arg-extrema, tile prefixes) in every mode.

Inputs are float32 device tensors (int32 keys); there is no CPU path.
"""
from __future__ import annotations

from typing import Optional

import torch

from . import (DIM, PcadError, matd_reduce_fwd, matd_reduce_vjp, matd_scan_fwd, matd_scan_vjp,
               reduce_fwd, reduce_vjp, rbi_fwd, rbi_vjp, saved_argk, scan_fwd, scan_vjp,
               scan_vjp_checkpoint, vrbi_fwd, vrbi_vjp, vreduce_fwd, vreduce_vjp, vscan_fwd,
               vscan_vjp)

MODES = ("auto", "recompute", "checkpoint")
CHECKPOINT_BUDGET_BYTES = 256 << 20


def _c(t: Optional[torch.Tensor]) -> Optional[torch.Tensor]:
    return None if t is None else t.contiguous()


def pick_mode(mode: str, tape_bytes: int) -> str:
    """The saved-state form a scan of ``tape_bytes`` of output uses."""
    if mode not in MODES:
        raise PcadError(f"mode must be one of {MODES}, not {mode!r}")
    if mode == "auto":
        return "checkpoint" if tape_bytes <= CHECKPOINT_BUDGET_BYTES else "recompute"
    return mode


class _Scan(torch.autograd.Function):
    @staticmethod
    def forward(ctx, op: str, mode: str, want_A: bool, x0, x1):
        x0, x1 = _c(x0), _c(x1)
        ckpt = mode == "checkpoint"
        y, A, saved = scan_fwd(op, x0, x1, want_A=want_A, keep_saved=not ckpt)
        ctx.op, ctx.ckpt, ctx.want_A = op, ckpt, want_A
        if ckpt:
            ctx.save_for_backward(x0, y, A)
        else:
            ctx.save_for_backward(x0, x1, saved)
        return (y, A) if want_A else y

    @staticmethod
    def backward(ctx, gy, gA=None):
        op = ctx.op
        if ctx.ckpt:
            x0, y, A = ctx.saved_tensors
        else:
            x0, x1, saved = ctx.saved_tensors
        gy = torch.zeros_like(x0) if gy is None else gy.contiguous()
        Abar = gA.contiguous() if (ctx.want_A and gA is not None) else None
        if ctx.ckpt:
            g = scan_vjp_checkpoint(op, x0, None, y, A if Abar is not None else None, gy, Abar)
        else:
            g = scan_vjp(op, x0, x1, saved, gy, Abar)
        if op == "linrec":
            return None, None, None, g[0], g[1]
        return None, None, None, g, None


def scan(op: str, x0: torch.Tensor, x1: Optional[torch.Tensor] = None, mode: str = "auto",
         return_A: bool = False):
    """Inclusive scan along the last axis (mat2: the axis before the trailing 4)."""
    if op != "linrec" and (x1 is not None or return_A):
        raise PcadError("x1 and return_A belong to the linear recurrence only")
    tape = x0.numel() * 4 * (2 if (op == "linrec" and return_A) else 1)
    return _Scan.apply(op, pick_mode(mode, tape), bool(return_A), x0, x1)


def scan_linrec(a: torch.Tensor, b: torch.Tensor, mode: str = "auto", return_A: bool = False):
    """y_i = a_i * y_{i-1} + b_i with y_{-1} = 0 (and A_i = a_0 ... a_i)."""
    return scan("linrec", a, b, mode=mode, return_A=return_A)


def scan_mat2(M: torch.Tensor, mode: str = "auto"):
    """P_i = M_0 M_1 ... M_i of row-major 2x2 matrices, shape (..., n, 4)."""
    return scan("mat2", M, mode=mode)


class _Reduce(torch.autograd.Function):
    @staticmethod
    def forward(ctx, op: str, x0, x1):
        x0, x1 = _c(x0), _c(x1)
        y, saved = reduce_fwd(op, x0, x1)
        ctx.op = op
        ctx.save_for_backward(x0, x1, saved)
        return y

    @staticmethod
    def backward(ctx, gy):
        x0, x1, saved = ctx.saved_tensors
        g = reduce_vjp(ctx.op, x0, x1, saved, gy.contiguous())
        if ctx.op == "linrec":
            return None, g[0], g[1]
        return None, g, None


def reduce(op: str, x0: torch.Tensor, x1: Optional[torch.Tensor] = None):
    """Fold along the last axis; linrec returns the composed (A, y) pair."""
    if op != "linrec" and x1 is not None:
        raise PcadError("x1 belongs to the linear recurrence only")
    return _Reduce.apply(op, x0, x1)


class _Rbi(torch.autograd.Function):
    @staticmethod
    def forward(ctx, op: str, m: int, want_argk: bool, idx, v):
        idx, v = _c(idx), _c(v)
        hist, saved = rbi_fwd(op, idx, v, m)
        ctx.op, ctx.m = op, m
        ctx.save_for_backward(idx, v, saved)
        if want_argk:
            batch = hist.numel() // m if m else 0
            argk = saved_argk(saved, batch, m).view(hist.shape).clone()
            ctx.mark_non_differentiable(argk)
            return hist, argk
        return hist

    @staticmethod
    def backward(ctx, gh, gk=None):
        idx, v, saved = ctx.saved_tensors
        vbar = rbi_vjp(ctx.op, idx, v, ctx.m, saved, gh.contiguous())
        return None, None, None, None, vbar


def reduce_by_index(op: str, idx: torch.Tensor, v: torch.Tensor, m: int,
                    return_argk: bool = False):
    """hist[..., k] = fold of v[..., i] over idx[..., i] == k (neutral start);
    keys outside [0, m) are skipped.  min/max can also return the per-bin
    lowest arg-extremum (n for an empty bin)."""
    if return_argk and op not in ("min", "max"):
        raise PcadError("return_argk belongs to min and max")
    if idx.dtype != torch.int32:
        raise PcadError("keys must be int32")
    return _Rbi.apply(op, int(m), bool(return_argk), idx, v)


class _MatdScan(torch.autograd.Function):
    @staticmethod
    def forward(ctx, M):
        M = M.contiguous()
        P, saved = matd_scan_fwd(M)
        ctx.save_for_backward(M, saved)
        return P

    @staticmethod
    def backward(ctx, gP):
        M, saved = ctx.saved_tensors
        return matd_scan_vjp(M, saved, gP.contiguous())


class _MatdReduce(torch.autograd.Function):
    @staticmethod
    def forward(ctx, M):
        M = M.contiguous()
        Y, saved = matd_reduce_fwd(M)
        ctx.save_for_backward(M, saved)
        return Y

    @staticmethod
    def backward(ctx, gY):
        M, saved = ctx.saved_tensors
        return matd_reduce_vjp(M, saved, gY.contiguous())


def scan_matd(M: torch.Tensor):
    """P[..., i, :, :] = M[..., 0, :, :] @ ... @ M[..., i, :, :] for 3x3 or 5x5
    matrices M (..., n, d, d); the adjoint recomputes the forward prefixes
    from the saved tile prefixes (Section 5.3's redundant block-diagonal
    form)."""
    return _MatdScan.apply(M)


def reduce_matd(M: torch.Tensor):
    """Y[...] = M[..., 0, :, :] @ ... @ M[..., n-1, :, :] (identity for n = 0)."""
    return _MatdReduce.apply(M)


class _VScan(torch.autograd.Function):
    @staticmethod
    def forward(ctx, op: str, x):
        x = x.contiguous()
        y, saved = vscan_fwd(op, x)
        ctx.op = op
        ctx.save_for_backward(x, saved)
        return y

    @staticmethod
    def backward(ctx, gy):
        x, saved = ctx.saved_tensors
        return None, vscan_vjp(ctx.op, x, saved, gy.contiguous())


class _VReduce(torch.autograd.Function):
    @staticmethod
    def forward(ctx, op: str, x):
        x = x.contiguous()
        y, saved = vreduce_fwd(op, x)
        ctx.op = op
        ctx.save_for_backward(x, saved)
        return y

    @staticmethod
    def backward(ctx, gy):
        x, saved = ctx.saved_tensors
        return None, vreduce_vjp(ctx.op, x, saved, gy.contiguous())


class _VRbi(torch.autograd.Function):
    @staticmethod
    def forward(ctx, op: str, m: int, idx, v):
        idx, v = _c(idx), _c(v)
        hist, saved = vrbi_fwd(op, idx, v, m)
        ctx.op, ctx.m = op, m
        ctx.save_for_backward(idx, v, saved)
        return hist

    @staticmethod
    def backward(ctx, gh):
        idx, v, saved = ctx.saved_tensors
        return None, None, None, vrbi_vjp(ctx.op, idx, v, ctx.m, saved, gh.contiguous())


def vscan(op: str, x: torch.Tensor):
    """Inclusive scan along n of x (..., n, d) with map2 op (+ * min max)."""
    return _VScan.apply(op, x)


def vreduce(op: str, x: torch.Tensor):
    """Fold of x (..., n, d) along n with map2 op -> (..., d)."""
    return _VReduce.apply(op, x)


def vreduce_by_index(op: str, idx: torch.Tensor, v: torch.Tensor, m: int):
    """hist[..., k, c] = fold of v[..., i, c] over idx[..., i] == k."""
    if idx.dtype != torch.int32:
        raise PcadError("keys must be int32")
    return _VRbi.apply(op, int(m), idx, v)


__all__ = ["MODES", "CHECKPOINT_BUDGET_BYTES", "pick_mode", "scan", "scan_linrec", "scan_mat2",
           "reduce", "reduce_by_index", "scan_matd", "reduce_matd", "vscan", "vreduce",
           "vreduce_by_index", "DIM"]
