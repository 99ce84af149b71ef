"""Differentiable contraction: a hand-written backward for torch.autograd.

For C = alpha * A . B + beta * C0 (labels idx_A, idx_B -> idx_C) and an
upstream gradient dC, the definition of the contraction (Sec. 4, eq.
gen-contraction) is bilinear in A and B, so

    dA[idx_A] = alpha * sum_{J} dC[idx_C] * B[idx_B]
    dB[idx_B] = alpha * sum_{I} A[idx_A] * dC[idx_C]
    dC0       = beta * dC

Each of dA and dB is itself a general contraction (its labels again appear in
exactly two of its three tensors), so both are computed by the same planner
and kernels, transpose-free, in the forward's precision mode.
"""
import torch

from . import tc


def _colmajor_like(shape, dtype, device):
    strides, s = [], 1
    for n in shape:
        strides.append(s)
        s *= max(int(n), 1)
    return torch.empty_strided(tuple(shape), tuple(strides), dtype=dtype, device=device)


def _dense(t):
    """The library needs positive strides on every dimension of length > 1
    (no broadcast views): materialise such gradients."""
    if any(st == 0 and n > 1 for n, st in zip(t.shape, t.stride())):
        return t.contiguous()
    return t


class Contract(torch.autograd.Function):
    """Contract.apply(A, idx_A, B, idx_B, idx_C, alpha=1, beta=0, C0=None, mode="native")"""

    @staticmethod
    def forward(ctx, A, idx_A, B, idx_B, idx_C, alpha=1.0, beta=0.0, C0=None, mode="native"):
        ext = {}
        for t, lab in ((A, idx_A), (B, idx_B)):
            for l, n in zip(lab, t.shape):
                ext[l] = int(n)
        out = _colmajor_like([ext[l] for l in idx_C], A.dtype, A.device)
        if C0 is not None and beta != 0.0:
            out.copy_(C0)
            tc.contract(A, idx_A, B, idx_B, idx_C, alpha=alpha, beta=beta, out=out, mode=mode)
        else:
            tc.contract(A, idx_A, B, idx_B, idx_C, alpha=alpha, beta=0.0, out=out, mode=mode)
        ctx.save_for_backward(A, B)
        ctx.meta = (idx_A, idx_B, idx_C, float(alpha), float(beta), mode, C0 is not None)
        return out

    @staticmethod
    def backward(ctx, dC):
        A, B = ctx.saved_tensors
        idx_A, idx_B, idx_C, alpha, beta, mode, has_c0 = ctx.meta
        dC = _dense(dC)
        dA = dB = dC0 = None
        if ctx.needs_input_grad[0]:
            dA = _colmajor_like(A.shape, A.dtype, A.device)
            tc.contract(dC, idx_C, B, idx_B, idx_A, alpha=alpha, beta=0.0, out=dA, mode=mode)
        if ctx.needs_input_grad[2]:
            dB = _colmajor_like(B.shape, B.dtype, B.device)
            tc.contract(A, idx_A, dC, idx_C, idx_B, alpha=alpha, beta=0.0, out=dB, mode=mode)
        if has_c0 and ctx.needs_input_grad[7]:
            # dC0 := beta * dC by the library: a copy of dC scaled by a call
            # with alpha = 0, which reads neither operand (C := beta * C)
            dC0 = _colmajor_like(dC.shape, dC.dtype, dC.device)
            dC0.copy_(dC)
            tc.contract(A, idx_A, B, idx_B, idx_C, alpha=0.0, beta=beta, out=dC0, mode=mode)
        return dA, None, dB, None, None, None, None, dC0, None


def contract(A, idx_A, B, idx_B, idx_C, alpha=1.0, beta=0.0, C0=None, mode="native"):
    """Differentiable C[idx_C] = alpha * A . B + beta * C0."""
    return Contract.apply(A, idx_A, B, idx_B, idx_C, alpha, beta, C0, mode)
