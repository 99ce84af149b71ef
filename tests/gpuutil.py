"""Helpers for GPU tests: moving numpy operands to the device with their
exact strides, and the error bounds of the parity checks."""
import numpy as np

U64 = 2.0 ** -53
U32 = 2.0 ** -24


def require_gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def to_dev(a, dtype=None):
    """Device tensor with a's shape and element strides (numpy layout kept)."""
    import torch
    a = np.asarray(a)
    if dtype is not None:
        a = a.astype(dtype, order="K")
    strides = [s // a.itemsize for s in a.strides]
    span = 1 + sum((n - 1) * s for n, s in zip(a.shape, strides)) if a.size else 0
    base = torch.zeros(max(span, 1), dtype=torch.from_numpy(np.zeros(1, a.dtype)).dtype, device="cuda")
    t = torch.as_strided(base, a.shape, strides)
    if a.size:
        t.copy_(torch.from_numpy(np.ascontiguousarray(a).reshape(a.shape)).to("cuda"))
    return t


def to_host(t):
    return t.detach().cpu().numpy()


def fp64_bound(K, alpha, maxA, maxB, beta=0.0, maxC0=0.0):
    """max|C - Cref| <= 1e-12 * K * |alpha| * max|A| * max|B| (+ beta term)."""
    return 1e-12 * max(K, 1) * abs(alpha) * maxA * maxB + 4 * U64 * abs(beta) * maxC0


def fp32_componentwise(K, alpha, absC, beta=0.0, C0=None):
    """|C - Cref| <= (K + 2) u32 (|alpha| absC + |beta| |C0|) elementwise."""
    b = (K + 2) * U32 * abs(alpha) * absC
    if beta != 0.0 and C0 is not None:
        b = b + (K + 2) * U32 * abs(beta) * np.abs(C0)
    return b


def split_bf16_componentwise(K, alpha, absC, beta=0.0, C0=None):
    """|C - Cref| <= (3 2^-16 (1 + 2^-7) + (3K + 2) u32) |alpha| absC + 2 u32 |beta C0|."""
    b = (3 * 2.0 ** -16 * (1 + 2.0 ** -7) + (3 * K + 2) * U32) * abs(alpha) * absC
    if beta != 0.0 and C0 is not None:
        b = b + 2 * U32 * abs(beta) * np.abs(C0)
    return b
