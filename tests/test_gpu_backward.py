"""Backward pass of the differentiable contraction on the GPU: the oracle's
gradient, central finite differences, the adjoint identity, and torch's
gradcheck on tiny FP64 problems."""
import numpy as np
import pytest

from paper_1607_00291_amd import inputs
from gpuutil import U32, require_gpu, to_dev, to_host

pytestmark = pytest.mark.gpu


def f32(x):
    return np.asfortranarray(np.asarray(x, dtype=np.float32).astype(np.float64))


def oracle_out(oracle_mod, A, ia, B, ib, shape, ic, absval=False):
    C = inputs.colmajor(shape, fill=0.0)
    oracle_mod.contract(1.0, A, ia, B, ib, 0.0, C, ic, absval=absval)
    return C


def test_cfg4_fp32_forward_backward(oracle_mod):
    torch = require_gpu()
    from paper_1607_00291_amd.autograd import contract
    p = inputs.cfg4()
    A64, B64, dC64 = f32(p.A), f32(p.B), f32(p.dC)  # FP32-rounded, widened
    A = to_dev(A64, np.float32).requires_grad_(True)
    B = to_dev(B64, np.float32).requires_grad_(True)
    print("case cfg4 forward+backward fp32", flush=True)
    C = contract(A, p.idx_A, B, p.idx_B, p.idx_C)
    C.backward(to_dev(dC64, np.float32))
    torch.cuda.synchronize()
    gC, gA, gB = to_host(C.detach()).astype(np.float64), to_host(A.grad).astype(np.float64), \
        to_host(B.grad).astype(np.float64)

    # forward vs oracle (componentwise FP32 bound)
    Cref = oracle_out(oracle_mod, A64, p.idx_A, B64, p.idx_B, p.C.shape, p.idx_C)
    absC = oracle_out(oracle_mod, A64, p.idx_A, B64, p.idx_B, p.C.shape, p.idx_C, absval=True)
    K = p.mnk()[2]
    assert np.all(np.abs(gC - Cref) <= (K + 2) * U32 * absC)

    # oracle gradients: dA = dC . B over J, dB = A . dC over I (contracted 2048 each)
    dAref = oracle_out(oracle_mod, dC64, p.idx_C, B64, p.idx_B, p.A.shape, p.idx_A)
    absdA = oracle_out(oracle_mod, dC64, p.idx_C, B64, p.idx_B, p.A.shape, p.idx_A, absval=True)
    dBref = oracle_out(oracle_mod, A64, p.idx_A, dC64, p.idx_C, p.B.shape, p.idx_B)
    absdB = oracle_out(oracle_mod, A64, p.idx_A, dC64, p.idx_C, p.B.shape, p.idx_B, absval=True)
    Kp = 2048
    assert np.all(np.abs(gA - dAref) <= (Kp + 2) * U32 * absdA)
    assert np.all(np.abs(gB - dBref) <= (Kp + 2) * U32 * absdB)

    # central differences (h = 1e-3, FP64) on 64 seeded entries of dA and dB.
    # L = <dC, C(A, B)> is linear in A, so only the outputs an entry touches
    # enter: for A[i,k,l,b] these are C[i, :, :, b]; for B[k,j,a,l], C[:, j, a, :].
    rng = np.random.default_rng(44)
    h = 1e-3
    e = p.extents

    def L_slice(Ap, Bp, pts):
        vals = oracle_mod.contract_points(1.0, Ap, p.idx_A, Bp, p.idx_B, 0.0, p.C, p.idx_C, pts)
        return float(np.dot(dC64[tuple(pts.T)], vals))

    jj, aa = np.meshgrid(np.arange(e["j"]), np.arange(e["a"]), indexing="ij")
    for _ in range(64):
        x = tuple(int(rng.integers(0, n)) for n in p.A.shape)  # (i, k, l, b)
        pts = np.stack([np.full(jj.size, x[0]), jj.ravel(), aa.ravel(), np.full(jj.size, x[3])], axis=1)
        Ap, Am = A64.copy(order="F"), A64.copy(order="F")
        Ap[x] += h
        Am[x] -= h
        g_fd = (L_slice(Ap, B64, pts) - L_slice(Am, B64, pts)) / (2 * h)
        tol = (Kp + 2) * U32 * absdA[x] + 1e-6 * (1 + abs(g_fd))
        assert abs(gA[x] - g_fd) <= tol, (x, gA[x], g_fd)
    ii, bb = np.meshgrid(np.arange(e["i"]), np.arange(e["b"]), indexing="ij")
    for _ in range(64):
        x = tuple(int(rng.integers(0, n)) for n in p.B.shape)  # (k, j, a, l)
        pts = np.stack([ii.ravel(), np.full(ii.size, x[1]), np.full(ii.size, x[2]), bb.ravel()], axis=1)
        Bp, Bm = B64.copy(order="F"), B64.copy(order="F")
        Bp[x] += h
        Bm[x] -= h
        g_fd = (L_slice(A64, Bp, pts) - L_slice(A64, Bm, pts)) / (2 * h)
        tol = (Kp + 2) * U32 * absdB[x] + 1e-6 * (1 + abs(g_fd))
        assert abs(gB[x] - g_fd) <= tol, (x, gB[x], g_fd)

    # adjoint identity <dC, C> = <dA, A> = <dB, B> (alpha = 1, beta = 0), each
    # side within the FP32 bound of the results it sums
    s_c = float(np.sum(dC64 * gC))
    s_a = float(np.sum(gA * A64))
    s_b = float(np.sum(gB * B64))
    b_c = float(np.sum(np.abs(dC64) * (K + 2) * U32 * absC))
    b_a = float(np.sum(np.abs(A64) * (Kp + 2) * U32 * absdA))
    b_b = float(np.sum(np.abs(B64) * (Kp + 2) * U32 * absdB))
    slack = 1e-9 * (abs(s_c) + 1)
    assert abs(s_a - s_c) <= b_a + b_c + slack
    assert abs(s_b - s_c) <= b_b + b_c + slack


def test_gradcheck_fp64_small():
    """torch.autograd.gradcheck (FP64 finite differences) through the library,
    with alpha, beta and C0, on tiny random permutations."""
    torch = require_gpu()
    from paper_1607_00291_amd.autograd import Contract
    for seed in range(3):
        p = inputs.random_problem(700 + seed, 2, 1, 2, lo=2, hi=4, beta=0.5, alpha=1.5)
        A = to_dev(p.A).requires_grad_(True)
        B = to_dev(p.B).requires_grad_(True)
        C0 = to_dev(p.C).requires_grad_(True)
        print(f"case gradcheck seed={seed}", flush=True)
        f = lambda a, b, c: Contract.apply(a, p.idx_A, b, p.idx_B, p.idx_C, p.alpha, p.beta, c, "native")
        assert torch.autograd.gradcheck(f, (A, B, C0), eps=1e-6, atol=1e-9, rtol=1e-7)


def test_backward_broadcast_gradient():
    """A gradient with zero strides (sum().backward()) is materialised."""
    torch = require_gpu()
    from paper_1607_00291_amd.autograd import contract
    p = inputs.random_problem(800, 2, 2, 1, lo=2, hi=6)
    A = to_dev(p.A).requires_grad_(True)
    B = to_dev(p.B).requires_grad_(True)
    contract(A, p.idx_A, B, p.idx_B, p.idx_C).sum().backward()
    torch.cuda.synchronize()
    # dA = sum over J of B (with dC = 1): compare with einsum on the host
    ones = np.ones(p.C.shape)
    want = np.einsum(f"{p.idx_C},{p.idx_B}->{p.idx_A}", ones, p.B)
    assert np.max(np.abs(to_host(A.grad) - want)) <= 1e-12 * max(1, p.mnk()[1])
