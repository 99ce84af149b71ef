"""GPU parity of the transpose-transpose-GEMM-transpose baseline (Sec. 5, fig. TTGT):
the permute-copy kernel against the definition of a copy (bit-exact), and the
whole TTGT contraction against the CPU oracle within the FP64 and FP32 bounds."""
import itertools

import numpy as np
import pytest

from paper_1607_00291_amd import inputs
from gpuutil import fp32_componentwise, fp64_bound, require_gpu, to_dev, to_host

pytestmark = pytest.mark.gpu


def _perm_case(shape, perm, dtype, src_gap=1, seed=0):
    """src: column-major with every stride scaled by src_gap (not dense when
    src_gap > 1); dst: column-major in the order `perm` of the dimensions."""
    from paper_1607_00291_amd import tc
    torch = require_gpu()
    rng = np.random.default_rng(seed)
    n = int(np.prod(shape)) if shape else 1
    vals = rng.standard_normal(n).astype(dtype)
    tdt = torch.float64 if dtype == np.float64 else torch.float32
    sstr, s = [], 1
    for x in shape:
        sstr.append(s * src_gap)
        s *= max(x, 1)
    base = torch.zeros(max(1, (s - 1) * src_gap + 1 if n else 1), dtype=tdt, device="cuda")
    src = torch.as_strided(base, shape, sstr)
    if n:
        src.copy_(torch.from_numpy(vals.reshape(shape, order="F")).to("cuda"))
    dstr, s = [0] * len(shape), 1
    for d in perm:
        dstr[d] = s
        s *= max(shape[d], 1)
    dst = torch.empty_strided(shape, dstr, dtype=tdt, device="cuda")
    if n:
        dst.fill_(float("nan"))
    print(f"case permute shape={shape} perm={perm} {np.dtype(dtype).name} gap={src_gap}", flush=True)
    tc.permute_into(src, dst)
    torch.cuda.synchronize()
    got = to_host(dst)
    ref = vals.reshape(shape, order="F")
    # bit-exact copy
    assert got.shape == ref.shape
    assert np.array_equal(got.view(np.uint64 if dtype == np.float64 else np.uint32),
                          np.ascontiguousarray(ref).view(np.uint64 if dtype == np.float64 else np.uint32)
                          .reshape(ref.shape))


@pytest.mark.parametrize("perm", list(itertools.permutations(range(4))))
def test_permute_rank4_every_order(perm):
    _perm_case((70, 5, 65, 3), perm, np.float64, seed=sum(p * 4 ** i for i, p in enumerate(perm)))


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("shape,perm,gap", [
    ((), (), 1),                       # scalar
    ((1000,), (0,), 1),                # one dimension: straight copy
    ((129, 1, 67), (2, 1, 0), 1),      # length-1 dimension, ragged tiles
    ((64, 64), (1, 0), 1),             # one full tile, transposed
    ((130, 7, 3, 66), (0, 3, 1, 2), 1),  # shared unit-stride dimension
    ((33, 40, 17), (1, 2, 0), 3),      # non-dense source
    ((96, 24, 24, 96), (0, 2, 1, 3), 1),  # W[akic] -> (a,i),(k,c) at v=96/o=24
])
def test_permute_cases(shape, perm, gap, dtype):
    _perm_case(shape, perm, dtype, src_gap=gap)


def test_permute_empty():
    from paper_1607_00291_amd import tc
    torch = require_gpu()
    src = torch.zeros((3, 0, 4), dtype=torch.float64, device="cuda")
    dst = torch.empty_strided((3, 0, 4), (4, 12, 1), dtype=torch.float64, device="cuda")
    tc.permute_into(src, dst)
    torch.cuda.synchronize()


def _oracle(oracle_mod, p, A, B, C0, absval=False):
    C = np.array(C0, order="F", copy=True)
    oracle_mod.contract(p.alpha, A, p.idx_A, B, p.idx_B, p.beta, C, p.idx_C, absval=absval)
    return C


def _ttgt(p, dtype):
    from paper_1607_00291_amd import tc
    torch = require_gpu()
    A, B, C = to_dev(p.A, dtype), to_dev(p.B, dtype), to_dev(p.C, dtype)
    t = tc.TTGT(A, p.idx_A, B, p.idx_B, C, p.idx_C, p.alpha, p.beta)
    t.run()
    torch.cuda.synchronize()
    out = to_host(C)
    t.close()
    return out


@pytest.mark.parametrize("case", ["cfg1", "ragged_beta", "ragged_beta0"])
def test_ttgt_fp64_vs_oracle(oracle_mod, case):
    if case == "cfg1":
        p = inputs.cfg1()
    else:
        p = inputs.random_problem(11 if case == "ragged_beta" else 12, lo=3, hi=19,
                                  beta=0.5 if case == "ragged_beta" else 0.0, alpha=-1.25)
    print(f"case ttgt fp64 {case} {p.idx_A},{p.idx_B}->{p.idx_C} mnk={p.mnk()}", flush=True)
    got = _ttgt(p, np.float64)
    ref = _oracle(oracle_mod, p, p.A, p.B, p.C)
    K = p.mnk()[2]
    bound = fp64_bound(K, p.alpha, np.max(np.abs(p.A)), np.max(np.abs(p.B)), p.beta, np.max(np.abs(p.C)))
    err = np.max(np.abs(got - ref))
    assert err <= bound, f"max err {err:.3e} > {bound:.3e}"


def test_ttgt_fp32_vs_oracle(oracle_mod):
    p = inputs.random_problem(13, lo=5, hi=21, beta=1.0)
    print(f"case ttgt fp32 {p.idx_A},{p.idx_B}->{p.idx_C} mnk={p.mnk()}", flush=True)
    A32, B32, C32 = (np.asarray(x, dtype=np.float32, order="K").astype(np.float64, order="K")
                     for x in (p.A, p.B, p.C))
    got = _ttgt(p, np.float32).astype(np.float64)
    ref = _oracle(oracle_mod, p, A32, B32, C32)
    q = inputs.Problem(p.idx_A, p.idx_B, p.idx_C, A32, B32, np.zeros_like(C32, order="F"), 1.0, 0.0)
    absC = _oracle(oracle_mod, q, A32, B32, q.C, absval=True)
    bound = fp32_componentwise(p.mnk()[2], p.alpha, absC, p.beta, C32)
    assert np.all(np.abs(got - ref) <= bound)
