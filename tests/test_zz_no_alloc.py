"""The allocation-free entry point (tc_contract_noalloc) against tc_contract
on the same inputs: two calls in a row on one GPU, the second with a smaller
problem (the static offset array keeps the first call's contents), each
bitwise equal to tc_contract's result (same kernels, same tile, the same
offset vectors built on the device instead of uploaded; where tc_contract runs
the packed split tile, which needs a workspace, the allocation-free call runs
its twin that splits in its own producer waves, with the same bits)."""
import numpy as np
import pytest

from paper_1607_00291_amd import inputs
from gpuutil import require_gpu, to_dev, to_host

pytestmark = pytest.mark.gpu


def both(p, dtype, mode="native"):
    """(tc_contract result, tc_contract_noalloc result) on fresh outputs."""
    torch = require_gpu()
    from paper_1607_00291_amd import tc
    A, B = to_dev(p.A, dtype), to_dev(p.B, dtype)
    C1, C2 = to_dev(p.C, dtype), to_dev(p.C, dtype)
    tc.contract(A, p.idx_A, B, p.idx_B, p.idx_C, alpha=p.alpha, beta=p.beta, out=C1, mode=mode)
    tc.contract_noalloc(A, p.idx_A, B, p.idx_B, p.idx_C, C2, alpha=p.alpha, beta=p.beta, mode=mode)
    torch.cuda.synchronize()
    return to_host(C1), to_host(C2)


@pytest.mark.parametrize("dtype,mode", [(np.float64, "native"), (np.float32, "native"), (np.float32, "split_bf16x3")])
def test_noalloc_matches_contract_large_then_small(dtype, mode):
    big = inputs.cfg2()
    small = inputs.random_problem(8100, 2, 2, 2, lo=3, hi=17, beta=0.5, alpha=1.25)
    # unit strides of A and B on different contracted indices: the device
    # builds the sub-blocked k order of the plan
    conflict = inputs.p_conflict_problem(8102, {"e": 13, "g": 3, "f": 10, "i": 40, "j": 30}, beta=0.5)
    for p in (big, small, conflict):
        print(f"case noalloc {np.dtype(dtype).name} {mode} {p.name} mnk={p.mnk()}", flush=True)
        ref, got = both(p, dtype, mode)
        assert np.array_equal(ref, got), p.name


def test_noalloc_alpha_zero_and_empty_contracted_extent():
    torch = require_gpu()
    from paper_1607_00291_amd import tc
    p = inputs.random_problem(8101, 2, 2, 2, lo=2, hi=9, beta=-2.0, alpha=0.0)
    print("case noalloc alpha=0", flush=True)
    ref, got = both(p, np.float64)
    assert np.array_equal(ref, got) and np.array_equal(got, -2.0 * p.C)
    C0 = np.asfortranarray(np.random.default_rng(3).uniform(-1, 1, (5, 6)))
    A = torch.zeros((5, 0), dtype=torch.float64, device="cuda")
    B = torch.zeros((0, 6), dtype=torch.float64, device="cuda")
    Cd = to_dev(C0)
    tc.contract_noalloc(A, "ip", B, "pj", "ij", Cd, alpha=1.0, beta=0.5)
    torch.cuda.synchronize()
    assert np.array_equal(to_host(Cd), 0.5 * C0)
