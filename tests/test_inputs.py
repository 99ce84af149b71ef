"""The seeded input generators: reproducibility and the shape of the
random-contraction sweep instances (Sec. 9.2)."""
import numpy as np
import pytest

from paper_1607_00291_amd import inputs


@pytest.mark.parametrize("target,dims", [(4096, 1), (4096, 2), (4096, 3), (50, 3), (7, 2), (300, 3)])
def test_split_extent(target, dims):
    for seed in range(20):
        lens = inputs.split_extent(np.random.default_rng(seed), target, dims)
        assert len(lens) == dims and all(x >= (1 if dims == 1 else 2) for x in lens)
        prod = int(np.prod(lens))
        if dims == 1:
            assert prod == target
        else:  # the last extent absorbs the rounding, unless the minimum of 2 binds
            # (then the product can exceed the target by up to about 2.5x)
            assert target / 2 - 1 <= prod <= 2.5 * target + 8


def test_sweep_instance_structure():
    for seed in range(50):
        rng = np.random.default_rng(seed)
        ext, ia, ib, ic = inputs.sweep_instance(rng, 1000, 700, 40)
        I = set(ia) & set(ic)
        J = set(ib) & set(ic)
        P = set(ia) & set(ib)
        # every label in exactly two operands, each bundle one to three labels
        for lab in ext:
            assert (lab in ia) + (lab in ib) + (lab in ic) == 2
        assert 1 <= len(I) <= 3 and 1 <= len(J) <= 3 and 1 <= len(P) <= 3
        assert len(set(ia)) == len(ia) and len(set(ib)) == len(ib) and len(set(ic)) == len(ic)
        for bundle, target in ((I, 1000), (J, 700), (P, 40)):
            prod = int(np.prod([ext[l] for l in bundle]))
            assert target / 2 - 1 <= prod <= 2.5 * target + 8


def test_sweep_problem_reproducible():
    p1 = inputs.sweep_problem(5, 120, 90, 30)
    p2 = inputs.sweep_problem(5, 120, 90, 30)
    assert (p1.idx_A, p1.idx_B, p1.idx_C) == (p2.idx_A, p2.idx_B, p2.idx_C)
    assert np.array_equal(p1.A, p2.A) and np.array_equal(p1.B, p2.B)
    assert p1.A.flags.f_contiguous and p1.B.flags.f_contiguous
    assert np.all(p1.C == 0) and p1.beta == 0.0
    m, n, k = p1.mnk()
    assert m * n * k > 0
