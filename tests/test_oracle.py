"""Pins for the CPU oracle: each test checks it against something other than
itself -- a library routine, a different algorithm from the paper, a closed
form, an exact special case or an invariant of the definition -- so that a
dropped term, a wrong sign, a wrong index or a transposed operand fails here.
"""
import itertools
import math

import numpy as np
import pytest

from paper_1607_00291_amd import inputs

U64 = 2.0 ** -53


def run_oracle(oracle_mod, p, alpha=None, beta=None, absval=False, threads=None):
    C = np.array(p.C, order="F", copy=True)
    oracle_mod.contract(p.alpha if alpha is None else alpha, p.A, p.idx_A, p.B, p.idx_B,
                        p.beta if beta is None else beta, C, p.idx_C, absval=absval, threads=threads)
    return C


def einsum_ref(p):
    s = np.einsum(f"{p.idx_A},{p.idx_B}->{p.idx_C}", p.A, p.B, optimize=False)
    return p.alpha * s + (p.beta * p.C if p.beta != 0 else 0.0)


def fp64_bound(p, K):
    """Two FP64 evaluations in any order differ by <= 2*gamma_K*sum|a||b|."""
    return 2 * K * U64 * K * abs(p.alpha) * np.max(np.abs(p.A)) * np.max(np.abs(p.B)) \
        + 4 * U64 * abs(p.beta) * (np.max(np.abs(p.C)) if p.C.size else 0)


def ttgt(p):
    """The transpose-transpose-GEMM-transpose route (Sec. 5, fig. TTGT):
    explicit permuted copies into A~[I,P] and B~[P,J] (column-major), a plain
    matrix multiply, then a transpose-and-sum back into C's layout."""
    I = [l for l in p.idx_C if l in p.idx_A]
    J = [l for l in p.idx_C if l in p.idx_B]
    P = [l for l in p.idx_A if l in p.idx_B]
    e = p.extents
    m = int(np.prod([e[l] for l in I], dtype=np.int64))
    n = int(np.prod([e[l] for l in J], dtype=np.int64))
    k = int(np.prod([e[l] for l in P], dtype=np.int64))
    At = np.transpose(p.A, [p.idx_A.index(l) for l in I + P]).copy(order="F")
    Bt = np.transpose(p.B, [p.idx_B.index(l) for l in P + J]).copy(order="F")
    Am = At.reshape((m, k), order="F")
    Bm = Bt.reshape((k, n), order="F")
    Cm = np.zeros((m, n))
    for pp in range(k):  # naive rank-1 updates, one contracted index at a time
        Cm += np.outer(Am[:, pp], Bm[pp, :])
    Ct = (p.alpha * Cm).reshape([e[l] for l in I + J], order="F")
    back = np.transpose(Ct, [(I + J).index(l) for l in p.idx_C])
    return back + (p.beta * p.C if p.beta != 0 else 0.0)


SHAPES = [(1, 1, 1), (2, 1, 1), (1, 2, 2), (2, 2, 2), (3, 1, 2), (0, 2, 2), (2, 0, 2), (2, 2, 0),
          (0, 0, 2), (2, 2, 1), (1, 3, 1)]


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("nb", SHAPES)
def test_oracle_matches_einsum(oracle_mod, nb, seed):
    p = inputs.random_problem(seed * 31 + sum(nb), *nb, lo=1, hi=5, beta=0.5 if seed % 2 else 0.0,
                              alpha=1.5 if seed % 3 else 1.0)
    got = run_oracle(oracle_mod, p)
    K = max(p.mnk()[2], 1)
    assert np.max(np.abs(got - einsum_ref(p)), initial=0.0) <= fp64_bound(p, K)


@pytest.mark.parametrize("seed", range(8))
def test_oracle_matches_ttgt(oracle_mod, seed):
    p = inputs.random_problem(100 + seed, 2, 2, 2, lo=1, hi=5, beta=-0.75, alpha=2.0)
    got = run_oracle(oracle_mod, p)
    K = max(p.mnk()[2], 1)
    assert np.max(np.abs(got - ttgt(p))) <= fp64_bound(p, K)


def test_paper_worked_example_shape(oracle_mod):
    """C_abcde := A_cfbd . B_fea with the lengths of the Sec. 5 example
    (A 2x4x3x3, B 4x4x6, C 6x3x2x3x4), checked against TTGT and einsum."""
    ext = {"a": 6, "b": 3, "c": 2, "d": 3, "e": 4, "f": 4}
    rng = np.random.default_rng(7)
    A = inputs.colmajor_from_flat(rng.uniform(-1, 1, 2 * 4 * 3 * 3), (2, 4, 3, 3))
    B = inputs.colmajor_from_flat(rng.uniform(-1, 1, 4 * 4 * 6), (4, 4, 6))
    C = inputs.colmajor((6, 3, 2, 3, 4), fill=0.0)
    p = inputs.Problem("cfbd", "fea", "abcde", A, B, C, 1.0, 0.0, "worked", ext)
    assert C.strides == tuple(8 * s for s in (1, 6, 18, 36, 108))  # the strides the paper lists
    got = run_oracle(oracle_mod, p)
    assert np.max(np.abs(got - ttgt(p))) <= fp64_bound(p, 4)
    assert np.max(np.abs(got - einsum_ref(p))) <= fp64_bound(p, 4)


def test_identity_tensor_is_exact_permutation(oracle_mod):
    """B = delta over (P, J) with n_J = n_P: C is exactly a permuted copy of A."""
    rng = np.random.default_rng(3)
    ext = {"a": 3, "b": 4, "c": 5, "p": 6, "j": 6}
    A = inputs.colmajor_from_flat(rng.standard_normal(3 * 4 * 5 * 6), (5, 6, 3, 4))  # A[c p a b]
    B = np.array(np.eye(6), order="F")  # B[p j]
    C = inputs.colmajor((6, 4, 3, 5), fill=np.nan)  # C[j b a c]
    p = inputs.Problem("cpab", "pj", "jbac", A, B, C, 1.0, 0.0, "identity", ext)
    got = run_oracle(oracle_mod, p)
    want = np.transpose(A, (1, 3, 2, 0))  # A permuted into C's label order j<-p
    assert np.array_equal(got, want)


@pytest.mark.parametrize("seed", range(5))
def test_integer_inputs_are_bitwise_exact(oracle_mod, seed):
    """Small integers: every partial sum is exact in FP64, so any correct
    summation order gives the same bits; the oracle must equal einsum bitwise."""
    p = inputs.random_problem(200 + seed, 2, 2, 2, lo=1, hi=6, integer=True, beta=2.0, alpha=3.0)
    got = run_oracle(oracle_mod, p)
    assert np.array_equal(got, einsum_ref(p))
    assert np.array_equal(got, ttgt(p))


def test_linearity_in_A_and_B(oracle_mod):
    base = inputs.random_problem(11, 2, 1, 2, lo=2, hi=6)
    rng = np.random.default_rng(12)
    A1, A2 = base.A, np.asfortranarray(rng.uniform(-1, 1, base.A.shape))
    B1, B2 = base.B, np.asfortranarray(rng.uniform(-1, 1, base.B.shape))
    a, b = 0.75, -1.25

    def c(A, B):
        q = inputs.Problem(base.idx_A, base.idx_B, base.idx_C, A, B, base.C, 1.0, 0.0, "", base.extents)
        return run_oracle(oracle_mod, q)

    K = base.mnk()[2]
    lhs = c(np.asfortranarray(a * A1 + b * A2), B1)
    rhs = a * c(A1, B1) + b * c(A2, B1)
    assert np.max(np.abs(lhs - rhs)) <= 6 * K * U64 * (abs(a) + abs(b)) * K
    lhs = c(A1, np.asfortranarray(a * B1 + b * B2))
    rhs = a * c(A1, B1) + b * c(A1, B2)
    assert np.max(np.abs(lhs - rhs)) <= 6 * K * U64 * (abs(a) + abs(b)) * K


def test_label_renaming_is_bitwise_invariant(oracle_mod):
    p = inputs.random_problem(21, 2, 2, 2, lo=2, hi=5, beta=0.5)
    ren = dict(zip("abcdef", "uvwxyz"))
    q = inputs.Problem("".join(ren[l] for l in p.idx_A), "".join(ren[l] for l in p.idx_B),
                       "".join(ren[l] for l in p.idx_C), p.A, p.B, p.C, p.alpha, p.beta)
    assert np.array_equal(run_oracle(oracle_mod, p), run_oracle(oracle_mod, q))


def test_storage_permutations(oracle_mod):
    """Moving labels together with the data: permuting C's storage is bitwise
    invariant (same sums, same order); permuting A or B is within the bound."""
    p = inputs.random_problem(31, 2, 2, 2, lo=2, hi=5, beta=0.0)
    ref = run_oracle(oracle_mod, p)
    K = p.mnk()[2]
    for perm in itertools.permutations(range(4)):
        idx_C = "".join(p.idx_C[i] for i in perm)
        C = np.asfortranarray(np.zeros([p.C.shape[i] for i in perm]))
        q = inputs.Problem(p.idx_A, p.idx_B, idx_C, p.A, p.B, C, p.alpha, p.beta)
        got = run_oracle(oracle_mod, q)
        assert np.array_equal(np.transpose(got, np.argsort(perm)), ref)
        idx_A = "".join(p.idx_A[i] for i in perm)
        A = np.asfortranarray(np.transpose(p.A, perm))
        q = inputs.Problem(idx_A, p.idx_B, p.idx_C, A, p.B, p.C, p.alpha, p.beta)
        got = run_oracle(oracle_mod, q)
        assert np.max(np.abs(got - ref)) <= fp64_bound(p, K)


def test_gemm_special_case_textbook_loop(oracle_mod):
    """One index per bundle: C_ij = sum_p A_ip B_pj, checked against a plain
    Python triple loop (pure-Python, so no shared library arithmetic)."""
    rng = np.random.default_rng(41)
    m, n, k = 5, 4, 7
    A = np.asfortranarray(rng.uniform(-1, 1, (m, k)))
    B = np.asfortranarray(rng.uniform(-1, 1, (k, n)))
    C0 = np.asfortranarray(rng.uniform(-1, 1, (m, n)))
    alpha, beta = 1.5, -0.5
    want = np.empty((m, n))
    for i in range(m):
        for j in range(n):
            s = 0.0
            for q in range(k):
                s = s + A[i, q] * B[q, j]
            want[i, j] = alpha * s + beta * C0[i, j]
    p = inputs.Problem("ip", "pj", "ij", A, B, C0, alpha, beta)
    got = run_oracle(oracle_mod, p)
    assert np.array_equal(got, want)  # same order, same roundings
    # transposed operand orders give the same numbers
    q = inputs.Problem("pi", "jp", "ji", np.asfortranarray(A.T), np.asfortranarray(B.T),
                       np.asfortranarray(C0.T), alpha, beta)
    assert np.array_equal(run_oracle(oracle_mod, q).T, want)


def test_dot_and_outer_products(oracle_mod):
    rng = np.random.default_rng(51)
    x = np.asfortranarray(rng.uniform(-1, 1, (3, 4)))
    y = np.asfortranarray(rng.uniform(-1, 1, (4, 3)))
    C = np.zeros((), order="F")
    p = inputs.Problem("ab", "ba", "", x, y, C, 1.0, 0.0)
    got = run_oracle(oracle_mod, p)
    assert abs(float(got) - math.fsum((x * y.T).ravel())) <= 24 * U64 * 12
    # outer product: a single product per output, exact
    u = rng.uniform(-1, 1, 5)
    v = rng.uniform(-1, 1, 3)
    C = np.asfortranarray(np.zeros((3, 5)))
    p = inputs.Problem("a", "b", "ba", u, v, C, 1.0, 0.0)
    assert np.array_equal(run_oracle(oracle_mod, p), np.outer(v, u))


def test_alpha_beta_semantics(oracle_mod):
    p = inputs.random_problem(61, 2, 1, 1, lo=2, hi=4)
    C = np.full(p.C.shape, np.nan, order="F")
    q = inputs.Problem(p.idx_A, p.idx_B, p.idx_C, p.A, p.B, C, 1.0, 0.0)
    assert not np.isnan(run_oracle(oracle_mod, q)).any()  # beta = 0: C not read
    C0 = np.asfortranarray(np.random.default_rng(1).uniform(-1, 1, p.C.shape))
    q = inputs.Problem(p.idx_A, p.idx_B, p.idx_C, p.A, p.B, C0, 0.0, 2.0)
    assert np.array_equal(run_oracle(oracle_mod, q), 2.0 * C0)
    # empty contracted bundle extent: C := beta * C
    A = np.zeros((3, 0), order="F")
    B = np.zeros((0, 2), order="F")
    q = inputs.Problem("ip", "pj", "ij", A, B, np.asfortranarray(C0[:3, :2] if C0.ndim == 2 else np.ones((3, 2))),
                       1.0, 0.5)
    assert np.array_equal(run_oracle(oracle_mod, q), 0.5 * q.C)


def test_alpha_zero_reads_neither_operand(oracle_mod):
    """alpha = 0 (Sec. 3 alpha/beta update, read with the BLAS convention):
    C := beta * C exactly, and NaN or Inf in A or B never reach C; with
    beta = 0 as well, C := 0 whatever it held."""
    p = inputs.random_problem(62, 2, 2, 2, lo=2, hi=5, beta=1.0)
    A = np.array(p.A, order="F", copy=True)
    B = np.array(p.B, order="F", copy=True)
    A.reshape(-1, order="F")[::3] = np.nan
    B.reshape(-1, order="F")[1::4] = np.inf
    C0 = np.asfortranarray(np.random.default_rng(2).uniform(-1, 1, p.C.shape))
    q = inputs.Problem(p.idx_A, p.idx_B, p.idx_C, A, B, C0, 0.0, -1.5)
    assert np.array_equal(run_oracle(oracle_mod, q), -1.5 * C0)
    pts = np.array(list(np.ndindex(*C0.shape)), dtype=np.int64)
    vals = oracle_mod.contract_points(0.0, A, p.idx_A, B, p.idx_B, -1.5, C0, p.idx_C, pts)
    assert np.array_equal(vals, np.array([-1.5 * C0[tuple(t)] for t in pts]))
    Cn = np.full(C0.shape, np.nan, order="F")
    q = inputs.Problem(p.idx_A, p.idx_B, p.idx_C, A, B, Cn, 0.0, 0.0)
    assert np.array_equal(run_oracle(oracle_mod, q), np.zeros(C0.shape))


def test_absval_variant(oracle_mod):
    p = inputs.random_problem(71, 2, 2, 1, lo=2, hi=5)
    got = run_oracle(oracle_mod, p, absval=True)
    want = np.einsum(f"{p.idx_A},{p.idx_B}->{p.idx_C}", np.abs(p.A), np.abs(p.B), optimize=False)
    assert np.max(np.abs(got - want)) <= fp64_bound(p, p.mnk()[2])


def test_points_match_full(oracle_mod):
    p = inputs.random_problem(81, 2, 2, 2, lo=2, hi=5, beta=0.25)
    full = run_oracle(oracle_mod, p)
    pts = np.array(list(np.ndindex(*p.C.shape)), dtype=np.int64)
    vals = oracle_mod.contract_points(p.alpha, p.A, p.idx_A, p.B, p.idx_B, p.beta, p.C, p.idx_C, pts)
    assert np.array_equal(vals, np.array([full[tuple(t)] for t in pts]))


def test_thread_count_does_not_change_bits(oracle_mod):
    p = inputs.random_problem(91, 2, 2, 2, lo=3, hi=7)
    assert np.array_equal(run_oracle(oracle_mod, p, threads=1), run_oracle(oracle_mod, p, threads=4))


@pytest.mark.parametrize("bad", [
    ("ab", "bc", "ad"),    # d only in C, c only in B
    ("aab", "bc", "ac"),   # repeated label in A
    ("ab", "bc", "abc"),   # b in all three (batch index)
])
def test_rejects_labels_outside_the_definition(oracle_mod, bad):
    ia, ib, ic = bad
    A = np.zeros([2] * len(ia), order="F")
    B = np.zeros([2] * len(ib), order="F")
    C = np.zeros([2] * len(ic), order="F")
    with pytest.raises(ValueError):
        oracle_mod.contract(1.0, A, ia, B, ib, 0.0, C, ic)


def test_rejects_extent_mismatch(oracle_mod):
    with pytest.raises(ValueError):
        oracle_mod.contract(1.0, np.zeros((2, 3), order="F"), "ab", np.zeros((4, 2), order="F"), "bc",
                            0.0, np.zeros((2, 2), order="F"), "ac")
