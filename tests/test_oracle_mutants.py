"""Plant plausible mistakes in copies of the oracle source (on the CPU only)
and check that the pins catch every one: a dropped term, a wrong sign, a wrong
stride, a transposed operand index, a lost beta term, an alpha = 0 update that
still forms the sum or drops beta."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

from paper_1607_00291_amd import inputs

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "tc_oracle.c")

MUTANTS = {
    "dropped_term": ("double prod = a * b;", "double prod = (q == 0) ? 0.0 : a * b;"),
    "wrong_sign": ("sum = sum + prod;", "sum = sum - prod;"),
    "wrong_stride": ("offB += p[i] * pr->psB[i];", "offB += p[i] * pr->psA[i];"),
    "transposed_free_index": ("pr->fsA[pr->nf] = (a >= 0) ? strA[a] : 0;",
                              "pr->fsA[pr->nf] = (a >= 0) ? strA[ndA - 1 - a] : 0;"),
    "lost_beta": ("if (beta != 0.0) r = r + beta * c0;", "(void)c0;"),
    "alpha_zero_still_sums": ("        if (alpha == 0.0) {\n            C[offC] = scale_only",
                              "        if (alpha == 0.0 && 0) {\n            C[offC] = scale_only"),
    "alpha_zero_drops_beta": ("return beta != 0.0 ? beta * c0 : 0.0;", "return c0;"),
}


def build_mutant(tmp_path, name):
    old, new = MUTANTS[name]
    text = open(SRC).read()
    assert text.count(old) == 1, name
    src = tmp_path / f"{name}.c"
    src.write_text(text.replace(old, new))
    so = tmp_path / f"{name}.so"
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fPIC", "-shared",
                           str(src), "-o", str(so), "-lm"])
    lib = ctypes.CDLL(str(so))
    return lib


def call(lib, p):
    C = np.array(p.C, order="F", copy=True)

    def d(arr, lab):
        return [arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), arr.ndim,
                (ctypes.c_int64 * max(arr.ndim, 1))(*arr.shape),
                (ctypes.c_int64 * max(arr.ndim, 1))(*[s // 8 for s in arr.strides]), lab.encode()]

    lib.oracle_contract.restype = ctypes.c_int
    st = lib.oracle_contract(ctypes.c_double(p.alpha), *d(p.A, p.idx_A), *d(p.B, p.idx_B),
                             ctypes.c_double(p.beta), *d(C, p.idx_C), 0, 1)
    assert st == 0
    return C


def pins_pass(lib):
    """The einsum and identity-tensor pins of test_oracle, on a few problems."""
    for seed in range(4):
        p = inputs.random_problem(500 + seed, 2, 2, 2, lo=2, hi=5, beta=0.5)
        want = np.einsum(f"{p.idx_A},{p.idx_B}->{p.idx_C}", p.A, p.B, optimize=False) * p.alpha + p.beta * p.C
        if np.max(np.abs(call(lib, p) - want)) > 1e-12:
            return False
    # alpha = 0: C := beta * C, with NaN in A never read
    p = inputs.random_problem(510, 2, 2, 2, lo=2, hi=5, beta=0.5)
    A = np.array(p.A, order="F", copy=True)
    A.reshape(-1, order="F")[::2] = np.nan
    q = inputs.Problem(p.idx_A, p.idx_B, p.idx_C, A, p.B, p.C, 0.0, -0.5)
    if not np.array_equal(call(lib, q), -0.5 * p.C):
        return False
    return True


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistake(tmp_path, name):
    assert not pins_pass(build_mutant(tmp_path, name))


def test_unmutated_copy_passes(tmp_path):
    so = tmp_path / "clean.so"
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fPIC", "-shared", SRC,
                           "-o", str(so), "-lm"])
    assert pins_pass(ctypes.CDLL(str(so)))
