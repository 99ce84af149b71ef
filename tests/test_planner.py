"""Host-side planner and C-ABI tests (no GPU): scatter vectors and block
strides against the paper's worked example, the reordering heuristic on the
workloads, brute-force addressing, and argument validation."""
import ctypes
import itertools
import json
import os
import re

import numpy as np
import pytest

import korder
from paper_1607_00291_amd import inputs, tc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLDEN = os.path.join(ROOT, "tests", "golden")


def strides_of(a):
    return [s // a.itemsize for s in a.strides]


def describe(p, dtype=tc.TC_F64, mode=tc.TC_NATIVE):
    return tc.describe(p.A.shape, strides_of(p.A), p.idx_A, p.B.shape, strides_of(p.B), p.idx_B,
                       p.C.shape, strides_of(p.C), p.idx_C, dtype, mode)


def test_library_exports_every_declared_symbol():
    header = open(os.path.join(ROOT, "include", "tc.h")).read()
    declared = set(re.findall(r"^(?:int|const char\*)\s+(tc_\w+)\(", header, re.M))
    assert declared == set(tc.EXPORTS)
    L = ctypes.CDLL(tc.LIB_PATH)
    for name in declared:
        assert hasattr(L, name), name


# --------------------------------------------------------------------------
# worked example of Sec. 6.1 / 6.2 (fig. bsm): C_abcde, lengths 6x3x2x3x4,
# strides 1, 6, 18, 36, 108, bundles I = cdb and J = ae, blocking 4
# --------------------------------------------------------------------------

def load_golden():
    with open(os.path.join(GOLDEN, "worked_example.json")) as fh:
        return json.load(fh)


def test_worked_example_scatter_vectors():
    g = load_golden()
    ln, st = g["lens"], g["strides"]
    I = [g["labels"].index(l) for l in g["I"]]
    J = [g["labels"].index(l) for l in g["J"]]
    rscat = tc.scatter_vector([ln[i] for i in I], [st[i] for i in I])
    cscat = tc.scatter_vector([ln[j] for j in J], [st[j] for j in J])
    # the printed stretch of cscat: 0..5, then a jump to 108..113
    assert cscat[:12] == g["cscat_prefix"]
    # the printed formula of rscat / cscat (eq. cscat-c) with floor division
    na, nb, nc, nd, ne = ln
    for Ibar in range(nc * nd * nb):
        want = (Ibar % nc) * na * nb + ((Ibar // nc) % nd) * na * nb * nc + ((Ibar // (nc * nd)) % nb) * na
        assert rscat[Ibar] == want
    for Jbar in range(na * ne):
        assert cscat[Jbar] == (Jbar % na) + ((Jbar // na) % ne) * na * nb * nc * nd
    # short stretches of rscat behave like a constant stride n_a n_b = 18
    assert rscat[1] - rscat[0] == g["rscat_short_stride"]


def test_worked_example_block_strides_and_53_percent():
    g = load_golden()
    ln, st = g["lens"], g["strides"]
    I = [g["labels"].index(l) for l in g["I"]]
    J = [g["labels"].index(l) for l in g["J"]]
    rscat = tc.scatter_vector([ln[i] for i in I], [st[i] for i in I])
    cscat = tc.scatter_vector([ln[j] for j in J], [st[j] for j in J])
    rbs = tc.block_strides(rscat, g["mR"])
    cbs = tc.block_strides(cscat, g["nR"])
    # every valid block stride is the constant difference of its block
    for bs, scat, b in ((rbs, rscat, g["mR"]), (cbs, cscat, g["nR"])):
        for i, s in enumerate(bs):
            blk = scat[i * b:(i + 1) * b]
            diffs = {y - x for x, y in zip(blk, blk[1:])}
            assert (s != 0) == (len(diffs) <= 1 and min(diffs, default=1) > 0)
            if s:
                assert diffs <= {s}
    both = sum(1 for r in rbs for c in cbs if r and c)
    total = len(rbs) * len(cbs)
    assert round(100 * both / total) == g["percent_constant_stride_tiles"]


def test_block_strides_edge_cases():
    assert tc.block_strides([5], 4) == [1]                 # one entry
    assert tc.block_strides([0, 3, 6, 9, 12], 4) == [3, 1]  # last block of one entry
    assert tc.block_strides([0, 2, 4, 5], 4) == [0]
    assert tc.block_strides([9, 6, 3, 0], 4) == [0]        # negative differences: no stride
    assert tc.block_strides([0, 0, 0], 4) == [0]           # zero difference: no stride
    assert tc.block_strides([], 4) == []


@pytest.mark.parametrize("seed", range(10))
def test_scatter_vectors_address_every_element(seed):
    """Brute force: for every (I, J, P) index of a random small contraction,
    the planned scatter vectors give the element offsets of A, B and C."""
    p = inputs.random_problem(300 + seed, 2, 2, 2, lo=1, hi=5)
    d = describe(p)
    if d["noop"]:
        return
    X, Y = (p.B, p.A) if d["swapped"] else (p.A, p.B)
    ix, iy = (p.idx_B, p.idx_A) if d["swapped"] else (p.idx_A, p.idx_B)

    def walk(dims):
        """label values of every linear index of a planned bundle"""
        lens = [x["len"] for x in dims]
        out = []
        for lin in range(int(np.prod(lens, dtype=np.int64)) if dims else 1):
            vals, r = {}, lin
            for x in dims:
                v = r % x["len"]
                r //= x["len"]
                # a folded dim covers several labels, first fastest
                for l in x["labels"]:
                    n = p.extents[l]
                    vals[l] = v % n
                    v //= n
            out.append(vals)
        return out

    def off(arr, labels, vals):
        return sum(vals[l] * s for l, s in zip(labels, strides_of(arr)) if l in vals)

    Iv, Jv = walk(d["I"]), walk(d["J"])
    Pv = korder.p_label_values(d["P"], d["k_sub"], p.extents)
    for mi, a in enumerate(Iv):
        assert d["rscat_X"][mi] == off(X, ix, a)
        assert d["rscat_C"][mi] == off(p.C, p.idx_C, a)
    for nj, b in enumerate(Jv):
        assert d["cscat_Y"][nj] == off(Y, iy, b)
        assert d["cscat_C"][nj] == off(p.C, p.idx_C, b)
    for kp, c in enumerate(Pv):
        assert d["cscat_X"][kp] == off(X, ix, c)
        assert d["rscat_Y"][kp] == off(Y, iy, c)


def test_heuristic_cfg1():
    """The paper's heuristic orders J = (c, d) by C's strides; B[dfce] has its
    unit stride on d, so the GPU amendment moves d to the front of J and B is
    gathered with unit stride along n."""
    d = describe(inputs.cfg1())
    assert not d["swapped"]
    assert d["paper_order"] == "ab|cd|ef"
    assert [x["labels"] for x in d["I"]] == ["a", "b"]
    assert [x["labels"] for x in d["J"]] == ["d", "c"]
    assert [x["labels"] for x in d["P"]] == ["e", "f"]
    assert d["unit_moves"] == 1 and d["J"][0]["sY"] == 1
    assert (d["m"], d["n"], d["k"]) == (256, 256, 256)
    assert d["x_lanes"] == "m" and d["y_lanes"] == "n"


def test_heuristic_cfg2_gpu_amendment():
    """Sort by A's stride would give P = (k, c); T[cbkj] has its unit stride
    on c, so the amended order is P = (c, k) and T is gathered along k."""
    d = describe(inputs.cfg2())
    assert not d["swapped"]
    assert d["paper_order"] == "ai|bj|kc" and d["unit_moves"] == 0
    assert [x["labels"] for x in d["I"]] == ["a", "i"]
    assert [x["labels"] for x in d["J"]] == ["b", "j"]
    assert [x["labels"] for x in d["P"]] == ["c", "k"]
    assert d["P"][0]["sY"] == 1
    assert (d["m"], d["n"], d["k"]) == (2304, 2304, 2304)
    assert d["x_lanes"] == "m" and d["y_lanes"] == "k"
    assert d["k_blocks_regular_x"] == d["k_blocks"] and d["k_blocks_regular_y"] == d["k_blocks"]


def test_heuristic_cfg4_fold_and_backward():
    p = inputs.cfg4()
    d = describe(p)
    # J = (j, a) is contiguous in C and B: folded into one index of length 2048
    assert [x["labels"] for x in d["J"]] == ["ja"]
    assert d["J"][0]["len"] == 2048
    assert (d["m"], d["n"], d["k"]) == (2048, 2048, 1024)
    assert d["folds"] >= 1
    # dA[iklb] = dC[ijab] . B[kjal]  (contracted j, a)
    dA = inputs.colmajor(p.A.shape, fill=0.0)
    q = inputs.Problem("ijab", "kjal", "iklb", p.dC, p.B, dA, 1.0, 0.0, "dA", p.extents)
    d = describe(q)
    assert (d["m"], d["n"], d["k"]) == (2048, 1024, 2048)
    # dB[kjal] = A[iklb] . dC[ijab]  (contracted i, b)
    dB = inputs.colmajor(p.B.shape, fill=0.0)
    q = inputs.Problem("iklb", "ijab", "kjal", p.A, p.dC, dB, 1.0, 0.0, "dB", p.extents)
    d = describe(q)
    assert d["m"] * d["n"] == 1024 * 2048 and d["k"] == 2048


def test_unit_stride_index_moved_to_front_of_free_bundle():
    """A[u v p] B[p j] -> C[v u j]: C's unit stride is on v, A's on u (Sec. 7.3
    notes that no order gives unit stride in both).  The paper's order is
    I = (v, u); the planner moves u to the front so that A's gather lanes run
    with unit stride (the C tile is written once; A's slivers are gathered by
    every tile column), and the scatter vectors still address every element."""
    e = {"u": 32, "v": 48, "p": 40, "j": 24}
    A = inputs.colmajor((32, 48, 40))
    B = inputs.colmajor((40, 24))
    C = inputs.colmajor((48, 32, 24))
    p = inputs.Problem("uvp", "pj", "vuj", A, B, C, 1.0, 0.0, "unit-first", e)
    d = describe(p)
    assert d["paper_order"] == "vu|j|p"
    assert [x["labels"] for x in d["I"]] == ["u", "v"] and d["unit_moves"] == 1
    assert d["x_lanes"] == "m" and d["I"][0]["sX"] == 1
    # rscat_X / rscat_C still pair each m with the same (u, v)
    rX, rC = d["rscat_X"], d["rscat_C"]
    for m in range(0, 32 * 48, 37):
        u, v = m % 32, m // 32
        assert rX[m] == u + 32 * v and rC[m] == v + 48 * u


@pytest.mark.parametrize("dtype", [tc.TC_F64, tc.TC_F32])
@pytest.mark.parametrize("ext", [(7, 5, 3), (8, 8, 2), (2, 9, 1), (13, 3, 4)])
def test_sub_blocked_k_order_when_unit_strides_disagree_in_P(dtype, ext):
    """A[e g f i] and B[f j e g] (e unit-stride in A, f in B, both contracted):
    no P order makes both operands contiguous along k, so the plan walks k in
    sub-blocks over (e, f) (GPU amendment 3).  The description states the
    sub-blocks; the k vectors address exactly the elements of that order
    (checked against the tensors' own strides), and each (e, f, g) appears
    once; every KT-sized k stage of either operand then reads runs of at
    least min(4, extent) contiguous elements."""
    ne, nf, ng = ext
    ni, nj = 6, 5
    A = np.zeros((ne, ng, nf, ni), order="F")
    B = np.zeros((nf, nj, ne, ng), order="F")
    C = np.zeros((ni, nj), order="F")
    d = tc.describe(A.shape, strides_of(A), "egfi", B.shape, strides_of(B), "fjeg", C.shape, strides_of(C), "ij",
                    dtype=dtype)
    P = d["P"]
    labs = "".join(x["labels"] for x in P)
    ks = d["k_sub"]
    if ne == 1 or nf == 1:
        return
    # sub-blocks only when B's best plain gather (along J[0] or P[0]) is
    # strided by more than the run the sub-blocks would give it
    ia = next(i for i, x in enumerate(P) if x["sX"] == 1)
    ib = next(i for i, x in enumerate(P) if x["sY"] == 1)
    La, Lb = P[ia]["len"], P[ib]["len"]  # e and f, possibly folded with g
    bx = min(4 if dtype == tc.TC_F64 else 8, La)
    by = min(d["KT"] // bx, Lb)
    ybest = min(x for x in (d["J"][0]["sY"], P[0]["sY"]) if x > 0)
    if ybest <= by:
        assert ks is None, d
        return
    assert ks is not None, d
    assert (ks["a"], ks["b"], ks["bx"], ks["by"]) == (ia, ib, bx, by)
    assert P[ks["a"]]["labels"][0] == "e" and P[ks["b"]]["labels"][0] == "f"
    assert d["x_lanes"] == "k" and d["y_lanes"] == "k"
    ext_of = {"e": ne, "f": nf, "g": ng}
    vals = korder.p_label_values(P, ks, ext_of)
    assert sorted((v["e"], v["f"], v.get("g", 0)) for v in vals) == sorted(
        itertools.product(range(ne), range(nf), range(ng)))
    sa, sb = strides_of(A), strides_of(B)
    for kp, v in enumerate(vals):
        assert d["cscat_X"][kp] == v["e"] * sa[0] + v.get("g", 0) * sa[1] + v["f"] * sa[2]
        assert d["rscat_Y"][kp] == v["f"] * sb[0] + v["e"] * sb[2] + v.get("g", 0) * sb[3]
    # contiguous runs inside each k stage, for both operands, where the
    # sub-blocks tile the plane exactly and fill a stage
    KT = d["KT"]
    if La % ks["bx"] or Lb % ks["by"] or ks["bx"] * ks["by"] != KT:
        return
    for vec, run in ((d["cscat_X"], ks["bx"]), (d["rscat_Y"], ks["by"])):
        for s0 in range(0, len(vec), KT):
            stage = sorted(vec[s0:s0 + KT])
            longest, cur = 1, 1
            for x, y in zip(stage, stage[1:]):
                cur = cur + 1 if y == x + 1 else 1
                longest = max(longest, cur)
            assert longest >= min(run, len(stage)), (labs, s0, stage)


def test_swap_when_C_unit_stride_in_J():
    A = inputs.colmajor((5, 7))   # A[i p]
    B = inputs.colmajor((7, 9))   # B[p j]
    C = inputs.colmajor((9, 5))   # C[j i]: unit stride on j
    p = inputs.Problem("ip", "pj", "ji", A, B, C)
    d = describe(p)
    assert d["swapped"]
    assert [x["labels"] for x in d["I"]] == ["j"] and d["I"][0]["sC"] == 1


def test_length_one_dims_dropped():
    A = inputs.colmajor((5, 1, 7))
    B = inputs.colmajor((7, 1, 9))
    C = inputs.colmajor((5, 1, 1, 9))
    p = inputs.Problem("iqp", "prj", "iqrj", A, B, C)
    d = describe(p)
    assert d["dropped"] == 2  # q (in A and C) and r (in B and C)
    assert (d["m"], d["n"], d["k"]) == (5, 9, 7)


def test_tile_table():
    for dt, mode in ((tc.TC_F64, tc.TC_NATIVE), (tc.TC_F32, tc.TC_NATIVE)):
        n = tc.tile_count(dt, mode)
        assert n >= 1
        for t in range(n):
            MT, NT, KT, waves = tc.tile_info(dt, mode, t)
            assert MT % 16 == 0 and NT % 16 == 0 and KT % 4 == 0 and waves >= 1


def test_packed_split_tile_workspace_and_choice():
    """The packed split tile needs one panel of 2 planes x 144 rows x 32
    bf16 per operand row (column) panel and k block; the cost model picks it
    for the split mode at the v=96/o=24 shape, and no other tile (or mode)
    reports a workspace."""
    p = inputs.cfg2()
    d = describe(p, tc.TC_F32, tc.TC_SPLIT_BF16X3)
    m, n, k = p.mnk()
    assert d["layout"] == 4 and (d["MT"], d["NT"], d["KT"]) == (144, 144, 32)
    panels = (-(-m // 144) + -(-n // 144)) * -(-k // 32)
    assert d["workspace_bytes"] == panels * 2 * 144 * 32 * 2 == 2 * 2304 * 2304 * 4
    assert describe(p, tc.TC_F32, tc.TC_NATIVE)["workspace_bytes"] == 0
    assert describe(p)["workspace_bytes"] == 0
    # ragged: partial panels are whole panels in the workspace
    e = {"a": 97, "b": 5, "c": 99, "d": 3, "e": 98, "f": 2}
    q = inputs.Problem("aebf", "dfce", "abcd", inputs.colmajor(inputs.shape_of("aebf", e)),
                       inputs.colmajor(inputs.shape_of("dfce", e)), inputs.colmajor(inputs.shape_of("abcd", e)),
                       1.0, 0.0, "ragged", e)
    m, n, k = q.mnk()
    d = describe(q, tc.TC_F32, tc.TC_SPLIT_BF16X3)
    if d["layout"] == 4:
        assert d["workspace_bytes"] == (-(-m // 144) + -(-n // 144)) * -(-k // 32) * 18432
    else:
        assert d["workspace_bytes"] == 0
    # above 8 GiB of panels the model leaves the packed tile out (m = n = 2^18,
    # k = 2^13: about 17 GB of panels); descriptors only, nothing is allocated
    big = tc.describe((1 << 18, 1 << 13), (1, 1 << 18), "ik", (1 << 13, 1 << 18), (1, 1 << 13), "kj",
                      (1 << 18, 1 << 18), (1, 1 << 18), "ij", tc.TC_F32, tc.TC_SPLIT_BF16X3)
    assert big["layout"] != 4 and big["workspace_bytes"] == 0


# --------------------------------------------------------------------------
# argument validation through the C ABI (no GPU work is started)
# --------------------------------------------------------------------------

def plan_status(shape_A, st_A, ia, shape_B, st_B, ib, shape_C, st_C, ic, dtype=tc.TC_F64, mode=tc.TC_NATIVE):
    try:
        tc.Plan(shape_A, st_A, ia, shape_B, st_B, ib, shape_C, st_C, ic, dtype, mode).close()
        return 0
    except tc.TCError as e:
        return e.status


def test_abi_errors():
    L = tc.lib()
    ok = ((2, 3), (1, 2), "ip", (3, 4), (1, 3), "pj", (2, 4), (1, 2), "ij")
    assert plan_status(*ok) == 0
    assert plan_status((2, 3), (1, 2), "ii", (3, 4), (1, 3), "pj", (2, 4), (1, 2), "ij") == -3  # repeated
    assert plan_status((2, 3), (1, 2), "ip", (3, 4), (1, 3), "pj", (2, 4), (1, 2), "ix") == -3  # x only in C
    assert plan_status((2, 3), (1, 2), "ip", (3, 4), (1, 3), "pi", (2, 4), (1, 2), "ij") == -3  # i in all / j in one
    assert plan_status((2, 3), (1, 2), "ip", (4, 4), (1, 4), "pj", (2, 4), (1, 2), "ij") == -4  # p: 3 vs 4
    assert plan_status((2, 3), (1, 0), "ip", (3, 4), (1, 3), "pj", (2, 4), (1, 2), "ij") == -5  # zero stride
    assert plan_status((2, 3), (1, -2), "ip", (3, 4), (1, 3), "pj", (2, 4), (1, 2), "ij") == -5
    assert plan_status((2, 3), (1, 2), "ip", (3, 4), (1, 3), "pj", (2, 4), (1, 1), "ij") == -6  # C overlaps itself
    assert plan_status(*ok[:-0] if False else ok, dtype=5) == -7
    assert plan_status(*ok, dtype=tc.TC_F64, mode=tc.TC_SPLIT_BF16X3) == -7
    # ndim out of range and NULL descriptors
    h = ctypes.c_void_p()
    lens = (ctypes.c_int64 * 17)(*([1] * 17))
    assert L.tc_plan_create(ctypes.byref(h), 17, lens, lens, b"abcdefghijklmnopq", 0, None, None, None,
                            17, lens, lens, b"abcdefghijklmnopq", 0, 0) == -2
    assert L.tc_plan_create(ctypes.byref(h), 2, None, None, None, 0, None, None, None, 0, None, None, None, 0, 0) == -1
    assert L.tc_plan_create(None, 0, None, None, None, 0, None, None, None, 0, None, None, None, 0, 0) == -1
    assert L.tc_plan_execute(None, 1.0, None, None, 0.0, None, None) == -1
    assert L.tc_plan_destroy(None) == 0
    assert L.tc_last_error()


def test_length_one_dim_may_have_any_stride():
    assert plan_status((2, 1, 3), (1, 0, 2), "iqp", (3, 4), (1, 3), "pj", (2, 1, 4), (1, -7, 2), "iqj") == 0


def test_describe_without_gpu_and_vectors_size_limit():
    p = inputs.cfg2()
    d = describe(p)
    assert d["vectors"] is True and len(d["rscat_X"]) == 2304
    big = inputs.Problem("ip", "pj", "ij", inputs.colmajor((8192, 2)), inputs.colmajor((2, 3)),
                         inputs.colmajor((8192, 3)))
    assert describe(big)["vectors"] is False


def test_permute_abi_errors():
    """tc_permute rejects bad descriptors on the host, before any launch."""
    L = tc.lib()
    lens = tc._arr([3, 4])
    ss = tc._arr([1, 3])
    ds = tc._arr([4, 1])
    assert L.tc_permute(None, None, 17, lens, ss, ds, tc.TC_F64, None) == -2
    assert L.tc_permute(None, None, 2, None, ss, ds, tc.TC_F64, None) == -1
    assert L.tc_permute(None, None, 2, lens, ss, ds, 9, None) == -7
    assert L.tc_permute(None, None, 2, tc._arr([3, -1]), ss, ds, tc.TC_F64, None) == -4
    assert L.tc_permute(None, None, 2, lens, tc._arr([1, 0]), ds, tc.TC_F64, None) == -5
    assert L.tc_permute(None, None, 2, lens, ss, tc._arr([-4, 1]), tc.TC_F32, None) == -5
    assert L.tc_permute(None, None, 2, lens, ss, ds, tc.TC_F64, None) == -1  # NULL data, non-empty
    # an empty index space is a no-op and needs no data
    assert L.tc_permute(None, None, 2, tc._arr([3, 0]), ss, ds, tc.TC_F64, None) == 0


def _batch_status(problems):
    """tc_batch_create on fake device addresses: every check below fails on
    the host before any HIP call is made."""
    L = tc.lib()
    plans = [tc.Plan(*desc) for desc, _ in problems]
    n = len(problems)
    hs = (ctypes.c_void_p * n)(*[p.handle for p in plans])
    al = (ctypes.c_double * n)(*([1.0] * n))
    be = (ctypes.c_double * n)(*([0.0] * n))
    As = (ctypes.c_void_p * n)(*[ptrs[0] for _, ptrs in problems])
    Bs = (ctypes.c_void_p * n)(*[ptrs[1] for _, ptrs in problems])
    Cs = (ctypes.c_void_p * n)(*[ptrs[2] for _, ptrs in problems])
    h = ctypes.c_void_p()
    st = L.tc_batch_create(ctypes.byref(h), n, hs, al, As, Bs, be, Cs)
    for p in plans:
        p.close()
    return st, L.tc_last_error().decode()


def test_batch_rejects_cross_problem_aliasing():
    """Outputs of two problems that overlap, and an operand of one problem
    inside another problem's output, are refused (TC_ERR_ALIAS)."""
    gemm = ((4, 3), (1, 4), "ip", (3, 5), (1, 3), "pj", (4, 5), (1, 4), "ij")  # C spans 20 doubles
    base = 1 << 40
    A0, B0, C0 = base, base + 4096, base + 8192
    A1, B1 = base + 16384, base + 20480
    st, msg = _batch_status([(gemm, (A0, B0, C0)), (gemm, (A1, B1, C0 + 8 * 19))])
    assert st == -6 and "outputs" in msg
    st, msg = _batch_status([(gemm, (A0, B0, C0)), (gemm, (C0 + 8 * 5, B1, base + 32768))])
    assert st == -6 and "operand of batch problem 1" in msg
    st, msg = _batch_status([(gemm, (A0, B0, C0)), (gemm, (A1, C0, base + 32768))])
    assert st == -6


def test_batch_problem_tile_abi_errors():
    L = tc.lib()
    t = ctypes.c_int()
    assert L.tc_batch_problem_tile(None, 0, ctypes.byref(t)) == -1


def test_contract_batched_abi_errors_and_host_tensors():
    """tc_contract_batched: argument errors before any device work, and the
    binding refuses host tensors."""
    import torch
    L = tc.lib()
    assert L.tc_contract_batched(0, None, tc.TC_F64, tc.TC_NATIVE, None) == 0
    assert L.tc_contract_batched(-1, None, tc.TC_F64, tc.TC_NATIVE, None) == -10  # TC_ERR_ARG
    assert L.tc_contract_batched(2, None, tc.TC_F64, tc.TC_NATIVE, None) == -1  # TC_ERR_NULL
    A = torch.zeros(3, 4, dtype=torch.float64)
    B = torch.zeros(4, 5, dtype=torch.float64)
    C = torch.zeros(3, 5, dtype=torch.float64)
    with pytest.raises(ValueError):
        tc.contract_batched([(A, "ik", B, "kj", C, "ij", 1.0, 0.0)])


def test_binding_refuses_host_tensors():
    """A CPU tensor never reaches the library: its host address would be
    meaningless to the kernels."""
    import pytest
    import torch
    A = torch.zeros(4, 3, dtype=torch.float64)
    B = torch.zeros(3, 5, dtype=torch.float64)
    C = torch.zeros(4, 5, dtype=torch.float64)
    with pytest.raises(ValueError, match="current HIP device"):
        tc.contract(A, "ip", B, "pj", "ij", out=C)
    with pytest.raises(ValueError, match="current HIP device"):
        tc.permute_into(A, torch.zeros(4, 3, dtype=torch.float64))


def test_noalloc_refuses_vectors_beyond_its_array():
    """tc_contract_noalloc refuses, before any launch or HIP call, a problem
    whose offset vectors exceed its static array (fake device addresses)."""
    L = tc.lib()
    m = (8 << 20) // 8 + 1024  # rscat_X and rscat_C alone pass 8 MiB of int32
    shpA, stA = tc._arr([m, 2]), tc._arr([1, m])
    shpB, stB = tc._arr([2, 3]), tc._arr([1, 2])
    shpC, stC = tc._arr([m, 3]), tc._arr([1, m])
    base = 1 << 40
    st = L.tc_contract_noalloc(1.0, base, 2, shpA, stA, b"ip", base + (1 << 30), 2, shpB, stB, b"pj", 0.0,
                               base + (1 << 31), 2, shpC, stC, b"ij", tc.TC_F64, tc.TC_NATIVE, None)
    assert st == -10 and b"allocation-free" in L.tc_last_error()
