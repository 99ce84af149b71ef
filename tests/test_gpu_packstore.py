"""The pack and store stages alone (tc_plan_pack, tc_plan_store), through the
C ABI: the tile-panel matrix of each operand equals, bit for bit, the
operand's matrix view rebuilt here in numpy from the tensor and the bundle
order of the plan (labels and lengths only); the store of an m x n matrix
equals, bit for bit, that matrix laid into C's layout plus beta C (alpha and
beta powers of two, so one rounding on either side)."""
import numpy as np
import pytest

import korder
from paper_1607_00291_amd import inputs
from gpuutil import require_gpu, to_dev, to_host

pytestmark = pytest.mark.gpu


def matrix_view(T, labels, row_labels, col_labels):
    """T as a (prod rows) x (prod cols) matrix, first label fastest on each side."""
    At = np.transpose(T, [labels.index(l) for l in row_labels + col_labels])
    m = int(np.prod([T.shape[labels.index(l)] for l in row_labels], dtype=np.int64))
    k = int(np.prod([T.shape[labels.index(l)] for l in col_labels], dtype=np.int64))
    return np.reshape(At, (m, k), order="F")


def panels(M, R, KT):
    """The tile-panel layout of tc_plan_pack: slivers R x KT in (row tile, k
    block) order, each stored k-major, zero padded."""
    m, k = M.shape
    tr, nkb = -(-m // R), -(-k // KT)
    P = np.zeros((tr * R, nkb * KT), dtype=M.dtype)
    P[:m, :k] = M
    out = np.empty(tr * nkb * KT * R, dtype=M.dtype)
    for t in range(tr):
        for b in range(nkb):
            blk = t * nkb + b
            out[blk * KT * R:(blk + 1) * KT * R] = P[t * R:(t + 1) * R, b * KT:(b + 1) * KT].T.reshape(-1)
    return out


def bundle_labels(d, key):
    return "".join(x["labels"] for x in d[key])


def k_columns(d, P, extents):
    """Column of the colexicographic P matrix view holding each k of the
    plan, in the plan's k order (sub-blocked when the plan says so)."""
    cols = []
    for vals in korder.p_label_values(d["P"], d["k_sub"], extents):
        c, w = 0, 1
        for l in P:
            c += vals[l] * w
            w *= extents[l]
        cols.append(c)
    return np.asarray(cols, dtype=np.int64)


def problems():
    yield inputs.cfg2(v=40, o=12)
    for seed in range(3):
        yield inputs.sweep_problem(300 + seed, 300, 200, 70)
    yield inputs.random_problem(301, 2, 2, 2, lo=3, hi=17, beta=0.5)
    yield inputs.p_conflict_problem(77)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_pack_matches_matrix_view(dtype):
    torch = require_gpu()
    from paper_1607_00291_amd import tc
    code = tc.TC_F64 if dtype == np.float64 else tc.TC_F32
    for q, p in enumerate(problems()):
        A, B, C = to_dev(p.A, dtype), to_dev(p.B, dtype), to_dev(p.C, dtype)
        plan = tc.Plan.for_tensors(A, p.idx_A, B, p.idx_B, C, p.idx_C)
        # every tile shape on the first problem (every sliver height R), the
        # planner's choice on the others
        for tile in (range(tc.tile_count(code)) if q == 0 else [plan.tile]):
            plan.tile = tile
            d = plan.describe()
            I, J, P = bundle_labels(d, "I"), bundle_labels(d, "J"), bundle_labels(d, "P")
            for operand, (T, lab) in enumerate(((p.A, p.idx_A), (p.B, p.idx_B))):
                x = (operand == 0) != d["swapped"]
                rows, R = (I, d["MT"]) if x else (J, d["NT"])
                M = matrix_view(np.asarray(T, dtype=dtype), lab, rows, P)
                want = panels(M[:, k_columns(d, P, p.extents)], R, d["KT"])
                dst = torch.full((plan.pack_elements(operand),), float("nan"), dtype=A.dtype, device="cuda")
                print(f"case pack {p.name} {np.dtype(dtype).name} tile {tile} operand {operand} rows {rows} k {P}",
                      flush=True)
                plan.pack(operand, A if operand == 0 else B, dst)
                torch.cuda.synchronize()
                assert np.array_equal(to_host(dst), want), (p.name, tile, operand)
        plan.close()


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_store_matches_layout(dtype):
    torch = require_gpu()
    from paper_1607_00291_amd import tc
    rng = np.random.default_rng(4)
    for p in problems():
        A, B = to_dev(p.A, dtype), to_dev(p.B, dtype)
        C0 = np.asfortranarray(rng.uniform(-1, 1, p.C.shape)).astype(dtype)
        plan = tc.Plan.for_tensors(A, p.idx_A, B, p.idx_B, to_dev(C0), p.idx_C)
        d = plan.describe()
        # the plan's m x n matrix: rows over its I bundle, columns over its J
        # bundle, each in the plan's order, first label fastest
        I, J = bundle_labels(d, "I"), bundle_labels(d, "J")
        src = rng.uniform(-1, 1, (d["m"], d["n"])).astype(dtype)
        T = np.reshape(src, [p.extents[l] for l in I + J], order="F")
        laid = np.transpose(T, [(I + J).index(l) for l in p.idx_C])
        for alpha, beta in ((1.0, 0.5), (-2.0, 0.0)):
            Cd = to_dev(C0)
            srcd = torch.from_numpy(np.asfortranarray(src).reshape(-1, order="F").copy()).to("cuda")
            print(f"case store {p.name} {np.dtype(dtype).name} alpha {alpha} beta {beta}", flush=True)
            plan.store(srcd, Cd, alpha=alpha, beta=beta)
            torch.cuda.synchronize()
            want = (alpha * laid + (beta * C0 if beta != 0 else 0)).astype(dtype)
            assert np.array_equal(to_host(Cd), want), (p.name, alpha, beta)
        plan.close()
