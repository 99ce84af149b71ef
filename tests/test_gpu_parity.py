"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the
same seeded inputs, element by element, within the stated tolerances."""
import itertools

import numpy as np
import pytest

from paper_1607_00291_amd import inputs
from gpuutil import fp32_componentwise, fp64_bound, require_gpu, to_dev, to_host

pytestmark = pytest.mark.gpu


def oracle_result(oracle_mod, p, A=None, B=None, C=None, absval=False):
    A = p.A if A is None else A
    B = p.B if B is None else B
    C = np.array(p.C if C is None else C, order="F", copy=True)
    oracle_mod.contract(p.alpha, A, p.idx_A, B, p.idx_B, p.beta, C, p.idx_C, absval=absval)
    return C


def gpu_result(p, dtype=np.float64, tile=None, mode="native"):
    from paper_1607_00291_amd import tc
    torch = require_gpu()
    A, B, C = to_dev(p.A, dtype), to_dev(p.B, dtype), to_dev(p.C, dtype)
    if tile is None:
        tc.contract(A, p.idx_A, B, p.idx_B, p.idx_C, alpha=p.alpha, beta=p.beta, out=C, mode=mode)
    else:
        plan = tc.Plan.for_tensors(A, p.idx_A, B, p.idx_B, C, p.idx_C, mode=mode)
        plan.tile = tile
        plan.execute(A, B, C, p.alpha, p.beta)
        plan.close()
    torch.cuda.synchronize()
    return to_host(C)


def check_fp64(oracle_mod, p, got):
    ref = oracle_result(oracle_mod, p)
    K = p.mnk()[2]
    maxA = np.max(np.abs(p.A), initial=0.0)
    maxB = np.max(np.abs(p.B), initial=0.0)
    bound = fp64_bound(K, p.alpha, maxA, maxB, p.beta, np.max(np.abs(p.C), initial=0.0))
    err = np.max(np.abs(got - ref), initial=0.0)
    assert err <= bound, f"{p.name}: max err {err:.3e} > bound {bound:.3e}"
    return err


def test_cfg1_fp64(oracle_mod):
    p = inputs.cfg1()
    print("case cfg1 fp64", flush=True)
    check_fp64(oracle_mod, p, gpu_result(p))


@pytest.mark.parametrize("seed", range(12))
def test_random_small_fp64(oracle_mod, seed):
    nb = [(2, 2, 2), (1, 2, 3), (3, 1, 1), (2, 3, 2), (1, 1, 1), (2, 2, 1)][seed % 6]
    p = inputs.random_problem(1000 + seed, *nb, lo=1, hi=13, beta=0.0 if seed % 3 == 0 else -0.5,
                              alpha=1.0 if seed % 2 == 0 else 1.75)
    print(f"case random seed={seed} {p.idx_A},{p.idx_B}->{p.idx_C} {p.extents}", flush=True)
    check_fp64(oracle_mod, p, gpu_result(p))


@pytest.mark.parametrize("shape", [(300, 200, 50), (160, 170, 9), (400, 64, 200), (97, 301, 33)])
def test_sweep_instances(oracle_mod, shape):
    """Random-contraction sweep instances (one to three labels per bundle,
    random storage orders), as timed by the bench sweep, at sizes the oracle
    finishes quickly."""
    for sd in range(3):
        p = inputs.sweep_problem(77 + sd, *shape)
        print(f"case sweep {shape} seed={77 + sd} {p.idx_A},{p.idx_B}->{p.idx_C} {p.extents}", flush=True)
        check_fp64(oracle_mod, p, gpu_result(p))


@pytest.mark.parametrize("f", [2, 1])
@pytest.mark.parametrize("ext", [1, 3, 17, 97])
def test_ragged_extents_every_tile(oracle_mod, ext, f):
    """Extents that leave ragged tiles in m, n and k, under every tile config.
    With f = 1 the contracted bundle is the single label e, whose k blocks all
    share one block stride, so the kernels' per-tile byte-offset path runs
    with a partial last k block."""
    from paper_1607_00291_amd import tc
    p = ragged_problem(ext, beta=0.5, f=f)
    for t in range(tc.tile_count(tc.TC_F64)):
        print(f"case ragged ext={ext} f={f} tile={t}", flush=True)
        check_fp64(oracle_mod, p, gpu_result(p, tile=t))


@pytest.mark.parametrize("seed", range(4))
def test_integer_inputs_bitwise_fp64(oracle_mod, seed):
    p = inputs.random_problem(2000 + seed, 2, 2, 2, lo=2, hi=11, integer=True, beta=2.0, alpha=1.0)
    print(f"case integer seed={seed}", flush=True)
    assert np.array_equal(gpu_result(p), oracle_result(oracle_mod, p))


def test_integer_inputs_bitwise_fp32(oracle_mod):
    p = inputs.random_problem(2100, 2, 2, 2, lo=2, hi=11, integer=True, beta=0.0)
    print("case integer fp32", flush=True)
    assert np.array_equal(gpu_result(p, np.float32).astype(np.float64), oracle_result(oracle_mod, p))


def test_storage_permutations(oracle_mod):
    """Every storage order of C, and every order of A with B, of a rank-4
    contraction with extents in {2, 3}: integer inputs, so results are exact."""
    rng = np.random.default_rng(7)
    e = {"a": 3, "b": 2, "c": 3, "d": 2, "e": 3, "f": 2}
    base_A, base_B, base_C = "aebf", "dfce", "abcd"

    def mk(lab):
        shp = inputs.shape_of(lab, e)
        return inputs.colmajor_from_flat(rng.integers(-4, 5, int(np.prod(shp))).astype(np.float64), shp)

    A0, B0 = mk(base_A), mk(base_B)
    perms = list(itertools.permutations(range(4)))
    cases = [(pa, pb, pc) for pa in perms[::5] for pb in perms[::5] for pc in perms[::7]]
    print(f"case storage permutations n={len(cases)}", flush=True)
    for pa, pb, pc in cases:
        ia = "".join(base_A[i] for i in pa)
        ib = "".join(base_B[i] for i in pb)
        ic = "".join(base_C[i] for i in pc)
        A = np.asfortranarray(np.transpose(A0, pa))
        B = np.asfortranarray(np.transpose(B0, pb))
        C = inputs.colmajor(inputs.shape_of(ic, e), fill=0.0)
        p = inputs.Problem(ia, ib, ic, A, B, C, 1.0, 0.0, f"perm {ia},{ib}->{ic}", e)
        got = gpu_result(p)
        ref = oracle_result(oracle_mod, p)
        assert np.array_equal(got, ref), p.name


def test_swapped_operands(oracle_mod):
    """C's unit stride in J: the planner computes C^T = B^T A^T."""
    p = inputs.random_problem(3000, 2, 2, 2, lo=3, hi=20, beta=0.25)
    # make C's first label come from B
    ib_first = [l for l in p.idx_C if l in p.idx_B][0]
    ic = ib_first + p.idx_C.replace(ib_first, "")
    C = inputs.colmajor(inputs.shape_of(ic, p.extents), fill=0.0)
    C[...] = np.random.default_rng(1).uniform(-1, 1, C.shape)
    q = inputs.Problem(p.idx_A, p.idx_B, ic, p.A, p.B, C, 1.0, 0.25, "swapped", p.extents)
    from paper_1607_00291_amd import tc
    s = lambda a: [x // a.itemsize for x in a.strides]
    assert tc.describe(q.A.shape, s(q.A), q.idx_A, q.B.shape, s(q.B), q.idx_B, q.C.shape, s(q.C), q.idx_C)["swapped"]
    check_fp64(oracle_mod, q, gpu_result(q))


def test_fp32_random(oracle_mod):
    for seed in range(4):
        p = inputs.random_problem(4000 + seed, 2, 2, 2, lo=3, hi=24, beta=0.5 if seed % 2 else 0.0)
        A32, B32, C32 = (x.astype(np.float32).astype(np.float64) for x in (p.A, p.B, p.C))
        q = inputs.Problem(p.idx_A, p.idx_B, p.idx_C, np.asfortranarray(A32), np.asfortranarray(B32),
                           np.asfortranarray(C32), p.alpha, p.beta, p.name, p.extents)
        print(f"case fp32 seed={seed}", flush=True)
        got = gpu_result(q, np.float32).astype(np.float64)
        ref = oracle_result(oracle_mod, q)
        absC = oracle_result(oracle_mod, inputs.Problem(q.idx_A, q.idx_B, q.idx_C, q.A, q.B,
                                                        np.zeros_like(q.C, order="F"), 1.0, 0.0), absval=True)
        bound = fp32_componentwise(q.mnk()[2], q.alpha, absC, q.beta, q.C)
        assert np.all(np.abs(got - ref) <= bound + 1e-30), f"fp32 seed {seed}"


def test_edge_cases(oracle_mod):
    torch = require_gpu()
    from paper_1607_00291_amd import tc
    rng = np.random.default_rng(5)
    # empty I (m = 1), empty P (outer product), scalar output (dot product)
    for ia, ib, ic, e in [("p", "pj", "j", {"p": 37, "j": 70}),
                          ("i", "j", "ij", {"i": 33, "j": 65}),
                          ("pq", "qp", "", {"p": 19, "q": 23}),
                          ("ip", "pj", "ij", {"i": 1, "p": 1, "j": 1})]:
        A = inputs.colmajor_from_flat(rng.uniform(-1, 1, int(np.prod(inputs.shape_of(ia, e)))), inputs.shape_of(ia, e))
        B = inputs.colmajor_from_flat(rng.uniform(-1, 1, int(np.prod(inputs.shape_of(ib, e)))), inputs.shape_of(ib, e))
        C = inputs.colmajor(inputs.shape_of(ic, e), fill=0.0)
        p = inputs.Problem(ia, ib, ic, A, B, C, 1.0, 0.0, f"edge {ia},{ib}->{ic}", e)
        print(f"case {p.name}", flush=True)
        check_fp64(oracle_mod, p, gpu_result(p))
    # beta = 0 never reads C (NaN does not propagate)
    p = inputs.random_problem(6000, 2, 2, 2, lo=2, hi=9)
    p.C[...] = np.nan
    got = gpu_result(p)
    assert not np.isnan(got).any()
    # alpha = 0: C := beta C, A and B not read (pass NULL-free but garbage-free tensors)
    p = inputs.random_problem(6001, 2, 2, 2, lo=2, hi=9, beta=-2.0, alpha=0.0)
    assert np.array_equal(gpu_result(p), -2.0 * p.C)
    # a contracted extent of 0: C := beta C
    e = {"i": 5, "p": 0, "j": 6}
    C0 = inputs.colmajor_from_flat(rng.uniform(-1, 1, 30), (5, 6))
    A = torch.zeros((5, 0), dtype=torch.float64, device="cuda")
    B = torch.zeros((0, 6), dtype=torch.float64, device="cuda")
    Cd = to_dev(C0)
    tc.contract(A, "ip", B, "pj", "ij", alpha=1.0, beta=0.5, out=Cd)
    torch.cuda.synchronize()
    assert np.array_equal(to_host(Cd), 0.5 * C0)
    # a free extent of 0: no-op, no error
    A = torch.zeros((0, 4), dtype=torch.float64, device="cuda")
    B = torch.zeros((4, 3), dtype=torch.float64, device="cuda")
    C = torch.zeros((0, 3), dtype=torch.float64, device="cuda")
    tc.contract(A, "ip", B, "pj", "ij", out=C)


def test_noncontiguous_views(oracle_mod):
    """Operands that are slices of larger buffers (strides with gaps)."""
    torch = require_gpu()
    from paper_1607_00291_amd import tc
    rng = np.random.default_rng(8)
    big = inputs.colmajor_from_flat(rng.uniform(-1, 1, 40 * 9 * 30), (40, 9, 30))
    A = big[3:35:2, 1:8, ::3]        # a[16] x b[7] x p[10] with gaps
    B = np.asfortranarray(rng.uniform(-1, 1, (10, 13)))[:, ::2]  # p x j[7]
    C = inputs.colmajor((7, 7, 16), fill=0.0)  # j[7] b[7] a[16]
    p = inputs.Problem("abp", "pj", "jba", A, B, C, 1.0, 0.0, "views",
                       {"a": 16, "b": 7, "p": 10, "j": 7})
    check_fp64(oracle_mod, p, gpu_result(p))


def test_cfg2_full_size_every_output(oracle_mod):
    """The v=96/o=24 coupled-cluster contraction at full size, in the launch
    configuration the benchmark times (the plan's own tile choice): every one
    of the 5.3 M outputs against the oracle, within the FP64 bound."""
    torch = require_gpu()
    from paper_1607_00291_amd import tc
    p = inputs.cfg2()
    A, B, C = to_dev(p.A), to_dev(p.B), to_dev(p.C)
    plan = tc.Plan.for_tensors(A, p.idx_A, B, p.idx_B, C, p.idx_C)
    d = plan.describe()
    print(f"case cfg2 full, tile {d['MT']}x{d['NT']}x{d['KT']} waves {d['waves']}", flush=True)
    plan.execute(A, B, C, p.alpha, p.beta)
    torch.cuda.synchronize()
    got = to_host(C)
    plan.close()
    err = check_fp64(oracle_mod, p, got)
    print(f"cfg2 full: max|C - Cref| = {err:.3e} over {got.size} outputs", flush=True)


def ragged_problem(ext, beta, f=2):
    """Extents that leave ragged tiles in m, n and k (m = ext * 5,
    n = (ext + 2) * 3, k = (ext + 1) * f), alpha = 1.25."""
    rng = np.random.default_rng(ext)
    e = {"a": ext, "b": 5, "c": ext + 2, "d": 3, "e": ext + 1, "f": f}
    mk = lambda lab: inputs.colmajor_from_flat(rng.uniform(-1, 1, int(np.prod(inputs.shape_of(lab, e)))),
                                               inputs.shape_of(lab, e))
    A, B, C = mk("aebf"), mk("dfce"), mk("abcd")
    return inputs.Problem("aebf", "dfce", "abcd", A, B, C, 1.25, beta, f"ragged{ext}", e)


@pytest.mark.parametrize("f", [2, 1])
@pytest.mark.parametrize("ext", [1, 3, 17, 97])
def test_ragged_extents_every_tile_fp32(oracle_mod, ext, f):
    """The FP32 kernels with 32-bit offsets at ragged m, n and k, beta != 0,
    under every tile configuration (including the specialised-wave pinwheel
    and its partial last k block), within the FP32 componentwise bound."""
    from paper_1607_00291_amd import tc
    p = ragged_problem(ext, beta=-0.75, f=f)
    q = inputs.Problem(p.idx_A, p.idx_B, p.idx_C, *(np.asfortranarray(x.astype(np.float32).astype(np.float64))
                                                      for x in (p.A, p.B, p.C)), p.alpha, p.beta, p.name, p.extents)
    ref = oracle_result(oracle_mod, q)
    absC = oracle_result(oracle_mod, inputs.Problem(q.idx_A, q.idx_B, q.idx_C, q.A, q.B,
                                                    np.zeros_like(q.C, order="F"), 1.0, 0.0), absval=True)
    bound = fp32_componentwise(q.mnk()[2], q.alpha, absC, q.beta, q.C)
    for t in range(tc.tile_count(tc.TC_F32)):
        print(f"case ragged fp32 ext={ext} f={f} tile={t}", flush=True)
        got = gpu_result(q, np.float32, tile=t).astype(np.float64)
        assert np.all(np.abs(got - ref) <= bound + 1e-30), f"tile {t}"


def test_alpha_zero_with_nan_operands(oracle_mod):
    """alpha = 0 reads neither A nor B: with NaN and Inf in both operands the
    GPU result equals the oracle's C := beta * C exactly (FP64 and FP32)."""
    p = inputs.random_problem(6002, 2, 2, 2, lo=3, hi=19, beta=-2.0, alpha=0.0)
    p.A.reshape(-1, order="F")[::3] = np.nan
    p.B.reshape(-1, order="F")[1::5] = np.inf
    ref = oracle_result(oracle_mod, p)
    print("case alpha=0 with NaN operands", flush=True)
    assert not np.isnan(ref).any()
    assert np.array_equal(gpu_result(p), ref)
    q = inputs.Problem(p.idx_A, p.idx_B, p.idx_C, p.A, p.B,
                       np.asfortranarray(p.C.astype(np.float32).astype(np.float64)), 0.0, -2.0, p.name, p.extents)
    assert np.array_equal(gpu_result(q, np.float32).astype(np.float64), oracle_result(oracle_mod, q))


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_int64_offsets(oracle_mod, dtype):
    """An operand whose span exceeds 2^31 bytes (one huge stride over a
    length-2 dimension) takes the 64-bit offset kernels; checked under every
    tile configuration."""
    from paper_1607_00291_amd import tc
    torch = require_gpu()
    rng = np.random.default_rng(91)
    e = {"a": 37, "e": 3, "b": 6, "f": 2, "d": 9, "c": 21}
    A = inputs.colmajor_from_flat(rng.uniform(-1, 1, 37 * 3 * 6 * 2), (37, 3, 6, 2))
    B = inputs.colmajor_from_flat(rng.uniform(-1, 1, 9 * 2 * 21 * 3), (9, 2, 21, 3))
    C0 = inputs.colmajor_from_flat(rng.uniform(-1, 1, 37 * 6 * 21 * 9), (37, 6, 21, 9))
    if dtype == np.float32:
        A, B, C0 = (np.asfortranarray(x.astype(np.float32).astype(np.float64)) for x in (A, B, C0))
    p = inputs.Problem("aebf", "dfce", "abcd", A, B, C0, 1.5, -0.5, "int64-offsets", e)
    elt = np.dtype(dtype).itemsize
    big = (1 << 31) // elt  # one step of this stride alone passes 2^31 bytes
    tdt = torch.float64 if dtype == np.float64 else torch.float32
    storage = torch.zeros(big + 37 * 3 * 6, dtype=tdt, device="cuda")
    Ad = torch.as_strided(storage, (37, 3, 6, 2), (1, 37, 111, big))
    Ad.copy_(torch.from_numpy(A.astype(dtype)).to("cuda"))
    Bd = to_dev(B, dtype)
    ref = oracle_result(oracle_mod, p)
    if dtype == np.float32:
        absC = oracle_result(oracle_mod, inputs.Problem(p.idx_A, p.idx_B, p.idx_C, p.A, p.B,
                                                        np.zeros_like(p.C, order="F"), 1.0, 0.0), absval=True)
        bound = fp32_componentwise(p.mnk()[2], p.alpha, absC, p.beta, p.C)
    code = tc.TC_F64 if dtype == np.float64 else tc.TC_F32
    for t in range(tc.tile_count(code)):
        Cd = to_dev(C0, dtype)
        plan = tc.Plan.for_tensors(Ad, p.idx_A, Bd, p.idx_B, Cd, p.idx_C)
        assert plan.describe()["off64"]
        plan.tile = t
        print(f"case int64 offsets dtype={np.dtype(dtype).name} tile={t}", flush=True)
        plan.execute(Ad, Bd, Cd, p.alpha, p.beta)
        plan.close()
        torch.cuda.synchronize()
        got = to_host(Cd).astype(np.float64)
        if dtype == np.float64:
            check_fp64(oracle_mod, p, got)
        else:
            assert np.all(np.abs(got - ref) <= bound + 1e-30), f"tile {t}"
    del storage
    torch.cuda.empty_cache()


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_unit_stride_index_not_first_in_free_bundle(oracle_mod, dtype):
    """Layouts where C orders a free bundle differently from the operand that
    holds it (no order gives unit stride in both, Sec. 7.3): A[u v p] B[p j]
    -> C[v u j] (A's unit stride on u, C's on v), and B[w j p] with C[i j w]
    (B's unit stride on w, C's order puts j first).  The planner moves the
    operand's unit-stride index to the front of its bundle; every output is
    compared with the oracle, beta != 0, tiles ragged in m, n and k."""
    from paper_1607_00291_amd import tc
    rng = np.random.default_rng(17)
    cases = [("uvp", "pj", "vuj", {"u": 40, "v": 48, "p": 72, "j": 100}),
             ("ip", "wjp", "ijw", {"i": 150, "p": 66, "w": 36, "j": 20})]
    for ia, ib, ic, e in cases:
        mk = lambda lab: inputs.colmajor_from_flat(rng.uniform(-1, 1, int(np.prod(inputs.shape_of(lab, e)))),
                                                   inputs.shape_of(lab, e))
        A, B, C = mk(ia), mk(ib), mk(ic)
        if dtype == np.float32:
            A, B, C = (np.asfortranarray(x.astype(np.float32).astype(np.float64)) for x in (A, B, C))
        p = inputs.Problem(ia, ib, ic, A, B, C, 1.5, -0.5, f"unit-first {ia},{ib}->{ic}", e)
        s = lambda a: [x // a.itemsize for x in a.strides]
        d = tc.describe(A.shape, s(A), ia, B.shape, s(B), ib, C.shape, s(C), ic,
                        tc.TC_F64 if dtype == np.float64 else tc.TC_F32)
        assert d["unit_moves"] == 1, d["paper_order"]
        print(f"case {p.name} {np.dtype(dtype).name} paper {d['paper_order']} lanes {d['x_lanes']}/{d['y_lanes']}",
              flush=True)
        got = gpu_result(p, dtype).astype(np.float64)
        if dtype == np.float64:
            check_fp64(oracle_mod, p, got)
        else:
            ref = oracle_result(oracle_mod, p)
            absC = oracle_result(oracle_mod, inputs.Problem(ia, ib, ic, A, B, np.zeros_like(C, order="F"), 1.0, 0.0),
                                 absval=True)
            assert np.all(np.abs(got - ref) <= fp32_componentwise(p.mnk()[2], p.alpha, absC, p.beta, p.C) + 1e-30)


@pytest.mark.parametrize("ext", [{"e": 13, "g": 3, "f": 10, "i": 150, "j": 70},
                                 {"e": 16, "g": 1, "f": 8, "i": 97, "j": 129},
                                 {"e": 5, "g": 7, "f": 37, "i": 33, "j": 300},
                                 {"e": 3, "g": 2, "f": 7, "i": 17, "j": 9}])
def test_unit_strides_disagree_in_contracted_bundle_every_tile(oracle_mod, ext):
    """A[e g f i] . B[f j e g] -> C[i j]: A's unit-stride index e and B's f
    are both contracted, so the plan walks k in sub-blocks over (e, f) (the
    layouts of Sec. 7.3 and Sec. 9.2 that call for dimension sub-division).
    Every output against the oracle, beta != 0, every FP64 and FP32 tile,
    extents ragged against the sub-blocks and the tiles."""
    from paper_1607_00291_amd import tc
    p = inputs.p_conflict_problem(31, ext, beta=0.5)
    s = lambda a: [x // a.itemsize for x in a.strides]
    d = tc.describe(p.A.shape, s(p.A), p.idx_A, p.B.shape, s(p.B), p.idx_B, p.C.shape, s(p.C), p.idx_C)
    assert d["k_sub"] is not None, d["P"]
    for t in range(tc.tile_count(tc.TC_F64)):
        print(f"case p-conflict fp64 {ext} tile={t}", flush=True)
        check_fp64(oracle_mod, p, gpu_result(p, tile=t))
    q = inputs.Problem(p.idx_A, p.idx_B, p.idx_C, *(np.asfortranarray(x.astype(np.float32).astype(np.float64))
                                                      for x in (p.A, p.B, p.C)), p.alpha, p.beta, p.name, p.extents)
    ref = oracle_result(oracle_mod, q)
    absC = oracle_result(oracle_mod, inputs.Problem(q.idx_A, q.idx_B, q.idx_C, q.A, q.B,
                                                    np.zeros_like(q.C, order="F"), 1.0, 0.0), absval=True)
    bound = fp32_componentwise(q.mnk()[2], q.alpha, absC, q.beta, q.C)
    for t in range(tc.tile_count(tc.TC_F32)):
        print(f"case p-conflict fp32 {ext} tile={t}", flush=True)
        got = gpu_result(q, np.float32, tile=t).astype(np.float64)
        assert np.all(np.abs(got - ref) <= bound + 1e-30), f"tile {t}"
