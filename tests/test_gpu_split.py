"""Split-BF16 mode (FP32 storage, hi/lo bf16 operands, three matrix-core
products, FP32 accumulation) against the FP64 oracle."""
import numpy as np
import pytest

from paper_1607_00291_amd import inputs
from gpuutil import fp32_componentwise, require_gpu, split_bf16_componentwise, to_dev, to_host

pytestmark = pytest.mark.gpu


def f32(x):
    return np.asfortranarray(np.asarray(x, dtype=np.float32).astype(np.float64))


def run(p, mode, tile=None):
    from paper_1607_00291_amd import tc
    torch = require_gpu()
    A, B, C = to_dev(p.A, np.float32), to_dev(p.B, np.float32), to_dev(p.C, np.float32)
    plan = tc.Plan.for_tensors(A, p.idx_A, B, p.idx_B, C, p.idx_C, mode=mode)
    if tile is not None:
        plan.tile = tile
    plan.execute(A, B, C, p.alpha, p.beta)
    torch.cuda.synchronize()
    plan.close()
    return to_host(C).astype(np.float64)


def oracle(oracle_mod, p, absval=False, C=None):
    out = np.array(p.C if C is None else C, order="F", copy=True)
    oracle_mod.contract(p.alpha if not absval else 1.0, p.A, p.idx_A, p.B, p.idx_B,
                        p.beta if not absval else 0.0, out, p.idx_C, absval=absval)
    return out


def rounded(p):
    """The problem with operands rounded to FP32 (what the GPU receives)."""
    return inputs.Problem(p.idx_A, p.idx_B, p.idx_C, f32(p.A), f32(p.B), f32(p.C), p.alpha, p.beta, p.name,
                          p.extents)


@pytest.mark.parametrize("seed", range(4))
def test_split_random(oracle_mod, seed):
    p = rounded(inputs.random_problem(5000 + seed, 2, 2, 2, lo=3, hi=20, beta=0.5 if seed % 2 else 0.0,
                                      alpha=1.25))
    print(f"case split random seed={seed}", flush=True)
    got = run(p, "split_bf16x3")
    ref = oracle(oracle_mod, p)
    absC = oracle(oracle_mod, p, absval=True, C=np.zeros_like(p.C, order="F"))
    bound = split_bf16_componentwise(p.mnk()[2], p.alpha, absC, p.beta, p.C)
    assert np.all(np.abs(got - ref) <= bound + 1e-30)


@pytest.mark.parametrize("beta,f", [(0.0, 2), (0.5, 2), (-1.5, 1)])
@pytest.mark.parametrize("ext", [1, 17, 45, 97])
def test_split_ragged_every_tile(oracle_mod, ext, beta, f):
    """Ragged m, n and k under every split tile configuration (the 144 x 144
    tile included), with beta = 0 and beta != 0; f = 1 leaves a single
    contracted label whose k blocks share one block stride."""
    from paper_1607_00291_amd import tc
    rng = np.random.default_rng(ext)
    e = {"a": ext, "b": 5, "c": ext + 2, "d": 3, "e": ext + 1, "f": f}
    mk = lambda lab: f32(inputs.colmajor_from_flat(rng.uniform(-1, 1, int(np.prod(inputs.shape_of(lab, e)))),
                                                  inputs.shape_of(lab, e)))
    C0 = mk("abcd") if beta != 0.0 else inputs.colmajor(inputs.shape_of("abcd", e), fill=0.0)
    p = inputs.Problem("aebf", "dfce", "abcd", mk("aebf"), mk("dfce"), C0, 1.0, beta, f"ragged{ext}", e)
    ref = oracle(oracle_mod, p)
    absC = oracle(oracle_mod, p, absval=True, C=np.zeros_like(p.C, order="F"))
    bound = split_bf16_componentwise(p.mnk()[2], 1.0, absC, beta, p.C)
    for t in range(tc.tile_count(tc.TC_F32, tc.TC_SPLIT_BF16X3)):
        print(f"case split ragged ext={ext} beta={beta} f={f} tile={t}", flush=True)
        got = run(p, "split_bf16x3", tile=t)
        assert np.all(np.abs(got - ref) <= bound + 1e-30), t


def test_split_integer_inputs_bitwise(oracle_mod):
    """Small integers are exact in bf16 (lo = 0) and every partial sum is
    exact in FP32: the split result equals the oracle bit for bit."""
    p = inputs.random_problem(5100, 2, 2, 2, lo=2, hi=11, integer=True)
    print("case split integer", flush=True)
    assert np.array_equal(run(p, "split_bf16x3"), oracle(oracle_mod, p))


@pytest.mark.parametrize("shape", ["cfg1", "cfg2"])
def test_cfg3_fp32_and_split_error_report(oracle_mod, shape):
    """Inputs N(0,1) with per-mode scales 10^U(-3,3): FP32 and split-BF16
    within their bounds against the oracle on the same FP32-rounded inputs,
    and the end-to-end error against the FP64 inputs reported."""
    p64 = inputs.cfg3(shape=shape)
    p = rounded(p64)
    K = p.mnk()[2]
    print(f"case cfg3 {shape}", flush=True)
    # every output, at both shapes
    ref = oracle(oracle_mod, p)
    absC = oracle(oracle_mod, p, absval=True)
    ref64 = oracle(oracle_mod, p64)
    for mode, bound_fn in (("native", fp32_componentwise), ("split_bf16x3", split_bf16_componentwise)):
        got = run(p, mode)
        err = np.abs(got - ref)
        bound = bound_fn(K, 1.0, absC)
        assert np.all(err <= bound + 1e-300), mode
        rel = np.max(np.abs(got - ref64) / np.maximum(np.abs(ref64), 1e-300))
        ratio = np.max(err / np.maximum(bound, 1e-300))
        print(f"{shape} {mode}: max|err| vs oracle {np.max(err):.3e}, max err/bound {ratio:.3e}, "
              f"max rel err vs FP64 inputs {rel:.3e}", flush=True)


@pytest.mark.parametrize("seed", [41, 42])
def test_split_unit_strides_disagree_in_contracted_bundle(oracle_mod, seed):
    """Split-BF16 under the sub-blocked k order (A[e g f i] . B[f j e g]),
    every split tile, beta != 0, within the split componentwise bound."""
    from paper_1607_00291_amd import tc
    ext = {"e": 13, "g": 3, "f": 10, "i": 150, "j": 70} if seed == 41 else {"e": 6, "g": 5, "f": 9, "i": 61, "j": 145}
    p0 = inputs.p_conflict_problem(seed, ext, beta=-0.5)
    p = inputs.Problem(p0.idx_A, p0.idx_B, p0.idx_C, f32(p0.A), f32(p0.B), f32(p0.C), 1.0, -0.5, p0.name, ext)
    ref = oracle(oracle_mod, p)
    absC = oracle(oracle_mod, p, absval=True, C=np.zeros_like(p.C, order="F"))
    bound = split_bf16_componentwise(p.mnk()[2], 1.0, absC, -0.5, p.C)
    for t in range(tc.tile_count(tc.TC_F32, tc.TC_SPLIT_BF16X3)):
        print(f"case split p-conflict seed={seed} tile={t}", flush=True)
        got = run(p, "split_bf16x3", tile=t)
        assert np.all(np.abs(got - ref) <= bound + 1e-30), t



def split_tiles_by_layout(plan):
    """{layout: tile id} of the split tile table, read through a plan."""
    from paper_1607_00291_amd import tc
    keep, out = plan.tile, {}
    for t in range(tc.tile_count(tc.TC_F32, tc.TC_SPLIT_BF16X3)):
        plan.tile = t
        out.setdefault(plan.describe()["layout"], t)
    plan.tile = keep
    return out


def run_tiles(p, tiles, Ad=None):
    """Results of one split plan under each tile (fresh C each)."""
    from paper_1607_00291_amd import tc
    torch = require_gpu()
    A = to_dev(p.A, np.float32) if Ad is None else Ad
    B = to_dev(p.B, np.float32)
    outs = []
    for t in tiles:
        C = to_dev(p.C, np.float32)
        plan = tc.Plan.for_tensors(A, p.idx_A, B, p.idx_B, C, p.idx_C, mode="split_bf16x3")
        plan.tile = t
        plan.execute(A, B, C, p.alpha, p.beta)
        torch.cuda.synchronize()
        plan.close()
        outs.append(to_host(C))
    return outs


def ragged(ext, f, beta, seed):
    rng = np.random.default_rng(seed)
    e = {"a": ext, "b": 5, "c": ext + 2, "d": 3, "e": ext + 1, "f": f}
    mk = lambda lab: f32(inputs.colmajor_from_flat(rng.uniform(-1, 1, int(np.prod(inputs.shape_of(lab, e)))),
                                                  inputs.shape_of(lab, e)))
    return inputs.Problem("aebf", "dfce", "abcd", mk("aebf"), mk("dfce"), mk("abcd"), 1.25, beta,
                          f"ragged{ext}", e)


def test_packed_split_tile_same_bits_as_in_kernel_split():
    """The packed split tile (operands split once into hi/lo panels by a
    separate pass, the tile's producer waves only copying them) gives the same
    bits as the specialised-wave tile that gathers and splits in its own
    producer waves: ragged m, n and k, beta != 0, both gather directions of
    each operand, the sub-blocked k order and scatter-vector k blocks."""
    from paper_1607_00291_amd import tc
    torch = require_gpu()
    probe = ragged(17, 2, 0.5, 0)
    A = to_dev(probe.A, np.float32)
    plan = tc.Plan.for_tensors(A, probe.idx_A, to_dev(probe.B, np.float32), probe.idx_B,
                               to_dev(probe.C, np.float32), probe.idx_C, mode="split_bf16x3")
    lay = split_tiles_by_layout(plan)
    plan.close()
    packed, twin = lay[4], lay[2]
    cases = [ragged(ext, f, beta, ext) for ext, f, beta in ((1, 2, 0.5), (17, 1, -1.5), (97, 2, 0.0),
                                                            (150, 1, 0.5))]
    cases += [inputs.random_problem(5300 + s, 2, 2, 2, lo=3, hi=40, beta=0.5, alpha=1.25) for s in range(4)]
    cases += [inputs.random_problem(5320 + s, 1 + s % 3, 1 + (s + 1) % 3, 1 + (s + 2) % 3, lo=2, hi=30, beta=-0.5)
              for s in range(6)]
    cases.append(inputs.p_conflict_problem(5310, {"e": 13, "g": 3, "f": 10, "i": 150, "j": 70}, beta=-0.5))
    for p in cases:
        p = rounded(p)
        print(f"case packed split {p.name} mnk={p.mnk()}", flush=True)
        a, b = run_tiles(p, (twin, packed))
        assert np.array_equal(a, b), p.name
    torch.cuda.synchronize()


def test_packed_split_tile_int64_offsets():
    """The split-and-pack pass and the packed tile with 64-bit offsets (one
    operand spanning more than 2^31 bytes): the same bits as the in-kernel
    split twin, and within the split bound of the oracle."""
    from paper_1607_00291_amd import tc
    torch = require_gpu()
    rng = np.random.default_rng(92)
    e = {"a": 37, "e": 3, "b": 6, "f": 2, "d": 9, "c": 21}
    A = f32(inputs.colmajor_from_flat(rng.uniform(-1, 1, 37 * 3 * 6 * 2), (37, 3, 6, 2)))
    B = f32(inputs.colmajor_from_flat(rng.uniform(-1, 1, 9 * 2 * 21 * 3), (9, 2, 21, 3)))
    C0 = f32(inputs.colmajor_from_flat(rng.uniform(-1, 1, 37 * 6 * 21 * 9), (37, 6, 21, 9)))
    p = inputs.Problem("aebf", "dfce", "abcd", A, B, C0, 1.5, -0.5, "int64-offsets", e)
    big = (1 << 31) // 4
    storage = torch.zeros(big + 37 * 3 * 6, dtype=torch.float32, device="cuda")
    Ad = torch.as_strided(storage, (37, 3, 6, 2), (1, 37, 111, big))
    Ad.copy_(torch.from_numpy(A.astype(np.float32)).to("cuda"))
    plan = tc.Plan.for_tensors(Ad, p.idx_A, to_dev(B, np.float32), p.idx_B, to_dev(C0, np.float32), p.idx_C,
                               mode="split_bf16x3")
    assert plan.describe()["off64"]
    lay = split_tiles_by_layout(plan)
    plan.close()
    print("case packed split int64 offsets", flush=True)
    a, b = run_tiles(p, (lay[2], lay[4]), Ad=Ad)
    assert np.array_equal(a, b)
    del storage, Ad
    torch.cuda.empty_cache()


def test_packed_split_workspace_per_stream_and_graph_replay():
    """One plan on the packed split tile run on two streams at once with
    different inputs (each stream has its own panels), then captured on a
    stream it ran on and replayed with eager work in between: every result
    equals the in-kernel split twin's, bit for bit."""
    from paper_1607_00291_amd import tc
    torch = require_gpu()
    p1, p2 = rounded(ragged(150, 2, 0.0, 11)), rounded(ragged(150, 2, 0.0, 12))
    A1, B1, C1 = to_dev(p1.A, np.float32), to_dev(p1.B, np.float32), to_dev(p1.C, np.float32)
    A2, B2, C2 = to_dev(p2.A, np.float32), to_dev(p2.B, np.float32), to_dev(p2.C, np.float32)
    plan = tc.Plan.for_tensors(A1, p1.idx_A, B1, p1.idx_B, C1, p1.idx_C, mode="split_bf16x3")
    lay = split_tiles_by_layout(plan)
    plan.tile = lay[2]
    plan.execute(A1, B1, C1, 1.25, 0.0)
    torch.cuda.synchronize()
    ref1 = to_host(C1)
    plan.execute(A2, B2, C2, 1.25, 0.0)
    torch.cuda.synchronize()
    ref2 = to_host(C2)
    plan.tile = lay[4]
    plan.upload()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    s1.wait_stream(torch.cuda.current_stream())
    s2.wait_stream(torch.cuda.current_stream())
    print("case packed split two streams", flush=True)
    for _ in range(3):
        C1.zero_()
        C2.zero_()
        s1.wait_stream(torch.cuda.current_stream())
        s2.wait_stream(torch.cuda.current_stream())
        plan.execute(A1, B1, C1, 1.25, 0.0, stream=s1)
        plan.execute(A2, B2, C2, 1.25, 0.0, stream=s2)
        torch.cuda.synchronize()
        assert np.array_equal(to_host(C1), ref1) and np.array_equal(to_host(C2), ref2)
    print("case packed split graph replay", flush=True)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s1):
        plan.execute(A1, B1, C1, 1.25, 0.0, stream=s1)
    for rep in range(3):
        C1.fill_(float(rep + 7))
        plan.execute(A2, B2, C2, 1.25, 0.0, stream=s2)  # eager work on another stream's panels
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(to_host(C1), ref1), f"replay {rep}"
        assert np.array_equal(to_host(C2), ref2)
    del g
    plan.close()
