"""The whole 512-contraction batch (extents 4..64, random permutations of
every operand), as the benchmark times it: every problem bitwise equal to a
sequential launch of the same tile configuration, under per-problem tile
classes and under every single class a batch runs; and a fixed seeded subset
(the 32 cheapest instances plus 32 drawn at random from the rest) against the
oracle within the FP64 bound."""
import numpy as np
import pytest

from paper_1607_00291_amd import inputs
from gpuutil import fp64_bound, require_gpu, to_dev, to_host

pytestmark = pytest.mark.gpu

COUNT = 512


def oracle_subset(probs):
    fl = np.array([p.flops() for p in probs], dtype=np.float64)
    order = np.argsort(fl, kind="stable")
    rest = order[32:]
    pick = np.random.default_rng(512).choice(rest, 32, replace=False)
    return sorted(int(i) for i in np.concatenate([order[:32], pick]))


@pytest.fixture(scope="module", params=[np.float64, np.float32], ids=["fp64", "fp32"])
def batch512(request):
    """All 512 problems on the device, bound into one batch.  Host copies are
    kept only for the oracle subset."""
    torch = require_gpu()
    from paper_1607_00291_amd import tc
    dtype = request.param
    probs, dev = [], []
    for i in range(COUNT):
        p = inputs.cfg5_instance(i)
        dev.append((to_dev(p.A, dtype), to_dev(p.B, dtype), to_dev(p.C, dtype)))
        probs.append(p)
    keep = set(oracle_subset(probs))
    for i, p in enumerate(probs):
        if i not in keep:
            p.A = p.B = p.C = None  # host copies only where the oracle needs them
    print(f"case batch512 {np.dtype(dtype).name}: {COUNT} problems on the device", flush=True)
    batch = tc.Batch([(A, p.idx_A, B, p.idx_B, C, p.idx_C, p.alpha, p.beta) for p, (A, B, C) in zip(probs, dev)])
    yield dtype, probs, dev, batch
    batch.close()
    del dev
    torch.cuda.empty_cache()


def run_and_compare(torch, tc, probs, dev, batch):
    """Run the batch, then every problem alone with the tile configuration the
    batch gave it, into separate outputs; compare bitwise on the device."""
    for _, _, C in dev:
        C.zero_()
    batch.execute()
    seq = []
    for i, (p, (A, B, C)) in enumerate(zip(probs, dev)):
        Cs = torch.zeros_like(C)
        t = batch.problem_tile(i)
        if t >= 0:
            plan = tc.Plan.for_tensors(A, p.idx_A, B, p.idx_B, Cs, p.idx_C)
            plan.tile = t
            plan.execute(A, B, Cs, p.alpha, p.beta)
            plan.close()
        seq.append(Cs)
    torch.cuda.synchronize()
    bad = [i for i, ((_, _, C), Cs) in enumerate(zip(dev, seq)) if not torch.equal(C, Cs)]
    assert not bad, f"batched != sequential for problems {bad[:10]}"


def test_batch512_per_class_equals_sequential(batch512):
    torch = require_gpu()
    from paper_1607_00291_amd import tc
    dtype, probs, dev, batch = batch512
    batch.tile = -1
    info = batch.info()
    classes = sorted({batch.problem_tile(i) for i in range(COUNT)})
    print(f"case batch512 {np.dtype(dtype).name} per-class {info} classes {classes}", flush=True)
    run_and_compare(torch, tc, probs, dev, batch)


def test_batch512_every_single_class_equals_sequential(batch512):
    torch = require_gpu()
    from paper_1607_00291_amd import tc
    dtype, probs, dev, batch = batch512
    code = tc.TC_F64 if dtype == np.float64 else tc.TC_F32
    for t in range(tc.tile_count(code)):
        MT, NT, KT, waves = tc.tile_info(code, tc.TC_NATIVE, t)
        try:
            batch.tile = t
        except tc.TCError:  # a layout batches do not run
            continue
        print(f"case batch512 {np.dtype(dtype).name} single class {t} ({MT}x{NT}x{KT})", flush=True)
        run_and_compare(torch, tc, probs, dev, batch)
    batch.tile = -1


def test_batch512_oracle_subset(batch512, oracle_mod):
    torch = require_gpu()
    dtype, probs, dev, batch = batch512
    if dtype != np.float64:
        pytest.skip("the oracle subset is checked on the FP64 batch")
    batch.tile = -1
    for _, _, C in dev:
        C.zero_()
    batch.execute()
    torch.cuda.synchronize()
    sub = oracle_subset(probs)
    print(f"case batch512 oracle subset ({len(sub)} problems, "
          f"{sum(probs[i].flops() for i in sub) / 1e9:.1f} GFLOP)", flush=True)
    for i in sub:
        p = probs[i]
        ref = np.array(p.C, order="F", copy=True)
        oracle_mod.contract(p.alpha, p.A, p.idx_A, p.B, p.idx_B, p.beta, ref, p.idx_C)
        bound = fp64_bound(p.mnk()[2], p.alpha, np.max(np.abs(p.A)), np.max(np.abs(p.B)))
        err = np.max(np.abs(to_host(dev[i][2]) - ref))
        assert err <= bound, f"{p.name}: {err:.3e} > {bound:.3e}"
