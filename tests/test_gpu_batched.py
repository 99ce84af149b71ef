"""Batched contractions in persistent launches (one per tile class): bitwise equality with
sequential launches with a regular tile configuration, parity with the oracle,
and graph capture with several replays."""
import numpy as np
import pytest

from paper_1607_00291_amd import inputs
from gpuutil import fp64_bound, require_gpu, to_dev, to_host

pytestmark = pytest.mark.gpu


def subset(n):
    """The n cheapest instances of the 512-problem workload, plus 4 large ones."""
    probs = [inputs.cfg5_instance(i) for i in range(64)]
    probs.sort(key=lambda p: p.flops())
    return probs[:n] + probs[-4:]


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_batched_equals_sequential_and_oracle(oracle_mod, dtype):
    torch = require_gpu()
    from paper_1607_00291_amd import tc
    probs = subset(24)
    dev = [(to_dev(p.A, dtype), to_dev(p.B, dtype), to_dev(p.C, dtype)) for p in probs]
    seq_out = [to_dev(p.C, dtype) for p in probs]
    batch = tc.Batch([(A, p.idx_A, B, p.idx_B, C, p.idx_C, p.alpha, p.beta) for p, (A, B, C) in zip(probs, dev)])
    batch.tile = 1  # one regular class: bitwise comparable with sequential launches
    info = batch.info()
    print(f"case batched dtype={dtype.__name__} {info}", flush=True)
    batch.execute()
    # sequential launches with a regular tile: every regular configuration
    # sums each output in the same order, so any of them matches bitwise
    for p, (A, B, _), Cs in zip(probs, dev, seq_out):
        plan = tc.Plan.for_tensors(A, p.idx_A, B, p.idx_B, Cs, p.idx_C)
        plan.tile = 1
        plan.execute(A, B, Cs, p.alpha, p.beta)
        plan.close()
    torch.cuda.synchronize()
    for p, (_, _, C), Cs in zip(probs, dev, seq_out):
        assert np.array_equal(to_host(C), to_host(Cs)), p.name
    if dtype == np.float64:
        for p, (_, _, C) in zip(probs[:8] + probs[-2:], dev[:8] + dev[-2:]):
            ref = np.array(p.C, order="F", copy=True)
            oracle_mod.contract(p.alpha, p.A, p.idx_A, p.B, p.idx_B, p.beta, ref, p.idx_C)
            bound = fp64_bound(p.mnk()[2], p.alpha, np.max(np.abs(p.A)), np.max(np.abs(p.B)))
            assert np.max(np.abs(to_host(C) - ref)) <= bound, p.name
    batch.close()


def test_batched_every_tile_and_graph_replay(oracle_mod):
    torch = require_gpu()
    from paper_1607_00291_amd import tc
    probs = subset(12)
    dev = [(to_dev(p.A), to_dev(p.B), to_dev(p.C)) for p in probs]
    batch = tc.Batch([(A, p.idx_A, B, p.idx_B, C, p.idx_C, 1.0, 0.0) for p, (A, B, C) in zip(probs, dev)])
    ref = None
    # regular tiles first (bitwise among themselves), then per-problem classes
    # and the specialised-wave pinwheel (which sums its centre in another
    # order: compared within the FP64 bound)
    order = [t for t in range(tc.tile_count(tc.TC_F64)) if tc.tile_info(tc.TC_F64, tc.TC_NATIVE, t)[0] != 144]
    order += [-1] + [t for t in range(tc.tile_count(tc.TC_F64)) if t not in order and t != 4]
    for t in order:
        MT = tc.tile_info(tc.TC_F64, tc.TC_NATIVE, t)[0] if t >= 0 else -1
        batch.tile = t
        for _, _, C in dev:
            C.zero_()
        batch.execute()
        torch.cuda.synchronize()
        outs = [to_host(C) for _, _, C in dev]
        print(f"case batched tile={t}", flush=True)
        if ref is None:
            ref = outs
        elif MT == 144 or t == -1:
            for p, a, b in zip(probs, ref, outs):
                bound = fp64_bound(p.mnk()[2], 1.0, np.max(np.abs(p.A)), np.max(np.abs(p.B)))
                assert np.max(np.abs(a - b), initial=0.0) <= 2 * bound, p.name
        else:  # every regular tile sums in the same order: bitwise equal
            for a, b in zip(ref, outs):
                assert np.array_equal(a, b)
    # graph capture of the persistent launches (one per tile class present),
    # replayed with eager work in between; every replay must reproduce the
    # eager result
    batch.tile = -1
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        batch.execute(stream=s)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    ref = [to_host(C) for _, _, C in dev]  # the eager result of this configuration
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        batch.execute()
    for rep in range(3):
        for _, _, C in dev:
            C.fill_(float(rep + 7))  # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for a, (_, _, C) in zip(ref, dev):
            assert np.array_equal(a, to_host(C)), f"replay {rep}"
    batch.close()


def test_autotune_batch_and_plan():
    torch = require_gpu()
    from paper_1607_00291_amd import tc
    probs = subset(6)
    dev = [(to_dev(p.A), to_dev(p.B), to_dev(p.C)) for p in probs]
    batch = tc.Batch([(A, p.idx_A, B, p.idx_B, C, p.idx_C, 1.0, 0.0) for p, (A, B, C) in zip(probs, dev)])
    tile, ms = batch.autotune(reps=2)
    assert ms > 0 and -1 <= tile < tc.tile_count(tc.TC_F64)
    p = probs[-1]
    A, B, C = dev[-1]
    plan = tc.Plan.for_tensors(A, p.idx_A, B, p.idx_B, C, p.idx_C)
    tile, ms = plan.autotune(A, B, C, reps=2)
    assert ms > 0
    # a new plan with the same signature starts from the tuned tile
    plan2 = tc.Plan.for_tensors(A, p.idx_A, B, p.idx_B, C, p.idx_C)
    assert plan2.tile == tile
    plan.close()
    plan2.close()
    batch.close()


def test_contract_batched_one_shot(oracle_mod):
    """tc_contract_batched (one call: plans, batch, run, free) gives, bit for
    bit, what a batch built with tc_batch_create gives (the same plans and
    per-problem tile classes), on cfg5 instances, a ragged problem with
    beta != 0 and one whose operands' unit strides lie on different
    contracted indices; every output against the oracle."""
    torch = require_gpu()
    from paper_1607_00291_amd import tc
    probs = subset(12) + [inputs.random_problem(7100, 2, 2, 2, lo=3, hi=23, beta=0.5, alpha=-1.5),
                          inputs.p_conflict_problem(7101, {"e": 13, "g": 3, "f": 10, "i": 150, "j": 70}, beta=0.25)]
    dev = [(to_dev(p.A), to_dev(p.B), to_dev(p.C)) for p in probs]
    one = [to_dev(p.C) for p in probs]
    print(f"case contract_batched {len(probs)} problems", flush=True)
    tc.contract_batched([(A, p.idx_A, B, p.idx_B, C1, p.idx_C, p.alpha, p.beta)
                         for p, (A, B, _), C1 in zip(probs, dev, one)])
    batch = tc.Batch([(A, p.idx_A, B, p.idx_B, C, p.idx_C, p.alpha, p.beta) for p, (A, B, C) in zip(probs, dev)])
    batch.execute()
    torch.cuda.synchronize()
    batch.close()
    for p, (_, _, C), C1 in zip(probs, dev, one):
        assert torch.equal(C, C1), p.name
        ref = np.array(p.C, order="F", copy=True)
        oracle_mod.contract(p.alpha, p.A, p.idx_A, p.B, p.idx_B, p.beta, ref, p.idx_C)
        bound = fp64_bound(p.mnk()[2], p.alpha, np.max(np.abs(p.A)), np.max(np.abs(p.B)), p.beta,
                           np.max(np.abs(p.C)))
        assert np.max(np.abs(to_host(C1) - ref)) <= bound, p.name
