"""Benchmark of the transpose-free contraction on one GPU.  Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--settle-ms S] [--no-cpu] [--quick] [--sections S]
                 [--tile T] [--copy-calibration]

Headline workload (value, roofline): the FP64 forward of the coupled-cluster
shaped contraction Z[abij] = sum_{k,c} W[akic] T[cbkj] + Z with a,b,c = 96 and
i,j,k = 24 (alpha = beta = 1), inputs resident in HBM.  A step is one full
contraction (one kernel launch); value = 2mnk / mean step time over the K
timed steps (two hipEvents around them).  Before the W warm-up steps the same
launch is repeated for --settle-ms of wall time (default 400) while the engine
clock is sampled, so that the timed steps do not run while the clock ramps up
from idle (it needs about 20 ms of sustained load after any idle gap of a
few milliseconds); the line reports the settle phase, the sampled clock, and
the median, min and max of per-launch times from a pass of K launches with a
hipEvent between consecutive launches, run between the warm-up and the timed
steps.

The same line carries, under "secondary", the other workloads measured on the
same GPU: FP32 and split-BF16 at the same shape, the FP32 forward + backward of
C[ijab] = A[iklb] B[kjal] (i,j,k,l = 32, a,b = 64), the FP64 extent-16
contraction C[abcd] = A[aebf] B[dfce], 512 batched FP64 contractions against
512 sequential launches, the transpose-transpose-GEMM-transpose method
(Sec. 5, fig. TTGT) on the same GPU at the v=96/o=24 and the FP32 forward
shapes, a sweep of random contractions (Sec. 9.2) against plain GEMMs of the
same size, and the pack and store stages alone with their HBM GB/s (unless
--quick; --sections fp32,fwdbwd,x16,packstore,ttgt,batched,sweep picks a
subset).

  --copy-calibration first runs a plain 1 GiB device copy three times in the
  same process: the reference that scales rocprofv3's HBM byte counters.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6
PEAK_FP32_TFLOPS = 157.3
PEAK_BF16_TFLOPS = 2500.0
WORKLOAD = "Z[abij]+=W[akic]T[cbkj] v=96 o=24 fp64"


# the sources that define the contraction kernels and the plans they run
KERNEL_SOURCES = ("kernels_impl.hpp", "tiles.hpp", "launch.hpp", "plan.hpp", "kernels.hip", "k_f64_i32.hip",
                  "k_f64_i64.hip", "k_f32_i32.hip", "k_f32_i64.hip", "plan.cpp")


def _code_only(text):
    """C++ source without its comments and blank lines (the hash below
    follows the code, not its commentary)."""
    import re
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    return "\n".join(line.rstrip() for line in text.splitlines() if line.strip())


def kernel_source_hash():
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_1607_00291_amd", "csrc")
    for f in KERNEL_SOURCES:
        with open(os.path.join(d, f), encoding="utf-8") as fh:
            h.update(_code_only(fh.read()).encode())
    return h.hexdigest()[:16]


def load_traffic(workload_key):
    """HBM bytes per launch of the dominant kernel from the committed
    rocprofv3 counter summary, or None when the kernel sources changed since
    the counters were taken."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as fh:
            rec = json.load(fh).get(workload_key)
    except (OSError, ValueError):
        return None
    if not rec or rec.get("kernel_hash") != kernel_source_hash():
        return None
    return rec.get("bytes_per_launch")


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(p, target_s=9.0):
    """The oracle timed on the host on a bounded sample of output elements
    (each a full-length contracted sum), scaled to GFLOP/s: once on every core
    this process may use (the reported value) and once on one thread."""
    import oracle
    threads = oracle.default_threads()
    K = p.mnk()[2]
    rng = np.random.default_rng(1234)

    def run(npts, nthr):
        pts = np.stack([rng.integers(0, n, npts) for n in p.C.shape], axis=1)
        t0 = time.perf_counter()
        oracle.contract_points(p.alpha, p.A, p.idx_A, p.B, p.idx_B, p.beta, p.C, p.idx_C, pts, threads=nthr)
        return time.perf_counter() - t0

    def rate(nthr, probe):
        t = run(probe, nthr)
        n2 = int(min(max(probe * target_s / max(t, 1e-3), probe), 20_000_000))
        t2 = run(n2, nthr)
        return 2.0 * K * n2 / t2 / 1e9, n2, t2

    g_all, n_all, t_all = rate(threads, 4096)
    g_one, n_one, t_one = rate(1, 256)
    return {"value": round(g_all, 4), "unit": "GFLOP/s", "cores": threads, "kind": "oracle",
            "single_thread_value": round(g_one, 4), "cpu_model": cpu_model(),
            "sample": f"random output elements of Z, each a full K={K} FP64 sum: {n_all} on {threads} threads "
                      f"({t_all:.1f} s), {n_one} on 1 thread ({t_one:.1f} s)"}


def dev(a, dtype=None):
    """Device tensor with the numpy array's shape and element strides."""
    import torch
    a = np.asarray(a) if dtype is None else np.asarray(a).astype(dtype, order="K")
    strides = [s // a.itemsize for s in a.strides]
    span = 1 + sum((d - 1) * s for d, s in zip(a.shape, strides)) if a.size else 1
    base = torch.zeros(span, dtype=torch.from_numpy(np.zeros(1, a.dtype)).dtype, device="cuda")
    t = torch.as_strided(base, a.shape, strides)
    if a.size:
        t.copy_(torch.from_numpy(np.ascontiguousarray(a).reshape(a.shape)).cuda())
    return t


def progress(msg):
    """One line on stderr when a section of the benchmark has finished."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def sclk_reader():
    """A function returning the current engine clock in MHz (the active level
    of the DPM table in sysfs) or None where it cannot be read."""
    import glob
    paths = sorted(glob.glob("/sys/class/drm/card*/device/pp_dpm_sclk"))

    def read():
        for path in paths:
            try:
                with open(path) as fh:
                    for line in fh:
                        if line.rstrip().endswith("*"):
                            return int(line.split(":")[1].strip().split("Mhz")[0].split("MHz")[0])
            except (OSError, ValueError, IndexError):
                continue
        return None
    return read


def time_launches(fn, steps, warmup, settle_ms=0.0):
    """Time `steps` back-to-back calls on the current stream.

    First, optionally, a clock-settle phase: calls repeated for `settle_ms`
    of wall time (synchronising every 16 calls) while the engine clock is
    sampled; the engine clock drops within milliseconds of the GPU going idle
    and needs about 20 ms of sustained load to come back, so the phases below
    follow it with no idle gap.  Then `warmup` untimed calls, a pass of
    `steps` calls with a hipEvent between consecutive calls (per-launch
    median, min and max; the events add a few microseconds between kernels),
    and the timed pass: `steps` calls bracketed by two hipEvents, whose mean
    is the reported time per step."""
    import threading
    import torch
    settle = {"launches": 0, "ms": 0.0, "sclk_mhz": []}
    th = stop = None
    samples = []
    if settle_ms > 0:
        read = sclk_reader()
        stop = threading.Event()

        def sample():
            while not stop.is_set():
                v = read()
                if v is not None:
                    samples.append(v)
                time.sleep(0.02)
        th = threading.Thread(target=sample, daemon=True)
        th.start()
        t0 = time.perf_counter()
        while (time.perf_counter() - t0) * 1e3 < settle_ms:
            for _ in range(16):
                fn()
            settle["launches"] += 16
            torch.cuda.synchronize()
        settle["ms"] = round((time.perf_counter() - t0) * 1e3, 1)
        stop.set()  # joined after the timed pass, so no idle gap here
    for _ in range(warmup):
        fn()
    s = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    ev[0].record(s)
    for i in range(steps):
        fn()
        ev[i + 1].record(s)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(s)
    for _ in range(steps):
        fn()
    e1.record(s)
    torch.cuda.synchronize()
    if th is not None:
        th.join()
        settle["sclk_mhz"] = sorted(set(samples))
    per = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(steps)])
    return {"mean": e0.elapsed_time(e1) / steps, "median": float(np.median(per)),
            "min": float(per.min()), "max": float(per.max()), "settle": settle}


def time_calls(fn, steps, warmup, settle_ms=60.0, hold=None):
    """Mean milliseconds per call, hipEvent timing on the current stream,
    after `warmup` untimed calls that continue (synchronising every 8 calls)
    until `settle_ms` of wall time have passed, so that the engine clock is
    back from idle when the timed calls start.  `hold`, when given, enqueues
    GPU work ahead of the start event that lasts longer than the host takes
    to enqueue the timed calls: they then run back to back, and the events
    time the kernels rather than the host's per-call overhead (for kernels
    shorter than that overhead)."""
    import torch
    t0 = time.perf_counter()
    done = 0
    while done < warmup or (time.perf_counter() - t0) * 1e3 < settle_ms:
        fn()
        done += 1
        if done % 8 == 0:
            torch.cuda.synchronize()
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    if hold is not None:
        hold()
    e0.record(s)
    for _ in range(steps):
        fn()
    e1.record(s)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def plan_runner(tc, A, ia, B, ib, C, ic, alpha, beta, mode="native"):
    import torch
    plan = tc.Plan.for_tensors(A, ia, B, ib, C, ic, mode=mode)
    plan.upload()
    lib, h = tc.lib(), plan.handle
    Ap, Bp, Cp = A.data_ptr(), B.data_ptr(), C.data_ptr()
    sp = torch.cuda.current_stream().cuda_stream

    def run():
        tc._check(lib.tc_plan_execute(h, alpha, Ap, Bp, beta, Cp, sp))
    return plan, run


SECTIONS = ("fp32", "fwdbwd", "x16", "packstore", "ttgt", "batched", "sweep")
PEAK_HBM_GBPS = 8000.0


def secondary(tc, inputs, steps, warmup, sections=SECTIONS):
    import torch
    out = {}
    if "fp32" in sections:
        _fp32(tc, inputs, steps, warmup, out)
    if "fwdbwd" in sections:
        _fwdbwd(tc, inputs, steps, warmup, out)
    if "x16" in sections:
        _x16(tc, inputs, steps, warmup, out)
    if "packstore" in sections:
        out["pack_store_fp64_v96_o24"] = pack_store(tc, inputs, steps, warmup)
        progress("pack and store stages done")
    if "ttgt" in sections:
        out["ttgt_baseline"] = ttgt_baseline(tc, inputs, steps, warmup)
        progress("TTGT baseline done")
    if "batched" in sections:
        out["batched_512_fp64"] = batched(tc, inputs, steps, warmup)
        progress("batched 512 done")
    if "sweep" in sections:
        out["random_sweep_fp64"] = sweep(tc, inputs, max(steps // 2, 5), 2)
    torch.cuda.empty_cache()
    return out


def _fp32(tc, inputs, steps, warmup, out):
    # FP32 and split-BF16 at the v=96/o=24 shape
    p = inputs.cfg2()
    m, n, k = p.mnk()
    fl = 2.0 * m * n * k
    A, B, C = dev(p.A, np.float32), dev(p.B, np.float32), dev(p.C, np.float32)
    for mode, peak, mult in (("native", PEAK_FP32_TFLOPS, 1), ("split_bf16x3", PEAK_BF16_TFLOPS, 3)):
        plan, run = plan_runner(tc, A, p.idx_A, B, p.idx_B, C, p.idx_C, 1.0, 1.0, mode)
        ms = time_calls(run, steps, warmup)
        d = plan.describe()
        key = "fp32_v96_o24" if mode == "native" else "split_bf16_v96_o24"
        out[key] = {"gflops": round(fl / ms / 1e6, 1), "ms": round(ms, 4),
                    "frac_of_peak": round(mult * fl / ms / 1e9 / peak, 4),
                    "peak_tflops": peak, "tile": [d["MT"], d["NT"], d["KT"]], "layout": d["layout"]}
        if mult == 3:
            out[key]["note"] = "frac counts the three bf16 products (3 * 2mnk) against the dense bf16 peak"
            if d["workspace_bytes"]:
                out[key]["workspace_bytes"] = d["workspace_bytes"]
                out[key]["note"] += "; layout 4: a split-and-pack pass, then the tile on the packed hi/lo panels (both timed)"
        plan.close()
    del A, B, C
    progress("FP32 and split-BF16 at v=96/o=24 done")


def _fwdbwd(tc, inputs, steps, warmup, out):
    # FP32 forward + backward, C[ijab] = A[iklb] B[kjal]
    p = inputs.cfg4()
    A, B, dC = dev(p.A, np.float32), dev(p.B, np.float32), dev(p.dC, np.float32)
    C = dev(p.C, np.float32)
    dA = dev(np.zeros_like(p.A, order="F"), np.float32)
    dB = dev(np.zeros_like(p.B, order="F"), np.float32)
    runs = {
        "fwd": plan_runner(tc, A, p.idx_A, B, p.idx_B, C, p.idx_C, 1.0, 0.0),
        "dA": plan_runner(tc, dC, p.idx_C, B, p.idx_B, dA, p.idx_A, 1.0, 0.0),
        "dB": plan_runner(tc, A, p.idx_A, dC, p.idx_C, dB, p.idx_B, 1.0, 0.0),
    }
    fl4 = 2.0 * 2048 * 2048 * 1024
    rec = {}
    tot = 0.0
    for name, (plan, run) in runs.items():
        ms = time_calls(run, steps, warmup)
        tot += ms
        rec[name] = {"gflops": round(fl4 / ms / 1e6, 1), "ms": round(ms, 4),
                     "frac_of_fp32_peak": round(fl4 / ms / 1e9 / PEAK_FP32_TFLOPS, 4)}
        plan.close()
    rec["fwd_bwd"] = {"gflops": round(3 * fl4 / tot / 1e6, 1), "ms": round(tot, 4),
                      "frac_of_fp32_peak": round(3 * fl4 / tot / 1e9 / PEAK_FP32_TFLOPS, 4)}
    # the same through torch.autograd (Contract.apply + backward)
    from paper_1607_00291_amd.autograd import contract
    Ag = A.detach().requires_grad_(True)
    Bg = B.detach().requires_grad_(True)

    def fb():
        Ag.grad = None
        Bg.grad = None
        contract(Ag, p.idx_A, Bg, p.idx_B, p.idx_C).backward(dC)
    ms = time_calls(fb, max(steps // 2, 3), 2)
    rec["autograd_fwd_bwd"] = {"gflops": round(3 * fl4 / ms / 1e6, 1), "ms": round(ms, 4)}
    out["fp32_fwd_bwd_ijab_iklb_kjal"] = rec
    progress("FP32 forward + backward done")
    del A, B, C, dA, dB, dC, Ag, Bg


def _x16(tc, inputs, steps, warmup, out):
    # FP64 extent-16 contraction (latency-bound)
    p = inputs.cfg1()
    A, B, C = dev(p.A), dev(p.B), dev(p.C)
    plan, run = plan_runner(tc, A, p.idx_A, B, p.idx_B, C, p.idx_C, 1.0, 0.0)
    ms = time_calls(run, steps * 4, warmup)
    out["fp64_abcd_aebf_dfce_x16"] = {"us_per_call": round(ms * 1e3, 2), "gflops": round(p.flops() / ms / 1e6, 1)}
    plan.close()
    del A, B, C


def pack_store(tc, inputs, steps, warmup):
    """The contraction's pack stage (gather of W and of T into tile panels)
    and store stage (Z := Z0 + src through the C offset vectors, beta = 1)
    run alone at the v=96/o=24 FP64 shape with the plan's own tile, against
    the HBM peak.  Algorithmic bytes: the operand elements gathered and the
    panel written (pack), src and C read and C written (store), plus 4 bytes
    per distinct offset entry each workgroup reads (a sliver's R row offsets
    and KT k offsets; a fragment's 16 row and 16 column offsets)."""
    import torch
    p = inputs.cfg2()
    W, T, Z = dev(p.A), dev(p.B), dev(p.C)
    plan = tc.Plan.for_tensors(W, p.idx_A, T, p.idx_B, Z, p.idx_C)
    plan.upload()
    d = plan.describe()
    lib, h = tc.lib(), plan.handle
    sp = torch.cuda.current_stream().cuda_stream
    res = {"tile": [d["MT"], d["NT"], d["KT"]]}
    nkb = -(-d["k"] // d["KT"])
    Wp, Tp, Zp = W.data_ptr(), T.data_ptr(), Z.data_ptr()
    n_hold = 4 + steps // 10  # about 0.4 ms of contraction per 10 timed calls of about 30 us of host time

    def hold():
        for _ in range(n_hold):
            tc._check(lib.tc_plan_execute(h, 1.0, Wp, Tp, 0.0, Zp, sp))
    for operand, (src, name) in enumerate(((W, "pack_W"), (T, "pack_T"))):
        elems = plan.pack_elements(operand)
        dst = torch.empty(elems, dtype=torch.float64, device="cuda")
        x = (operand == 0) != d["swapped"]
        R = d["MT"] if x else d["NT"]
        rows = d["m"] if x else d["n"]
        slivers = -(-rows // R) * nkb
        sp_, dp_ = src.data_ptr(), dst.data_ptr()

        def run(op=operand, a=sp_, b=dp_):
            tc._check(lib.tc_plan_pack(h, op, a, b, sp))
        ms = time_calls(run, steps, warmup, hold=hold)
        moved = 8 * (rows * d["k"] + elems) + 4 * slivers * (R + d["KT"])
        res[name] = {"us": round(ms * 1e3, 2), "bytes": moved, "gbps": round(moved / ms / 1e6, 1),
                     "frac_of_hbm_peak": round(moved / ms / 1e6 / PEAK_HBM_GBPS, 4)}
        del dst
    m, n = d["m"], d["n"]
    src = torch.empty(m * n, dtype=torch.float64, device="cuda").normal_()
    frags = d["tiles_m"] * d["tiles_n"] * (d["MT"] // 16) * (d["NT"] // 16)
    a, b = src.data_ptr(), Z.data_ptr()

    def store():
        tc._check(lib.tc_plan_store(h, 1.0, a, 1.0, b, sp))
    ms = time_calls(store, steps, warmup, hold=hold)
    moved = 8 * 3 * m * n + 4 * 32 * frags
    res["store_Z_beta1"] = {"us": round(ms * 1e3, 2), "bytes": moved, "gbps": round(moved / ms / 1e6, 1),
                            "frac_of_hbm_peak": round(moved / ms / 1e6 / PEAK_HBM_GBPS, 4)}
    plan.close()
    del W, T, Z, src
    torch.cuda.empty_cache()
    return res


def ttgt_baseline(tc, inputs, steps, warmup):
    """The transpose-transpose-GEMM-transpose method (Sec. 5, fig. TTGT) on the same
    GPU: permute-copies into matrix layout, one matrix product of the same
    kernels, permute-copy back; against the transpose-free contraction."""
    import torch
    res = {}
    cases = (("fp64_v96_o24", inputs.cfg2(), None, 1.0),
             ("fp32_ijab_iklb_kjal_fwd", inputs.cfg4(), np.float32, 0.0))
    for key, p, dt, beta in cases:
        A, B, C = dev(p.A, dt), dev(p.B, dt), dev(p.C, dt)
        plan, run = plan_runner(tc, A, p.idx_A, B, p.idx_B, C, p.idx_C, 1.0, beta)
        ms_free = time_calls(run, steps, warmup)
        plan.close()
        t = tc.TTGT(A, p.idx_A, B, p.idx_B, C, p.idx_C, 1.0, beta)
        ms_in = time_calls(t.transpose_in, steps, warmup)
        ms_gemm = time_calls(t.gemm, steps, warmup)
        ms_out = time_calls(t.transpose_out, steps, warmup)
        ms_all = time_calls(t.run, steps, warmup)
        elt = A.element_size()
        moved = A.numel() + B.numel() + C.numel() * (2 if beta != 0.0 else 1)  # elements permuted per run
        fl = 2.0 * t.m * t.n * t.k
        res[key] = {
            "transpose_free_ms": round(ms_free, 4),
            "ttgt_ms": round(ms_all, 4),
            "ttgt_over_transpose_free": round(ms_all / ms_free, 3),
            "transpose_ms": round(ms_in + ms_out, 4),
            "gemm_ms": round(ms_gemm, 4),
            "transpose_fraction": round((ms_in + ms_out) / (ms_in + ms_gemm + ms_out), 4),
            "permute_gbps": round(2.0 * elt * moved / ((ms_in + ms_out) * 1e6), 1),
            "gemm_gflops": round(fl / ms_gemm / 1e6, 1),
            "extra_workspace_bytes": t.workspace_bytes(),
        }
        t.close()
        del A, B, C, t
        torch.cuda.empty_cache()
    return res


def sweep(tc, inputs, steps, warmup, square=(512, 1024, 2048, 4096), rankk=(8, 32, 128, 512), big=4096, seeds=3):
    """Random contractions in the manner of the paper's generator (Sec. 9.2),
    FP64: square shapes m ~ n ~ k and rank-k shapes m ~ n ~ 4096 with small k,
    each timed against a plain column-major GEMM of the same m, n, k run by
    the same library (the transpose-free path's cost of arbitrary layouts).
    Also reports the fraction of C tiles and k blocks with a constant block
    stride (the fast-path share, Sec. 6.2)."""
    import torch
    rows = []
    cases = [("square", t, t, t) for t in square] + [("rank-k", big, big, kk) for kk in rankk]
    for kind, m0, n0, k0 in cases:
        rates, gemm_rates, fast_c, fast_k = [], [], [], []
        for sd in range(seeds):
            p = inputs.sweep_problem(1000 * sd + m0 + k0, m0, n0, k0)
            m, n, k = p.mnk()
            A, B, C = dev(p.A), dev(p.B), dev(p.C)
            plan, run = plan_runner(tc, A, p.idx_A, B, p.idx_B, C, p.idx_C, 1.0, 0.0)
            d = plan.describe()
            ms = time_calls(run, steps, warmup)
            plan.close()
            del A, B, C
            A2 = torch.zeros(k, m, dtype=torch.float64, device="cuda").t()
            B2 = torch.zeros(n, k, dtype=torch.float64, device="cuda").t()
            C2 = torch.zeros(n, m, dtype=torch.float64, device="cuda").t()
            A2.normal_()
            B2.normal_()
            plan, run = plan_runner(tc, A2, "ik", B2, "kj", C2, "ij", 1.0, 0.0)
            ms_g = time_calls(run, steps, warmup)
            plan.close()
            del A2, B2, C2
            rates.append(2.0 * m * n * k / ms / 1e6)
            gemm_rates.append(2.0 * m * n * k / ms_g / 1e6)
            fast_c.append(d["c_tiles_regular"] / max(d["tiles_m"] * d["tiles_n"], 1))
            kb = max(d["k_blocks"], 1)
            fast_k.append(min(d["k_blocks_regular_x"], d["k_blocks_regular_y"]) / kb)
        progress(f"sweep {kind} {m0}x{n0}x{k0} done")
        rows.append({"kind": kind, "target_mnk": [m0, n0, k0], "instances": seeds,
                     "gflops_mean": round(float(np.mean(rates)), 1), "gflops_min": round(float(np.min(rates)), 1),
                     "gemm_gflops_mean": round(float(np.mean(gemm_rates)), 1),
                     "ratio_to_gemm": round(float(np.mean(np.array(rates) / np.array(gemm_rates))), 3),
                     "fast_c_tiles": round(float(np.mean(fast_c)), 3),
                     "fast_k_blocks": round(float(np.mean(fast_k)), 3)})
    torch.cuda.empty_cache()
    return rows


def batched(tc, inputs, steps, warmup):
    """512 contractions (extents 4..64, random permutations) as one batch
    (persistent launches, one per tile class, or one class for all if the
    autotuner finds that faster) against 512 sequential plan launches.  Also
    reports the default mode (every problem in the class the planner picks for
    it): its total time and, per tile class, the problems, flop share and the
    time of that class's launch timed alone."""
    import torch
    probs, tensors, total = [], [], 0.0
    for i in range(512):
        p = inputs.cfg5_instance(i)
        A, B, C = dev(p.A), dev(p.B), dev(p.C)
        probs.append(p)
        tensors.append((A, B, C))
        total += p.flops()
    items = [(A, p.idx_A, B, p.idx_B, C, p.idx_C, 1.0, 0.0) for p, (A, B, C) in zip(probs, tensors)]
    batch = tc.Batch(items)
    reps = max(steps // 5, 3)
    ms_pc = time_calls(batch.execute, reps, 1)
    classes = {}
    for i in range(len(probs)):
        t = batch.problem_tile(i)
        if t >= 0:
            classes.setdefault(t, []).append(i)
    per_class = {}
    for t, idx in sorted(classes.items()):
        sub = tc.Batch([items[i] for i in idx])
        sub.tile = t
        ms = time_calls(sub.execute, reps, 1)
        fl = sum(probs[i].flops() for i in idx)
        per_class[str(t)] = {"problems": len(idx), "flop_share": round(fl / total, 4), "ms": round(ms, 3),
                             "gflops": round(fl / ms / 1e6, 1)}
        sub.close()
    tile, _ = batch.autotune(reps=2)
    ms_b = time_calls(batch.execute, reps, 1)
    plans = [plan_runner(tc, A, p.idx_A, B, p.idx_B, C, p.idx_C, 1.0, 0.0) for p, (A, B, C) in zip(probs, tensors)]

    def seq():
        for _, run in plans:
            run()
    ms_s = time_calls(seq, max(steps // 5, 3), 1)
    info = batch.info()
    for plan, _ in plans:
        plan.close()
    batch.close()
    del tensors
    torch.cuda.empty_cache()
    return {"problems": 512, "total_gflop": round(total / 1e9, 1), "batched_ms": round(ms_b, 3),
            "sequential_ms": round(ms_s, 3), "speedup": round(ms_s / ms_b, 3),
            "batched_gflops": round(total / ms_b / 1e6, 1),
            "batched_frac_of_fp64_peak": round(total / ms_b / 1e9 / PEAK_FP64_TFLOPS, 4),
            "sequential_gflops": round(total / ms_s / 1e6, 1), "batch_tile": tile,
            "work_items": info["work_items"], "grid": info["grid"],
            "default_per_class": {"ms": round(ms_pc, 3), "gflops": round(total / ms_pc / 1e6, 1),
                                  "classes": per_class}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    # 100 untimed launches bring the matrix cores to their sustained clock
    # (5 left the first timed launches measurably slower)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--quick", action="store_true", help="headline workload only (no secondary workloads)")
    ap.add_argument("--sections", default=",".join(SECTIONS),
                    help="comma-separated secondary workloads to run after the headline: " + ",".join(SECTIONS))
    ap.add_argument("--tile", type=int, default=None, help="force a tile configuration")
    ap.add_argument("--settle-ms", type=float, default=400.0,
                    help="before the warm-up steps, repeat the headline launch for this long (wall time) so the "
                         "engine clock has left its idle level; the clock is sampled meanwhile (0: off)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a plain 1 GiB device copy three times (the reference for HBM byte "
                         "counters, taken in the same process as the contraction)")
    args = ap.parse_args()
    sections = [x for x in args.sections.split(",") if x]
    bad = [x for x in sections if x not in SECTIONS]
    if bad:
        print(f"bench.py: unknown section(s) {bad}; choose from {list(SECTIONS)}", file=sys.stderr)
        sys.exit(2)
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1607_00291_amd import inputs, tc

    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    torch.cuda.set_device(0)
    if args.copy_calibration:
        x = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": x.numel() * 8, "copy_bytes_written": y.numel() * 8, "launches": 3}),
              file=sys.stderr, flush=True)
        del x, y
    p = inputs.cfg2()
    m, n, k = p.mnk()
    flops = 2.0 * m * n * k
    W, T, Z = dev(p.A), dev(p.B), dev(p.C)
    plan, run = plan_runner(tc, W, p.idx_A, T, p.idx_B, Z, p.idx_C, p.alpha, p.beta)
    if args.tile is not None:
        plan.tile = args.tile
        plan.upload()
    desc = plan.describe()
    t_wall = time.perf_counter()
    tm = time_launches(run, args.steps, args.warmup, settle_ms=args.settle_ms)
    wall = time.perf_counter() - t_wall
    ms = tm["mean"]
    gflops = flops / (ms * 1e-3) / 1e9
    achieved_tf = gflops / 1e3
    sclk_after = sclk_reader()()
    plan.close()
    del W, T, Z

    line = {
        "metric": "contraction GFLOP/s (FP64 forward; % of FP64 matrix-core peak in roofline)",
        "value": round(gflops, 2),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded normal inputs, column-major)",
        "config": {"workload": WORKLOAD, "m": m, "n": n, "k": k, "alpha": p.alpha, "beta": p.beta,
                   "tile": [desc["MT"], desc["NT"], desc["KT"]], "waves": desc["waves"],
                   "x_lanes": desc["x_lanes"], "y_lanes": desc["y_lanes"], "parallelism": "single GPU"},
        "roofline": {"bound": "mfma", "achieved": round(achieved_tf, 3), "peak": PEAK_FP64_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(achieved_tf / PEAK_FP64_TFLOPS, 4),
                     "traffic": load_traffic(WORKLOAD), "algorithmic_flops_per_launch": flops,
                     "mean_launch_ms": round(ms, 5), "median_launch_ms": round(tm["median"], 5),
                     "min_launch_ms": round(tm["min"], 5), "max_launch_ms": round(tm["max"], 5),
                     "frac_at_median": round(flops / (tm["median"] * 1e-3) / 1e12 / PEAK_FP64_TFLOPS, 4),
                     "per_launch_note": "median/min/max from a pass with a hipEvent between launches"},
        "clock": {"settle_launches": tm["settle"]["launches"], "settle_ms": tm["settle"]["ms"],
                  "sclk_mhz_sysfs_during_settle": tm["settle"]["sclk_mhz"], "sclk_mhz_sysfs_after_timed": sclk_after,
                  "sclk_note": "active DPM level read from sysfs pp_dpm_sclk (a slowly averaged value)"},
        "wall_s_timed_region": round(wall, 3),
    }
    if not args.quick:
        line["secondary"] = secondary(tc, inputs, max(args.steps // 2, 10), max(args.warmup, 5), sections)
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(p)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
