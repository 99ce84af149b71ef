"""ctypes binding of libtc.so (the C ABI declared in include/tc.h).

Argument marshalling only: descriptors are read from torch tensors (shape,
element strides, data pointer, current HIP stream) and handed to the library;
every step of the contraction runs in the library's kernels.  A missing
library raises; there is no fallback path.
"""
import ctypes
import json
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtc.so")

TC_F64, TC_F32 = 0, 1
TC_NATIVE, TC_SPLIT_BF16X3 = 0, 1
MODES = {"native": TC_NATIVE, "split_bf16x3": TC_SPLIT_BF16X3, "split-bf16": TC_SPLIT_BF16X3}

# every symbol include/tc.h declares
EXPORTS = [
    "tc_contract", "tc_contract_noalloc", "tc_plan_create", "tc_plan_upload", "tc_plan_execute", "tc_plan_destroy",
    "tc_plan_describe", "tc_plan_pack_elements", "tc_plan_pack", "tc_plan_store", "tc_tile_count", "tc_tile_info", "tc_plan_set_tile", "tc_plan_get_tile",
    "tc_plan_autotune", "tc_batch_create", "tc_batch_execute", "tc_batch_destroy", "tc_batch_info",
    "tc_batch_set_tile", "tc_batch_autotune", "tc_batch_problem_tile", "tc_contract_batched",
    "tc_scatter_vector", "tc_block_strides", "tc_permute", "tc_status_string", "tc_last_error",
]


class TCError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"tc status {status}: {msg}")
        self.status = status


_lib = None
_i64p = ctypes.POINTER(ctypes.c_int64)
_vp = ctypes.c_void_p


class _Problem(ctypes.Structure):
    """One problem of tc_contract_batched (the arguments of tc_contract)."""
    _fields_ = [("alpha", ctypes.c_double),
                ("A", _vp), ("ndim_A", ctypes.c_int), ("lens_A", _i64p), ("strides_A", _i64p), ("idx_A", ctypes.c_char_p),
                ("B", _vp), ("ndim_B", ctypes.c_int), ("lens_B", _i64p), ("strides_B", _i64p), ("idx_B", ctypes.c_char_p),
                ("beta", ctypes.c_double),
                ("C", _vp), ("ndim_C", ctypes.c_int), ("lens_C", _i64p), ("strides_C", _i64p), ("idx_C", ctypes.c_char_p)]


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1607_00291_amd.build`")
        # torch ships its own HIP runtime under the same soname as the system
        # one that libtc.so links against.  Loaded after torch, libtc.so binds
        # to torch's copy; loaded first, it would bring in a second runtime,
        # and of two runtimes in one process only the first to initialise
        # sees the GPU.  So torch is always loaded first.
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        desc = [ctypes.c_int, _i64p, _i64p, ctypes.c_char_p]
        L.tc_contract.argtypes = ([ctypes.c_double, _vp] + desc + [_vp] + desc + [ctypes.c_double, _vp] + desc
                                  + [ctypes.c_int, ctypes.c_int, _vp])
        L.tc_contract_noalloc.argtypes = L.tc_contract.argtypes
        L.tc_plan_create.argtypes = [ctypes.POINTER(_vp)] + desc * 3 + [ctypes.c_int, ctypes.c_int]
        L.tc_plan_upload.argtypes = [_vp]
        L.tc_plan_execute.argtypes = [_vp, ctypes.c_double, _vp, _vp, ctypes.c_double, _vp, _vp]
        L.tc_plan_destroy.argtypes = [_vp]
        L.tc_plan_pack_elements.argtypes = [_vp, ctypes.c_int, _i64p]
        L.tc_plan_pack.argtypes = [_vp, ctypes.c_int, _vp, _vp, _vp]
        L.tc_plan_store.argtypes = [_vp, ctypes.c_double, _vp, ctypes.c_double, _vp, _vp]
        L.tc_plan_describe.argtypes = [_vp, ctypes.c_char_p, ctypes.c_size_t]
        L.tc_tile_count.argtypes = [ctypes.c_int, ctypes.c_int]
        ip = ctypes.POINTER(ctypes.c_int)
        L.tc_tile_info.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ip, ip, ip, ip]
        L.tc_plan_set_tile.argtypes = [_vp, ctypes.c_int]
        L.tc_plan_get_tile.argtypes = [_vp]
        L.tc_plan_autotune.argtypes = [_vp, _vp, _vp, _vp, ctypes.c_int, _vp, ctypes.POINTER(ctypes.c_double)]
        L.tc_batch_create.argtypes = [ctypes.POINTER(_vp), ctypes.c_int, ctypes.POINTER(_vp),
                                      ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_vp), ctypes.POINTER(_vp),
                                      ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_vp)]
        L.tc_batch_execute.argtypes = [_vp, _vp]
        L.tc_batch_destroy.argtypes = [_vp]
        L.tc_batch_info.argtypes = [_vp, _i64p, ip, ip]
        L.tc_batch_set_tile.argtypes = [_vp, ctypes.c_int]
        L.tc_batch_autotune.argtypes = [_vp, ctypes.c_int, _vp, ctypes.POINTER(ctypes.c_double)]
        L.tc_batch_problem_tile.argtypes = [_vp, ctypes.c_int, ip]
        L.tc_contract_batched.argtypes = [ctypes.c_int, ctypes.POINTER(_Problem), ctypes.c_int, ctypes.c_int, _vp]
        L.tc_scatter_vector.argtypes = [ctypes.c_int, _i64p, _i64p, _i64p]
        L.tc_block_strides.argtypes = [_i64p, ctypes.c_int64, ctypes.c_int64, _i64p]
        L.tc_permute.argtypes = [_vp, _vp, ctypes.c_int, _i64p, _i64p, _i64p, ctypes.c_int, _vp]
        L.tc_status_string.argtypes = [ctypes.c_int]
        L.tc_status_string.restype = ctypes.c_char_p
        L.tc_last_error.argtypes = []
        L.tc_last_error.restype = ctypes.c_char_p
        for name in EXPORTS:
            if name not in ("tc_status_string", "tc_last_error"):
                getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(st):
    if st < 0:
        L = lib()
        raise TCError(st, f"{L.tc_status_string(st).decode()}: {L.tc_last_error().decode()}")
    return st


def _arr(vals):
    vals = list(vals)
    return (ctypes.c_int64 * max(len(vals), 1))(*vals)


def _desc(shape, strides, labels):
    labels = labels.encode() if isinstance(labels, str) else labels
    if len(labels) != len(shape) or len(strides) != len(shape):
        raise ValueError("labels, shape and strides must have one entry per dimension")
    return [len(shape), _arr(shape), _arr(strides), labels]


def _dtype_code(dtype):
    import torch
    if dtype == torch.float64:
        return TC_F64
    if dtype == torch.float32:
        return TC_F32
    raise TypeError(f"unsupported dtype {dtype} (float64 or float32)")


def _stream_ptr(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return s.cuda_stream


def scatter_vector(lens, strides):
    """Offsets of every linear index of a bundle (first index fastest)."""
    n = 1
    for x in lens:
        n *= x
    out = (ctypes.c_int64 * max(n, 1))()
    _check(lib().tc_scatter_vector(len(lens), _arr(lens), _arr(strides), out))
    return list(out[:n])


def block_strides(scat, b):
    """Block-stride vector of a scatter vector for blocking b (0 = none)."""
    n = len(scat)
    nb = (n + b - 1) // b
    out = (ctypes.c_int64 * max(nb, 1))()
    _check(lib().tc_block_strides(_arr(scat), n, b, out))
    return list(out[:nb])


def tile_count(dtype=TC_F64, mode=TC_NATIVE):
    return _check(lib().tc_tile_count(dtype, mode))


def tile_info(dtype, mode, tile):
    v = [ctypes.c_int() for _ in range(4)]
    _check(lib().tc_tile_info(dtype, mode, tile, *[ctypes.byref(x) for x in v]))
    return tuple(x.value for x in v)


class Plan:
    """A planned contraction (descriptors only; data bound at execute)."""

    def __init__(self, shape_A, strides_A, idx_A, shape_B, strides_B, idx_B, shape_C, strides_C, idx_C,
                 dtype=TC_F64, mode=TC_NATIVE):
        self._h = _vp()
        self.dtype, self.mode = dtype, mode
        _check(lib().tc_plan_create(ctypes.byref(self._h), *_desc(shape_A, strides_A, idx_A),
                                    *_desc(shape_B, strides_B, idx_B), *_desc(shape_C, strides_C, idx_C),
                                    dtype, mode))

    @classmethod
    def for_tensors(cls, A, idx_A, B, idx_B, C, idx_C, mode="native"):
        mode = MODES[mode] if isinstance(mode, str) else mode
        return cls(tuple(A.shape), A.stride(), idx_A, tuple(B.shape), B.stride(), idx_B, tuple(C.shape), C.stride(),
                   idx_C, _dtype_code(C.dtype), mode)

    def describe(self):
        n = _check(lib().tc_plan_describe(self._h, None, 0))
        buf = ctypes.create_string_buffer(n + 1)
        _check(lib().tc_plan_describe(self._h, buf, n + 1))
        return json.loads(buf.value.decode())

    def upload(self):
        _check(lib().tc_plan_upload(self._h))

    def execute(self, A, B, C, alpha=1.0, beta=0.0, stream=None):
        _check(lib().tc_plan_execute(self._h, float(alpha), _ptr(A), _ptr(B), float(beta), _ptr(C),
                                     _stream_ptr(stream)))
        return C

    def execute_ptrs(self, A, B, C, alpha, beta, stream_ptr):
        return _check(lib().tc_plan_execute(self._h, float(alpha), A, B, float(beta), C, stream_ptr))

    def pack_elements(self, operand):
        """Elements of the tile-panel matrix of operand 0 (A) or 1 (B)."""
        n = ctypes.c_int64()
        _check(lib().tc_plan_pack_elements(self._h, int(operand), ctypes.byref(n)))
        return n.value

    def pack(self, operand, src, dst, stream=None):
        """Gather operand 0 (A) or 1 (B) into the tile-panel matrix dst (the
        contraction's pack stage alone)."""
        _check(lib().tc_plan_pack(self._h, int(operand), _ptr(src), _ptr(dst), _stream_ptr(stream)))
        return dst

    def store(self, src, C, alpha=1.0, beta=0.0, stream=None):
        """C[rscat_C[i] + cscat_C[j]] = alpha src[i + m j] + beta C (the
        contraction's tile store alone; src is an m x n column-major matrix)."""
        _check(lib().tc_plan_store(self._h, float(alpha), _ptr(src), float(beta), _ptr(C), _stream_ptr(stream)))
        return C

    @property
    def tile(self):
        return _check(lib().tc_plan_get_tile(self._h))

    @tile.setter
    def tile(self, t):
        _check(lib().tc_plan_set_tile(self._h, int(t)))

    def autotune(self, A, B, C_scratch, reps=3, stream=None):
        best = ctypes.c_double()
        _check(lib().tc_plan_autotune(self._h, _ptr(A), _ptr(B), _ptr(C_scratch), int(reps), _stream_ptr(stream),
                                      ctypes.byref(best)))
        return self.tile, best.value

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h:
            lib().tc_plan_destroy(self._h)
            self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many independent contractions run by one persistent kernel launch.

    ``problems`` is a list of (A, idx_A, B, idx_B, C, idx_C, alpha, beta) with
    torch tensors on the current device, all of one dtype.  The tensors are
    bound at construction (their pointers go into the device work table), so
    they must stay alive while the batch is used.  ``execute`` issues one
    persistent launch per tile class present (``tile`` = -1: every problem with
    the class the planner picks for it; else one class for all) and may be
    recorded in a HIP graph.
    """

    def __init__(self, problems, mode="native"):
        self._h = _vp()
        self.plans = [Plan.for_tensors(A, ia, B, ib, C, ic, mode=mode) for (A, ia, B, ib, C, ic, _, _) in problems]
        n = len(problems)
        self.tensors = [(p[0], p[2], p[4]) for p in problems]  # keep alive
        hs = (_vp * max(n, 1))(*[p.handle for p in self.plans])
        al = (ctypes.c_double * max(n, 1))(*[float(p[6]) for p in problems])
        be = (ctypes.c_double * max(n, 1))(*[float(p[7]) for p in problems])
        As = (_vp * max(n, 1))(*[_ptr(p[0]) for p in problems])
        Bs = (_vp * max(n, 1))(*[_ptr(p[2]) for p in problems])
        Cs = (_vp * max(n, 1))(*[_ptr(p[4]) for p in problems])
        _check(lib().tc_batch_create(ctypes.byref(self._h), n, hs, al, As, Bs, be, Cs))

    def execute(self, stream=None):
        _check(lib().tc_batch_execute(self._h, _stream_ptr(stream)))

    def info(self):
        w, t, g = ctypes.c_int64(), ctypes.c_int(), ctypes.c_int()
        _check(lib().tc_batch_info(self._h, ctypes.byref(w), ctypes.byref(t), ctypes.byref(g)))
        return {"work_items": w.value, "tile": t.value, "grid": g.value}

    @property
    def tile(self):
        return self.info()["tile"]

    @tile.setter
    def tile(self, t):
        _check(lib().tc_batch_set_tile(self._h, int(t)))

    def problem_tile(self, i):
        """Tile configuration problem i runs with (-1: it launches no work)."""
        t = ctypes.c_int()
        _check(lib().tc_batch_problem_tile(self._h, int(i), ctypes.byref(t)))
        return t.value

    def autotune(self, reps=3, stream=None):
        best = ctypes.c_double()
        _check(lib().tc_batch_autotune(self._h, int(reps), _stream_ptr(stream), ctypes.byref(best)))
        return self.tile, best.value

    def close(self):
        if self._h:
            lib().tc_batch_destroy(self._h)
            self._h = _vp()
        for p in getattr(self, "plans", []):
            p.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _ptr(t):
    """Data pointer of a tensor on the current HIP device (None when empty).
    A tensor anywhere else is refused before the library is called: its
    address would be meaningless to the kernels."""
    if t is None:
        return None
    if t.device.type != "cuda":
        raise ValueError(f"tensor on {t.device}: the contraction needs tensors on the current HIP device")
    import torch
    if t.device.index != torch.cuda.current_device():
        raise ValueError(f"tensor on {t.device}, but the current HIP device is cuda:{torch.cuda.current_device()}")
    return t.data_ptr() if t.numel() else None


def contract(A, idx_A, B, idx_B, idx_C, alpha=1.0, beta=0.0, out=None, mode="native", stream=None):
    """C[idx_C] = alpha * A[idx_A] . B[idx_B] + beta * out, on the GPU.

    A, B (and out) are torch tensors on the current HIP device with any
    strides.  Without ``out`` a new column-major C is allocated (beta is then
    ignored).  Returns C.
    """
    import torch
    mode_code = MODES[mode] if isinstance(mode, str) else mode
    if A.dtype != B.dtype:
        raise TypeError("A and B must have the same dtype")
    if out is None:
        ext = {}
        for t, lab in ((A, idx_A), (B, idx_B)):
            for l, n in zip(lab, t.shape):
                ext[l] = n
        shape = [ext[l] for l in idx_C]
        strides, s = [], 1
        for n in shape:
            strides.append(s)
            s *= max(n, 1)
        out = torch.empty_strided(shape, strides, dtype=A.dtype, device=A.device)
        beta = 0.0
    if out.dtype != A.dtype:
        raise TypeError("C must have the dtype of A and B")
    _check(lib().tc_contract(float(alpha), _ptr(A), *_desc(tuple(A.shape), A.stride(), idx_A), _ptr(B),
                             *_desc(tuple(B.shape), B.stride(), idx_B), float(beta), _ptr(out),
                             *_desc(tuple(out.shape), out.stride(), idx_C), _dtype_code(A.dtype), mode_code,
                             _stream_ptr(stream)))
    return out


def contract_batched(problems, mode="native", stream=None):
    """One-shot batch: C_i[idx_C] = alpha_i * A_i . B_i + beta_i * C_i for
    every (A, idx_A, B, idx_B, C, idx_C, alpha, beta) in ``problems`` (torch
    tensors on the current device, one dtype), in persistent launches.
    Synchronous (waits for the stream); for repeated use build a ``Batch``."""
    mode_code = MODES[mode] if isinstance(mode, str) else mode
    n = len(problems)
    if n == 0:
        return
    dt = problems[0][0].dtype
    keep, arr = [], (_Problem * n)()
    for i, (A, ia, B, ib, C, ic, alpha, beta) in enumerate(problems):
        if A.dtype != dt or B.dtype != dt or C.dtype != dt:
            raise TypeError("every tensor of a batch must have the same dtype")
        ds = [_desc(tuple(t.shape), t.stride(), lab) for t, lab in ((A, ia), (B, ib), (C, ic))]
        keep.append(ds)
        f = [(nd, ctypes.cast(ln, _i64p), ctypes.cast(st, _i64p), lab) for nd, ln, st, lab in ds]
        arr[i] = _Problem(float(alpha), _ptr(A), *f[0], _ptr(B), *f[1], float(beta), _ptr(C), *f[2])
    _check(lib().tc_contract_batched(n, arr, _dtype_code(dt), mode_code, _stream_ptr(stream)))


def contract_noalloc(A, idx_A, B, idx_B, idx_C, out, alpha=1.0, beta=0.0, mode="native", stream=None):
    """The same as ``contract`` with a given ``out``, through the entry point
    that allocates no device memory (tc_contract_noalloc): for callers that
    cannot allocate.  Calls that overlap in time on one GPU race on the
    library's static array; serialise them.  Returns out."""
    mode_code = MODES[mode] if isinstance(mode, str) else mode
    if A.dtype != B.dtype or out.dtype != A.dtype:
        raise TypeError("A, B and out must have one dtype")
    _check(lib().tc_contract_noalloc(float(alpha), _ptr(A), *_desc(tuple(A.shape), A.stride(), idx_A), _ptr(B),
                                     *_desc(tuple(B.shape), B.stride(), idx_B), float(beta), _ptr(out),
                                     *_desc(tuple(out.shape), out.stride(), idx_C), _dtype_code(A.dtype), mode_code,
                                     _stream_ptr(stream)))
    return out


def describe(A_shape, A_strides, idx_A, B_shape, B_strides, idx_B, C_shape, C_strides, idx_C, dtype=TC_F64,
             mode=TC_NATIVE):
    """Plan description (no GPU needed)."""
    p = Plan(A_shape, A_strides, idx_A, B_shape, B_strides, idx_B, C_shape, C_strides, idx_C, dtype, mode)
    try:
        return p.describe()
    finally:
        p.close()


def permute_into(src, dst, stream=None):
    """dst[...] = src[...] elementwise (same shape, any strides) through the
    library's permute-copy kernel; returns dst."""
    if tuple(src.shape) != tuple(dst.shape) or src.dtype != dst.dtype:
        raise ValueError("src and dst must have one shape and one dtype")
    n = len(src.shape)
    _check(lib().tc_permute(_ptr(src), _ptr(dst), n, _arr(src.shape), _arr(src.stride()), _arr(dst.stride()),
                            _dtype_code(src.dtype), _stream_ptr(stream)))
    return dst


def _colmajor_strides(labels, ext):
    out, s = {}, 1
    for l in labels:
        out[l] = s
        s *= max(ext[l], 1)
    return out


class TTGT:
    """The transpose-transpose-GEMM-transpose method (Sec. 5, fig. TTGT) on the GPU,
    as the baseline the transpose-free contraction is measured against.

    A is copied into a column-major m x k matrix (rows I, columns P), B into a
    k x n matrix (P, J) and, when beta != 0, C into an m x n matrix (I, J), with
    the library's permute-copy kernel; one plain matrix product then runs on
    the linearised operands (the same contraction kernels, two-dimensional
    descriptors), and the m x n result is copied back into C's layout.  I and
    J are ordered as in C, P as in A.  The three matrices are the method's
    extra workspace, allocated once here.
    """

    def __init__(self, A, idx_A, B, idx_B, C, idx_C, alpha=1.0, beta=0.0):
        import torch
        self.A, self.B, self.C = A, B, C
        self.alpha, self.beta = float(alpha), float(beta)
        ext = {}
        for t, lab in ((A, idx_A), (B, idx_B), (C, idx_C)):
            for l, n in zip(lab, t.shape):
                ext[l] = n
        I = [l for l in idx_C if l in idx_A]
        J = [l for l in idx_C if l in idx_B]
        P = [l for l in idx_A if l in idx_B]

        def prod(ls):
            r = 1
            for l in ls:
                r *= ext[l]
            return r
        self.m, self.n, self.k = prod(I), prod(J), prod(P)
        m, n, k = self.m, self.n, self.k
        dt, dv = A.dtype, A.device
        self.Am = torch.empty(m * k, dtype=dt, device=dv)
        self.Bm = torch.empty(k * n, dtype=dt, device=dv)
        self.Cm = torch.empty(m * n, dtype=dt, device=dv)
        sA = _colmajor_strides(I + P, ext)
        sB = _colmajor_strides(P + J, ext)
        sC = _colmajor_strides(I + J, ext)
        # the matrices seen with each tensor's own index order
        self.Av = torch.as_strided(self.Am, tuple(A.shape), [sA[l] for l in idx_A])
        self.Bv = torch.as_strided(self.Bm, tuple(B.shape), [sB[l] for l in idx_B])
        self.Cv = torch.as_strided(self.Cm, tuple(C.shape), [sC[l] for l in idx_C])
        self.A2 = torch.as_strided(self.Am, (m, k), (1, m))
        self.B2 = torch.as_strided(self.Bm, (k, n), (1, k))
        self.C2 = torch.as_strided(self.Cm, (m, n), (1, m))
        self.gemm_plan = Plan.for_tensors(self.A2, "ip", self.B2, "pj", self.C2, "ij")
        self.gemm_plan.upload()

    def workspace_bytes(self):
        return (self.Am.numel() + self.Bm.numel() + self.Cm.numel()) * self.Am.element_size()

    def transpose_in(self, stream=None):
        permute_into(self.A, self.Av, stream)
        permute_into(self.B, self.Bv, stream)
        if self.beta != 0.0:
            permute_into(self.C, self.Cv, stream)

    def gemm(self, stream=None):
        self.gemm_plan.execute(self.A2, self.B2, self.C2, self.alpha, self.beta, stream)

    def transpose_out(self, stream=None):
        permute_into(self.Cv, self.C, stream)

    def run(self, stream=None):
        self.transpose_in(stream)
        self.gemm(stream)
        self.transpose_out(stream)
        return self.C

    def close(self):
        self.gemm_plan.close()


def ttgt(A, idx_A, B, idx_B, C, idx_C, alpha=1.0, beta=0.0, stream=None):
    """C[idx_C] = alpha A . B + beta C by transpose-transpose-GEMM-transpose."""
    t = TTGT(A, idx_A, B, idx_B, C, idx_C, alpha, beta)
    try:
        return t.run(stream)
    finally:
        t.close()
