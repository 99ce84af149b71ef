"""Seeded synthetic inputs for the contraction workloads.

This module only draws random numbers and lays them out in memory; it holds
none of the contraction's arithmetic and imports neither the GPU library nor
the oracle, so both sides can share it.

Storage is generalized column-major (first index fastest), the layout the
paper uses for its examples (Sec. 5, eq. loc).  Random numbers come from
``numpy.random.default_rng`` (PCG64), each tensor filled as one flat vector in
its own column-major order, tensors drawn in the order they are listed.
"""
from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np


@dataclass
class Problem:
    """One contraction C[idx_C] = alpha * A[idx_A] . B[idx_B] + beta * C."""
    idx_A: str
    idx_B: str
    idx_C: str
    A: np.ndarray
    B: np.ndarray
    C: np.ndarray
    alpha: float = 1.0
    beta: float = 0.0
    name: str = ""
    extents: Dict[str, int] = field(default_factory=dict)

    def mnk(self):
        e = self.extents
        m = int(np.prod([e[l] for l in self.idx_A if l in self.idx_C], dtype=np.int64))
        n = int(np.prod([e[l] for l in self.idx_B if l in self.idx_C], dtype=np.int64))
        k = int(np.prod([e[l] for l in self.idx_A if l in self.idx_B], dtype=np.int64))
        return m, n, k

    def flops(self):
        m, n, k = self.mnk()
        return 2 * m * n * k


def colmajor(shape, dtype=np.float64, fill=None):
    """A new array of ``shape`` in generalized column-major order."""
    a = np.empty(tuple(shape), dtype=dtype, order="F")
    if fill is not None:
        a[...] = fill
    return a


def colmajor_from_flat(flat, shape):
    """Lay a flat vector out in column-major order (first index fastest)."""
    return np.asarray(flat).reshape(tuple(shape), order="F")


def shape_of(labels, extents):
    return tuple(extents[l] for l in labels)


def _uniform(rng, labels, extents, lo=-1.0, hi=1.0):
    shp = shape_of(labels, extents)
    return colmajor_from_flat(rng.uniform(lo, hi, size=int(np.prod(shp, dtype=np.int64))), shp)


def _normal(rng, labels, extents, scale=1.0):
    shp = shape_of(labels, extents)
    return colmajor_from_flat(rng.standard_normal(int(np.prod(shp, dtype=np.int64))) * scale, shp)


# ---------------------------------------------------------------------------
# The five workloads
# ---------------------------------------------------------------------------

def cfg1(seed=0):
    """C[abcd] = sum_{e,f} A[aebf] B[dfce], every extent 16, A,B ~ U[-1,1], C=0."""
    ext = {l: 16 for l in "abcdef"}
    rng = np.random.default_rng(seed)
    A = _uniform(rng, "aebf", ext)
    B = _uniform(rng, "dfce", ext)
    C = colmajor(shape_of("abcd", ext), fill=0.0)
    return Problem("aebf", "dfce", "abcd", A, B, C, 1.0, 0.0, "abcd-aebf-dfce x16", ext)


def cfg2(seed=0, v=96, o=24):
    """Z[abij] = sum_{k,c} W[akic] T[cbkj] + Z; a,b,c = v; i,j,k = o.

    W, T ~ N(0,1) * 1e-2, Z0 ~ N(0,1), alpha = beta = 1, drawn W, T, Z.
    """
    ext = {"a": v, "b": v, "c": v, "i": o, "j": o, "k": o}
    rng = np.random.default_rng(seed)
    W = _normal(rng, "akic", ext, 1e-2)
    T = _normal(rng, "cbkj", ext, 1e-2)
    Z = _normal(rng, "abij", ext, 1.0)
    return Problem("akic", "cbkj", "abij", W, T, Z, 1.0, 1.0, f"Z[abij]+=W[akic]T[cbkj] v={v} o={o}", ext)


def scaled_normal(rng, labels, extents, lo=-3.0, hi=3.0):
    """N(0,1) entries times a per-mode scale 10^U(lo,hi) along every mode."""
    shp = shape_of(labels, extents)
    z = colmajor_from_flat(rng.standard_normal(int(np.prod(shp, dtype=np.int64))), shp)
    out = np.array(z, order="F")
    for ax, n in enumerate(shp):
        s = 10.0 ** rng.uniform(lo, hi, size=n)
        bshape = [1] * len(shp)
        bshape[ax] = n
        out *= s.reshape(bshape)
    return out


def cfg3(seed=0, shape="cfg1"):
    """The cfg1 (or cfg2) index pattern with magnitudes spread by 10^U(-3,3) per mode.

    Inputs are FP64; the FP32 / split-BF16 runs round them to FP32 outside
    any timed region.  alpha = 1, beta = 0.
    """
    rng = np.random.default_rng(seed)
    if shape == "cfg1":
        ext = {l: 16 for l in "abcdef"}
        ia, ib, ic = "aebf", "dfce", "abcd"
    else:
        ext = {"a": 96, "b": 96, "c": 96, "i": 24, "j": 24, "k": 24}
        ia, ib, ic = "akic", "cbkj", "abij"
    A = scaled_normal(rng, ia, ext)
    B = scaled_normal(rng, ib, ext)
    C = colmajor(shape_of(ic, ext), fill=0.0)
    return Problem(ia, ib, ic, A, B, C, 1.0, 0.0, f"cfg3 scaled {shape}", ext)


def cfg4(seed=0, o=32, v=64):
    """C[ijab] = sum_{k,l} A[iklb] B[kjal]; i,j,k,l = 32, a,b = 64.

    A, B ~ U[-1,1]; the upstream gradient dC ~ N(0,1) is returned as ``C``'s
    companion in ``extra['dC']``.  Drawn A, B, dC.
    """
    ext = {"i": o, "j": o, "k": o, "l": o, "a": v, "b": v}
    rng = np.random.default_rng(seed)
    A = _uniform(rng, "iklb", ext)
    B = _uniform(rng, "kjal", ext)
    dC = _normal(rng, "ijab", ext)
    C = colmajor(shape_of("ijab", ext), fill=0.0)
    p = Problem("iklb", "kjal", "ijab", A, B, C, 1.0, 0.0, "C[ijab]=A[iklb]B[kjal]", ext)
    p.dC = dC
    return p


def random_instance(rng, n_i=2, n_j=2, n_p=2, lo=4, hi=64, dist="uniform"):
    """A random contraction: bundles of the given sizes, extents U{lo..hi},
    every operand's storage order an independent random permutation."""
    labels = "abcdefghijklmnopqrstuvwxyz"
    I = list(labels[:n_i])
    J = list(labels[n_i:n_i + n_j])
    P = list(labels[n_i + n_j:n_i + n_j + n_p])
    ext = {l: int(rng.integers(lo, hi + 1)) for l in I + J + P}
    ic = "".join(rng.permutation(I + J)) if I + J else ""
    ia = "".join(rng.permutation(I + P)) if I + P else ""
    ib = "".join(rng.permutation(P + J)) if P + J else ""
    return ext, ia, ib, ic


def cfg5_instance(i, dtype=np.float64):
    """Instance i of the 512-problem batch: 2 I, 2 J, 2 P labels, extents
    U{4..64}, random permutations, entries U[-1,1], seed default_rng([5, i])."""
    rng = np.random.default_rng([5, i])
    ext, ia, ib, ic = random_instance(rng, 2, 2, 2, 4, 64)
    A = _uniform(rng, ia, ext).astype(dtype, order="F")
    B = _uniform(rng, ib, ext).astype(dtype, order="F")
    C = colmajor(shape_of(ic, ext), dtype=dtype, fill=0.0)
    return Problem(ia, ib, ic, A, B, C, 1.0, 0.0, f"cfg5[{i}]", ext)


def cfg5(count=512, dtype=np.float64):
    return [cfg5_instance(i, dtype) for i in range(count)]


def random_problem(seed, n_i=2, n_j=2, n_p=2, lo=1, hi=7, beta=0.0, alpha=1.0, integer=False):
    """A small random contraction for parity tests (column-major operands,
    random label orders).  ``integer`` draws entries from {-4..4}."""
    rng = np.random.default_rng(seed)
    ext, ia, ib, ic = random_instance(rng, n_i, n_j, n_p, lo, hi)
    if integer:
        mk = lambda lab: colmajor_from_flat(
            rng.integers(-4, 5, size=int(np.prod(shape_of(lab, ext), dtype=np.int64))).astype(np.float64),
            shape_of(lab, ext))
    else:
        mk = lambda lab: _uniform(rng, lab, ext)
    A = mk(ia)
    B = mk(ib)
    C = mk(ic) if beta != 0.0 else colmajor(shape_of(ic, ext), fill=0.0)
    return Problem(ia, ib, ic, A, B, C, alpha, beta, f"random[{seed}]", ext)


def p_conflict_problem(seed, ext=None, beta=0.0):
    """C[i j] = A[e g f i] . B[f j e g] with every operand column-major:
    e is A's unit-stride index and f is B's, and both are contracted, so the
    storage orders of A and B disagree inside the contracted bundle (the
    layouts the paper discusses with dimension sub-division).  ``ext`` maps
    the labels e, f, g, i, j to extents."""
    rng = np.random.default_rng(seed)
    ext = dict(ext or {"e": 13, "g": 3, "f": 10, "i": 150, "j": 70})
    A = _uniform(rng, "egfi", ext)
    B = _uniform(rng, "fjeg", ext)
    C = _uniform(rng, "ij", ext) if beta != 0.0 else colmajor(shape_of("ij", ext), fill=0.0)
    return Problem("egfi", "fjeg", "ij", A, B, C, 1.0, beta, f"p_conflict[{seed}]", ext)


def split_extent(rng, target, dims):
    """``dims`` extents (each >= 2) whose product is close to ``target``: the
    log of the target cut at dims - 1 uniform random points, the last extent
    then absorbing the rounding of the others."""
    if dims <= 1:
        return [max(int(target), 1)]
    cuts = np.sort(rng.random(dims - 1))
    parts = np.diff(np.concatenate([[0.0], cuts, [1.0]])) * np.log(max(target, 1))
    lens = [max(int(round(float(np.exp(x)))), 2) for x in parts[:-1]]
    lens.append(max(int(round(target / float(np.prod(lens)))), 2))
    return lens


def sweep_instance(rng, m, n, k):
    """A contraction whose matrix view is about m x n x k, in the manner of
    the paper's random-contraction generator (Sec. 9.2): each of the bundles
    I, J and P gets one to three labels whose extents multiply to about m, n
    and k, and every operand's storage order is an independent random
    permutation of its labels."""
    labels = iter("abcdefghijklmnopqrstuvwxyz")
    ext, bundles = {}, []
    for target in (m, n, k):
        lens = split_extent(rng, target, int(rng.integers(1, 4)))
        labs = [next(labels) for _ in lens]
        ext.update(zip(labs, lens))
        bundles.append(labs)
    I, J, P = bundles
    ic = "".join(rng.permutation(I + J))
    ia = "".join(rng.permutation(I + P))
    ib = "".join(rng.permutation(P + J))
    return ext, ia, ib, ic


def sweep_problem(seed, m, n, k, dtype=np.float64):
    """Seeded sweep instance with U[-1,1] operands (A then B), C = 0, alpha 1,
    beta 0."""
    rng = np.random.default_rng(seed)
    ext, ia, ib, ic = sweep_instance(rng, m, n, k)
    A = _uniform(rng, ia, ext).astype(dtype, order="F")
    B = _uniform(rng, ib, ext).astype(dtype, order="F")
    C = colmajor(shape_of(ic, ext), dtype=dtype, fill=0.0)
    return Problem(ia, ib, ic, A, B, C, 1.0, 0.0, f"sweep[{seed}:{m}x{n}x{k}]", ext)
