// Strided permute-copy dst[i] = src[i] over one index space with two stride
// sets: the "transpose" step of the transpose-transpose-GEMM-transpose
// (TTGT) method of Sec. 5 (fig. TTGT), which the block-scatter-matrix contraction
// avoids.  It exists to measure that method on the same device.
//
// Bandwidth-bound.  Two dimensions are picked: `a`, the unit-stride (or
// smallest-stride) dimension of src, and `b`, that of dst.  A workgroup moves
// a PA x PB tile of (a, b) at one position of the remaining ("outer")
// dimensions: it reads with lanes along a, stages the tile in LDS and writes
// with lanes along b, so both HBM sides are coalesced.  When src and dst share
// their unit-stride dimension the tile is copied straight through, lanes
// along a on both sides.  The tile edges are chosen per call from 16 to 64 so
// that the tiles cover the (a, b) extents with the least padding (the
// coupled-cluster shapes have extents such as 96 and 24, which 64 x 64 tiles
// cover at under a third of their slots), and the LDS stage is sized to the
// tile so that more workgroups share a CU.  The copy moves element bits
// unchanged.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <string>

#include "plan.hpp"
#include "tc.h"

namespace tc {

namespace {

constexpr int PTHREADS = 256;  // threads per workgroup
constexpr int PMAX = 64;       // largest tile edge

struct PermArgs {
    int nout;
    int64_t olen[TC_MAX_NDIM];
    int64_t osrc[TC_MAX_NDIM];
    int64_t odst[TC_MAX_NDIM];
    int64_t la, lb;
    int64_t sa_src, sa_dst, sb_src, sb_dst;
    int64_t tiles_a, tiles_b, total;
    int pa, pb;  // tile edges along a and b, each in [16, PMAX]
    int same;    // src and dst share dimension a as their fastest one
};

template <typename W>
__global__ __launch_bounds__(PTHREADS) void permute_kernel(const W* __restrict__ src, W* __restrict__ dst,
                                                           PermArgs p) {
    // tile[b][a] with row pitch pa + 1 (pb * (pa + 1) elements, dynamic LDS)
    extern __shared__ unsigned char permute_lds[];
    W* tile = reinterpret_cast<W*>(permute_lds);
    const int pa = p.pa, pb = p.pb, ld = pa + 1;
    // read mapping: lanes along a; threads past the last whole row idle
    const int ra = threadIdx.x % pa, rr = threadIdx.x / pa, rstep = PTHREADS / pa;
    // write mapping: lanes along b
    const int wb = threadIdx.x % pb, wr = threadIdx.x / pb, wstep = PTHREADS / pb;
    for (int64_t t = blockIdx.x; t < p.total; t += gridDim.x) {
        int64_t r = t;
        const int64_t ta = r % p.tiles_a;
        r /= p.tiles_a;
        const int64_t tb = r % p.tiles_b;
        r /= p.tiles_b;
        int64_t sbase = 0, dbase = 0;
        for (int d = 0; d < p.nout; ++d) {
            const int64_t i = r % p.olen[d];
            r /= p.olen[d];
            sbase += i * p.osrc[d];
            dbase += i * p.odst[d];
        }
        const int64_t a0 = ta * pa, b0 = tb * pb;
        if (p.same) {
            const int64_t ia = a0 + ra;
            if (rr < rstep && ia < p.la) {
                for (int k = rr; k < pb; k += rstep) {
                    const int64_t ib = b0 + k;
                    if (ib < p.lb)
                        dst[dbase + ia * p.sa_dst + ib * p.sb_dst] = src[sbase + ia * p.sa_src + ib * p.sb_src];
                }
            }
            continue;
        }
        // read: lanes along a (src's fast dimension)
        if (rr < rstep) {
            const int64_t ia = a0 + ra;
            for (int k = rr; k < pb; k += rstep) {
                const int64_t ib = b0 + k;
                if (ia < p.la && ib < p.lb) tile[k * ld + ra] = src[sbase + ia * p.sa_src + ib * p.sb_src];
            }
        }
        __syncthreads();
        // write: lanes along b (dst's fast dimension)
        if (wr < wstep) {
            const int64_t ib = b0 + wb;
            for (int k = wr; k < pa; k += wstep) {
                const int64_t ia = a0 + k;
                if (ia < p.la && ib < p.lb) dst[dbase + ia * p.sa_dst + ib * p.sb_dst] = tile[wb * ld + k];
            }
        }
        __syncthreads();
    }
}

// Tile edge for an extent: the candidate whose tiles cover it with the least
// padding, the larger one on a tie.
int permute_edge(int64_t len) {
    static const int cand[] = {16, 24, 32, 48, PMAX};
    int best = PMAX;
    int64_t best_pad = -1;
    for (int c : cand) {
        const int64_t pad = (len + c - 1) / c * c - len;
        if (best_pad < 0 || pad < best_pad || (pad == best_pad && c > best)) {
            best = c;
            best_pad = pad;
        }
    }
    return best;
}

}  // namespace

int launch_permute(const void* src, void* dst, int ndim, const int64_t* lens, const int64_t* ss, const int64_t* ds,
                   int dtype, hipStream_t stream) {
    // keep dimensions of length > 1; an empty index space is a no-op
    int keep[TC_MAX_NDIM];
    int nk = 0;
    for (int d = 0; d < ndim; ++d) {
        if (lens[d] == 0) return TC_OK;
        if (lens[d] > 1) keep[nk++] = d;
    }
    PermArgs p{};
    int a = -1, b = -1;
    for (int q = 0; q < nk; ++q) {
        const int d = keep[q];
        if (a < 0 || ss[d] < ss[a]) a = d;
        if (b < 0 || ds[d] < ds[b]) b = d;
    }
    p.same = (a == b) ? 1 : 0;
    if (p.same && nk > 1) {
        // second tile dimension: the smallest dst stride among the rest
        b = -1;
        for (int q = 0; q < nk; ++q) {
            const int d = keep[q];
            if (d != a && (b < 0 || ds[d] < ds[b])) b = d;
        }
    }
    p.la = a >= 0 ? lens[a] : 1;
    p.sa_src = a >= 0 ? ss[a] : 0;
    p.sa_dst = a >= 0 ? ds[a] : 0;
    const bool hasb = b >= 0 && b != a;
    p.lb = hasb ? lens[b] : 1;
    p.sb_src = hasb ? ss[b] : 0;
    p.sb_dst = hasb ? ds[b] : 0;
    p.nout = 0;
    int64_t outer = 1;
    for (int q = 0; q < nk; ++q) {
        const int d = keep[q];
        if (d == a || d == b) continue;
        p.olen[p.nout] = lens[d];
        p.osrc[p.nout] = ss[d];
        p.odst[p.nout] = ds[d];
        ++p.nout;
        outer *= lens[d];
    }
    p.pa = permute_edge(p.la);
    p.pb = permute_edge(p.lb);
    p.tiles_a = (p.la + p.pa - 1) / p.pa;
    p.tiles_b = (p.lb + p.pb - 1) / p.pb;
    p.total = p.tiles_a * p.tiles_b * outer;
    const int grid = (int)std::min<int64_t>(p.total, int64_t(1) << 20);
    const size_t esz = dtype == TC_F64 ? sizeof(uint64_t) : sizeof(uint32_t);
    const size_t lds = p.same ? 0 : (size_t)p.pb * (size_t)(p.pa + 1) * esz;
    if (dtype == TC_F64)
        hipLaunchKernelGGL(permute_kernel<uint64_t>, dim3(grid), dim3(PTHREADS), lds, stream,
                           (const uint64_t*)src, (uint64_t*)dst, p);
    else
        hipLaunchKernelGGL(permute_kernel<uint32_t>, dim3(grid), dim3(PTHREADS), lds, stream,
                           (const uint32_t*)src, (uint32_t*)dst, p);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error(std::string("permute launch: ") + hipGetErrorString(e));
        return TC_ERR_HIP;
    }
    return TC_OK;
}

}  // namespace tc
