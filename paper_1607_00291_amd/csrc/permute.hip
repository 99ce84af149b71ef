// Strided permute-copy dst[i] = src[i] over one index space with two stride
// sets: the "transpose" step of the transpose-transpose-GEMM-transpose
// (TTGT) method of Sec. 3.2, which the block-scatter-matrix contraction
// avoids.  It exists to measure that method on the same device.
//
// Bandwidth-bound.  Two dimensions are picked: `a`, the unit-stride (or
// smallest-stride) dimension of src, and `b`, that of dst.  A workgroup moves
// a 64 x 64 tile of (a, b) at one position of the remaining ("outer")
// dimensions: it reads with lanes along a, stages the tile in LDS and writes
// with lanes along b, so both HBM sides are coalesced.  When src and dst share
// their unit-stride dimension the tile is copied straight through, lanes
// along a on both sides.  The copy moves element bits unchanged.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <string>

#include "plan.hpp"
#include "tc.h"

namespace tc {

namespace {

constexpr int PT = 64;       // tile edge
constexpr int PROWS = 4;     // rows of threads (PT x PROWS = 256 threads)

struct PermArgs {
    int nout;
    int64_t olen[TC_MAX_NDIM];
    int64_t osrc[TC_MAX_NDIM];
    int64_t odst[TC_MAX_NDIM];
    int64_t la, lb;
    int64_t sa_src, sa_dst, sb_src, sb_dst;
    int64_t tiles_a, tiles_b, total;
    int same;  // src and dst share dimension a as their fastest one
};

template <typename W>
__global__ __launch_bounds__(PT* PROWS) void permute_kernel(const W* __restrict__ src, W* __restrict__ dst,
                                                            PermArgs p) {
    __shared__ W tile[PT][PT + 1];
    const int tx = threadIdx.x % PT;
    const int ty = threadIdx.x / PT;
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
        const int64_t a0 = ta * PT, b0 = tb * PT;
        if (p.same) {
            const int64_t ia = a0 + tx;
            if (ia < p.la) {
                for (int k = ty; k < PT; k += PROWS) {
                    const int64_t ib = b0 + k;
                    if (ib < p.lb)
                        dst[dbase + ia * p.sa_dst + ib * p.sb_dst] = src[sbase + ia * p.sa_src + ib * p.sb_src];
                }
            }
            continue;
        }
        // read: lanes along a (src's fast dimension)
        {
            const int64_t ia = a0 + tx;
            for (int k = ty; k < PT; k += PROWS) {
                const int64_t ib = b0 + k;
                if (ia < p.la && ib < p.lb) tile[k][tx] = src[sbase + ia * p.sa_src + ib * p.sb_src];
            }
        }
        __syncthreads();
        // write: lanes along b (dst's fast dimension)
        {
            const int64_t ib = b0 + tx;
            for (int k = ty; k < PT; k += PROWS) {
                const int64_t ia = a0 + k;
                if (ia < p.la && ib < p.lb) dst[dbase + ia * p.sa_dst + ib * p.sb_dst] = tile[tx][k];
            }
        }
        __syncthreads();
    }
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
    p.tiles_a = (p.la + PT - 1) / PT;
    p.tiles_b = (p.lb + PT - 1) / PT;
    p.total = p.tiles_a * p.tiles_b * outer;
    const int grid = (int)std::min<int64_t>(p.total, int64_t(1) << 20);
    if (dtype == TC_F64)
        hipLaunchKernelGGL(permute_kernel<uint64_t>, dim3(grid), dim3(PT * PROWS), 0, stream,
                           (const uint64_t*)src, (uint64_t*)dst, p);
    else
        hipLaunchKernelGGL(permute_kernel<uint32_t>, dim3(grid), dim3(PT * PROWS), 0, stream,
                           (const uint32_t*)src, (uint32_t*)dst, p);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error(std::string("permute launch: ") + hipGetErrorString(e));
        return TC_ERR_HIP;
    }
    return TC_OK;
}

}  // namespace tc
