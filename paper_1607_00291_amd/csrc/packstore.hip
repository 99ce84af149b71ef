// The contraction's pack and store stages run alone, to measure their memory
// traffic (the scatter packing of Sec. 6.1 with the block strides of
// Sec. 6.2, and the alpha/beta scatter-store of the C tiles):
//   pack  : every (row tile, k block) sliver of one operand is gathered
//           through the plan's offset vectors by the same code as the
//           contraction (PackRole: per-tile row offsets, k offsets from the
//           block stride when valid, bounds-checked buffer loads, lanes along
//           the operand's unit-stride index), staged k-major in LDS, and
//           written out densely as that sliver of a tile-panel matrix;
//   store : every C tile reads an m x n column-major matrix into the
//           fragment layout of the regular tiles and writes it with the same
//           scatter-store code as the contraction (store_rect through
//           rscat_C / cscat_C, C read only when beta != 0).
#include "kernels_impl.hpp"

namespace tc {

namespace {

template <typename T, typename OffT, int R, int KT>
__global__ __launch_bounds__(256) void pack_kernel(const T* __restrict__ src, int64_t span, const OffT* rowvec,
                                                   const OffT* kvec, const OffT* kbs, OffT rows, OffT K, int64_t nkb,
                                                   int lanes_row, T* __restrict__ dst) {
    typedef PackRole<T, OffT, R, KT, 256, 1> PR;
    __shared__ T stage[KT * (R + 1)];
    const int64_t blk = blockIdx.x;
    const int64_t tr = blk / nkb, kb = blk % nkb;
    const int ld = lanes_row ? Pitch<R, true>::value : Pitch<R, false>::value;
    PR pk;
    pk.init(rowvec, (OffT)(tr * R), rows, threadIdx.x, lanes_row != 0, ld);
    pk.template load<0>(src, span, kvec, kbs, (OffT)kb, K, threadIdx.x);
    pk.template store<0>(stage, threadIdx.x);
    __syncthreads();
    T* out = dst + blk * (int64_t)(KT * R);
    for (int e = threadIdx.x; e < KT * R; e += 256) out[e] = stage[(e / R) * ld + e % R];
}

// One wave per 16 x 16 fragment of the tile grid (fragment f of tile t is
// wave t * nfrag + f), four waves per workgroup: enough waves in flight to
// cover the gather latency of the offset and C reads.
template <typename T, typename OffT>
__global__ __launch_bounds__(256) void store_kernel(KArgs<T, OffT> a, const T* __restrict__ src, int MT, int NT,
                                                    int64_t frags) {
    typedef Mfma<T> M;
    const int lane = threadIdx.x & 63;
    const int64_t g = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (g >= frags) return;
    const int fm = MT / 16, nfrag = fm * (NT / 16);
    const int64_t tile = g / nfrag;
    const int f = (int)(g - tile * nfrag);
    const int64_t tm = tile % a.tiles_m, tn = tile / a.tiles_m;
    const OffT fm0 = (OffT)(tm * MT + 16 * (f % fm)), fn0 = (OffT)(tn * NT + 16 * (f / fm));
    typename M::acc_t acc;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const OffT r = fm0 + M::row(lane, t), c = fn0 + M::col(lane, t);
        acc[t] = r < a.m && c < a.n ? src[(int64_t)r + (int64_t)a.m * c] : T(0);
    }
    store_frag<T, OffT, M>(a, fm0, fn0, acc, lane);
}

template <typename T, typename OffT, int R, int KT>
int launch_pack_r(const T* src, int64_t span, const OffT* rowvec, const OffT* kvec, const OffT* kbs, int64_t rows,
                  int64_t K, bool lanes_row, T* dst, hipStream_t s) {
    const int64_t tiles = (rows + R - 1) / R, nkb = (K + KT - 1) / KT;
    if (tiles * nkb == 0) return TC_OK;
    if (tiles * nkb > 0x7fffffffLL) {
        set_error("too many slivers for one launch");
        return TC_ERR_ARG;
    }
    hipLaunchKernelGGL((pack_kernel<T, OffT, R, KT>), dim3((unsigned)(tiles * nkb)), dim3(256), 0, s, src, span, rowvec,
                       kvec, kbs, (OffT)rows, (OffT)K, nkb, (int)lanes_row, dst);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? TC_OK : hip_fail(e, "pack kernel launch");
}

template <typename T, typename OffT>
int pack_typed(const Plan& p, const DeviceVectors& dv, int operand, const void* src, void* dst, hipStream_t s) {
    const OffT* base = (const OffT*)dv.buf;
    const TileCfg& t = tile_table(p.dtype, p.mode)[p.tile];
    const bool x = (operand == 0) != p.swapped;  // the operand plays X (rows m) or Y (rows n)
    const OffT* rowvec = base + (x ? dv.o_rX : dv.o_cY);
    const OffT* kvec = base + (x ? dv.o_cX : dv.o_rY);
    const OffT* kbs = base + (x ? dv.o_kbsX : dv.o_kbsY);
    const int64_t rows = x ? p.m : p.n;
    const int64_t span = operand == 0 ? p.spanA : p.spanB;
    const bool lr = x ? p.x_lanes_m : p.y_lanes_n;
    const int R = x ? t.MT : t.NT;
    const T* sp = (const T*)src;
    T* dp = (T*)dst;
    if (t.KT == 16) {
        switch (R) {
            case 32: return launch_pack_r<T, OffT, 32, 16>(sp, span, rowvec, kvec, kbs, rows, p.k, lr, dp, s);
            case 64: return launch_pack_r<T, OffT, 64, 16>(sp, span, rowvec, kvec, kbs, rows, p.k, lr, dp, s);
            case 128: return launch_pack_r<T, OffT, 128, 16>(sp, span, rowvec, kvec, kbs, rows, p.k, lr, dp, s);
            case 144: return launch_pack_r<T, OffT, 144, 16>(sp, span, rowvec, kvec, kbs, rows, p.k, lr, dp, s);
        }
    } else if (t.KT == 32) {
        switch (R) {
            case 32: return launch_pack_r<T, OffT, 32, 32>(sp, span, rowvec, kvec, kbs, rows, p.k, lr, dp, s);
            case 64: return launch_pack_r<T, OffT, 64, 32>(sp, span, rowvec, kvec, kbs, rows, p.k, lr, dp, s);
            case 128: return launch_pack_r<T, OffT, 128, 32>(sp, span, rowvec, kvec, kbs, rows, p.k, lr, dp, s);
            case 144: return launch_pack_r<T, OffT, 144, 32>(sp, span, rowvec, kvec, kbs, rows, p.k, lr, dp, s);
        }
    }
    set_error("no pack kernel for this tile shape");
    return TC_ERR_ARG;
}

template <typename T, typename OffT>
int store_typed(const Plan& p, const DeviceVectors& dv, double alpha, const void* src, double beta, void* C,
                hipStream_t s) {
    const OffT* base = (const OffT*)dv.buf;
    const TileCfg& t = tile_table(p.dtype, p.mode)[p.tile];
    KArgs<T, OffT> a{};
    a.C = (T*)C;
    a.rC = base + dv.o_rC;
    a.cC = base + dv.o_cC;
    a.m = (OffT)p.m;
    a.n = (OffT)p.n;
    a.tiles_m = p.tiles_m;
    a.tiles_n = p.tiles_n;
    a.alpha = (T)alpha;
    a.beta = (T)beta;
    const int64_t frags = p.tiles_m * p.tiles_n * (t.MT / 16) * (t.NT / 16), blocks = (frags + 3) / 4;
    if (frags == 0) return TC_OK;
    if (blocks > 0x7fffffffLL) {
        set_error("too many fragments for one launch");
        return TC_ERR_ARG;
    }
    hipLaunchKernelGGL((store_kernel<T, OffT>), dim3((unsigned)blocks), dim3(256), 0, s, a, (const T*)src, t.MT, t.NT,
                       frags);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? TC_OK : hip_fail(e, "store kernel launch");
}

}  // namespace

int64_t pack_elements(const Plan& p, int operand) {
    const TileCfg& t = tile_table(p.dtype, p.mode)[p.tile];
    const bool x = (operand == 0) != p.swapped;
    const int64_t rows = x ? p.m : p.n, R = x ? t.MT : t.NT;
    return ((rows + R - 1) / R) * R * ((p.k + t.KT - 1) / t.KT) * t.KT;
}

int launch_pack(const Plan& p, const DeviceVectors& dv, int operand, const void* src, void* dst, hipStream_t s) {
    if (p.dtype == TC_F64)
        return p.off64 ? pack_typed<double, int64_t>(p, dv, operand, src, dst, s)
                       : pack_typed<double, int32_t>(p, dv, operand, src, dst, s);
    return p.off64 ? pack_typed<float, int64_t>(p, dv, operand, src, dst, s)
                   : pack_typed<float, int32_t>(p, dv, operand, src, dst, s);
}

int launch_store(const Plan& p, const DeviceVectors& dv, double alpha, const void* src, double beta, void* C,
                 hipStream_t s) {
    if (p.dtype == TC_F64)
        return p.off64 ? store_typed<double, int64_t>(p, dv, alpha, src, beta, C, s)
                       : store_typed<double, int32_t>(p, dv, alpha, src, beta, C, s);
    return p.off64 ? store_typed<float, int64_t>(p, dv, alpha, src, beta, C, s)
                   : store_typed<float, int32_t>(p, dv, alpha, src, beta, C, s);
}

}  // namespace tc
