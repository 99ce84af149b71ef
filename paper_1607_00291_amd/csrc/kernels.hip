// gfx950 kernels of the transpose-free contraction (block-scatter-matrix
// tensor contraction, Sec. 6.2) and their launchers.
//
// One workgroup computes one MT x NT tile of the matrix view C[m, n] of the
// output.  Its K loop runs over LDS stages of depth KT:
//   pack   : every thread gathers its share of the MT x KT sliver of X and
//            the KT x NT sliver of Y straight from the tensors' own layouts,
//            element (m, k) of X at X + rscat_X[m] + cscat_X[k] (Sec. 6.1).
//            The per-thread row / column offsets are loaded once per tile;
//            the k offsets come from the block stride of the current k block
//            when it is valid (Sec. 6.2, the k_P blocking) and from the
//            scatter vector otherwise.  Lanes run along each operand's
//            unit-stride index, so global reads coalesce whatever the
//            permutation of the tensor's dimensions.  The stage is written
//            to LDS in the k-major order the matrix-core fragments read,
//            which is where the tensor-to-matrix reshape is folded in.
//   micro  : waves run 16x16x4 matrix-core instructions on register tiles
//            (FP64 or FP32 accumulation in the storage type).
//   store  : accumulators are scaled by alpha and written to
//            C + rscat_C[m] + cscat_C[n], reading C only when beta != 0.
// LDS is double-buffered: global loads for stage s+1 are in flight while the
// matrix cores consume stage s; one barrier per stage.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>

#include "launch.hpp"
#include "tc.h"
#include "tiles.hpp"

namespace tc {

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

template <typename T>
struct Mfma;

template <>
struct Mfma<double> {
    typedef f64x4 acc_t;
    // D(16x16) += A(16x4) B(4x16); lane l holds A[l%16][l/16], B[l/16][l%16]
    // and D[l/16 + 4r][l%16] in element r.
    static __device__ __forceinline__ acc_t run(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};

template <>
struct Mfma<float> {
    typedef f32x4 acc_t;
    // same operand layout as FP64; D[4*(l/16) + r][l%16] in element r
    static __device__ __forceinline__ acc_t run(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

template <typename T, typename OffT>
struct KArgs {
    const T* X;
    const T* Y;
    T* C;
    const OffT* rX;
    const OffT* cX;
    const OffT* rY;
    const OffT* cY;
    const OffT* rC;
    const OffT* cC;
    const OffT* kbsX;
    const OffT* kbsY;
    OffT m, n, k;
    int64_t tiles_m, tiles_n;
    T alpha, beta;
};

// LDS row pitch (in elements) of a k-major stage: one element of padding when
// the lanes of the gather run along k (consecutive lanes then write to
// consecutive LDS rows, and the pad spreads them over the banks).
template <int W, bool LANES_ALONG_ROW>
struct Pitch {
    static constexpr int value = LANES_ALONG_ROW ? W : W + 1;
};

// The pack stage of one tile: MT x KT slivers of X and KT x NT slivers of Y
// gathered through the offset vectors into registers, then written to a
// k-major LDS stage.  Element e = tid + NTHR * i of a stage is (row, kk) with
// the row index fastest when the operand's lanes run along m (XM) / n (YN),
// and kk fastest otherwise.
template <typename T, typename OffT, int MT, int NT, int KT, int NTHR, bool XM, bool YN>
struct Pack {
    static constexpr int EX = MT * KT / NTHR, EY = NT * KT / NTHR;
    static constexpr int LDX = Pitch<MT, XM>::value, LDY = Pitch<NT, YN>::value;
    static constexpr int XS = KT * LDX, YS = KT * LDY;  // elements of one stage
    static constexpr int ELEMS = 2 * (XS + YS);          // double-buffered
    static_assert((MT * KT) % NTHR == 0 && (NT * KT) % NTHR == 0, "stage must split evenly over threads");

    static __device__ __forceinline__ int xrow(int e) { return XM ? e % MT : e / KT; }
    static __device__ __forceinline__ int xk(int e) { return XM ? e / MT : e % KT; }
    static __device__ __forceinline__ int ycol(int e) { return YN ? e % NT : e / KT; }
    static __device__ __forceinline__ int yk(int e) { return YN ? e / NT : e % KT; }

    OffT xo[EX], yo[EY];  // row offsets of X / column offsets of Y, fixed per tile
    bool xv[EX], yv[EY];
    T rx[EX], ry[EY];     // one stage in flight

    __device__ __forceinline__ void init(const KArgs<T, OffT>& a, OffT m0, OffT n0, int tid) {
#pragma unroll
        for (int i = 0; i < EX; ++i) {
            const OffT mm = m0 + xrow(tid + NTHR * i);
            xv[i] = mm < a.m;
            xo[i] = xv[i] ? a.rX[mm] : OffT(0);
        }
#pragma unroll
        for (int i = 0; i < EY; ++i) {
            const OffT nn = n0 + ycol(tid + NTHR * i);
            yv[i] = nn < a.n;
            yo[i] = yv[i] ? a.cY[nn] : OffT(0);
        }
    }

    // Global gather of k block kb.  A valid block stride (Sec. 6.2) replaces
    // the per-element scatter-vector reads along k.
    __device__ __forceinline__ void load(const KArgs<T, OffT>& a, OffT kb, int tid) {
        const OffT k0 = kb * KT;
        const OffT sx = a.kbsX[kb], sy = a.kbsY[kb];
        const OffT bx = a.cX[k0], by = a.rY[k0];
#pragma unroll
        for (int i = 0; i < EX; ++i) {
            const int kk = xk(tid + NTHR * i);
            const OffT kg = k0 + kk;
            T v = T(0);
            if (xv[i] && kg < a.k) v = a.X[xo[i] + (sx ? bx + (OffT)kk * sx : a.cX[kg])];
            rx[i] = v;
        }
#pragma unroll
        for (int i = 0; i < EY; ++i) {
            const int kk = yk(tid + NTHR * i);
            const OffT kg = k0 + kk;
            T v = T(0);
            if (yv[i] && kg < a.k) v = a.Y[yo[i] + (sy ? by + (OffT)kk * sy : a.rY[kg])];
            ry[i] = v;
        }
    }

    __device__ __forceinline__ void store(T* smem, int buf, int tid) const {
        T* bx = smem + buf * XS;
        T* by = smem + 2 * XS + buf * YS;
#pragma unroll
        for (int i = 0; i < EX; ++i) {
            const int e = tid + NTHR * i;
            bx[xk(e) * LDX + xrow(e)] = rx[i];
        }
#pragma unroll
        for (int i = 0; i < EY; ++i) {
            const int e = tid + NTHR * i;
            by[yk(e) * LDY + ycol(e)] = ry[i];
        }
    }
};

template <typename T, typename OffT>
__device__ __forceinline__ void store_c(const KArgs<T, OffT>& a, OffT mm, OffT co, T acc) {
    if (mm < a.m) {
        const OffT o = a.rC[mm] + co;
        T v = a.alpha * acc;
        if (a.beta != T(0)) v += a.beta * a.C[o];
        a.C[o] = v;
    }
}

// Regular layout: a WM x WN grid of waves, each owning FM x FN fragments.
template <typename T, typename OffT, int MT, int NT, int KT, int WM, int WN, bool XM, bool YN>
struct TileRegular {
    static constexpr int NTHR = WM * WN * 64;
    static constexpr int WTM = MT / WM, WTN = NT / WN;
    static constexpr int FM = WTM / 16, FN = WTN / 16;
    static_assert(KT % 4 == 0, "KT must be a multiple of the MFMA depth");
    static_assert(WTM % 16 == 0 && WTN % 16 == 0, "wave tiles are made of 16x16 fragments");
    typedef Pack<T, OffT, MT, NT, KT, NTHR, XM, YN> P;
    static constexpr int SMEM = P::ELEMS;

    static __device__ __forceinline__ void run(const KArgs<T, OffT>& a, int64_t tile, T* smem) {
        typedef Mfma<T> M;
        typedef typename M::acc_t acc_t;
        const int tid = threadIdx.x;
        const int lane = tid & 63, wave = tid >> 6;
        const int wm = wave % WM, wn = wave / WM;
        const int64_t tm = tile % a.tiles_m, tn = tile / a.tiles_m;
        const OffT m0 = (OffT)(tm * MT), n0 = (OffT)(tn * NT);

        P pk;
        pk.init(a, m0, n0, tid);
        acc_t acc[FM][FN];
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r) acc[i][j][r] = T(0);

        const OffT nkb = (a.k + KT - 1) / KT;
        if (nkb > 0) {
            pk.load(a, 0, tid);
            pk.store(smem, 0, tid);
            __syncthreads();
            for (OffT kb = 0; kb < nkb; ++kb) {
                const int buf = (int)(kb & 1);
                const bool more = kb + 1 < nkb;
                if (more) pk.load(a, kb + 1, tid);
                const T* bx = smem + buf * P::XS + wm * WTM + (lane & 15);
                const T* by = smem + 2 * P::XS + buf * P::YS + wn * WTN + (lane & 15);
#pragma unroll
                for (int s = 0; s < KT / 4; ++s) {
                    const int kr = 4 * s + (lane >> 4);
                    T fa[FM], fb[FN];
#pragma unroll
                    for (int i = 0; i < FM; ++i) fa[i] = bx[kr * P::LDX + 16 * i];
#pragma unroll
                    for (int j = 0; j < FN; ++j) fb[j] = by[kr * P::LDY + 16 * j];
#pragma unroll
                    for (int i = 0; i < FM; ++i)
#pragma unroll
                        for (int j = 0; j < FN; ++j) acc[i][j] = M::run(fa[i], fb[j], acc[i][j]);
                }
                if (more) pk.store(smem, buf ^ 1, tid);
                __syncthreads();
            }
        }
        // alpha/beta scatter-store through rscat_C / cscat_C (Sec. 6.1)
#pragma unroll
        for (int j = 0; j < FN; ++j) {
            const OffT nn = n0 + wn * WTN + 16 * j + (lane & 15);
            if (nn >= a.n) continue;
            const OffT co = a.cC[nn];
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int r = 0; r < 4; ++r) store_c(a, (OffT)(m0 + wm * WTM + 16 * i + M::row(lane, r)), co, acc[i][j][r]);
        }
    }
};

// Pinwheel layout for MT = NT = 144 on four waves: the 9 x 9 grid of 16 x 16
// fragments is covered by four rectangles of 20 fragments (4x5 at (0,0), 5x4
// at (0,5), 4x5 at (5,4), 5x4 at (4,0)) around the centre fragment (4,4),
// whose k-steps are dealt round-robin to the four waves and summed in LDS at
// the end.  Every SIMD then issues exactly 20.25 fragment updates per k-step,
// and a 2304 x 2304 output is exactly 256 tiles, one per compute unit.
template <typename T, typename OffT, int KT, bool XM, bool YN>
struct TilePinwheel {
    static constexpr int MT = 144, NT = 144, NTHR = 256;
    static_assert(KT % 16 == 0, "the centre k-split needs KT a multiple of 16");
    typedef Pack<T, OffT, MT, NT, KT, NTHR, XM, YN> P;
    static constexpr int SMEM = P::ELEMS > 4 * 256 ? P::ELEMS : 4 * 256;

    template <int R, int C>
    static __device__ __forceinline__ void step(typename Mfma<T>::acc_t* acc, const T* bx, const T* by, int kr, int fr0,
                                                int fc0) {
        T fa[R], fb[C];
#pragma unroll
        for (int i = 0; i < R; ++i) fa[i] = bx[kr * P::LDX + 16 * (fr0 + i)];
#pragma unroll
        for (int j = 0; j < C; ++j) fb[j] = by[kr * P::LDY + 16 * (fc0 + j)];
#pragma unroll
        for (int i = 0; i < R; ++i)
#pragma unroll
            for (int j = 0; j < C; ++j) acc[i * C + j] = Mfma<T>::run(fa[i], fb[j], acc[i * C + j]);
    }

    template <int R, int C>
    static __device__ __forceinline__ void epilogue(const KArgs<T, OffT>& a, const typename Mfma<T>::acc_t* acc,
                                                    OffT m0, OffT n0, int fr0, int fc0, int lane) {
#pragma unroll
        for (int j = 0; j < C; ++j) {
            const OffT nn = n0 + 16 * (fc0 + j) + (lane & 15);
            if (nn >= a.n) continue;
            const OffT co = a.cC[nn];
#pragma unroll
            for (int i = 0; i < R; ++i)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    store_c(a, (OffT)(m0 + 16 * (fr0 + i) + Mfma<T>::row(lane, r)), co, acc[i * C + j][r]);
        }
    }

    static __device__ __forceinline__ void run(const KArgs<T, OffT>& a, int64_t tile, T* smem) {
        typedef Mfma<T> M;
        typedef typename M::acc_t acc_t;
        const int tid = threadIdx.x;
        const int lane = tid & 63, wave = tid >> 6;
        // rectangle of this wave (in fragments)
        const bool wide = (wave & 1) == 0;  // 4 x 5 for waves 0 and 2, 5 x 4 for 1 and 3
        const int fr0 = wave == 2 ? 5 : wave == 3 ? 4 : 0;
        const int fc0 = wave == 1 ? 5 : wave == 2 ? 4 : 0;
        const int64_t tm = tile % a.tiles_m, tn = tile / a.tiles_m;
        const OffT m0 = (OffT)(tm * MT), n0 = (OffT)(tn * NT);

        P pk;
        pk.init(a, m0, n0, tid);
        acc_t acc[20], accc;
#pragma unroll
        for (int f = 0; f < 20; ++f)
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[f][r] = T(0);
#pragma unroll
        for (int r = 0; r < 4; ++r) accc[r] = T(0);

        const OffT nkb = (a.k + KT - 1) / KT;
        if (nkb > 0) {
            pk.load(a, 0, tid);
            pk.store(smem, 0, tid);
            __syncthreads();
            for (OffT kb = 0; kb < nkb; ++kb) {
                const int buf = (int)(kb & 1);
                const bool more = kb + 1 < nkb;
                if (more) pk.load(a, kb + 1, tid);
                const T* bx = smem + buf * P::XS + (lane & 15);
                const T* by = smem + 2 * P::XS + buf * P::YS + (lane & 15);
#pragma unroll
                for (int s = 0; s < KT / 4; ++s) {
                    const int kr = 4 * s + (lane >> 4);
                    if (wide) step<4, 5>(acc, bx, by, kr, fr0, fc0);
                    else step<5, 4>(acc, bx, by, kr, fr0, fc0);
                    if ((s & 3) == wave) accc = M::run(bx[kr * P::LDX + 64], by[kr * P::LDY + 64], accc);
                }
                if (more) pk.store(smem, buf ^ 1, tid);
                __syncthreads();
            }
        }
        if (wide) epilogue<4, 5>(a, acc, m0, n0, fr0, fc0, lane);
        else epilogue<5, 4>(a, acc, m0, n0, fr0, fc0, lane);
        // centre fragment: partial sums of the four waves added in wave order
#pragma unroll
        for (int r = 0; r < 4; ++r) smem[wave * 256 + r * 64 + lane] = accc[r];
        __syncthreads();
        if (wave == 0) {
            const OffT nn = n0 + 64 + (lane & 15);
            if (nn < a.n) {
                const OffT co = a.cC[nn];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    T v = smem[r * 64 + lane];
                    v += smem[256 + r * 64 + lane];
                    v += smem[512 + r * 64 + lane];
                    v += smem[768 + r * 64 + lane];
                    store_c(a, (OffT)(m0 + 64 + M::row(lane, r)), co, v);
                }
            }
        }
    }
};

template <typename T, typename OffT, int MT, int NT, int KT, int WM, int WN, int LAYOUT, bool XM, bool YN>
struct TileOf {
    typedef TileRegular<T, OffT, MT, NT, KT, WM, WN, XM, YN> type;
    static constexpr int threads = WM * WN * 64;
};
template <typename T, typename OffT, int MT, int NT, int KT, int WM, int WN, bool XM, bool YN>
struct TileOf<T, OffT, MT, NT, KT, WM, WN, 1, XM, YN> {
    typedef TilePinwheel<T, OffT, KT, XM, YN> type;
    static constexpr int threads = 256;
};

template <typename T, typename OffT, int MT, int NT, int KT, int WM, int WN, int LAYOUT, bool XM, bool YN>
__global__ __launch_bounds__((TileOf<T, OffT, MT, NT, KT, WM, WN, LAYOUT, XM, YN>::threads)) void contract_kernel(
    KArgs<T, OffT> a) {
    typedef typename TileOf<T, OffT, MT, NT, KT, WM, WN, LAYOUT, XM, YN>::type Tile;
    __shared__ T smem[Tile::SMEM];
    Tile::run(a, blockIdx.x, smem);
}

// C := beta * C over the matrix view (k == 0 or alpha == 0).
template <typename T, typename OffT>
__global__ __launch_bounds__(256) void scale_kernel(T* C, const OffT* rC, const OffT* cC, OffT m, OffT n, T beta) {
    const int64_t total = (int64_t)m * n;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        const OffT i = (OffT)(t % m), j = (OffT)(t / m);
        const OffT o = rC[i] + cC[j];
        C[o] = beta == T(0) ? T(0) : beta * C[o];
    }
}

static int hip_fail(hipError_t e, const char* what) {
    set_error(std::string(what) + ": " + hipGetErrorString(e));
    return TC_ERR_HIP;
}

template <typename T, typename OffT, int MT, int NT, int KT, int WM, int WN, int LAYOUT>
static int launch_tile(const KArgs<T, OffT>& a, bool xm, bool yn, hipStream_t s) {
    const int64_t tiles = a.tiles_m * a.tiles_n;
    if (tiles <= 0) return TC_OK;
    if (tiles > 0x7fffffffLL) {
        set_error("too many tiles for one launch");
        return TC_ERR_ARG;
    }
    dim3 grid((unsigned)tiles), block(TileOf<T, OffT, MT, NT, KT, WM, WN, LAYOUT, true, true>::threads);
    if (xm && yn)
        hipLaunchKernelGGL((contract_kernel<T, OffT, MT, NT, KT, WM, WN, LAYOUT, true, true>), grid, block, 0, s, a);
    else if (xm)
        hipLaunchKernelGGL((contract_kernel<T, OffT, MT, NT, KT, WM, WN, LAYOUT, true, false>), grid, block, 0, s, a);
    else if (yn)
        hipLaunchKernelGGL((contract_kernel<T, OffT, MT, NT, KT, WM, WN, LAYOUT, false, true>), grid, block, 0, s, a);
    else
        hipLaunchKernelGGL((contract_kernel<T, OffT, MT, NT, KT, WM, WN, LAYOUT, false, false>), grid, block, 0, s, a);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? TC_OK : hip_fail(e, "kernel launch");
}

template <typename T, typename OffT>
static int launch_typed(const Plan& p, const DeviceVectors& dv, double alpha, const void* A, const void* B,
                        double beta, void* C, hipStream_t s) {
    const OffT* base = (const OffT*)dv.buf;
    KArgs<T, OffT> a;
    a.X = (const T*)(p.swapped ? B : A);
    a.Y = (const T*)(p.swapped ? A : B);
    a.C = (T*)C;
    a.rX = base + dv.o_rX;
    a.cX = base + dv.o_cX;
    a.rY = base + dv.o_rY;
    a.cY = base + dv.o_cY;
    a.rC = base + dv.o_rC;
    a.cC = base + dv.o_cC;
    a.kbsX = base + dv.o_kbsX;
    a.kbsY = base + dv.o_kbsY;
    a.m = (OffT)p.m;
    a.n = (OffT)p.n;
    a.k = (OffT)p.k;
    a.tiles_m = p.tiles_m;
    a.tiles_n = p.tiles_n;
    a.alpha = (T)alpha;
    a.beta = (T)beta;
    if (p.m == 0 || p.n == 0) return TC_OK;
    if (p.k_empty || p.k == 0 || alpha == 0.0) {
        int64_t total = p.m * p.n;
        int64_t blocks = (total + 255) / 256;
        if (blocks > 65536) blocks = 65536;
        hipLaunchKernelGGL((scale_kernel<T, OffT>), dim3((unsigned)blocks), dim3(256), 0, s, (T*)C, a.rC, a.cC, a.m,
                           a.n, (T)beta);
        hipError_t e = hipGetLastError();
        return e == hipSuccess ? TC_OK : hip_fail(e, "kernel launch");
    }
    const bool xm = p.x_lanes_m, yn = p.y_lanes_n;
#define TC_CASE(id, MT, NT, KT, WM, WN, L) \
    case id:                               \
        return launch_tile<T, OffT, MT, NT, KT, WM, WN, L>(a, xm, yn, s);
    if (p.dtype == TC_F64) {
        switch (p.tile) { TC_TILES_F64(TC_CASE) }
    } else {
        switch (p.tile) { TC_TILES_F32(TC_CASE) }
    }
#undef TC_CASE
    set_error("unknown tile configuration");
    return TC_ERR_ARG;
}

int launch_plan(const Plan& p, const DeviceVectors& dv, double alpha, const void* A, const void* B, double beta,
                void* C, hipStream_t s) {
    if (p.mode != TC_NATIVE) {
        set_error("split-bf16 mode is not built into this library");
        return TC_ERR_DTYPE;
    }
    if (p.dtype == TC_F64)
        return p.off64 ? launch_typed<double, int64_t>(p, dv, alpha, A, B, beta, C, s)
                       : launch_typed<double, int32_t>(p, dv, alpha, A, B, beta, C, s);
    return p.off64 ? launch_typed<float, int64_t>(p, dv, alpha, A, B, beta, C, s)
                   : launch_typed<float, int32_t>(p, dv, alpha, A, B, beta, C, s);
}

int launch_batch(int, int, int, bool, const BatchItemDev*, int, int64_t, int, hipStream_t) {
    set_error("batched launch not built into this library");
    return TC_ERR_ARG;
}

int batch_grid(int, int, int, int64_t) { return 0; }

}  // namespace tc
