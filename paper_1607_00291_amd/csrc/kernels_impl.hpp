#pragma once
// Kernel templates of the transpose-free contraction (block-scatter-matrix
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
#include <type_traits>
#include <utility>
#include <cstdio>

#include "launch.hpp"
#include "tc.h"
#include "tiles.hpp"

namespace tc {

static int hip_fail(hipError_t e, const char* what) {
    set_error(std::string(what) + ": " + hipGetErrorString(e));
    return TC_ERR_HIP;
}

typedef float f32x4 __attribute__((ext_vector_type(4)));

// Four FP64 accumulators kept as independent scalars, so every matrix-core
// instruction can update its accumulator in place.
struct f64acc {
    double v[4];
    __device__ __forceinline__ double& operator[](int i) { return v[i]; }
    __device__ __forceinline__ const double& operator[](int i) const { return v[i]; }
};

// Matrix-core update of one 16 x 16 output fragment by a 16 x 4 sliver of X
// and a 4 x 16 sliver of Y, both read from k-major LDS stages.  Each trait
// gives the operand loads, the update, and the (row, column) inside the
// fragment of accumulator element t of a lane.
template <typename T>
struct Mfma;

// FP64: four v_mfma_f64_4x4x4_4b per fragment update.  One such instruction
// holds four independent 4x4x4 blocks; lane l = i + 4*blk + 16*k carries
// A[blk][i][k] and B[blk][k][j = l%4], and receives D[blk][i = l/16][j = l%4]
// at l = j + 4*blk + 16*i.  Instruction t pairs A rows 4*blk.. with B columns
// 4*((blk + t) % 4).., so the four instructions cover the whole 16 x 16
// fragment with one shared A register and four B registers.  (On gfx950 this
// form issues at close to the FP64 matrix peak; the 16x16x4 FP64 form
// sustains about half of it.)
template <>
struct Mfma<double> {
    typedef f64acc acc_t;
    typedef double afrag;
    struct bfrag {
        double v[4];
    };
    static __device__ __forceinline__ int bcol(int lane, int t) { return 4 * ((((lane >> 2) & 3) + t) & 3) + (lane & 3); }
    static __device__ __forceinline__ afrag load_a(const double* row, int lane) { return row[lane & 15]; }
    static __device__ __forceinline__ bfrag load_b(const double* row, int lane) {
        bfrag f;
#pragma unroll
        for (int t = 0; t < 4; ++t) f.v[t] = row[bcol(lane, t)];
        return f;
    }
    static __device__ __forceinline__ void run(afrag a, const bfrag& b, acc_t& c) {
        c.v[0] = __builtin_amdgcn_mfma_f64_4x4x4f64(a, b.v[0], c.v[0], 0, 0, 0);
        c.v[1] = __builtin_amdgcn_mfma_f64_4x4x4f64(a, b.v[1], c.v[1], 0, 0, 0);
        c.v[2] = __builtin_amdgcn_mfma_f64_4x4x4f64(a, b.v[2], c.v[2], 0, 0, 0);
        c.v[3] = __builtin_amdgcn_mfma_f64_4x4x4f64(a, b.v[3], c.v[3], 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int) { return 4 * ((lane >> 2) & 3) + (lane >> 4); }
    static __device__ __forceinline__ int col(int lane, int t) { return bcol(lane, t); }
};

// FP64 with the diagonal on the A side: instruction t pairs B columns
// 4*blk.. with A rows 4*((blk + t) % 4).., so one B register is shared and
// four A registers are read.  Used where a wave holds more B fragments than
// A fragments (fewer operand registers live).
struct Mfma64DiagA {
    typedef f64acc acc_t;
    struct afrag {
        double v[4];
    };
    typedef double bfrag;
    static __device__ __forceinline__ afrag load_a(const double* row, int lane) {
        afrag f;
#pragma unroll
        for (int t = 0; t < 4; ++t) f.v[t] = row[Mfma<double>::bcol(lane, t)];
        return f;
    }
    static __device__ __forceinline__ bfrag load_b(const double* row, int lane) { return row[lane & 15]; }
    static __device__ __forceinline__ void run(const afrag& a, bfrag b, acc_t& c) {
        c.v[0] = __builtin_amdgcn_mfma_f64_4x4x4f64(a.v[0], b, c.v[0], 0, 0, 0);
        c.v[1] = __builtin_amdgcn_mfma_f64_4x4x4f64(a.v[1], b, c.v[1], 0, 0, 0);
        c.v[2] = __builtin_amdgcn_mfma_f64_4x4x4f64(a.v[2], b, c.v[2], 0, 0, 0);
        c.v[3] = __builtin_amdgcn_mfma_f64_4x4x4f64(a.v[3], b, c.v[3], 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int t) { return Mfma<double>::bcol(lane, t) - (lane & 3) + (lane >> 4); }
    static __device__ __forceinline__ int col(int lane, int) { return lane & 15; }
};

// Operand schedule for a wave rectangle of R x C fragments: FP64 puts the
// diagonal on the side with fewer fragments.
template <typename T, bool WIDE>
struct MfmaFor {
    typedef Mfma<T> type;
};
template <>
struct MfmaFor<double, true> {
    typedef Mfma64DiagA type;
};

// FP32: v_mfma_f32_16x16x4_f32; lane l carries A[l%16][l/16], B[l/16][l%16]
// and receives D[4*(l/16) + t][l%16] in element t.
template <>
struct Mfma<float> {
    typedef f32x4 acc_t;
    typedef float afrag;
    typedef float bfrag;
    static __device__ __forceinline__ afrag load_a(const float* row, int lane) { return row[lane & 15]; }
    static __device__ __forceinline__ bfrag load_b(const float* row, int lane) { return row[lane & 15]; }
    static __device__ __forceinline__ void run(afrag a, bfrag b, acc_t& c) {
        c = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int t) { return 4 * (lane >> 4) + t; }
    static __device__ __forceinline__ int col(int lane, int) { return lane & 15; }
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
    int64_t spanX, spanY;  // element spans of X and Y (bounds of the buffer loads)
    T alpha, beta;
    int kregX, kregY;  // 1: every k block of X (Y) has a nonzero block stride
    OffT ksX, ksY;     // the block stride shared by every k block of X (Y), else 0
    int xm, yn;        // X gathered with lanes along m (else k), Y along n (else k)
    const void* packed;  // split panels of X then Y (the packed split tile), else unused
};

// LDS row pitch (in elements) of a k-major stage: one element of padding when
// the lanes of the gather run along k (consecutive lanes then write to
// consecutive LDS rows, and the pad spreads them over the banks).
template <int W, bool LANES_ALONG_ROW>
struct Pitch {
    static constexpr int value = LANES_ALONG_ROW ? W : W + 1;
};

// Values every lane of a wave holds equally (loaded from a uniform address),
// moved to scalar registers so that they can serve as a buffer load's scalar
// offset and as branch conditions without per-lane handling.
__device__ __forceinline__ int32_t uniform(int32_t x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ int64_t uniform(int64_t x) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)(uint64_t)x);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)((uint64_t)x >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Calls f(std::integral_constant<int, I>()) for I = 0 .. N-1 in order.
template <typename F, int... I>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, I...>) {
    (f(std::integral_constant<int, I>()), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
    static_for_impl(f, std::make_integer_sequence<int, N>());
}

// XCD-aware tile order.  Workgroups are dispatched round-robin over the 8
// XCDs (workgroup w runs on XCD w % 8), each with its own L2.  Workgroup w is
// given tile g = (w % 8) * T/8 + w / 8 of a grouped enumeration that walks
// G rows of tiles at a time (tm fastest inside a group), so every XCD works
// on a compact G x (T/8G) block and reads about G + T/(8G) operand panels
// instead of (for the plain column-major order) a few rows and every column.
// Identity when T is not a multiple of 8 or too small to matter.
__device__ __forceinline__ int64_t xcd_tile(int64_t w, int64_t tiles_m, int64_t tiles_n) {
    const int64_t T = tiles_m * tiles_n;
    if (T % 8 != 0 || T < 64) return w;
    const int64_t c = T / 8;
    const int64_t g = (w % 8) * c + w / 8;
    int64_t G = 1;
    while (G * G * 4 <= c && G * 2 <= tiles_m) G *= 2;  // G ~ sqrt(c), a power of two
    const int64_t per = G * tiles_n;
    const int64_t grp = g / per, within = g % per;
    const int64_t gh = (tiles_m - grp * G) < G ? (tiles_m - grp * G) : G;
    const int64_t tm = grp * G + within % gh, tn = within / gh;
    return tm + tiles_m * tn;
}

// Bounds-checked buffer loads (32-bit-offset plans): a byte offset at or past
// the buffer's size reads 0, so ragged edges need no select after the load
// and every load of a stage can stay in flight until the LDS write.
#define TC_BUF_DWORD3 0x00020000
static constexpr uint32_t kOutOfRange = 0x80000000u;

template <typename T>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const T* p, int64_t elems) {
    return __builtin_amdgcn_make_buffer_rsrc((void*)p, (short)0, (int)(elems * (int64_t)sizeof(T)), TC_BUF_DWORD3);
}
template <typename T>
__device__ __forceinline__ T buf_load(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff);
template <>
__device__ __forceinline__ double buf_load<double>(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0));
}
template <>
__device__ __forceinline__ float buf_load<float>(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0));
}

// The pack stage of one operand of one tile: an R x KT sliver (R rows of m
// for X, of n for Y) gathered through the offset vectors into registers, then
// written to a k-major LDS stage.  Element e = t + NTHR * i of a stage is
// (row, kk) with the row index fastest when the operand's lanes run along its
// free index (LR), and kk fastest when they run along k.
template <typename T, typename OffT, int R, int KT, int NTHR, bool LR, int SLOTS = 1>
struct PackOp {
    static constexpr int E = R * KT / NTHR;
    static constexpr int LD = Pitch<R, LR>::value;
    static constexpr int S = KT * LD;  // elements of one stage
    static_assert((R * KT) % NTHR == 0, "stage must split evenly over threads");

    static __device__ __forceinline__ int ridx(int e) { return LR ? e % R : e / KT; }
    static __device__ __forceinline__ int kidx(int e) { return LR ? e / R : e % KT; }

    OffT o[E];       // offsets of this thread's rows, fixed per tile; -1 past the edge
    T r[SLOTS][E];  // stages in flight

    __device__ __forceinline__ void init(const OffT* rowvec, OffT r0, OffT rmax, int t) {
#pragma unroll
        for (int i = 0; i < E; ++i) {
            const OffT rr = r0 + ridx(t + NTHR * i);
            const OffT x = rowvec[rr < rmax ? rr : rmax - 1];
            o[i] = rr < rmax ? x : OffT(-1);
        }
    }

    // Global gather of k block kb.  A valid block stride (Sec. 6.2) replaces
    // the per-element scatter-vector reads along k; the choice is uniform.
    // REG = 1: every block of this operand is known to have one (no per-k
    // offset reads compiled in); REG = -1: decided per block.  SL: the
    // register slot that receives the stage.
    template <int REG = -1, int SL = 0>
    __device__ __forceinline__ void load(const T* base, int64_t span, const OffT* kvec, const OffT* kbs, OffT kb, OffT K,
                                         int t) {
        const OffT k0 = kb * KT;
        const OffT sk = uniform(kbs[kb]);
        OffT ko[E];
        OffT kbase = 0;
        if (REG == 1 || sk) {
            kbase = uniform(kvec[k0]);
#pragma unroll
            for (int i = 0; i < E; ++i) ko[i] = (OffT)kidx(t + NTHR * i) * sk;
        } else if (LR && NTHR % R == 0 && R % 64 == 0) {
            // lanes along the free index, R a multiple of the wave size:
            // element i's k is the same in every lane of a wave, so its
            // offset is one scalar load
#pragma unroll
            for (int i = 0; i < E; ++i) {
                const OffT kg = k0 + uniform((int32_t)kidx(t + NTHR * i));
                ko[i] = uniform(kvec[kg < K ? kg : K - 1]);
            }
        } else {
#pragma unroll
            for (int i = 0; i < E; ++i) {
                const OffT kg = k0 + kidx(t + NTHR * i);
                ko[i] = kvec[kg < K ? kg : K - 1];
            }
        }
        if constexpr (sizeof(OffT) == 4) {
            const __amdgpu_buffer_rsrc_t rs = make_rsrc(base, span);
            const uint32_t soff = (uint32_t)uniform((int32_t)((uint32_t)kbase * (uint32_t)sizeof(T)));
#pragma unroll
            for (int i = 0; i < E; ++i) {
                const bool ok = o[i] >= 0 && k0 + kidx(t + NTHR * i) < K;
                const uint32_t vo = ok ? (uint32_t)(o[i] + ko[i]) * (uint32_t)sizeof(T) : kOutOfRange;
                r[SL][i] = buf_load<T>(rs, vo, soff);
            }
        } else {
#pragma unroll
            for (int i = 0; i < E; ++i) {
                const bool ok = o[i] >= 0 && k0 + kidx(t + NTHR * i) < K;
                const T x = base[ok ? kbase + o[i] + ko[i] : OffT(0)];
                r[SL][i] = ok ? x : T(0);
            }
        }
    }

    template <int SL = 0>
    __device__ __forceinline__ void store(T* stage, int t) const {
#pragma unroll
        for (int i = 0; i < E; ++i) {
            const int e = t + NTHR * i;
            stage[kidx(e) * LD + ridx(e)] = r[SL][i];
        }
    }
};

// Both operands of a tile, every thread gathering its share of each.
template <typename T, typename OffT, int MT, int NT, int KT, int NTHR, bool XM, bool YN, int SLOTS = 1>
struct Pack {
    typedef PackOp<T, OffT, MT, KT, NTHR, XM, SLOTS> PX;
    typedef PackOp<T, OffT, NT, KT, NTHR, YN, SLOTS> PY;
    static constexpr int LDX = PX::LD, LDY = PY::LD, XS = PX::S, YS = PY::S;
    static constexpr int ELEMS = 2 * (XS + YS);  // [X0][X1][Y0][Y1]
    PX px;
    PY py;
    __device__ __forceinline__ void init(const KArgs<T, OffT>& a, OffT m0, OffT n0, int t) {
        px.init(a.rX, m0, a.m, t);
        py.init(a.cY, n0, a.n, t);
    }
    template <int REG = -1, int SL = 0>
    __device__ __forceinline__ void load(const KArgs<T, OffT>& a, OffT kb, int t) {
        px.template load<REG, SL>(a.X, a.spanX, a.cX, a.kbsX, kb, a.k, t);
        py.template load<REG, SL>(a.Y, a.spanY, a.rY, a.kbsY, kb, a.k, t);
    }
    template <int SL = 0>
    __device__ __forceinline__ void store(T* smem, int buf, int t) const {
        px.template store<SL>(smem + buf * XS, t);
        py.template store<SL>(smem + 2 * XS + buf * YS, t);
    }
};

// alpha/beta update of an R x C rectangle of accumulator fragments through
// rscat_C / cscat_C (Sec. 6.1); C is read only when beta != 0.  Fragment
// (i, j) covers fragment rows r0 + 16 i + M::row and columns c0 + 16 j +
// M::col; they are C's m and n, or n and m when TR (a rectangle computed as
// C^T).  The offset reads, the C reads of a fragment row and its stores are
// each issued as one group, so a lane waits for two memory round trips per
// fragment row rather than two per element.
template <typename T, typename OffT, typename M, int R, int C, bool TR>
__device__ __forceinline__ void store_rect(const KArgs<T, OffT>& a, const typename M::acc_t* acc, OffT r0, OffT c0,
                                           int lane) {
    const OffT rmax = TR ? a.n : a.m, cmax = TR ? a.m : a.n;
    const OffT* rvec = TR ? a.cC : a.rC;
    const OffT* cvec = TR ? a.rC : a.cC;
    OffT co[C][4];
    bool cok[C][4];
#pragma unroll
    for (int j = 0; j < C; ++j)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const OffT c = (OffT)(c0 + 16 * j + M::col(lane, t));
            cok[j][t] = c < cmax;
            co[j][t] = cvec[cok[j][t] ? c : OffT(0)];
        }
#pragma unroll
    for (int i = 0; i < R; ++i) {
        OffT ro[4];
        bool rok[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const OffT r = (OffT)(r0 + 16 * i + M::row(lane, t));
            rok[t] = r < rmax;
            ro[t] = rvec[rok[t] ? r : OffT(0)];
        }
        T cv[C][4];
        if (a.beta != T(0)) {
#pragma unroll
            for (int j = 0; j < C; ++j)
#pragma unroll
                for (int t = 0; t < 4; ++t) cv[j][t] = a.C[rok[t] && cok[j][t] ? ro[t] + co[j][t] : OffT(0)];
        }
#pragma unroll
        for (int j = 0; j < C; ++j)
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                if (rok[t] && cok[j][t]) {
                    T v = a.alpha * acc[i * C + j][t];
                    if (a.beta != T(0)) v += a.beta * cv[j][t];
                    a.C[ro[t] + co[j][t]] = v;
                }
            }
    }
}

// Store of one accumulator fragment whose origin in C's matrix view is
// (fm0, fn0).
template <typename T, typename OffT, typename M = Mfma<T>>
__device__ __forceinline__ void store_frag(const KArgs<T, OffT>& a, OffT fm0, OffT fn0, const typename M::acc_t& acc,
                                           int lane) {
    store_rect<T, OffT, M, 1, 1, false>(a, &acc, fm0, fn0, lane);
}

// One k-step (depth 4) of an R x C rectangle of fragments: the products of
// A fragment rows fa[0..R) with B fragment columns fb[0..C).
template <typename T, typename M, int R, int C>
__device__ __forceinline__ void rect_mma(typename M::acc_t* acc, const typename M::afrag* fa,
                                         const typename M::bfrag* fb) {
#pragma unroll
    for (int i = 0; i < R; ++i)
#pragma unroll
        for (int j = 0; j < C; ++j) M::run(fa[i], fb[j], acc[i * C + j]);
}

template <typename T, typename OffT, typename M, int R, int C>
__device__ __forceinline__ void rect_store(const KArgs<T, OffT>& a, const typename M::acc_t* acc, OffT m0, OffT n0,
                                           int fr0, int fc0, int lane) {
    store_rect<T, OffT, M, R, C, false>(a, acc, (OffT)(m0 + 16 * fr0), (OffT)(n0 + 16 * fc0), lane);
}

// Store of a rectangle computed as C^T: fragment (i, j) covers n-fragment
// fp0 + i and m-fragment fq0 + j; its element rows are n, columns m.
template <typename T, typename OffT, typename M, int R, int C>
__device__ __forceinline__ void rect_store_t(const KArgs<T, OffT>& a, const typename M::acc_t* acc, OffT m0, OffT n0,
                                             int fp0, int fq0, int lane) {
    store_rect<T, OffT, M, R, C, true>(a, acc, (OffT)(n0 + 16 * fp0), (OffT)(m0 + 16 * fq0), lane);
}

// Regular layout: a WM x WN grid of waves, each owning FM x FN fragments.
template <typename T, typename OffT, int MT, int NT, int KT, int WM, int WN, bool XM, bool YN>
struct TileRegular {
    static constexpr int NTHR = WM * WN * 64;
    static constexpr int WTM = MT / WM, WTN = NT / WN;
    static constexpr int FM = WTM / 16, FN = WTN / 16;
    static_assert(KT % 4 == 0, "KT must be a multiple of the MFMA depth");
    static_assert(WTM % 16 == 0 && WTN % 16 == 0, "wave tiles are made of 16x16 fragments");
    // gathered stages in flight per thread: one, except on the 32 x 32 tile
    // of four one-fragment waves, whose stages are short against a
    // gather's latency (a few, within the 63 loads the memory counter tracks)
    static constexpr int LOADS = (MT + NT) * KT / NTHR;
    static constexpr int SLOTS = !(MT == 32 && NT == 32 && WM * WN == 4) ? 1
                                 : 4 * LOADS <= 63                       ? 4
                                 : 3 * LOADS <= 63                       ? 3
                                                                         : 1;
    typedef Pack<T, OffT, MT, NT, KT, NTHR, XM, YN, SLOTS> P;
    static constexpr int SMEM = P::ELEMS;

    static __device__ __forceinline__ void run(const KArgs<T, OffT>& a, int64_t tile, T* smem) {
        typedef Mfma<T> M;
        typedef typename M::acc_t acc_t;
        const int tid = threadIdx.x;
        const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
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
        auto compute = [&](int buf) {
            const T* bx = smem + buf * P::XS + wm * WTM;
            const T* by = smem + 2 * P::XS + buf * P::YS + wn * WTN;
#pragma unroll
            for (int s = 0; s < KT / 4; ++s) {
                const int kr = 4 * s + (lane >> 4);
                typename M::afrag fa[FM];
                typename M::bfrag fb[FN];
#pragma unroll
                for (int i = 0; i < FM; ++i) fa[i] = M::load_a(bx + kr * P::LDX + 16 * i, lane);
#pragma unroll
                for (int j = 0; j < FN; ++j) fb[j] = M::load_b(by + kr * P::LDY + 16 * j, lane);
#pragma unroll
                for (int i = 0; i < FM; ++i)
#pragma unroll
                    for (int j = 0; j < FN; ++j) M::run(fa[i], fb[j], acc[i][j]);
            }
        };
        // The gathers of stage kb + 1 and their LDS store run with no branch
        // around them: past the last stage they re-read the last block and
        // fill the LDS buffer that no stage reads any more.
        auto pipeline = [&](auto reg) {
            constexpr int RG = decltype(reg)::value;
            if constexpr (SLOTS == 1) {
                pk.template load<RG>(a, 0, tid);
                pk.store(smem, 0, tid);
                __syncthreads();
                for (OffT kb = 0; kb < nkb; ++kb) {
                    const int buf = (int)(kb & 1);
                    pk.template load<RG>(a, kb + 1 < nkb ? kb + 1 : kb, tid);
                    compute(buf);
                    pk.store(smem, buf ^ 1, tid);
                    __syncthreads();
                }
            } else {
                // stages kb + 1 .. kb + SLOTS in flight in registers while
                // stage kb is computed from LDS
                static_for<SLOTS>([&](auto ic) {
                    constexpr int i = decltype(ic)::value;
                    pk.template load<RG, i>(a, nkb > i ? (OffT)i : nkb - 1, tid);
                });
                pk.template store<0>(smem, 0, tid);
                __syncthreads();
                for (OffT kb0 = 0; kb0 < nkb; kb0 += SLOTS)
                    static_for<SLOTS>([&](auto ic) {
                        constexpr int i = decltype(ic)::value;
                        const OffT kb = kb0 + i;
                        const int buf = (int)(kb & 1);
                        // slot i held stage kb, already in LDS: refill it
                        pk.template load<RG, i>(a, kb + SLOTS < nkb ? kb + SLOTS : nkb - 1, tid);
                        if (kb < nkb) compute(buf);
                        // stage kb + 1, gathered SLOTS - 1 stages ago
                        pk.template store<(i + 1) % SLOTS>(smem, buf ^ 1, tid);
                        __syncthreads();
                    });
            }
        };
        if (nkb > 0) {
            if (a.kregX && a.kregY) pipeline(std::integral_constant<int, 1>());
            else pipeline(std::integral_constant<int, -1>());
        }
        // alpha/beta scatter-store through rscat_C / cscat_C (Sec. 6.1)
        store_rect<T, OffT, M, FM, FN, false>(a, &acc[0][0], (OffT)(m0 + wm * WTM), (OffT)(n0 + wn * WTN), lane);
    }
};

// The pack stage of one operand, with the operand (and so the lane
// direction and LDS pitch) chosen at run time: used where a wave gathers
// either X or Y, so that only one set of gather registers is live.
template <typename T, typename OffT, int R, int KT, int NTHR, int SLOTS = 1>
struct PackRole {
    static constexpr int E = R * KT / NTHR;
    static_assert((R * KT) % NTHR == 0, "stage must split evenly over threads");
    OffT o[E];  // -1 past the edge
    T r[SLOTS][E];  // stages in flight
    bool lr;  // lanes along the free index
    int ld;   // LDS pitch
    __device__ __forceinline__ int ridx(int e) const { return lr ? e % R : e / KT; }
    __device__ __forceinline__ int kidx(int e) const { return lr ? e / R : e % KT; }
    __device__ __forceinline__ void init(const OffT* rowvec, OffT r0, OffT rmax, int t, bool lanes_row, int pitch) {
        lr = lanes_row;
        ld = pitch;
#pragma unroll
        for (int i = 0; i < E; ++i) {
            const OffT rr = r0 + ridx(t + NTHR * i);
            const OffT x = rowvec[rr < rmax ? rr : rmax - 1];
            o[i] = rr < rmax ? x : OffT(-1);
        }
    }
    template <int SL = 0>
    __device__ __forceinline__ void load(const T* base, int64_t span, const OffT* kvec, const OffT* kbs, OffT kb, OffT K,
                                         int t) {
        load_with<SL>(uniform(kbs[kb]), uniform(kvec[kb * KT]), base, span, kvec, kb, K, t);
    }
    // Every k block shares the block stride s (REG = 2 below): the offset of
    // element i relative to its block's first k offset is the same in every
    // block, so it is formed once per tile, in bytes (out of range past the
    // edge), and the k offsets of a block reach the loads as one scalar.
    // tail: the elements that stay inside the last, partial block (bit i;
    // one bit per element of a thread's share, so at most 64 elements).
    static_assert(E <= 64, "the partial-block mask holds one bit per element");
    uint64_t tail = 0;
    __device__ __forceinline__ void fix_offsets(OffT s, OffT K, int t) {
        const OffT rem = K % KT;
#pragma unroll
        for (int i = 0; i < E; ++i) {
            const OffT kk = (OffT)kidx(t + NTHR * i);
            o[i] = o[i] >= 0 ? (OffT)((uint32_t)(o[i] + kk * s) * (uint32_t)sizeof(T)) : (OffT)kOutOfRange;
            tail |= (uint64_t)(kk < rem) << i;
        }
    }
    // The same with the k block's stride and first k offset already in
    // scalar registers (fetched ahead by the caller).  REG = 1: the caller
    // knows every k block of this operand has a nonzero stride (no per-k
    // offset reads); REG = 0: always read the per-k offsets (right for any
    // block); REG = -1: decide per block.  A compile-time choice keeps the
    // per-k offset reads (vector memory loads) off the regular path, so the
    // counter waits they need do not hold back gathers already in flight.
    template <int SL = 0, int REG = -1>
    __device__ __forceinline__ void load_with(OffT sk, OffT kfirst, const T* base, int64_t span, const OffT* kvec,
                                              OffT kb, OffT K, int t) {
        const OffT k0 = kb * KT;
        if constexpr (REG == 2 && sizeof(OffT) == 4) {
            const __amdgpu_buffer_rsrc_t rs = make_rsrc(base, span);
            const uint32_t soff = (uint32_t)uniform((int32_t)((uint32_t)kfirst * (uint32_t)sizeof(T)));
            const bool partial = k0 + KT > K;
#pragma unroll
            for (int i = 0; i < E; ++i) {
                const uint32_t vo = partial && !((tail >> i) & 1ull) ? kOutOfRange : (uint32_t)o[i];
                r[SL][i] = buf_load<T>(rs, vo, soff);
            }
            return;
        }
        OffT ko[E];
        OffT kbase = 0;
        if (REG >= 1 || (REG == -1 && sk)) {
            kbase = kfirst;
#pragma unroll
            for (int i = 0; i < E; ++i) ko[i] = (OffT)kidx(t + NTHR * i) * sk;
        } else if (lr && NTHR % R == 0 && R % 64 == 0) {
            // lanes along the free index, R a multiple of the wave size:
            // element i's k, (t + NTHR i) / R, is the same in every lane of a
            // wave, so its offset is one scalar load
#pragma unroll
            for (int i = 0; i < E; ++i) {
                const OffT kg = k0 + uniform((int32_t)((t + NTHR * i) / R));
                ko[i] = uniform(kvec[kg < K ? kg : K - 1]);
            }
        } else {
#pragma unroll
            for (int i = 0; i < E; ++i) {
                const OffT kg = k0 + kidx(t + NTHR * i);
                ko[i] = kvec[kg < K ? kg : K - 1];
            }
        }
        if constexpr (sizeof(OffT) == 4) {
            const __amdgpu_buffer_rsrc_t rs = make_rsrc(base, span);
            const uint32_t soff = (uint32_t)uniform((int32_t)((uint32_t)kbase * (uint32_t)sizeof(T)));
#pragma unroll
            for (int i = 0; i < E; ++i) {
                const bool ok = o[i] >= 0 && k0 + kidx(t + NTHR * i) < K;
                const uint32_t vo = ok ? (uint32_t)(o[i] + ko[i]) * (uint32_t)sizeof(T) : kOutOfRange;
                r[SL][i] = buf_load<T>(rs, vo, soff);
            }
        } else {
#pragma unroll
            for (int i = 0; i < E; ++i) {
                const bool ok = o[i] >= 0 && k0 + kidx(t + NTHR * i) < K;
                const T x = base[ok ? kbase + o[i] + ko[i] : OffT(0)];
                r[SL][i] = ok ? x : T(0);
            }
        }
    }
    template <int SL = 0>
    __device__ __forceinline__ void store(T* stage, int t) const {
#pragma unroll
        for (int i = 0; i < E; ++i) {
            const int e = t + NTHR * i;
            stage[kidx(e) * ld + ridx(e)] = r[SL][i];
        }
    }
};

// Pinwheel layout for MT = NT = 144 on eight waves (two per SIMD).  The 9 x 9
// grid of 16 x 16 fragments minus its centre fragment (4,4) is covered by
// four 4x5 / 5x4 rectangles arranged as a pinwheel around it (4x5 at (0,0),
// 5x4 at (0,5), 4x5 at (5,4), 5x4 at (4,0)); each wave owns half a rectangle
// (2 x 5 or 5 x 2 fragments) and the centre fragment's k-steps are dealt
// round-robin over the eight waves and summed in LDS at the end.  Every SIMD
// then issues exactly 20.25 fragment updates per k-step, and a 2304 x 2304
// output is exactly 256 tiles, one per compute unit.  Waves 0-3 gather the X
// sliver and waves 4-7 the Y sliver of each stage.
template <typename T, typename OffT, int KT, bool XM, bool YN>
struct TilePinwheel8 {
    static constexpr int MT = 144, NT = 144, NTHR = 512;
    static_assert(KT % 4 == 0, "KT must be a multiple of the MFMA depth");
    // gather register slots: two (a three-stage pipeline) when one stage's
    // share is small, else one (two stages: gathers of kb + 1 in flight)
    static constexpr int SLOTS = (144 * KT / 256) * (int)sizeof(T) <= 72 ? 2 : 1;
    typedef PackRole<T, OffT, 144, KT, 256, SLOTS> PR;
    static constexpr int LDX = Pitch<MT, XM>::value, LDY = Pitch<NT, YN>::value;
    static constexpr int XS = KT * LDX, YS = KT * LDY;
    static constexpr int ELEMS = 2 * (XS + YS);
    static constexpr int SMEM = ELEMS > 8 * 256 ? ELEMS : 8 * 256;
    typedef typename MfmaFor<T, true>::type MW;  // every wave runs a 2 x 5 rectangle

    static __device__ __forceinline__ void run(const KArgs<T, OffT>& a, int64_t tile, T* smem) {
        typedef Mfma<T> M;
        typedef typename M::acc_t acc_t;
        const int tid = threadIdx.x;
        const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
        const int tt = tid & 255;  // thread index inside the gathering half
        const int q = wave >> 1, h = wave & 1;
        const bool wide = (q & 1) == 0;
        const int fr0 = q == 0 ? 2 * h : q == 1 ? 0 : q == 2 ? 5 + 2 * h : 4;
        const int fc0 = q == 0 ? 0 : q == 1 ? 5 + 2 * h : q == 2 ? 4 : 2 * h;
        const int64_t tm = tile % a.tiles_m, tn = tile / a.tiles_m;
        const OffT m0 = (OffT)(tm * MT), n0 = (OffT)(tn * NT);
        const bool gx = wave < 4;
        const int p0 = wide ? fr0 : fc0, q0 = wide ? fc0 : fr0;
        const int ldp = wide ? LDX : LDY, ldq = wide ? LDY : LDX;
        // this wave's operand
        const T* gbase = gx ? a.X : a.Y;
        const int64_t gspan = gx ? a.spanX : a.spanY;
        const OffT* gk = gx ? a.cX : a.rY;
        const OffT* gbs = gx ? a.kbsX : a.kbsY;
        T* gstage = gx ? smem : smem + 2 * XS;
        const int gsz = gx ? XS : YS;

        PR pk;
        if (gx) pk.init(a.rX, m0, a.m, tt, XM, LDX);
        else pk.init(a.cY, n0, a.n, tt, YN, LDY);
        acc_t acc[10], accc;
#pragma unroll
        for (int f = 0; f < 10; ++f)
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[f][r] = T(0);
#pragma unroll
        for (int r = 0; r < 4; ++r) accc[r] = T(0);

        const OffT nkb = (a.k + KT - 1) / KT;
        // Three-stage pipeline: while the matrix cores consume LDS stage kb,
        // the gathers of stage kb + 2 are in flight in one register slot and
        // stage kb + 1 (gathered one iteration earlier) goes from the other
        // slot to LDS, so each gather has two stages of compute to land.
        // block stride and first k offset of the next gather, fetched one
        // stage ahead so their scalar-load latency is hidden
        OffT pre_sk = 0, pre_k = 0;
        auto fetch = [&](OffT kb) {
            pre_sk = uniform(gbs[kb]);
            pre_k = uniform(gk[kb * KT]);
        };
        // Every stage issues its gathers and its LDS store with no branch
        // around them: a gather past the last stage re-reads the last stage
        // and is stored into the LDS buffer no stage reads any more, and with
        // two slots an odd stage count ends with one stage that only moves
        // data.  The counter waits the compiler places then see the same
        // memory operations in flight on every path, and the gathers of later
        // stages stay in flight over the compute.
        auto body = [&](OffT kb, auto slot, auto reg) {
            constexpr int SL = decltype(slot)::value;
            constexpr int RG = decltype(reg)::value;
            constexpr int AHEAD = SLOTS;  // stages between a gather and its use
            const int buf = (int)(kb & 1);
            const OffT lk = kb + AHEAD < nkb ? kb + AHEAD : nkb - 1;
            pk.template load_with<SL, RG>(pre_sk, pre_k, gbase, gspan, gk, lk, a.k, tt);
            fetch(kb + AHEAD + 1 < nkb ? kb + AHEAD + 1 : nkb - 1);
            if (kb < nkb) {
                const T* bx = smem + buf * XS;
                const T* by = smem + 2 * XS + buf * YS;
                // a 5 x 2 rectangle of C is run as the 2 x 5 rectangle of C^T:
                // the Y stage feeds the A side and the X stage the B side
                const T* bp = wide ? bx : by;
                const T* bq = wide ? by : bx;
                typename M::afrag ca;
                typename M::bfrag cb;
                const int kr0 = lane >> 4;
                // the centre fragment's k-steps go round-robin over the waves
                const int cs = (wave - (int)((kb * (KT / 4)) & 7)) & 7;  // this wave's centre k-step, if < KT/4
                // The B-side fragments of k-step s + 1 are read while the
                // products of k-step s issue; the A side and the centre
                // operands are read in their own k-step (two waves per SIMD
                // leave no registers for a second A set).
                typename MW::afrag fa[2];
                typename MW::bfrag fb[2][5];
#pragma unroll
                for (int j = 0; j < 5; ++j) fb[0][j] = MW::load_b(bq + kr0 * ldq + 16 * (q0 + j), lane);
#pragma unroll
                for (int s = 0; s < KT / 4; ++s) {
                    const int kr = 4 * s + kr0;
#pragma unroll
                    for (int i = 0; i < 2; ++i) fa[i] = MW::load_a(bp + kr * ldp + 16 * (p0 + i), lane);
                    if (s + 1 < KT / 4) {
                        const int kn = kr + 4;
#pragma unroll
                        for (int j = 0; j < 5; ++j) fb[(s + 1) & 1][j] = MW::load_b(bq + kn * ldq + 16 * (q0 + j), lane);
                    }
                    rect_mma<T, MW, 2, 5>(acc, fa, fb[s & 1]);
                    if (cs == s) {
                        ca = M::load_a(bx + (4 * cs + kr0) * LDX + 64, lane);
                        cb = M::load_b(by + (4 * cs + kr0) * LDY + 64, lane);
                    }
                    if (cs == s) M::run(ca, cb, accc);
                }
            }
            pk.template store<(SL + 1) % SLOTS>(gstage + (buf ^ 1) * gsz, tt);
            __syncthreads();
        };
        typedef std::integral_constant<int, 0> S0;
        typedef std::integral_constant<int, 1> S1;
        auto pipeline = [&](auto reg) {
            constexpr int RG = decltype(reg)::value;
            fetch(0);
            pk.template load_with<0, RG>(pre_sk, pre_k, gbase, gspan, gk, 0, a.k, tt);
            pk.template store<0>(gstage, tt);
            if constexpr (SLOTS == 2) {
                fetch(nkb > 1 ? 1 : 0);
                pk.template load_with<1, RG>(pre_sk, pre_k, gbase, gspan, gk, nkb > 1 ? 1 : 0, a.k, tt);
            }
            fetch(nkb > SLOTS ? SLOTS : nkb - 1);
            __syncthreads();
            if constexpr (SLOTS == 2) {
                for (OffT kb = 0; kb < nkb; kb += 2) {
                    body(kb, S0(), reg);
                    body(kb + 1, S1(), reg);
                }
            } else {
                for (OffT kb = 0; kb < nkb; ++kb) body(kb, S0(), reg);
            }
        };
        if (nkb > 0) {
            const OffT ks = gx ? a.ksX : a.ksY;
            if (sizeof(OffT) == 4 && ks != 0) {
                pk.fix_offsets(ks, a.k, tt);
                pipeline(std::integral_constant<int, 2>());
            } else if (gx ? a.kregX : a.kregY) {
                pipeline(std::integral_constant<int, 1>());
            } else {
                pipeline(std::integral_constant<int, 0>());
            }
        }
        if (wide) rect_store<T, OffT, MW, 2, 5>(a, acc, m0, n0, fr0, fc0, lane);
        else rect_store_t<T, OffT, MW, 2, 5>(a, acc, m0, n0, fc0, fr0, lane);
        // centre fragment: partial sums of the eight waves added in wave order
#pragma unroll
        for (int r = 0; r < 4; ++r) smem[wave * 256 + r * 64 + lane] = accc[r];
        __syncthreads();
        if (wave == 0) {
            acc_t v;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                T x = smem[r * 64 + lane];
#pragma unroll
                for (int w = 1; w < 8; ++w) x += smem[w * 256 + r * 64 + lane];
                v[r] = x;
            }
            store_frag(a, (OffT)(m0 + 64), (OffT)(n0 + 64), v, lane);
        }
    }
};

// ---------------------------------------------------------------------------
// Split-BF16 mode (FP32 storage): every FP32 operand element x is split at
// pack time into hi = rn_bf16(x) and lo = rn_bf16(x - hi), and each 16x16
// fragment update over depth 32 is three bf16 matrix-core products
// lo*hi + hi*lo + hi*hi (the small terms first) accumulated in FP32.  The
// lo*lo term and the residual of the split (|x - hi - lo| <= 2^-16 |x|) are
// dropped, so the result carries a relative error of about 3 * 2^-16 per
// product plus FP32 accumulation; FP64 stays the path for ill-conditioned
// inputs.
// ---------------------------------------------------------------------------

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

// hi and lo halves of a pair (x0, x1) as packed bf16 words (x0 in the low
// half): hi = rn_bf16(x) by the hardware round-to-nearest-even conversion
// (one instruction for the pair), lo = rn_bf16(x - hi), where x - hi is exact;
// lo = 0 where x - hi is not finite (x NaN or infinite, or hi rounded up to
// infinity), so that no lo product turns a finite or infinite result into NaN.
__device__ __forceinline__ void split_pair(float x0, float x1, uint32_t& hi, uint32_t& lo) {
    const f32x2 x = {x0, x1};
    hi = __builtin_bit_cast(uint32_t, __builtin_convertvector(x, bf16x2));
    float r0 = x0 - __builtin_bit_cast(float, hi << 16);
    float r1 = x1 - __builtin_bit_cast(float, hi & 0xffff0000u);
    r0 = __builtin_isfinite(r0) ? r0 : 0.f;
    r1 = __builtin_isfinite(r1) ? r1 : 0.f;
    const f32x2 r = {r0, r1};
    lo = __builtin_bit_cast(uint32_t, __builtin_convertvector(r, bf16x2));
}

// Pack stage of one operand for the split mode: each thread gathers pairs of
// consecutive k of one row (the pair is one 32-bit LDS word per plane).
// Planes are row-major [R][KTP] bf16 (k contiguous), the order in which the
// bf16 matrix-core operands read 8 consecutive k per lane.
template <typename OffT, int R, int KT, int NTHR, bool LR, int SLOTS = 1>
struct PackPair {
    static constexpr int KP = KT / 2;
    static constexpr int EP = R * KP / NTHR;  // pairs per thread
    static constexpr int KTP = KT + 8;        // plane pitch in bf16 (16-byte multiple, spreads the banks)
    static constexpr int PLANE = R * KTP;     // bf16 elements of one plane
    static_assert((R * KP) % NTHR == 0, "stage must split evenly over threads");
    static __device__ __forceinline__ int ridx(int q) { return LR ? q % R : q / KP; }
    static __device__ __forceinline__ int pidx(int q) { return LR ? q / R : q % KP; }
    OffT o[EP];
    float r0[SLOTS][EP], r1[SLOTS][EP];  // stages in flight
    __device__ __forceinline__ void init(const OffT* rowvec, OffT r0_, OffT rmax, int t) {
#pragma unroll
        for (int i = 0; i < EP; ++i) {
            const OffT rr = r0_ + ridx(t + NTHR * i);
            const OffT x = rowvec[rr < rmax ? rr : rmax - 1];
            o[i] = rr < rmax ? x : OffT(-1);
        }
    }
    // REG = 1: every k block of this operand has a block stride (no per-k
    // offset reads compiled in); REG = -1: decided per block.
    template <int REG = -1, int SL = 0>
    __device__ __forceinline__ void load(const float* base, int64_t span, const OffT* kvec, const OffT* kbs, OffT kb,
                                         OffT K, int t) {
        const OffT k0 = kb * KT;
        const OffT sk = uniform(kbs[kb]);
        OffT kbase = 0;
        OffT ko0[EP], ko1[EP];
        if (REG == 1 || sk) {
            kbase = uniform(kvec[k0]);
#pragma unroll
            for (int i = 0; i < EP; ++i) {
                const OffT kk = 2 * pidx(t + NTHR * i);
                ko0[i] = kk * sk;
                ko1[i] = (kk + 1) * sk;
            }
        } else {
#pragma unroll
            for (int i = 0; i < EP; ++i) {
                const OffT kg = k0 + 2 * pidx(t + NTHR * i);
                ko0[i] = kvec[kg < K ? kg : K - 1];
                ko1[i] = kvec[kg + 1 < K ? kg + 1 : K - 1];
            }
        }
        if constexpr (sizeof(OffT) == 4) {
            const __amdgpu_buffer_rsrc_t rs = make_rsrc(base, span);
            const uint32_t soff = (uint32_t)uniform((int32_t)((uint32_t)kbase * 4u));
#pragma unroll
            for (int i = 0; i < EP; ++i) {
                const OffT kg = k0 + 2 * pidx(t + NTHR * i);
                const bool ok0 = o[i] >= 0 && kg < K, ok1 = o[i] >= 0 && kg + 1 < K;
                r0[SL][i] = buf_load<float>(rs, ok0 ? (uint32_t)(o[i] + ko0[i]) * 4u : kOutOfRange, soff);
                r1[SL][i] = buf_load<float>(rs, ok1 ? (uint32_t)(o[i] + ko1[i]) * 4u : kOutOfRange, soff);
            }
        } else {
#pragma unroll
            for (int i = 0; i < EP; ++i) {
                const OffT kg = k0 + 2 * pidx(t + NTHR * i);
                const bool ok0 = o[i] >= 0 && kg < K, ok1 = o[i] >= 0 && kg + 1 < K;
                const float x0 = base[ok0 ? kbase + o[i] + ko0[i] : OffT(0)];
                const float x1 = base[ok1 ? kbase + o[i] + ko1[i] : OffT(0)];
                r0[SL][i] = ok0 ? x0 : 0.f;
                r1[SL][i] = ok1 ? x1 : 0.f;
            }
        }
    }
    // hi plane at `hi`, lo plane at hi + PLANE (both as 32-bit words)
    template <int SL = 0>
    __device__ __forceinline__ void store(uint32_t* hi, int t) const {
        uint32_t* lo = hi + PLANE / 2;
#pragma unroll
        for (int i = 0; i < EP; ++i) {
            const int q = t + NTHR * i;
            uint32_t h, l;
            split_pair(r0[SL][i], r1[SL][i], h, l);
            const int w = (ridx(q) * KTP + 2 * pidx(q)) >> 1;
            hi[w] = h;
            lo[w] = l;
        }
    }
};

// Regular wave grid for the split mode (KT a multiple of 32).
template <typename OffT, int MT, int NT, int KT, int WM, int WN, bool XM, bool YN>
struct TileSplit {
    static constexpr int NTHR = WM * WN * 64;
    static constexpr int WTM = MT / WM, WTN = NT / WN;
    static constexpr int FM = WTM / 16, FN = WTN / 16;
    static_assert(KT % 32 == 0, "KT must be a multiple of the bf16 matrix-core depth");
    // gathered stages in flight in registers (measured: one for the 3 x 3
    // wave 144 tile, whose 576 threads leave 168 registers per thread)
    static constexpr int SLOTS = MT == 144 ? 1 : 2;
    typedef PackPair<OffT, MT, KT, NTHR, XM, SLOTS> PX;
    typedef PackPair<OffT, NT, KT, NTHR, YN, SLOTS> PY;
    // one stage: X hi, X lo, Y hi, Y lo planes (in bf16 elements)
    static constexpr int STAGE = 2 * PX::PLANE + 2 * PY::PLANE;
    static constexpr int SMEM = 2 * STAGE / 2;  // in floats (two stages of bf16 = STAGE floats)

    static __device__ __forceinline__ bf16x8 ld8(const __bf16* p) { return *(const bf16x8*)p; }

    static __device__ __forceinline__ void run(const KArgs<float, OffT>& a, int64_t tile, float* smemf) {
        typedef Mfma<float> M;
        __bf16* smem = (__bf16*)smemf;
        const int tid = threadIdx.x;
        const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
        const int wm = wave % WM, wn = wave / WM;
        const int64_t tm = tile % a.tiles_m, tn = tile / a.tiles_m;
        const OffT m0 = (OffT)(tm * MT), n0 = (OffT)(tn * NT);
        PX px;
        PY py;
        px.init(a.rX, m0, a.m, tid);
        py.init(a.cY, n0, a.n, tid);
        f32x4 acc[FM][FN];
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r) acc[i][j][r] = 0.f;
        auto xs = [&](int buf) { return smem + buf * STAGE; };
        auto ys = [&](int buf) { return smem + buf * STAGE + 2 * PX::PLANE; };
        const OffT nkb = (a.k + KT - 1) / KT;
        // Stage kb + SLOTS is gathered into register slot kb % SLOTS while
        // the matrix cores consume LDS stage kb, and stage kb + 1 (gathered
        // SLOTS - 1 stages earlier) is split into the other LDS buffer.  The
        // gathers and stores run with no branch around them: past the last
        // stage they re-read the last block into a buffer no stage reads.
        auto body = [&](OffT kb, auto slot, auto reg) {
            constexpr int SL = decltype(slot)::value;
            constexpr int RG = decltype(reg)::value;
            const int buf = (int)(kb & 1);
            const OffT lk = kb + SLOTS < nkb ? kb + SLOTS : nkb - 1;
            px.template load<RG, SL>(a.X, a.spanX, a.cX, a.kbsX, lk, a.k, tid);
            py.template load<RG, SL>(a.Y, a.spanY, a.rY, a.kbsY, lk, a.k, tid);
            if (kb < nkb) {
                const __bf16* xh = xs(buf) + (wm * WTM + (lane & 15)) * PX::KTP + 8 * (lane >> 4);
                const __bf16* yh = ys(buf) + (wn * WTN + (lane & 15)) * PY::KTP + 8 * (lane >> 4);
#pragma unroll
                for (int s = 0; s < KT / 32; ++s) {
                    bf16x8 ah[FM], al[FM], bh[FN], bl[FN];
#pragma unroll
                    for (int i = 0; i < FM; ++i) {
                        ah[i] = ld8(xh + 16 * i * PX::KTP + 32 * s);
                        al[i] = ld8(xh + PX::PLANE + 16 * i * PX::KTP + 32 * s);
                    }
#pragma unroll
                    for (int j = 0; j < FN; ++j) {
                        bh[j] = ld8(yh + 16 * j * PY::KTP + 32 * s);
                        bl[j] = ld8(yh + PY::PLANE + 16 * j * PY::KTP + 32 * s);
                    }
#pragma unroll
                    for (int i = 0; i < FM; ++i)
#pragma unroll
                        for (int j = 0; j < FN; ++j) {
                            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
                            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
                            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
                        }
                }
            }
            px.template store<(SL + 1) % SLOTS>((uint32_t*)xs(buf ^ 1), tid);
            py.template store<(SL + 1) % SLOTS>((uint32_t*)ys(buf ^ 1), tid);
            __syncthreads();
        };
        auto pipeline = [&](auto reg) {
            constexpr int RG = decltype(reg)::value;
            static_for<SLOTS>([&](auto ic) {
                constexpr int i = decltype(ic)::value;
                const OffT lk = nkb > i ? (OffT)i : nkb - 1;
                px.template load<RG, i>(a.X, a.spanX, a.cX, a.kbsX, lk, a.k, tid);
                py.template load<RG, i>(a.Y, a.spanY, a.rY, a.kbsY, lk, a.k, tid);
            });
            px.template store<0>((uint32_t*)xs(0), tid);
            py.template store<0>((uint32_t*)ys(0), tid);
            __syncthreads();
            for (OffT kb = 0; kb < nkb; kb += SLOTS)
                static_for<SLOTS>([&](auto ic) { body(kb + decltype(ic)::value, ic, reg); });
        };
        if (nkb > 0) {
            if (a.kregX && a.kregY) pipeline(std::integral_constant<int, 1>());
            else pipeline(std::integral_constant<int, -1>());
        }
        store_rect<float, OffT, M, FM, FN, false>(a, &acc[0][0], (OffT)(m0 + wm * WTM), (OffT)(n0 + wn * WTN), lane);
    }
};

// Pack stage of one operand for the warp-specialised split tile: a thread
// gathers quads of four consecutive k of one row (four loads in flight per
// quad), splits them into two hi and two lo words and writes each pair of
// words with one 64-bit LDS store.  Planes are [R][KTP] bf16 (k contiguous);
// a quad's element order follows the operand's lanes, as in PackRole.
template <typename OffT, int R, int KT, int NTHR, int KTP, int SLOTS>
struct PackQuad {
    static constexpr int KQ = KT / 4;         // quads per row
    static constexpr int EQ = R * KQ / NTHR;  // quads per thread
    static constexpr int PLANE = R * KTP;     // bf16 elements of one plane
    static_assert((R * KQ) % NTHR == 0, "stage must split evenly over threads");
    static_assert(KTP % 4 == 0, "64-bit LDS stores need an even word pitch");
    OffT o[EQ];  // row offsets, -1 past the edge
    float v[SLOTS][EQ][4];
    bool lr;  // lanes along the free index (else along k)
    __device__ __forceinline__ int ridx(int q) const { return lr ? q % R : q / KQ; }
    __device__ __forceinline__ int qidx(int q) const { return lr ? q / R : q % KQ; }
    __device__ __forceinline__ void init(const OffT* rowvec, OffT r0, OffT rmax, int t, bool lanes_row) {
        lr = lanes_row;
#pragma unroll
        for (int i = 0; i < EQ; ++i) {
            const OffT rr = r0 + ridx(t + NTHR * i);
            const OffT x = rowvec[rr < rmax ? rr : rmax - 1];
            o[i] = rr < rmax ? x : OffT(-1);
        }
    }
    // Gather of k block kb.  REG = 1: every k block has a block stride sk,
    // so k offsets are kk * sk from the block's first k offset (one scalar);
    // REG = 0: per-k offsets from the scatter vector.
    template <int SL, int REG>
    __device__ __forceinline__ void load_with(OffT sk, OffT kfirst, const float* base, int64_t span, const OffT* kvec,
                                              OffT kb, OffT K, int t) {
        const OffT k0 = kb * KT;
        if constexpr (sizeof(OffT) == 4) {
            const __amdgpu_buffer_rsrc_t rs = make_rsrc(base, span);
            const uint32_t soff = REG >= 1 ? (uint32_t)uniform((int32_t)((uint32_t)kfirst * 4u)) : 0u;
#pragma unroll
            for (int i = 0; i < EQ; ++i) {
                const OffT kq = 4 * (OffT)qidx(t + NTHR * i);
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const OffT kg = k0 + kq + j;
                    const bool ok = o[i] >= 0 && kg < K;
                    const OffT ko = REG >= 1 ? (kq + j) * sk : kvec[kg < K ? kg : K - 1];
                    v[SL][i][j] = buf_load<float>(rs, ok ? (uint32_t)(o[i] + ko) * 4u : kOutOfRange, soff);
                }
            }
        } else {
#pragma unroll
            for (int i = 0; i < EQ; ++i) {
                const OffT kq = 4 * (OffT)qidx(t + NTHR * i);
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const OffT kg = k0 + kq + j;
                    const bool ok = o[i] >= 0 && kg < K;
                    const OffT ko = REG >= 1 ? kfirst + (kq + j) * sk : kvec[kg < K ? kg : K - 1];
                    const float x = base[ok ? o[i] + ko : OffT(0)];
                    v[SL][i][j] = ok ? x : 0.f;
                }
            }
        }
    }
    // split and store: hi plane at `hi`, lo plane at hi + PLANE (as words)
    template <int SL>
    __device__ __forceinline__ void store(uint32_t* hi, int t) const {
        uint32_t* lo = hi + PLANE / 2;
#pragma unroll
        for (int i = 0; i < EQ; ++i) {
            const int q = t + NTHR * i;
            uint32_t h0, l0, h1, l1;
            split_pair(v[SL][i][0], v[SL][i][1], h0, l0);
            split_pair(v[SL][i][2], v[SL][i][3], h1, l1);
            const int w = (ridx(q) * KTP + 4 * qidx(q)) >> 1;
            typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
            *(u32x2*)(hi + w) = u32x2{h0, h1};
            *(u32x2*)(lo + w) = u32x2{l0, l1};
        }
    }
};

// Split mode on the pinwheel with specialised waves (MT = NT = 144, eight
// waves): waves 0-3 (one per SIMD) each own one whole 4x5 / 5x4 rectangle of
// the 9 x 9 fragment grid (a 5x4 one run as the 4x5 rectangle of C^T) and only
// read bf16 fragments from LDS and issue the three products per fragment;
// waves 4-7 gather, split and store both operands (4 and 5 the X sliver, 6
// and 7 the Y sliver), two stages in flight, and waves 4, 5 and 6 each run
// one of the three products of the centre fragment.  This keeps the split's
// vector work off the compute waves and gives every SIMD the same matrix work
// (the 3 x 3 wave grid puts three waves on one SIMD).
//
// PACKED: the operands were split once beforehand (split_pack_kernel) into
// panels of 16-byte chunks (unpadded rows of hi, then of lo), so the producer
// waves only copy each stage's two panels with 16-byte loads into the padded
// LDS rows; the compute side is the same, and so are the results, bit for
// bit.
template <typename OffT, int KT, bool XM, bool YN, bool PACKED = false>
struct TileSplitWS {
    static constexpr int MT = 144, NT = 144, NTHR = 512;
    static_assert(KT % 32 == 0, "KT must be a multiple of the bf16 matrix-core depth");
    static constexpr int KTP = KT + 8;  // plane pitch in bf16 (16-byte multiple)
    static constexpr int SLOTS = 2;     // gathered stages in flight per producer thread
    typedef PackQuad<OffT, 144, KT, 128, KTP, SLOTS> PQ;
    // a packed panel (one operand's 144 rows x KT of one k block): its hi
    // plane then its lo plane, rows of KT bf16, as CH 16-byte chunks; chunk
    // c is plane c / (144 CPR), row (c mod 144 CPR) / CPR, k-chunk c mod CPR
    static constexpr int CPR = KT / 8;
    static constexpr int CH = 2 * 144 * CPR;
    static constexpr int CPT = CH / 128;  // chunks per producer thread
    static_assert(CH % 128 == 0, "a panel splits evenly over two producer waves");
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    // LDS position (in bf16) of chunk c inside one operand's two planes
    static __device__ __forceinline__ int chunk_lds(int c) {
        const int pl = c / (144 * CPR), rem = c % (144 * CPR);
        return pl * PQ::PLANE + (rem / CPR) * KTP + 8 * (rem % CPR);
    }
    static constexpr int PLANE = PQ::PLANE;
    static constexpr int STAGE = 4 * PLANE;  // X hi, X lo, Y hi, Y lo (bf16 elements)
    static constexpr int SMEM = STAGE > 3 * 256 ? STAGE : 3 * 256;  // two stages, in floats

    static __device__ __forceinline__ bf16x8 ld8(const __bf16* p) { return *(const bf16x8*)p; }

    static __device__ __forceinline__ void run(const KArgs<float, OffT>& a, int64_t tile, float* smemf) {
        typedef Mfma<float> M;
        __bf16* smem = (__bf16*)smemf;
        const int tid = threadIdx.x;
        const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
        const int64_t tm = tile % a.tiles_m, tn = tile / a.tiles_m;
        const OffT m0 = (OffT)(tm * MT), n0 = (OffT)(tn * NT);
        const OffT nkb = (a.k + KT - 1) / KT;
        // operand planes of stage buffer b: X at [0, 2 PLANE), Y at [2 PLANE, 4 PLANE)
        auto xplane = [&](int b) { return smem + b * STAGE; };
        auto yplane = [&](int b) { return smem + b * STAGE + 2 * PLANE; };
        const int rl = lane & 15, kl = 8 * (lane >> 4);
        if (wave >= 4) {
            // ---- producer waves ----
            const bool gx = wave < 6;
            const int tt = tid & 127;
            const float* gbase = gx ? a.X : a.Y;
            const int64_t gspan = gx ? a.spanX : a.spanY;
            const OffT* gk = gx ? a.cX : a.rY;
            const OffT* gbs = gx ? a.kbsX : a.kbsY;
            PQ pk;
            if constexpr (!PACKED) {
                if (gx) pk.init(a.rX, m0, a.m, tt, XM);
                else pk.init(a.cY, n0, a.n, tt, YN);
            }
            f32x4 accc = {0.f, 0.f, 0.f, 0.f};
            OffT pre_sk = 0, pre_k = 0;
            auto fetch = [&](OffT kb) {
                if constexpr (!PACKED) {
                    pre_sk = uniform(gbs[kb]);
                    pre_k = uniform(gk[kb * KT]);
                }
            };
            // packed: this operand's panels of the tile's row (column) panel
            u32x4 cv[PACKED ? SLOTS : 1][PACKED ? CPT : 1];
            const u32x4* panels =
                PACKED ? (const u32x4*)a.packed + (gx ? tm : a.tiles_m + tn) * (int64_t)nkb * CH + tt : nullptr;
            auto load = [&](auto slot, auto reg, OffT kb) {
                constexpr int SL = decltype(slot)::value;
                constexpr int RG = decltype(reg)::value;
                if constexpr (PACKED) {
                    const u32x4* src = panels + (int64_t)kb * CH;
#pragma unroll
                    for (int i = 0; i < CPT; ++i) cv[SL][i] = src[128 * i];
                } else {
                    pk.template load_with<SL, RG>(pre_sk, pre_k, gbase, gspan, gk, kb, a.k, tt);
                }
            };
            auto store = [&](auto slot, __bf16* planes) {
                constexpr int SL = decltype(slot)::value;
                if constexpr (PACKED) {
#pragma unroll
                    for (int i = 0; i < CPT; ++i) *(u32x4*)(planes + chunk_lds(128 * i + tt)) = cv[SL][i];
                } else {
                    pk.template store<SL>((uint32_t*)planes, tt);
                }
            };
            auto body = [&](OffT kb, auto slot, auto reg) {
                constexpr int SL = decltype(slot)::value;
                constexpr int RG = decltype(reg)::value;
                const int buf = (int)(kb & 1);
                const OffT lk = kb + SLOTS < nkb ? kb + SLOTS : nkb - 1;
                load(slot, reg, lk);
                fetch(kb + SLOTS + 1 < nkb ? kb + SLOTS + 1 : nkb - 1);
                if (kb < nkb && wave < 7) {
                    // one of the centre fragment's three products: wave 4
                    // lo*hi, wave 5 hi*lo, wave 6 hi*hi
                    const __bf16* xc = xplane(buf) + (64 + rl) * KTP + kl;
                    const __bf16* yc = yplane(buf) + (64 + rl) * KTP + kl;
#pragma unroll
                    for (int s = 0; s < KT / 32; ++s) {
                        const bf16x8 ca = ld8(xc + (wave == 4 ? PLANE : 0) + 32 * s);
                        const bf16x8 cb = ld8(yc + (wave == 5 ? PLANE : 0) + 32 * s);
                        accc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ca, cb, accc, 0, 0, 0);
                    }
                }
                store(std::integral_constant<int, (SL + 1) % SLOTS>(), gx ? xplane(buf ^ 1) : yplane(buf ^ 1));
                __syncthreads();
            };
            auto pipeline = [&](auto reg) {
                static_for<SLOTS>([&](auto ic) {
                    constexpr int i = decltype(ic)::value;
                    fetch(nkb > i ? i : nkb - 1);
                    load(ic, reg, nkb > i ? (OffT)i : nkb - 1);
                });
                store(std::integral_constant<int, 0>(), gx ? xplane(0) : yplane(0));
                fetch(nkb > SLOTS ? SLOTS : nkb - 1);
                __syncthreads();
                for (OffT kb = 0; kb < nkb; kb += SLOTS)
                    static_for<SLOTS>([&](auto ic) { body(kb + decltype(ic)::value, ic, reg); });
            };
            if (nkb > 0) {
                if (PACKED || (gx ? a.kregX : a.kregY)) pipeline(std::integral_constant<int, 1>());
                else pipeline(std::integral_constant<int, 0>());
            }
            // centre fragment: the three products added in a fixed order
            if (wave < 7) {
#pragma unroll
                for (int r = 0; r < 4; ++r) smemf[(wave - 4) * 256 + r * 64 + lane] = accc[r];
            }
            __syncthreads();
            if (wave == 4) {
                f32x4 v;
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    v[r] = (smemf[r * 64 + lane] + smemf[256 + r * 64 + lane]) + smemf[512 + r * 64 + lane];
                store_frag<float, OffT>(a, (OffT)(m0 + 64), (OffT)(n0 + 64), v, lane);
            }
            return;
        }
        // ---- compute waves ----
        const int q = wave;
        const bool wide = (q & 1) == 0;
        const int fr0 = q == 0 ? 0 : q == 1 ? 0 : q == 2 ? 5 : 4;
        const int fc0 = q == 0 ? 0 : q == 1 ? 5 : q == 2 ? 4 : 0;
        const int p0 = wide ? fr0 : fc0, q0 = wide ? fc0 : fr0;
        f32x4 acc[20];
#pragma unroll
        for (int f = 0; f < 20; ++f) acc[f] = f32x4{0.f, 0.f, 0.f, 0.f};
        auto stage = [&](OffT kb) {
            const int buf = (int)(kb & 1);
            if (kb < nkb) {
                const __bf16* pp = (wide ? xplane(buf) : yplane(buf)) + (16 * p0 + rl) * KTP + kl;
                const __bf16* qp = (wide ? yplane(buf) : xplane(buf)) + (16 * q0 + rl) * KTP + kl;
#pragma unroll
                for (int s = 0; s < KT / 32; ++s) {
                    bf16x8 bh[5], bl[5];
#pragma unroll
                    for (int j = 0; j < 5; ++j) {
                        bh[j] = ld8(qp + 16 * j * KTP + 32 * s);
                        bl[j] = ld8(qp + PLANE + 16 * j * KTP + 32 * s);
                    }
                    // one A fragment row at a time, the next read over the
                    // current row's products
                    bf16x8 ah[2], al[2];
                    ah[0] = ld8(pp + 32 * s);
                    al[0] = ld8(pp + PLANE + 32 * s);
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        if (i + 1 < 4) {
                            ah[(i + 1) & 1] = ld8(pp + 16 * (i + 1) * KTP + 32 * s);
                            al[(i + 1) & 1] = ld8(pp + PLANE + 16 * (i + 1) * KTP + 32 * s);
                        }
#pragma unroll
                        for (int j = 0; j < 5; ++j) {
                            f32x4& c = acc[i * 5 + j];
                            c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i & 1], bh[j], c, 0, 0, 0);
                            c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i & 1], bl[j], c, 0, 0, 0);
                            c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i & 1], bh[j], c, 0, 0, 0);
                        }
                    }
                }
            }
            __syncthreads();
        };
        if (nkb > 0) {
            __syncthreads();  // the producers' first stage
            for (OffT kb = 0; kb < nkb; kb += SLOTS)
#pragma unroll
                for (int i = 0; i < SLOTS; ++i) stage(kb + i);
        }
        __syncthreads();  // the producers' centre reduction
        if (wide) rect_store<float, OffT, M, 4, 5>(a, acc, m0, n0, fr0, fc0, lane);
        else rect_store_t<float, OffT, M, 4, 5>(a, acc, m0, n0, fc0, fr0, lane);
    }
};

template <typename OffT, int MT, int NT, int KT, int WM, int WN, int LAYOUT, bool XM, bool YN>
struct SplitTileOf {
    typedef TileSplit<OffT, MT, NT, KT, WM, WN, XM, YN> type;
    static constexpr int threads = WM * WN * 64;
};
template <typename OffT, int MT, int NT, int KT, int WM, int WN, bool XM, bool YN>
struct SplitTileOf<OffT, MT, NT, KT, WM, WN, 2, XM, YN> {
    typedef TileSplitWS<OffT, KT, XM, YN> type;
    static constexpr int threads = 512;
};
template <typename OffT, int MT, int NT, int KT, int WM, int WN, bool XM, bool YN>
struct SplitTileOf<OffT, MT, NT, KT, WM, WN, 4, XM, YN> {
    typedef TileSplitWS<OffT, KT, XM, YN, true> type;
    static constexpr int threads = 512;
};

// Split-and-pack pass of the packed split tile: workgroup b packs panel b of
// X (b < tiles_m * nkb: row panel b / nkb, k block b mod nkb) or of Y (the
// rest, by column panel).  It gathers the panel's 144 x KT sliver through the
// offset vectors with the specialised-wave tile's own gather code, splits
// every element into hi and lo in LDS, and writes the panel out as 16-byte
// chunks in the order the tile's producer waves copy them.  Rows past m (n)
// and k past K are packed as zeros, as the tile itself would gather them.
template <typename OffT, int KT>
__global__ __launch_bounds__(128) void split_pack_kernel(KArgs<float, OffT> a, void* __restrict__ out) {
    typedef TileSplitWS<OffT, KT, true, true, true> W;
    typedef PackQuad<OffT, 144, KT, 128, W::KTP, 1> PQ;
    typedef typename W::u32x4 u32x4;
    __shared__ __align__(16) uint32_t planes[PQ::PLANE];  // hi and lo planes, PLANE bf16 each
    const int tid = threadIdx.x;
    const OffT nkb = (a.k + KT - 1) / KT;
    const int64_t b = blockIdx.x, nx = a.tiles_m * (int64_t)nkb;
    const bool gx = b < nx;
    const int64_t q = gx ? b : b - nx;
    const OffT r0 = (OffT)(q / nkb) * 144, kb = (OffT)(q % nkb);
    PQ pk;
    if (gx) pk.init(a.rX, r0, a.m, tid, a.xm != 0);
    else pk.init(a.cY, r0, a.n, tid, a.yn != 0);
    const float* base = gx ? a.X : a.Y;
    const int64_t span = gx ? a.spanX : a.spanY;
    const OffT* gk = gx ? a.cX : a.rY;
    const OffT sk = uniform((gx ? a.kbsX : a.kbsY)[kb]), kf = uniform(gk[kb * KT]);
    if (gx ? a.kregX : a.kregY) pk.template load_with<0, 1>(sk, kf, base, span, gk, kb, a.k, tid);
    else pk.template load_with<0, 0>(sk, kf, base, span, gk, kb, a.k, tid);
    pk.template store<0>(planes, tid);
    __syncthreads();
    const __bf16* lb = (const __bf16*)planes;
    u32x4* dst = (u32x4*)out + b * W::CH;
#pragma unroll
    for (int i = 0; i < W::CPT; ++i) {
        const int c = 128 * i + tid;
        dst[c] = *(const u32x4*)(lb + W::chunk_lds(c));
    }
}

template <typename OffT, int MT, int NT, int KT, int WM, int WN, int LAYOUT, bool XM, bool YN>
__global__ __launch_bounds__((SplitTileOf<OffT, MT, NT, KT, WM, WN, LAYOUT, XM, YN>::threads)) void split_kernel(
    KArgs<float, OffT> a) {
    typedef typename SplitTileOf<OffT, MT, NT, KT, WM, WN, LAYOUT, XM, YN>::type Tile;
    __shared__ float smem[Tile::SMEM];
    Tile::run(a, xcd_tile(blockIdx.x, a.tiles_m, a.tiles_n), smem);
}

template <typename OffT, int MT, int NT, int KT, int WM, int WN, int L>
static int launch_split_tile(const KArgs<float, OffT>& a, bool xm, bool yn, hipStream_t s) {
    const int64_t tiles = a.tiles_m * a.tiles_n;
    if (tiles <= 0) return TC_OK;
    if (tiles > 0x7fffffffLL) {
        set_error("too many tiles for one launch");
        return TC_ERR_ARG;
    }
    dim3 grid((unsigned)tiles), block(SplitTileOf<OffT, MT, NT, KT, WM, WN, L, true, true>::threads);
    if constexpr (L == 4) {
        // the split-and-pack pass, then the tile on the packed panels (the
        // lane directions matter only to the pass)
        static_assert(MT == 144 && NT == 144, "the packed split tile is the 144 x 144 pinwheel");
        if (!a.packed) {
            set_error("the packed split tile needs its workspace");
            return TC_ERR_ARG;
        }
        const int64_t panels = (a.tiles_m + a.tiles_n) * (int64_t)((a.k + KT - 1) / KT);
        if (panels > 0x7fffffffLL) {
            set_error("too many panels for one pack launch");
            return TC_ERR_ARG;
        }
        hipLaunchKernelGGL((split_pack_kernel<OffT, KT>), dim3((unsigned)panels), dim3(128), 0, s, a,
                           (void*)a.packed);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(e, "kernel launch");
        hipLaunchKernelGGL((split_kernel<OffT, MT, NT, KT, WM, WN, L, true, true>), grid, block, 0, s, a);
        e = hipGetLastError();
        return e == hipSuccess ? TC_OK : hip_fail(e, "kernel launch");
    } else {
        if (xm && yn) hipLaunchKernelGGL((split_kernel<OffT, MT, NT, KT, WM, WN, L, true, true>), grid, block, 0, s, a);
        else if (xm) hipLaunchKernelGGL((split_kernel<OffT, MT, NT, KT, WM, WN, L, true, false>), grid, block, 0, s, a);
        else if (yn) hipLaunchKernelGGL((split_kernel<OffT, MT, NT, KT, WM, WN, L, false, true>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((split_kernel<OffT, MT, NT, KT, WM, WN, L, false, false>), grid, block, 0, s, a);
        hipError_t e = hipGetLastError();
        return e == hipSuccess ? TC_OK : hip_fail(e, "kernel launch");
    }
}

template <typename T, typename OffT, int MT, int NT, int KT, int WM, int WN, int LAYOUT, bool XM, bool YN>
struct TileOf {
    typedef TileRegular<T, OffT, MT, NT, KT, WM, WN, XM, YN> type;
    static constexpr int threads = WM * WN * 64;
};
// Pinwheel with specialised waves: waves 0-3 (one per SIMD) each own one
// whole 4x5 / 5x4 rectangle of the pinwheel (a 5x4 one run as the 4x5
// rectangle of C^T) plus one k-step of the centre fragment per stage, and only
// read LDS and issue matrix instructions; waves 4-7 (one per SIMD) do every
// gather (4 and 5 the X sliver, 6 and 7 the Y sliver) and the LDS stores, so
// the compute waves never wait on vector-memory gathers.
template <typename T, typename OffT, int KT, bool XM, bool YN>
struct TilePinwheelWS {
    static constexpr int MT = 144, NT = 144, NTHR = 512;
    static_assert(KT % 16 == 0, "the centre's k-steps split evenly over the four producer waves");
    // gathered stages in flight per producer thread (three measured best for
    // FP64; FP32's larger stages leave registers for one)
    static constexpr int SLOTS = sizeof(T) == 8 ? 3 : 1;
    typedef PackRole<T, OffT, 144, KT, 128, SLOTS> PR;
    static constexpr int LDX = Pitch<MT, XM>::value, LDY = Pitch<NT, YN>::value;
    static constexpr int XS = KT * LDX, YS = KT * LDY;
    static constexpr int ELEMS = 2 * (XS + YS);
    static constexpr int SMEM = ELEMS > 4 * 256 ? ELEMS : 4 * 256;
    typedef typename MfmaFor<T, true>::type MW;

    static __device__ __forceinline__ void run(const KArgs<T, OffT>& a, int64_t tile, T* smem) {
        typedef Mfma<T> M;
        typedef typename M::acc_t acc_t;
        const int tid = threadIdx.x;
        const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
        const int64_t tm = tile % a.tiles_m, tn = tile / a.tiles_m;
        const OffT m0 = (OffT)(tm * MT), n0 = (OffT)(tn * NT);
        const OffT nkb = (a.k + KT - 1) / KT;
        if (wave >= 4) {
            // ---- producer waves ----
            const bool gx = wave < 6;
            const int tt = tid & 127;
            const T* gbase = gx ? a.X : a.Y;
            const int64_t gspan = gx ? a.spanX : a.spanY;
            const OffT* gk = gx ? a.cX : a.rY;
            const OffT* gbs = gx ? a.kbsX : a.kbsY;
            T* gstage = gx ? smem : smem + 2 * XS;
            const int gsz = gx ? XS : YS;
            PR pk;
            if (gx) pk.init(a.rX, m0, a.m, tt, a.xm != 0, LDX);
            else pk.init(a.cY, n0, a.n, tt, a.yn != 0, LDY);
            // the centre fragment: producer wave w does k-steps w - 4, w, ...
            // of every stage
            acc_t accc;
#pragma unroll
            for (int r = 0; r < 4; ++r) accc[r] = T(0);
            const int kc = 4 * (wave - 4) + (lane >> 4);
            OffT pre_sk = 0, pre_k = 0;
            auto fetch = [&](OffT kb) {
                pre_sk = uniform(gbs[kb]);
                pre_k = uniform(gk[kb * KT]);
            };
            auto body = [&](OffT kb, auto slot, auto reg) {
                constexpr int SL = decltype(slot)::value;
                constexpr int RG = decltype(reg)::value;
                const int buf = (int)(kb & 1);
                const OffT lk = kb + SLOTS < nkb ? kb + SLOTS : nkb - 1;
                pk.template load_with<SL, RG>(pre_sk, pre_k, gbase, gspan, gk, lk, a.k, tt);
                fetch(kb + SLOTS + 1 < nkb ? kb + SLOTS + 1 : nkb - 1);
                if (kb < nkb) {
#pragma unroll
                    for (int c = 0; c < KT / 16; ++c) {
                        const int kk = kc + 16 * c;
                        const typename M::afrag ca = M::load_a(smem + buf * XS + kk * LDX + 64, lane);
                        const typename M::bfrag cb = M::load_b(smem + 2 * XS + buf * YS + kk * LDY + 64, lane);
                        M::run(ca, cb, accc);
                    }
                }
                pk.template store<(SL + 1) % SLOTS>(gstage + (buf ^ 1) * gsz, tt);
                __syncthreads();
            };
            auto pipeline = [&](auto reg) {
                constexpr int RG = decltype(reg)::value;
                fetch(0);
                pk.template load_with<0, RG>(pre_sk, pre_k, gbase, gspan, gk, 0, a.k, tt);
                pk.template store<0>(gstage, tt);
                static_for<SLOTS - 1>([&](auto ic) {
                    constexpr int i = decltype(ic)::value + 1;
                    fetch(nkb > i ? i : nkb - 1);
                    pk.template load_with<i, RG>(pre_sk, pre_k, gbase, gspan, gk, nkb > i ? i : nkb - 1, a.k, tt);
                });
                fetch(nkb > SLOTS ? SLOTS : nkb - 1);
                __syncthreads();
                for (OffT kb = 0; kb < nkb; kb += SLOTS)
                    static_for<SLOTS>([&](auto ic) { body(kb + decltype(ic)::value, ic, reg); });
            };
            if (nkb > 0) {
                const OffT ks = gx ? a.ksX : a.ksY;
                if (sizeof(OffT) == 4 && ks != 0) {
                    pk.fix_offsets(ks, a.k, tt);
                    pipeline(std::integral_constant<int, 2>());
                } else if (gx ? a.kregX : a.kregY) {
                    pipeline(std::integral_constant<int, 1>());
                } else {
                    pipeline(std::integral_constant<int, 0>());
                }
            }
            // centre fragment: partial sums of the four producer waves added
            // in wave order (the stage buffers are free after the last stage)
#pragma unroll
            for (int r = 0; r < 4; ++r) smem[(wave - 4) * 256 + r * 64 + lane] = accc[r];
            __syncthreads();
            if (wave == 4) {
                acc_t v;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    T x = smem[r * 64 + lane];
#pragma unroll
                    for (int w = 1; w < 4; ++w) x += smem[w * 256 + r * 64 + lane];
                    v[r] = x;
                }
                store_frag(a, (OffT)(m0 + 64), (OffT)(n0 + 64), v, lane);
            }
            return;
        }
        // ---- compute waves ----
        const int q = wave;
        const bool wide = (q & 1) == 0;
        const int fr0 = q == 0 ? 0 : q == 1 ? 0 : q == 2 ? 5 : 4;
        const int fc0 = q == 0 ? 0 : q == 1 ? 5 : q == 2 ? 4 : 0;
        const int p0 = wide ? fr0 : fc0, q0 = wide ? fc0 : fr0;
        const int ldp = wide ? LDX : LDY, ldq = wide ? LDY : LDX;
        acc_t acc[20];
#pragma unroll
        for (int f = 0; f < 20; ++f)
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[f][r] = T(0);
        const int kr0 = lane >> 4;
        auto stage = [&](OffT kb) {
            const int buf = (int)(kb & 1);
            if (kb < nkb) {
                const T* bx = smem + buf * XS;
                const T* by = smem + 2 * XS + buf * YS;
                const T* bp = wide ? bx : by;
                const T* bq = wide ? by : bx;
                typename MW::bfrag fb[5];
#pragma unroll
                for (int s = 0; s < KT / 4; ++s) {
                    const int kr = 4 * s + kr0;
#pragma unroll
                    for (int j = 0; j < 5; ++j) fb[j] = MW::load_b(bq + kr * ldq + 16 * (q0 + j), lane);
                    // one A fragment row at a time, the next one read over
                    // the current row's products
                    typename MW::afrag fa[2];
                    fa[0] = MW::load_a(bp + kr * ldp + 16 * p0, lane);
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        if (i + 1 < 4) fa[(i + 1) & 1] = MW::load_a(bp + kr * ldp + 16 * (p0 + i + 1), lane);
#pragma unroll
                        for (int j = 0; j < 5; ++j) MW::run(fa[i & 1], fb[j], acc[i * 5 + j]);
                    }
                }
            }
            __syncthreads();
        };
        if (nkb > 0) {
            __syncthreads();  // the producers' first stage
            for (OffT kb = 0; kb < nkb; kb += SLOTS)
#pragma unroll
                for (int i = 0; i < SLOTS; ++i) stage(kb + i);
        }
        __syncthreads();  // the producers' centre reduction
        if (wide) rect_store<T, OffT, MW, 4, 5>(a, acc, m0, n0, fr0, fc0, lane);
        else rect_store_t<T, OffT, MW, 4, 5>(a, acc, m0, n0, fc0, fr0, lane);
    }
};

template <typename T, typename OffT, int MT, int NT, int KT, int WM, int WN, bool XM, bool YN>
struct TileOf<T, OffT, MT, NT, KT, WM, WN, 1, XM, YN> {
    typedef TilePinwheel8<T, OffT, KT, XM, YN> type;
    static constexpr int threads = 512;
};
template <typename T, typename OffT, int MT, int NT, int KT, int WM, int WN, bool XM, bool YN>
struct TileOf<T, OffT, MT, NT, KT, WM, WN, 2, XM, YN> {
    typedef TilePinwheelWS<T, OffT, KT, XM, YN> type;
    static constexpr int threads = 512;
};

// Specialised waves on a regular tile (layout 3): waves 0-3 (one per SIMD)
// form a 2 x 2 grid, each owning an (MT/2) x (NT/2) block of fragments, and
// only read LDS and issue matrix instructions; waves 4-7 (one per SIMD) do
// every gather (4 and 5 the X sliver, 6 and 7 the Y sliver) and the LDS
// stores.  The tile edges are free, so the output grid can be matched to the
// 256 compute units (2048 x 2048 is exactly 256 tiles of 128 x 128, 2048 x
// 1024 exactly 256 of 128 x 64), where the 144 pinwheel leaves CUs idle.
template <typename T, typename OffT, int MT, int NT, int KT, bool XM, bool YN>
struct TileWSGrid {
    static constexpr int NTHR = 512;
    static constexpr int FM = MT / 32, FN = NT / 32;  // fragments per compute wave
    static_assert(MT % 32 == 0 && NT % 32 == 0, "each compute wave owns whole 16 x 16 fragments");
    static_assert(KT % 4 == 0, "KT must be a multiple of the MFMA depth");
    // gathered stages in flight per producer thread, about within the 63
    // loads the memory counter tracks (two stages of 32 loads, one past it,
    // measured faster for the FP32 128 x 64 tile with 32-bit offsets; the
    // 128 x 128 FP32 tile and 64-bit offsets spill registers with two)
    static constexpr int EMAX = (MT > NT ? MT : NT) * KT / 128;
    static constexpr int SLOTS = 3 * EMAX <= 63                                                   ? 3
                                 : (2 * EMAX <= 64 && MT * NT <= 128 * 64 && sizeof(OffT) == 4) ? 2
                                                                                                 : 1;
    typedef PackRole<T, OffT, MT, KT, 128, SLOTS> PRX;
    typedef PackRole<T, OffT, NT, KT, 128, SLOTS> PRY;
    static constexpr int LDX = Pitch<MT, XM>::value, LDY = Pitch<NT, YN>::value;
    static constexpr int XS = KT * LDX, YS = KT * LDY;
    static constexpr int SMEM = 2 * (XS + YS);
    typedef typename MfmaFor<T, (FN >= FM)>::type MW;

    static __device__ __forceinline__ void run(const KArgs<T, OffT>& a, int64_t tile, T* smem) {
        const int tid = threadIdx.x;
        const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
        const int64_t tm = tile % a.tiles_m, tn = tile / a.tiles_m;
        const OffT m0 = (OffT)(tm * MT), n0 = (OffT)(tn * NT);
        const OffT nkb = (a.k + KT - 1) / KT;
        if (wave >= 4) {
            // ---- producer waves ----
            const bool gx = wave < 6;
            const int tt = tid & 127;
            auto produce = [&](auto& pk, const T* gbase, int64_t gspan, const OffT* gk, const OffT* gbs, T* gstage,
                               int gsz, OffT ks, int kreg) {
                OffT pre_sk = 0, pre_k = 0;
                auto fetch = [&](OffT kb) {
                    pre_sk = uniform(gbs[kb]);
                    pre_k = uniform(gk[kb * KT]);
                };
                auto body = [&](OffT kb, auto slot, auto reg) {
                    constexpr int SL = decltype(slot)::value;
                    constexpr int RG = decltype(reg)::value;
                    const int buf = (int)(kb & 1);
                    const OffT lk = kb + SLOTS < nkb ? kb + SLOTS : nkb - 1;
                    pk.template load_with<SL, RG>(pre_sk, pre_k, gbase, gspan, gk, lk, a.k, tt);
                    fetch(kb + SLOTS + 1 < nkb ? kb + SLOTS + 1 : nkb - 1);
                    pk.template store<(SL + 1) % SLOTS>(gstage + (buf ^ 1) * gsz, tt);
                    __syncthreads();
                };
                auto pipeline = [&](auto reg) {
                    constexpr int RG = decltype(reg)::value;
                    fetch(0);
                    pk.template load_with<0, RG>(pre_sk, pre_k, gbase, gspan, gk, 0, a.k, tt);
                    pk.template store<0>(gstage, tt);
                    static_for<SLOTS - 1>([&](auto ic) {
                        constexpr int i = decltype(ic)::value + 1;
                        fetch(nkb > i ? i : nkb - 1);
                        pk.template load_with<i, RG>(pre_sk, pre_k, gbase, gspan, gk, nkb > i ? i : nkb - 1, a.k, tt);
                    });
                    fetch(nkb > SLOTS ? SLOTS : nkb - 1);
                    __syncthreads();
                    for (OffT kb = 0; kb < nkb; kb += SLOTS)
                        static_for<SLOTS>([&](auto ic) { body(kb + decltype(ic)::value, ic, reg); });
                };
                if (nkb > 0) {
                    if (sizeof(OffT) == 4 && ks != 0) {
                        pk.fix_offsets(ks, a.k, tt);
                        pipeline(std::integral_constant<int, 2>());
                    } else if (kreg) {
                        pipeline(std::integral_constant<int, 1>());
                    } else {
                        pipeline(std::integral_constant<int, 0>());
                    }
                }
            };
            if (gx) {
                PRX pk;
                pk.init(a.rX, m0, a.m, tt, a.xm != 0, LDX);
                produce(pk, a.X, a.spanX, a.cX, a.kbsX, smem, XS, a.ksX, a.kregX);
            } else {
                PRY pk;
                pk.init(a.cY, n0, a.n, tt, a.yn != 0, LDY);
                produce(pk, a.Y, a.spanY, a.rY, a.kbsY, smem + 2 * XS, YS, a.ksY, a.kregY);
            }
            return;
        }
        // ---- compute waves ----
        typedef typename MW::acc_t acc_t;
        const int wm = wave & 1, wn = wave >> 1;
        acc_t acc[FM * FN];
#pragma unroll
        for (int f = 0; f < FM * FN; ++f)
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[f][r] = T(0);
        const int kr0 = lane >> 4;
        auto stage = [&](OffT kb) {
            const int buf = (int)(kb & 1);
            if (kb < nkb) {
                const T* bx = smem + buf * XS + 16 * FM * wm;
                const T* by = smem + 2 * XS + buf * YS + 16 * FN * wn;
                typename MW::bfrag fb[FN];
#pragma unroll
                for (int s = 0; s < KT / 4; ++s) {
                    const int kr = 4 * s + kr0;
#pragma unroll
                    for (int j = 0; j < FN; ++j) fb[j] = MW::load_b(by + kr * LDY + 16 * j, lane);
                    // one A fragment row at a time, the next one read over
                    // the current row's products
                    typename MW::afrag fa[2];
                    fa[0] = MW::load_a(bx + kr * LDX, lane);
#pragma unroll
                    for (int i = 0; i < FM; ++i) {
                        if (i + 1 < FM) fa[(i + 1) & 1] = MW::load_a(bx + kr * LDX + 16 * (i + 1), lane);
#pragma unroll
                        for (int j = 0; j < FN; ++j) MW::run(fa[i & 1], fb[j], acc[i * FN + j]);
                    }
                }
            }
            __syncthreads();
        };
        if (nkb > 0) {
            __syncthreads();  // the producers' first stage
            for (OffT kb = 0; kb < nkb; kb += SLOTS)
#pragma unroll
                for (int i = 0; i < SLOTS; ++i) stage(kb + i);
        }
        store_rect<T, OffT, MW, FM, FN, false>(a, acc, (OffT)(m0 + 16 * FM * wm), (OffT)(n0 + 16 * FN * wn), lane);
    }
};

template <typename T, typename OffT, int MT, int NT, int KT, int WM, int WN, bool XM, bool YN>
struct TileOf<T, OffT, MT, NT, KT, WM, WN, 3, XM, YN> {
    typedef TileWSGrid<T, OffT, MT, NT, KT, XM, YN> type;
    static constexpr int threads = 512;
};

template <typename T, typename OffT, int MT, int NT, int KT, int WM, int WN, int LAYOUT, bool XM, bool YN>
__global__ __launch_bounds__((TileOf<T, OffT, MT, NT, KT, WM, WN, LAYOUT, XM, YN>::threads)) void contract_kernel(
    KArgs<T, OffT> a) {
    typedef typename TileOf<T, OffT, MT, NT, KT, WM, WN, LAYOUT, XM, YN>::type Tile;
    __shared__ T smem[Tile::SMEM];
    Tile::run(a, xcd_tile(blockIdx.x, a.tiles_m, a.tiles_n), smem);
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

// The block stride shared by every k block, or 0 when they differ or one
// has none.
static inline int64_t common_stride(const std::vector<int64_t>& kbs) {
    if (kbs.empty() || kbs[0] == 0) return 0;
    for (int64_t v : kbs)
        if (v != kbs[0]) return 0;
    return kbs[0];
}

template <typename T, typename OffT>
static int launch_typed(const Plan& p, const DeviceVectors& dv, double alpha, const void* A, const void* B,
                        double beta, void* C, hipStream_t s, void* ws) {
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
    a.spanX = p.swapped ? p.spanB : p.spanA;
    a.spanY = p.swapped ? p.spanA : p.spanB;
    a.alpha = (T)alpha;
    a.beta = (T)beta;
    a.kregX = p.k_blocks_regular_x == (int64_t)p.kbsX.size();
    a.kregY = p.k_blocks_regular_y == (int64_t)p.kbsY.size();
    a.ksX = (OffT)common_stride(p.kbsX);
    a.ksY = (OffT)common_stride(p.kbsY);
    a.xm = p.x_lanes_m;
    a.yn = p.y_lanes_n;
    a.packed = ws;
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
    if constexpr (sizeof(T) == 4) {
        if (p.mode == TC_SPLIT_BF16X3) {
            // without a workspace the packed split tile runs as its twin that
            // splits in its own producer waves (the same bits)
            const int tile = !ws && split_unpacked_twin(p.tile) >= 0 ? split_unpacked_twin(p.tile) : p.tile;
#define TC_SCASE(id, MT, NT, KT, WM, WN, L) \
    case id:                                \
        return launch_split_tile<OffT, MT, NT, KT, WM, WN, L>(a, xm, yn, s);
            switch (tile) { TC_TILES_BF16X3(TC_SCASE) }
#undef TC_SCASE
            set_error("unknown tile configuration");
            return TC_ERR_ARG;
        }
    }
#define TC_CASE(id, MT, NT, KT, WM, WN, L) \
    case id:                               \
        return launch_tile<T, OffT, MT, NT, KT, WM, WN, L>(a, xm, yn, s);
    if constexpr (sizeof(T) == 8) {
        switch (p.tile) { TC_TILES_F64(TC_CASE) }
    } else {
        switch (p.tile) { TC_TILES_F32(TC_CASE) }
    }
#undef TC_CASE
    set_error("unknown tile configuration");
    return TC_ERR_ARG;
}

// Persistent batched kernel: workgroup g runs its own list of (problem,
// tile) work items, fixed on the host by a longest-processing-time-first
// assignment.  Every problem may have its own lane directions, so the four
// pack variants are dispatched per item.
template <typename T, typename OffT, int MT, int NT, int KT, int WM, int WN, int L>
__global__ __launch_bounds__((TileOf<T, OffT, MT, NT, KT, WM, WN, L, true, true>::threads)) void batch_kernel(
    const BatchItemDev* __restrict__ items, const int32_t* __restrict__ off, const int32_t* __restrict__ ent) {
    typedef typename TileOf<T, OffT, MT, NT, KT, WM, WN, L, true, true>::type TTT;
    typedef typename TileOf<T, OffT, MT, NT, KT, WM, WN, L, true, false>::type TTF;
    typedef typename TileOf<T, OffT, MT, NT, KT, WM, WN, L, false, true>::type TFT;
    typedef typename TileOf<T, OffT, MT, NT, KT, WM, WN, L, false, false>::type TFF;
    constexpr int S1 = TTT::SMEM > TTF::SMEM ? TTT::SMEM : TTF::SMEM;
    constexpr int S2 = TFT::SMEM > TFF::SMEM ? TFT::SMEM : TFF::SMEM;
    __shared__ T smem[S1 > S2 ? S1 : S2];
    const int32_t j0 = uniform(off[blockIdx.x]), j1 = uniform(off[blockIdx.x + 1]);
    for (int32_t j = j0; j < j1; ++j) {
        const BatchItemDev& it = items[uniform(ent[2 * j])];
        const int64_t tile = uniform(ent[2 * j + 1]);
        KArgs<T, OffT> a;
        a.X = (const T*)it.X;
        a.Y = (const T*)it.Y;
        a.C = (T*)it.C;
        a.rX = (const OffT*)it.rX;
        a.cX = (const OffT*)it.cX;
        a.rY = (const OffT*)it.rY;
        a.cY = (const OffT*)it.cY;
        a.rC = (const OffT*)it.rC;
        a.cC = (const OffT*)it.cC;
        a.kbsX = (const OffT*)it.kbsX;
        a.kbsY = (const OffT*)it.kbsY;
        a.m = (OffT)it.m;
        a.n = (OffT)it.n;
        a.k = (OffT)it.k;
        a.tiles_m = it.tiles_m;
        a.tiles_n = it.tiles_n;
        a.spanX = it.spanX;
        a.spanY = it.spanY;
        a.alpha = (T)it.alpha;
        a.beta = (T)it.beta;
        a.kregX = it.kregX;
        a.kregY = it.kregY;
        a.ksX = (OffT)it.ksX;
        a.ksY = (OffT)it.ksY;
        a.packed = nullptr;
        a.xm = it.x_lanes_m;
        a.yn = it.y_lanes_n;
        if (it.x_lanes_m) {
            if (it.y_lanes_n) TTT::run(a, tile, smem);
            else TTF::run(a, tile, smem);
        } else {
            if (it.y_lanes_n) TFT::run(a, tile, smem);
            else TFF::run(a, tile, smem);
        }
        __syncthreads();  // LDS is reused by the next item
    }
}

template <typename T, typename OffT, int MT, int NT, int KT, int WM, int WN, int L>
struct BatchLaunch {
    static constexpr int threads = TileOf<T, OffT, MT, NT, KT, WM, WN, L, true, true>::threads;
    static int launch(const BatchItemDev* items, const int32_t* off, const int32_t* ent, int grid, hipStream_t s) {
        if constexpr (L == 1) {
            set_error("batched launches use the regular and specialised-wave layouts");
            return TC_ERR_ARG;
        } else {
            hipLaunchKernelGGL((batch_kernel<T, OffT, MT, NT, KT, WM, WN, L>), dim3(grid), dim3(threads), 0, s,
                               items, off, ent);
            hipError_t e = hipGetLastError();
            return e == hipSuccess ? TC_OK : hip_fail(e, "batched kernel launch");
        }
    }
    static int grid(int64_t total) {
        if constexpr (L == 1) {
            return 0;
        } else {
            int dev = 0, cus = 0, per_cu = 0;
            if (hipGetDevice(&dev) != hipSuccess) return 0;
            if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
                    &per_cu, (const void*)batch_kernel<T, OffT, MT, NT, KT, WM, WN, L>, threads, 0) != hipSuccess)
                return 0;
            int64_t g = (int64_t)cus * (per_cu > 0 ? per_cu : 1);
            return (int)(total < g ? total : g);
        }
    }
};

template <typename T, typename OffT>
static int batch_dispatch(int dtype, int tile, bool launch, const BatchItemDev* items, const int32_t* off,
                          const int32_t* ent, int64_t total, int grid, hipStream_t s) {
#define TC_BCASE(id, MT, NT, KT, WM, WN, L)                                                            \
    case id:                                                                                           \
        return launch ? BatchLaunch<T, OffT, MT, NT, KT, WM, WN, L>::launch(items, off, ent, grid, s) \
                      : BatchLaunch<T, OffT, MT, NT, KT, WM, WN, L>::grid(total);
    (void)dtype;  // the storage type T fixes the tile table
    if constexpr (sizeof(T) == 8) {
        switch (tile) { TC_TILES_F64(TC_BCASE) }
    } else {
        switch (tile) { TC_TILES_F32(TC_BCASE) }
    }
#undef TC_BCASE
    set_error("unknown tile configuration");
    return launch ? TC_ERR_ARG : 0;
}

}  // namespace tc
