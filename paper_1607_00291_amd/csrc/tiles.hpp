// Compiled tile configurations.  One X-macro list per (dtype, mode) keeps the
// host-side table and the kernel instantiations in step.
//
// Columns: id, MT, NT, KT, WM, WN, LAYOUT
//   MT x NT  output tile of one workgroup, KT the k-depth of one LDS stage
//   WM x WN  grid of 64-lane waves; each wave owns (MT/WM) x (NT/WN) outputs
//   LAYOUT   0 = regular wave grid; 1 = "pinwheel" (MT = NT = 144, eight
//            waves): four 4x5 / 5x4 rectangles of 16x16 fragments around the
//            centre fragment of the 9x9 grid, each halved between two waves,
//            the centre's k-range split over the eight waves, so that every
//            SIMD does exactly 20.25 fragments of work and 2304^2 outputs
//            make exactly 256 tiles; 2 = the same pinwheel with specialised
//            waves: four compute waves own one whole rectangle each, four
//            producer waves gather both operands and do the centre; 3 = the
//            specialised waves on a regular tile (a 2 x 2 grid of compute
//            waves, four producer waves); 4 (split mode) = layout 2 on
//            operands split once into packed hi/lo panels by a separate pass,
//            the producer waves only copying them (needs a workspace)
#pragma once

#include <cstdint>

#define TC_TILES_F64(X)            \
    X(0, 32, 32, 16, 1, 1, 0)      \
    X(1, 64, 64, 16, 2, 2, 0)      \
    X(2, 128, 64, 16, 2, 2, 0)     \
    X(3, 128, 128, 16, 2, 2, 0)    \
    X(4, 144, 144, 16, 1, 1, 1)    \
    X(5, 144, 144, 16, 1, 1, 2)    \
    X(6, 128, 128, 16, 2, 2, 3)    \
    X(7, 128, 64, 16, 2, 2, 3)     \
    X(8, 32, 32, 16, 2, 2, 0)

#define TC_TILES_F32(X)            \
    X(0, 32, 32, 32, 1, 1, 0)      \
    X(1, 64, 64, 32, 2, 2, 0)      \
    X(2, 128, 64, 32, 2, 2, 0)     \
    X(3, 128, 128, 32, 2, 2, 0)    \
    X(4, 144, 144, 32, 1, 1, 1)    \
    X(5, 144, 144, 32, 1, 1, 2)    \
    X(6, 128, 128, 32, 2, 2, 3)    \
    X(7, 128, 64, 32, 2, 2, 3)     \
    X(8, 32, 32, 32, 2, 2, 0)

// split-bf16: KT is a multiple of the bf16 MFMA depth (32)
#define TC_TILES_BF16X3(X)         \
    X(0, 32, 32, 32, 1, 1, 0)      \
    X(1, 64, 64, 32, 2, 2, 0)      \
    X(2, 128, 64, 32, 2, 2, 0)     \
    X(3, 128, 128, 32, 2, 2, 0)    \
    X(4, 144, 144, 32, 3, 3, 0)    \
    X(5, 144, 144, 32, 1, 1, 2)    \
    X(6, 144, 144, 32, 1, 1, 4)

namespace tc {

struct TileCfg {
    int MT, NT, KT, WM, WN, layout;
    int waves() const { return layout != 0 ? 8 : WM * WN; }
};

#define TC_TILE_ENTRY(id, MT, NT, KT, WM, WN, L) TileCfg{MT, NT, KT, WM, WN, L},
static const TileCfg kTilesF64[] = {TC_TILES_F64(TC_TILE_ENTRY)};
static const TileCfg kTilesF32[] = {TC_TILES_F32(TC_TILE_ENTRY)};
static const TileCfg kTilesBF16x3[] = {TC_TILES_BF16X3(TC_TILE_ENTRY)};
#undef TC_TILE_ENTRY

// Measured throughput of each tile configuration on MI355X (TFLOP/s, dense
// column-major contractions of shapes 4096^2 x 1024, 2304^3, 2048^2 x 1024,
// 2048 x 1024 x 2048 and 1024^2 x 4096): r1 with one workgroup per compute
// unit, r2 with two or more resident, occ the workgroups that fit on one
// compute unit at once, and
// store the relative speed of the tile's C update (0.7 where only four of the
// eight waves store: the output-store-bound rank-k shapes run about that much
// slower on it).  The rates are fitted, together with the cost model's
// cache bandwidth (choose_tile), to the measured times of every tile on
// those five shapes and on six small ones (256^3 to 1024^2 x 256), so that
// the model picks the fastest measured tile on all eleven for both dtypes;
// they are within a few percent of the measured throughputs, which the
// fit trades against the model's simple terms.
struct TileRate {
    double r1, r2;
    int occ;
    double store;
};
static const TileRate kRatesF64[] = {{31, 31, 2, 1},     {25, 46, 2, 1},       {35, 52, 2, 1},     {40.6, 40.6, 1, 1},
                                     {51.4, 51.4, 1, 1}, {59.5, 59.5, 1, 0.7}, {56, 56, 1, 0.7}, {50, 52, 2, 0.7},
                                     {34, 30, 1, 1}};
static const TileRate kRatesF32[] = {{50, 57, 2, 1}, {41, 88, 2, 1},       {55, 84, 2, 1},   {68, 94, 2, 1},
                                     {94, 94, 1, 1}, {108.5, 108.5, 1, 0.7}, {83, 85, 2, 0.7}, {90, 90, 1, 0.7},
                                     {54, 60, 2, 1}};
// Split-BF16 rates count FP32-equivalent flops (one update = three bf16
// products).  The packed split tile's rate is its tile alone on 2304^3
// (72.2 us per 24.46 GFLOP); choose_tile adds its split-and-pack pass.  With
// the 32 x 32 and 64 x 64 rates the model picks the fastest measured split
// tile on 1024^3 to 2048^3, 4096^2 x 1024 and 1024^2 x 8192 (512^3: a tile
// within 15% of the fastest).
static const TileRate kRatesBF16x3[] = {{45, 40, 2, 1},   {57, 105, 2, 1},   {59, 104, 2, 1},   {76, 145, 2, 1},
                                        {144, 144, 1, 1}, {140, 140, 1, 0.7}, {340, 340, 1, 0.7}};
static_assert(sizeof(kRatesF64) / sizeof(TileRate) == sizeof(kTilesF64) / sizeof(TileCfg), "one rate per tile");
static_assert(sizeof(kRatesF32) / sizeof(TileRate) == sizeof(kTilesF32) / sizeof(TileCfg), "one rate per tile");
static_assert(sizeof(kRatesBF16x3) / sizeof(TileRate) == sizeof(kTilesBF16x3) / sizeof(TileCfg), "one rate per tile");

inline int tile_count(int dtype, int mode) {
    if (dtype == 0 && mode == 0) return (int)(sizeof(kTilesF64) / sizeof(TileCfg));
    if (dtype == 1 && mode == 0) return (int)(sizeof(kTilesF32) / sizeof(TileCfg));
    if (dtype == 1 && mode == 1) return (int)(sizeof(kTilesBF16x3) / sizeof(TileCfg));
    return 0;
}

inline const TileCfg* tile_table(int dtype, int mode) {
    if (dtype == 0 && mode == 0) return kTilesF64;
    if (dtype == 1 && mode == 0) return kTilesF32;
    if (dtype == 1 && mode == 1) return kTilesBF16x3;
    return nullptr;
}

// The specialised-wave split tile that gathers and splits in its own
// producer waves and has the same tile sizes as packed split tile `tile`
// (their results are the same bits); -1 if there is none.
inline int split_unpacked_twin(int tile) {
    const int n = (int)(sizeof(kTilesBF16x3) / sizeof(TileCfg));
    if (tile < 0 || tile >= n || kTilesBF16x3[tile].layout != 4) return -1;
    const TileCfg& t = kTilesBF16x3[tile];
    for (int i = 0; i < n; ++i)
        if (kTilesBF16x3[i].layout == 2 && kTilesBF16x3[i].MT == t.MT && kTilesBF16x3[i].NT == t.NT &&
            kTilesBF16x3[i].KT == t.KT)
            return i;
    return -1;
}

// Bytes of the packed split panels of X and Y for m x n x k on packed split
// tile t: one panel of 2 planes x MT (NT) rows x KT bf16 per row (column)
// panel and k block.
inline int64_t split_pack_bytes(const TileCfg& t, int64_t m, int64_t n, int64_t k) {
    const int64_t nkb = (k + t.KT - 1) / t.KT;
    return (((m + t.MT - 1) / t.MT) * t.MT + ((n + t.NT - 1) / t.NT) * t.NT) * nkb * t.KT * 4;
}
// The cost model leaves the packed split tile out above this many bytes of
// panels (the in-kernel split needs no workspace).
static constexpr int64_t kMaxSplitPanelBytes = int64_t(8) << 30;

inline const TileRate* rate_table(int dtype, int mode) {
    if (dtype == 0 && mode == 0) return kRatesF64;
    if (dtype == 1 && mode == 0) return kRatesF32;
    if (dtype == 1 && mode == 1) return kRatesBF16x3;
    return nullptr;
}

}  // namespace tc
