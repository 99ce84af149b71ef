// Compiled tile configurations.  One X-macro list per (dtype, mode) keeps the
// host-side table and the kernel instantiations in step.
//
// Columns: id, MT, NT, KT, WM, WN, LAYOUT
//   MT x NT  output tile of one workgroup, KT the k-depth of one LDS stage
//   WM x WN  grid of 64-lane waves; each wave owns (MT/WM) x (NT/WN) outputs
//   LAYOUT   0 = regular wave grid; 1 = "pinwheel": 4 waves on a 9x9 grid of
//            16x16 fragments, four 4x5 / 5x4 rectangles around the centre
//            fragment whose k-range is split over the 4 waves, so that every
//            SIMD does exactly 20.25 fragments of work; 2 = the same on 8
//            waves (two per SIMD), each owning half a rectangle
#pragma once

#define TC_TILES_F64(X)            \
    X(0, 32, 32, 16, 1, 1, 0)      \
    X(1, 64, 64, 16, 2, 2, 0)      \
    X(2, 128, 64, 16, 2, 2, 0)     \
    X(3, 128, 128, 16, 2, 2, 0)    \
    X(4, 144, 144, 16, 1, 1, 1)    \
    X(5, 144, 144, 16, 1, 1, 2)

#define TC_TILES_F32(X)            \
    X(0, 32, 32, 32, 1, 1, 0)      \
    X(1, 64, 64, 32, 2, 2, 0)      \
    X(2, 128, 64, 32, 2, 2, 0)     \
    X(3, 128, 128, 32, 2, 2, 0)    \
    X(4, 144, 144, 32, 1, 1, 1)    \
    X(5, 144, 144, 32, 1, 1, 2)

// split-bf16: KT is a multiple of the bf16 MFMA depth (32)
#define TC_TILES_BF16X3(X)         \
    X(0, 32, 32, 32, 1, 1, 0)      \
    X(1, 64, 64, 32, 2, 2, 0)      \
    X(2, 128, 64, 32, 2, 2, 0)     \
    X(3, 128, 128, 32, 2, 2, 0)

namespace tc {

struct TileCfg {
    int MT, NT, KT, WM, WN, layout;
    int waves() const { return layout == 1 ? 4 : layout == 2 ? 8 : WM * WN; }
};

#define TC_TILE_ENTRY(id, MT, NT, KT, WM, WN, L) TileCfg{MT, NT, KT, WM, WN, L},
static const TileCfg kTilesF64[] = {TC_TILES_F64(TC_TILE_ENTRY)};
static const TileCfg kTilesF32[] = {TC_TILES_F32(TC_TILE_ENTRY)};
static const TileCfg kTilesBF16x3[] = {TC_TILES_BF16X3(TC_TILE_ENTRY)};
#undef TC_TILE_ENTRY

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

}  // namespace tc
