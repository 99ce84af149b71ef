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
//            make exactly 256 tiles
#pragma once

#define TC_TILES_F64(X)            \
    X(0, 32, 32, 16, 1, 1, 0)      \
    X(1, 64, 64, 16, 2, 2, 0)      \
    X(2, 128, 64, 16, 2, 2, 0)     \
    X(3, 128, 128, 16, 2, 2, 0)    \
    X(4, 144, 144, 16, 1, 1, 1)

#define TC_TILES_F32(X)            \
    X(0, 32, 32, 32, 1, 1, 0)      \
    X(1, 64, 64, 32, 2, 2, 0)      \
    X(2, 128, 64, 32, 2, 2, 0)     \
    X(3, 128, 128, 32, 2, 2, 0)    \
    X(4, 144, 144, 32, 1, 1, 1)

// split-bf16: KT is a multiple of the bf16 MFMA depth (32)
#define TC_TILES_BF16X3(X)         \
    X(0, 32, 32, 32, 1, 1, 0)      \
    X(1, 64, 64, 32, 2, 2, 0)      \
    X(2, 128, 64, 32, 2, 2, 0)     \
    X(3, 128, 128, 32, 2, 2, 0)

namespace tc {

struct TileCfg {
    int MT, NT, KT, WM, WN, layout;
    int waves() const { return layout == 1 ? 8 : WM * WN; }
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
