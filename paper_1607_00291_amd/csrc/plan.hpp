// Host-side plan of one contraction: bundles, ordering, scatter and
// block-stride vectors (Sec. 4, 6.1-6.3, 7.3).  Internal to libtc.so.
#pragma once

#include <cstdint>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "tiles.hpp"

namespace tc {

constexpr int kMaxDim = 16;
constexpr int kMaxDevices = 16;

// One (possibly folded) index of a bundle.  Strides are in elements, in the
// planned operand roles: X holds I and P, Y holds P and J (X is A unless the
// operands were swapped).  A stride is 0 where the tensor lacks the index.
struct Dim {
    int64_t len = 1;
    int64_t sX = 0, sY = 0, sC = 0;
    std::string labels;  // original labels, several when folded
};

struct TensorDesc {
    int ndim = 0;
    int64_t lens[kMaxDim] = {};
    int64_t strides[kMaxDim] = {};
    char idx[kMaxDim] = {};
};

// Device copy of a plan's vectors.
struct DeviceVectors {
    void* buf = nullptr;  // one allocation holding every vector below
    size_t bytes = 0;
    // element offsets (in units of the offset type) of each vector inside buf
    size_t o_rX = 0, o_cX = 0, o_rY = 0, o_cY = 0, o_rC = 0, o_cC = 0, o_kbsX = 0, o_kbsY = 0;
};

struct Plan {
    int dtype = 0, mode = 0;
    TensorDesc dA, dB, dC;
    bool swapped = false;
    std::vector<Dim> I, J, P;
    int64_t m = 1, n = 1, k = 1;
    bool noop = false;        // some free index has length 0
    bool k_empty = false;     // some contracted index has length 0: C := beta C
    int64_t spanA = 0, spanB = 0, spanC = 0;  // element spans (max offset + 1)
    bool off64 = false;       // offsets need 64 bits
    int folds = 0;            // number of fold steps performed
    int dropped = 0;          // number of length-1 dims dropped
    int unit_moves = 0;       // operands whose unit-stride index was moved to the front of their free bundle
    std::string paper_order;  // "I|J|P" labels in the order of the paper's heuristic (before the GPU amendments and the fold)
    // Sub-blocked k order (GPU amendment 3), used when X and Y have their
    // unit strides on two different P dims: P dims sub_a (X's) and sub_b
    // (Y's) are walked in sub-blocks of sub_bx x sub_by (sub_a fastest, then
    // sub_b, then the blocks along sub_a, then the bands along sub_b), the
    // other P dims outside in P order.  sub_a = -1: plain colexicographic.
    int sub_a = -1, sub_b = -1;
    int64_t sub_bx = 1, sub_by = 1;

    // scatter vectors (Sec. 6.1): rows of X and C over I, columns of Y and C
    // over J, columns of X and rows of Y over P
    std::vector<int64_t> rX, cX, rY, cY, rC, cC;
    // lane-fast dimension of each operand for the gather: X along m or k,
    // Y along n or k
    bool x_lanes_m = true, y_lanes_n = true;

    int tile = 0;  // index into the tile table of (dtype, mode)
    // block strides (Sec. 6.2) at the tile granularity: along k by KT for X
    // and Y; along m by MT for X and C; along n by NT for Y and C
    std::vector<int64_t> kbsX, kbsY, rbsX, cbsY, rbsC, cbsC;
    int64_t tiles_m = 0, tiles_n = 0, c_tiles_regular = 0, k_blocks_regular_x = 0, k_blocks_regular_y = 0;

    mutable std::mutex dev_mu;
    mutable DeviceVectors dev[kMaxDevices];
    // packed split panels (the packed split tile's workspace), per device:
    // stream -> (buffer, bytes); guarded by dev_mu
    mutable std::map<void*, std::pair<void*, size_t>> ws[kMaxDevices];

    ~Plan();
};

// Build a plan; returns TC_OK or a TC_ERR_* status with a message set.
int build_plan(const TensorDesc& A, const TensorDesc& B, const TensorDesc& C, int dtype, int mode,
               std::unique_ptr<Plan>* out);
// (Re)compute block strides and tile counts for plan->tile.
void set_plan_tile(Plan* p, int tile);
// Pick a tile configuration from the shape (wave-quantisation aware model).
// Tile configuration of least estimated time; batched skips the pinwheel
// layouts (a batched launch does not run the all-compute one, and the
// specialised-wave one spills registers inside the batched kernel), the
// packed split tile and the 32 x 32 tiles.
int choose_tile(const Plan& p, bool batched = false);
// Shape signature used by the autotuner cache.
std::string plan_signature(const Plan& p);
std::string describe_plan(const Plan& p);

// scatter / block-stride primitives (Sec. 6.1 eq. cscat-c generalised; Sec. 6.2)
void scatter_vector(const std::vector<Dim>& dims, int which, std::vector<int64_t>* out);
// The same over P in the sub-blocked order of a plan (sub_a >= 0).
void scatter_vector_sub(const std::vector<Dim>& dims, int which, int a, int b, int64_t bx, int64_t by,
                        std::vector<int64_t>* out);
void block_strides(const int64_t* scat, int64_t len, int64_t b, int64_t* out);

// thread-local error message
void set_error(const std::string& msg);
const char* last_error();

}  // namespace tc
