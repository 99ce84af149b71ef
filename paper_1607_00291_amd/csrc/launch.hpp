// Kernel launchers (defined in kernels.hip), called by the C ABI layer.
#pragma once

#include <hip/hip_runtime.h>

#include "plan.hpp"

namespace tc {

// Launch one planned contraction on `stream`.  dv holds the plan's vectors on
// the current device; ws the packed split tile's panels (split_pack_bytes),
// or null: the packed split tile then runs as its in-kernel-split twin.
// Returns TC_OK or TC_ERR_*.
int launch_plan(const Plan& p, const DeviceVectors& dv, double alpha, const void* A, const void* B, double beta,
                void* C, hipStream_t stream, void* ws);

// One problem of a batched launch, as seen by the device.  Offset vectors
// are int32 or int64 for the whole batch.
struct BatchItemDev {
    const void* X;
    const void* Y;
    void* C;
    const void* rX;
    const void* cX;
    const void* rY;
    const void* cY;
    const void* rC;
    const void* cC;
    const void* kbsX;
    const void* kbsY;
    int64_t m, n, k;  // k = 0 when only C := beta C is needed
    int64_t tiles_m, tiles_n;
    int64_t first_item;  // index of this problem's first work item
    int64_t spanX, spanY;
    double alpha, beta;
    int32_t x_lanes_m, y_lanes_n;
    int32_t kregX, kregY;  // 1: every k block of X (Y) has a nonzero block stride
    int64_t ksX, ksY;      // the block stride shared by every k block of X (Y), else 0
};

// Launch the persistent batched kernel of tile configuration `tile` with
// `grid` workgroups: workgroup g runs the work items ent[2j] (problem index
// into items_dev) and ent[2j + 1] (tile of that problem) for j in
// [off[g], off[g + 1]).  total_items (> 0) is the number of work items.
int launch_batch(int dtype, int mode, int tile, bool off64, const BatchItemDev* items_dev, const int32_t* off,
                 const int32_t* ent, int64_t total_items, int grid, hipStream_t stream);
// Workgroups of a persistent batched launch: min(total_items, resident
// workgroups of the tile's kernel on the current device).
int batch_grid(int dtype, int mode, int tile, bool off64, int64_t total_items);

// Allocation-free execution (noalloc.hip): the byte size of a plan's vectors
// laid out as in an upload (offsets into *dv), and a kernel writing them into
// the current device's static array on `stream` (*dv then points there).
size_t noalloc_layout(const Plan& p, DeviceVectors* dv);
int noalloc_vectors(const Plan& p, hipStream_t stream, DeviceVectors* dv);

// The pack and store stages alone (packstore.hip): elements of an operand's
// tile-panel matrix, its gather into dst, and the alpha/beta scatter-store of
// an m x n column-major matrix into C.  Arguments already validated.
int64_t pack_elements(const Plan& p, int operand);
int launch_pack(const Plan& p, const DeviceVectors& dv, int operand, const void* src, void* dst, hipStream_t stream);
int launch_store(const Plan& p, const DeviceVectors& dv, double alpha, const void* src, double beta, void* C,
                 hipStream_t stream);

// Strided permute-copy dst[i] = src[i] (element bits copied) on `stream`.
// Arguments already validated by tc_permute.
int launch_permute(const void* src, void* dst, int ndim, const int64_t* lens, const int64_t* src_strides,
                   const int64_t* dst_strides, int dtype, hipStream_t stream);

}  // namespace tc
