// Kernel launchers (defined in kernels.hip), called by the C ABI layer.
#pragma once

#include <hip/hip_runtime.h>

#include "plan.hpp"

namespace tc {

// Launch one planned contraction on `stream`.  dv holds the plan's vectors on
// the current device.  Returns TC_OK or TC_ERR_*.
int launch_plan(const Plan& p, const DeviceVectors& dv, double alpha, const void* A, const void* B, double beta,
                void* C, hipStream_t stream);

// One problem of a batched launch, as seen by the device.
struct BatchItemDev {
    const void* X;
    const void* Y;
    void* C;
    const void* rX;  // offset vectors (int32 or int64, see off64 of the batch)
    const void* cX;
    const void* rY;
    const void* cY;
    const void* rC;
    const void* cC;
    const void* kbsX;
    const void* kbsY;
    int64_t m, n, k;
    int64_t tiles_m, tiles_n;
    int64_t first_item;  // prefix sum of tile counts
    double alpha, beta;
    int x_lanes_m, y_lanes_n;
    int scale_only;  // k == 0 or alpha == 0: C := beta C
    int pad_;
};

// Launch the persistent batched kernel over `count` items (table on device).
int launch_batch(int dtype, int mode, int tile, bool off64, const BatchItemDev* items_dev, int count,
                 int64_t total_items, int grid, hipStream_t stream);
// Persistent grid size for a batched launch of the given tile.
int batch_grid(int dtype, int mode, int tile, int64_t total_items);

}  // namespace tc
