// Launch dispatch of the transpose-free contraction (block-scatter-matrix
// tensor contraction, Sec. 6.2): picks the instantiation for the plan's
// storage type, offset width and tile configuration.  The kernels themselves
// are in kernels_impl.hpp, instantiated by the k_*.hip units.
#include <hip/hip_runtime.h>

#include "launch.hpp"
#include "tc.h"

namespace tc {

int launch_typed_f64_i32(const Plan& p, const DeviceVectors& dv, double alpha, const void* A, const void* B, double beta,
                       void* C, hipStream_t s, void* ws);
int batch_dispatch_f64_i32(int dtype, int tile, bool launch, const BatchItemDev* items, const int32_t* off,
                         const int32_t* ent, int64_t total, int grid, hipStream_t s);
int launch_typed_f64_i64(const Plan& p, const DeviceVectors& dv, double alpha, const void* A, const void* B, double beta,
                       void* C, hipStream_t s, void* ws);
int batch_dispatch_f64_i64(int dtype, int tile, bool launch, const BatchItemDev* items, const int32_t* off,
                         const int32_t* ent, int64_t total, int grid, hipStream_t s);
int launch_typed_f32_i32(const Plan& p, const DeviceVectors& dv, double alpha, const void* A, const void* B, double beta,
                       void* C, hipStream_t s, void* ws);
int batch_dispatch_f32_i32(int dtype, int tile, bool launch, const BatchItemDev* items, const int32_t* off,
                         const int32_t* ent, int64_t total, int grid, hipStream_t s);
int launch_typed_f32_i64(const Plan& p, const DeviceVectors& dv, double alpha, const void* A, const void* B, double beta,
                       void* C, hipStream_t s, void* ws);
int batch_dispatch_f32_i64(int dtype, int tile, bool launch, const BatchItemDev* items, const int32_t* off,
                         const int32_t* ent, int64_t total, int grid, hipStream_t s);

int launch_plan(const Plan& p, const DeviceVectors& dv, double alpha, const void* A, const void* B, double beta,
                void* C, hipStream_t s, void* ws) {
    if (p.mode != TC_NATIVE && !(p.mode == TC_SPLIT_BF16X3 && p.dtype == TC_F32)) {
        set_error("split-bf16 mode needs FP32 storage");
        return TC_ERR_DTYPE;
    }
    if (p.dtype == TC_F64)
        return p.off64 ? launch_typed_f64_i64(p, dv, alpha, A, B, beta, C, s, ws)
                       : launch_typed_f64_i32(p, dv, alpha, A, B, beta, C, s, ws);
    return p.off64 ? launch_typed_f32_i64(p, dv, alpha, A, B, beta, C, s, ws)
                   : launch_typed_f32_i32(p, dv, alpha, A, B, beta, C, s, ws);
}

int launch_batch(int dtype, int mode, int tile, bool off64, const BatchItemDev* items, const int32_t* off,
                 const int32_t* ent, int64_t total, int grid, hipStream_t s) {
    if (mode != TC_NATIVE) {
        set_error("batched launches support the native modes");
        return TC_ERR_DTYPE;
    }
    if (total <= 0) return TC_OK;
    if (dtype == TC_F64)
        return off64 ? batch_dispatch_f64_i64(dtype, tile, true, items, off, ent, total, grid, s)
                     : batch_dispatch_f64_i32(dtype, tile, true, items, off, ent, total, grid, s);
    return off64 ? batch_dispatch_f32_i64(dtype, tile, true, items, off, ent, total, grid, s)
                 : batch_dispatch_f32_i32(dtype, tile, true, items, off, ent, total, grid, s);
}

int batch_grid(int dtype, int mode, int tile, bool off64, int64_t total) {
    if (mode != TC_NATIVE || total <= 0) return 0;
    if (dtype == TC_F64)
        return off64 ? batch_dispatch_f64_i64(dtype, tile, false, nullptr, nullptr, nullptr, total, 0, nullptr)
                     : batch_dispatch_f64_i32(dtype, tile, false, nullptr, nullptr, nullptr, total, 0, nullptr);
    return off64 ? batch_dispatch_f32_i64(dtype, tile, false, nullptr, nullptr, nullptr, total, 0, nullptr)
                 : batch_dispatch_f32_i32(dtype, tile, false, nullptr, nullptr, nullptr, total, 0, nullptr);
}

}  // namespace tc
