// Instantiation of the contraction and batched kernels for one storage type
// and one offset width (one translation unit each, compiled in parallel).
#include "kernels_impl.hpp"

namespace tc {

int launch_typed_f64_i32(const Plan& p, const DeviceVectors& dv, double alpha, const void* A, const void* B, double beta,
                       void* C, hipStream_t s, void* ws) {
    return launch_typed<double, int32_t>(p, dv, alpha, A, B, beta, C, s, ws);
}

int batch_dispatch_f64_i32(int dtype, int tile, bool launch, const BatchItemDev* items, const int32_t* off,
                         const int32_t* ent, int64_t total, int grid, hipStream_t s) {
    return batch_dispatch<double, int32_t>(dtype, tile, launch, items, off, ent, total, grid, s);
}

}  // namespace tc
