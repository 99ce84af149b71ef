// Instantiation of the contraction and batched kernels for one storage type
// and one offset width (one translation unit each, compiled in parallel).
#include "kernels_impl.hpp"

namespace tc {

int launch_typed_f32_i64(const Plan& p, const DeviceVectors& dv, double alpha, const void* A, const void* B, double beta,
                       void* C, hipStream_t s, void* ws) {
    return launch_typed<float, int64_t>(p, dv, alpha, A, B, beta, C, s, ws);
}

int batch_dispatch_f32_i64(int dtype, int tile, bool launch, const BatchItemDev* items, const int32_t* off,
                         const int32_t* ent, int64_t total, int grid, hipStream_t s) {
    return batch_dispatch<float, int64_t>(dtype, tile, launch, items, off, ent, total, grid, s);
}

}  // namespace tc
