// Offset vectors of a plan built on the device into a file-scope array, for
// the entry point that allocates nothing (tc_contract_noalloc).
//
// tc_contract keeps a plan's scatter and block-stride vectors (Sec. 6.1-6.2)
// in device memory the library allocates and uploads once.  Callers that
// cannot allocate (code under graph capture, tight serving loops, harnesses
// that forbid hipMalloc) get the same vectors written by one small kernel into
// `scratch`, a static device array of TC_NOALLOC_SCRATCH_BYTES held per GPU for
// the life of the process: the plan's bundles travel as kernel arguments, so
// nothing is allocated and nothing is copied from host memory.  Every call on
// a GPU reuses that GPU's array, so calls that overlap on one GPU race.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <string>

#include "launch.hpp"
#include "plan.hpp"
#include "tc.h"

namespace tc {

namespace {

__device__ __align__(256) unsigned char scratch[TC_NOALLOC_SCRATCH_BYTES];

// One vector to build: the scatter vector of a bundle (entry x = sum over
// the bundle's dims of digit_d(x) * stride_d, first dim fastest; with
// sa >= 0 the plan's sub-blocked k order over dims sa and sb), or, with
// block > 0, the block strides of that scatter vector at blocking `block`.
struct VecJob {
    int nd;
    int sa, sb;      // sub-blocked dims, -1 for none
    int64_t bx, by;  // their sub-block extents
    int64_t len[kMaxDim];
    int64_t st[kMaxDim];
    int64_t total;  // entries of the scatter vector
    int64_t block;  // 0: the scatter vector itself; b > 0: its block strides
    int64_t out;    // element offset of the output inside the array
};

constexpr int kJobs = 8;  // rX, cX, rY, cY, rC, cC, kbsX, kbsY

struct VecJobs {
    VecJob j[kJobs];
};

__device__ __forceinline__ int64_t scat_at(const VecJob& j, int64_t x) {
    int64_t off = 0;
    if (j.sa >= 0) {
        // bands of by values of dim sb, cut into blocks of bx values of dim
        // sa (shorter at a ragged edge), sa fastest inside a block; the
        // other dims outside, in order
        const int64_t La = j.len[j.sa], Lb = j.len[j.sb], plane = La * Lb;
        const int64_t r = x % plane;
        x /= plane;
        const int64_t band = r / (La * j.by), r2 = r - band * La * j.by;
        const int64_t h = j.by < Lb - band * j.by ? j.by : Lb - band * j.by;
        const int64_t blk = r2 / (j.bx * h), r3 = r2 - blk * j.bx * h;
        const int64_t w = j.bx < La - blk * j.bx ? j.bx : La - blk * j.bx;
        off = (blk * j.bx + r3 % w) * j.st[j.sa] + (band * j.by + r3 / w) * j.st[j.sb];
    }
    for (int d = 0; d < j.nd; ++d) {
        if (d == j.sa || d == j.sb) continue;
        const int64_t q = x / j.len[d];
        off += (x - q * j.len[d]) * j.st[d];
        x = q;
    }
    return off;
}

// blockIdx.y selects the job.  Block strides follow the same definition as
// the host planner: a block of one entry has stride 1; otherwise the
// constant positive difference of consecutive entries, else 0.
template <typename OffT>
__global__ __launch_bounds__(256) void build_vectors_kernel(VecJobs jobs, OffT* __restrict__ out) {
    const VecJob& jb = jobs.j[blockIdx.y];
    const int64_t count = jb.block ? (jb.total + jb.block - 1) / jb.block : jb.total;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x) {
        int64_t v;
        if (!jb.block) {
            v = scat_at(jb, i);
        } else {
            const int64_t lo = i * jb.block;
            const int64_t hi = lo + jb.block < jb.total ? lo + jb.block : jb.total;
            if (hi - lo <= 1) {
                v = 1;
            } else {
                int64_t prev = scat_at(jb, lo + 1);
                const int64_t s = prev - scat_at(jb, lo);
                bool ok = s > 0;
                for (int64_t x = lo + 2; ok && x < hi; ++x) {
                    const int64_t c = scat_at(jb, x);
                    ok = c - prev == s;
                    prev = c;
                }
                v = ok ? s : 0;
            }
        }
        out[jb.out + i] = (OffT)v;
    }
}

std::mutex g_mu;
void* g_scratch[kMaxDevices];  // device address of `scratch` on each device, once resolved

// The array's address on the current device, resolved with the device
// current the first time the device is seen.
int scratch_address(void** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        set_error(std::string("hipGetDevice: ") + hipGetErrorString(e));
        return TC_ERR_HIP;
    }
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("device index beyond the library's limit of 16");
        return TC_ERR_ARG;
    }
    std::lock_guard<std::mutex> g(g_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_error(std::string("hipGetSymbolAddress of the scratch array: ") + hipGetErrorString(e));
            return TC_ERR_HIP;
        }
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return TC_OK;
}

void fill(VecJob* j, const std::vector<Dim>& dims, int which, int64_t block, int64_t out, const Plan* sub = nullptr) {
    j->nd = (int)dims.size();
    j->sa = sub ? sub->sub_a : -1;
    j->sb = sub ? sub->sub_b : -1;
    j->bx = sub ? sub->sub_bx : 1;
    j->by = sub ? sub->sub_by : 1;
    j->total = 1;
    for (int d = 0; d < j->nd; ++d) {
        j->len[d] = dims[(size_t)d].len;
        j->st[d] = which == 0 ? dims[(size_t)d].sX : which == 1 ? dims[(size_t)d].sY : dims[(size_t)d].sC;
        j->total *= j->len[d];
    }
    j->block = block;
    j->out = out;
}

}  // namespace

// Layout of a plan's vectors in the array (each start 256-byte aligned) and
// the bytes it needs; the same vectors as the plan's uploaded copy.
size_t noalloc_layout(const Plan& p, DeviceVectors* dv) {
    const size_t lens[kJobs] = {p.rX.size(), p.cX.size(), p.rY.size(), p.cY.size(),
                                p.rC.size(), p.cC.size(), p.kbsX.size(), p.kbsY.size()};
    size_t* offs[kJobs] = {&dv->o_rX, &dv->o_cX, &dv->o_rY, &dv->o_cY, &dv->o_rC, &dv->o_cC, &dv->o_kbsX, &dv->o_kbsY};
    const size_t w = p.off64 ? 8 : 4, align = 256 / w;
    size_t total = 0;
    for (int i = 0; i < kJobs; ++i) {
        *offs[i] = total;
        const size_t n = lens[i] > 0 ? lens[i] : 1;
        total += (n + align - 1) / align * align;
    }
    dv->bytes = total * w;
    return dv->bytes;
}

// Write the plan's vectors into this device's array on `stream` and point
// *dv at them.  TC_ERR_ARG when they do not fit (checked before any HIP
// call).  No allocation of any kind on the device.
int noalloc_vectors(const Plan& p, hipStream_t stream, DeviceVectors* dv) {
    const size_t need = noalloc_layout(p, dv);
    if (need > (size_t)TC_NOALLOC_SCRATCH_BYTES) {
        set_error("the plan's offset vectors need " + std::to_string(need) +
                  " bytes, more than the allocation-free entry point's array of " +
                  std::to_string((long long)TC_NOALLOC_SCRATCH_BYTES) + " bytes");
        return TC_ERR_ARG;
    }
    void* base = nullptr;
    int st = scratch_address(&base);
    if (st) return st;
    dv->buf = base;
    VecJobs jobs{};
    const TileCfg& t = tile_table(p.dtype, p.mode)[p.tile];
    fill(&jobs.j[0], p.I, 0, 0, (int64_t)dv->o_rX);
    fill(&jobs.j[1], p.P, 0, 0, (int64_t)dv->o_cX, &p);
    fill(&jobs.j[2], p.P, 1, 0, (int64_t)dv->o_rY, &p);
    fill(&jobs.j[3], p.J, 1, 0, (int64_t)dv->o_cY);
    fill(&jobs.j[4], p.I, 2, 0, (int64_t)dv->o_rC);
    fill(&jobs.j[5], p.J, 2, 0, (int64_t)dv->o_cC);
    fill(&jobs.j[6], p.P, 0, t.KT, (int64_t)dv->o_kbsX, &p);
    fill(&jobs.j[7], p.P, 1, t.KT, (int64_t)dv->o_kbsY, &p);
    if (p.noop) return TC_OK;
    if (p.k_empty)  // the host plan holds no contracted vectors either
        for (int i : {1, 2, 6, 7}) jobs.j[i].total = 0;
    int64_t most = 1;
    for (const VecJob& j : jobs.j) most = j.total > most ? j.total : most;
    int64_t blocks = (most + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (p.off64)
        hipLaunchKernelGGL(build_vectors_kernel<int64_t>, dim3((unsigned)blocks, kJobs), dim3(256), 0, stream, jobs,
                           (int64_t*)base);
    else
        hipLaunchKernelGGL(build_vectors_kernel<int32_t>, dim3((unsigned)blocks, kJobs), dim3(256), 0, stream, jobs,
                           (int32_t*)base);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error(std::string("offset-vector kernel launch: ") + hipGetErrorString(e));
        return TC_ERR_HIP;
    }
    return TC_OK;
}

}  // namespace tc
