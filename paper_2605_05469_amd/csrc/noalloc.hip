// noalloc.hip -- pic_deposit_cic_noalloc: the CIC deposit (Sec. 2, Fig.
// pic-loop: scatter) for callers that cannot allocate device memory.
//
// pic_deposit_cic takes its scratch (four n^3 row-sum arrays, reduction
// partials, the reduction state) from a context that pic_create allocated.
// This entry point needs no context: its scratch is the file-scope device
// array `scratch` below, sized for grids up to kNoallocMaxN^3, which every
// GPU the library runs on holds until the process ends.  The array's address
// on each device comes from hipGetSymbolAddress, taken once per device with
// that device current; host code uses only that address (the array's name
// is a host-side stand-in, not a device address).  Calls on one GPU share the
// array: calls that overlap in time on one GPU race.  The kernels are those
// of pic_deposit_cic, so both entry points return the same bits.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

#include "../../include/pic.h"
#include "particles.hpp"
#include "solver_state.hpp"

extern "C" int pic_set_error_(int code, const char* msg);

namespace pic {
namespace {

constexpr int kNoallocMaxN = PIC_NOALLOC_MAX_N;
constexpr size_t kAlign = 256;
constexpr size_t align_up(size_t b) { return (b + kAlign - 1) & ~(kAlign - 1); }
constexpr size_t kVecBytes = align_up((size_t)kNoallocMaxN * kNoallocMaxN * kNoallocMaxN * 8);
constexpr size_t kPartBytes = align_up((size_t)2 * 4096 * 8);  // 2 * deposit_partials()
constexpr size_t kStateBytes = align_up(sizeof(DevState));
constexpr size_t kScratchBytes = 4 * kVecBytes + kPartBytes + kStateBytes;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// The scratch array's device address on the current device (taken once).
int scratch_ptr(void** out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
        return pic_set_error_(PIC_ERR_HIP, "pic_deposit_cic_noalloc: no current HIP device");
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return pic_set_error_(PIC_ERR_HIP, "pic_deposit_cic_noalloc: hipGetSymbolAddress failed");
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return PIC_OK;
}

// Zero the reduction state (its "last block" tickets must start at zero);
// a kernel rather than a memset, so the call can be captured into a graph.
__global__ void clear_words_kernel(uint32_t* w, int n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) w[i] = 0u;
}

}  // namespace
}  // namespace pic

using namespace pic;

extern "C" int pic_deposit_cic_noalloc(const pic_params* p, int64_t np, const double* x,
                                       const double* y, const double* z,
                                       const uint32_t* cell_start, double* rho, double* norm_b,
                                       void* stream) {
    if (!p) return pic_set_error_(PIC_ERR_INVALID, "params is NULL");
    const int n = p->n;
    if (n < 32 || n > kNoallocMaxN || (n % 32) != 0)
        return pic_set_error_(PIC_ERR_INVALID,
                              "pic_deposit_cic_noalloc: n must be a multiple of 32 in "
                              "[32, PIC_NOALLOC_MAX_N]");
    if (p->bc != PIC_BC_PERIODIC)
        return pic_set_error_(PIC_ERR_INVALID, "pic_deposit_cic_noalloc: the periodic box only");
    if (!(p->length > 0.0) || !std::isfinite(p->length) || !std::isfinite(p->charge) ||
        !std::isfinite(p->rho_bg))
        return pic_set_error_(PIC_ERR_INVALID,
                              "pic_deposit_cic_noalloc: length must be positive, charge and "
                              "rho_bg finite");
    if (np < 0 || np >= ((int64_t)1 << 32))
        return pic_set_error_(PIC_ERR_INVALID, "pic_deposit_cic_noalloc: np must be in [0, 2^32)");
    if (!rho) return pic_set_error_(PIC_ERR_INVALID, "rho is NULL");
    if (np > 0 && (!x || !y || !z))
        return pic_set_error_(PIC_ERR_INVALID, "x, y and z are required when np > 0");
    const uintptr_t mis = (uintptr_t)rho | (uintptr_t)x | (uintptr_t)y | (uintptr_t)z |
                          (uintptr_t)cell_start;
    if (mis & 7u) return pic_set_error_(PIC_ERR_INVALID, "arrays must be 8-byte aligned");

    void* base = nullptr;
    const int rc = scratch_ptr(&base);
    if (rc != PIC_OK) return rc;
    unsigned char* b = (unsigned char*)base;
    double* T[4];
    for (int k = 0; k < 4; ++k) T[k] = (double*)(b + k * kVecBytes);
    double* part = (double*)(b + 4 * kVecBytes);
    DevState* st = (DevState*)(b + 4 * kVecBytes + kPartBytes);

    const double inv_h = (double)n / p->length;
    const double qh3 = p->charge * (inv_h * inv_h * inv_h);
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(clear_words_kernel, dim3(1), dim3(256), 0, s, (uint32_t*)st,
                       (int)(sizeof(DevState) / 4));
    hipError_t e = hipGetLastError();
    if (e == hipSuccess)
        e = launch_deposit(np, x, y, z, np > 0 ? cell_start : nullptr, rho, n, inv_h, qh3,
                           p->rho_bg, st, part, T, s);
    if (e != hipSuccess) return pic_set_error_(PIC_ERR_HIP, hipGetErrorString(e));
    if (norm_b) {
        double bb = 0.0;
        e = hipMemcpyAsync(&bb, &st->bb, sizeof bb, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return pic_set_error_(PIC_ERR_HIP, hipGetErrorString(e));
        *norm_b = std::sqrt(bb);
    }
    return PIC_OK;
}
