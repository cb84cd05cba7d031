// fft.hip -- FFT Poisson solve on the periodic grid (the paper's comparison
// solver, Sec. 3.1: pseudo-spectral, phi_hat = rho_hat / |k|^2, E = -i k
// phi_hat), and the variant with the 7-point operator's eigenvalues
// lambda(m) = sum_d (2 - 2 cos(2 pi m_d / N)) / h^2, which solves the PCG's
// own system exactly (the system is circulant).  Transforms are rocFFT's
// real-to-complex / complex-to-real plans on the [z][y][x] grid (x fastest:
// the half-spectrum has N/2 + 1 entries along x); the multiplier kernels are
// this library's.
#include <rocfft/rocfft.h>

#include <cmath>
#include <string>

#include "common.hpp"
#include "fft.hpp"

namespace pic {

struct FftPlans {
    int n = 0;
    rocfft_plan fwd = nullptr, inv = nullptr;
    rocfft_execution_info info = nullptr;
    void* work = nullptr;
    size_t work_bytes = 0;
};

static std::string g_fft_err;
const char* fft_last_error() { return g_fft_err.c_str(); }

static bool rchk(rocfft_status st, const char* what) {
    if (st == rocfft_status_success) return true;
    g_fft_err = std::string(what) + " failed (rocfft status " + std::to_string((int)st) + ")";
    return false;
}

int fft_create(FftPlans** out, int n) {
    *out = nullptr;
    static bool setup = false;
    if (!setup) {
        if (!rchk(rocfft_setup(), "rocfft_setup")) return -1;
        setup = true;
    }
    FftPlans* f = new FftPlans();
    f->n = n;
    const size_t len[3] = {(size_t)n, (size_t)n, (size_t)n};
    size_t wf = 0, wi = 0;
    bool ok = rchk(rocfft_plan_create(&f->fwd, rocfft_placement_notinplace,
                                      rocfft_transform_type_real_forward, rocfft_precision_double, 3,
                                      len, 1, nullptr),
                   "forward plan") &&
              rchk(rocfft_plan_create(&f->inv, rocfft_placement_notinplace,
                                      rocfft_transform_type_real_inverse, rocfft_precision_double, 3,
                                      len, 1, nullptr),
                   "inverse plan") &&
              rchk(rocfft_plan_get_work_buffer_size(f->fwd, &wf), "work size") &&
              rchk(rocfft_plan_get_work_buffer_size(f->inv, &wi), "work size") &&
              rchk(rocfft_execution_info_create(&f->info), "execution info");
    if (ok) {
        f->work_bytes = wf > wi ? wf : wi;
        if (f->work_bytes > 0 && hipMalloc(&f->work, f->work_bytes) != hipSuccess) {
            g_fft_err = "work buffer allocation failed";
            ok = false;
        }
        if (ok && f->work_bytes > 0)
            ok = rchk(rocfft_execution_info_set_work_buffer(f->info, f->work, f->work_bytes),
                      "set work buffer");
    }
    if (!ok) {
        fft_destroy(f);
        return -1;
    }
    *out = f;
    return 0;
}

void fft_destroy(FftPlans* f) {
    if (!f) return;
    if (f->info) rocfft_execution_info_destroy(f->info);
    if (f->fwd) rocfft_plan_destroy(f->fwd);
    if (f->inv) rocfft_plan_destroy(f->inv);
    if (f->work) (void)hipFree(f->work);
    delete f;
}

int fft_forward(FftPlans* f, double* in, double2* out, hipStream_t s) {
    if (!rchk(rocfft_execution_info_set_stream(f->info, s), "set stream")) return -1;
    void* ib[1] = {in};
    void* ob[1] = {out};
    return rchk(rocfft_execute(f->fwd, ib, ob, f->info), "forward transform") ? 0 : -1;
}

int fft_inverse(FftPlans* f, double2* in, double* out, hipStream_t s) {
    if (!rchk(rocfft_execution_info_set_stream(f->info, s), "set stream")) return -1;
    void* ib[1] = {in};
    void* ob[1] = {out};
    return rchk(rocfft_execute(f->inv, ib, ob, f->info), "inverse transform") ? 0 : -1;
}

// ------------------------------------------------------------ multipliers --
// Half spectrum index e -> (mx in [0, n/2], signed my, mz).
struct Mode {
    int mx, my, mz;
};
__device__ __forceinline__ Mode mode_of(int64_t e, int n) {
    const int nh = n / 2 + 1;
    Mode m;
    m.mx = (int)(e % nh);
    const int64_t r = e / nh;
    const int ky = (int)(r % n), kz = (int)(r / n);
    m.my = ky <= n / 2 ? ky : ky - n;
    m.mz = kz <= n / 2 ? kz : kz - n;
    return m;
}

// phi_hat = b_hat / symbol / n^3 (mode 0 -> 0).  kind 0: 7-point eigenvalues,
// kind 1: |k|^2.
__global__ void fft_divide_kernel(int64_t nspec, int n, double inv_h2, double kf, int kind,
                                  double inv_n3, double2* __restrict__ a) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nspec;
         e += (int64_t)gridDim.x * blockDim.x) {
        const Mode m = mode_of(e, n);
        double lam;
        if (kind == 0) {
            const double w = 2.0 * M_PI / n;
            lam = ((2.0 - 2.0 * cos(w * m.mx)) + (2.0 - 2.0 * cos(w * m.my)) +
                   (2.0 - 2.0 * cos(w * m.mz))) * inv_h2;
        } else {
            const double kx = kf * m.mx, ky = kf * m.my, kz = kf * m.mz;
            lam = (kx * kx + ky * ky) + kz * kz;
        }
        double2 v = a[e];
        if (e == 0) {
            v.x = 0.0;
            v.y = 0.0;
        } else {
            const double sc = inv_n3 / lam;
            v.x *= sc;
            v.y *= sc;
        }
        a[e] = v;
    }
}

// w = -i k_d phi_hat (the Nyquist derivative set to zero).
__global__ void fft_grad_kernel(int64_t nspec, int n, double kf, int dir,
                                const double2* __restrict__ a, double2* __restrict__ w) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nspec;
         e += (int64_t)gridDim.x * blockDim.x) {
        const Mode m = mode_of(e, n);
        int md = dir == 0 ? m.mx : (dir == 1 ? m.my : m.mz);
        if (2 * md == n || -2 * md == n) md = 0;
        const double k = kf * md;
        const double2 v = a[e];
        w[e] = make_double2(k * v.y, -k * v.x);  // -i k (vx + i vy) = k vy - i k vx
    }
}

static int spec_blocks(int64_t m) {
    int64_t b = (m + 255) / 256;
    return (int)(b < 8192 ? (b < 1 ? 1 : b) : 8192);
}

hipError_t launch_fft_divide(int64_t nspec, int n, double inv_h2, double kf, int kind,
                             double inv_n3, double2* a, hipStream_t s) {
    hipLaunchKernelGGL(fft_divide_kernel, dim3(spec_blocks(nspec)), dim3(256), 0, s, nspec, n,
                       inv_h2, kf, kind, inv_n3, a);
    return hipGetLastError();
}

hipError_t launch_fft_grad(int64_t nspec, int n, double kf, int dir, const double2* a, double2* w,
                           hipStream_t s) {
    hipLaunchKernelGGL(fft_grad_kernel, dim3(spec_blocks(nspec)), dim3(256), 0, s, nspec, n, kf,
                       dir, a, w);
    return hipGetLastError();
}

}  // namespace pic
