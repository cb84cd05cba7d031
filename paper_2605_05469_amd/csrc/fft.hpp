// fft.hpp -- FFT Poisson solve: rocFFT plans and multiplier kernels (internal).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pic {

struct FftPlans;
int fft_create(FftPlans** out, int n);
void fft_destroy(FftPlans* f);
const char* fft_last_error();
// Real n^3 -> half spectrum (n/2 + 1) x n x n; the input may be overwritten.
int fft_forward(FftPlans* f, double* in, double2* out, hipStream_t s);
// Half spectrum -> real n^3 (unnormalised); the input may be overwritten.
int fft_inverse(FftPlans* f, double2* in, double* out, hipStream_t s);
hipError_t launch_fft_divide(int64_t nspec, int n, double inv_h2, double kf, int kind,
                             double inv_n3, double2* a, hipStream_t s);
hipError_t launch_fft_grad(int64_t nspec, int n, double kf, int dir, const double2* a, double2* w,
                           hipStream_t s);

}  // namespace pic
