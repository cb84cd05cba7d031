// particle_math.hpp -- per-particle arithmetic shared by the PIC and PIF
// pushes (internal): cell index and CIC fraction, periodic wrap, cell key.
// Operation by operation the CPU oracle's definition (no contraction).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pic {

__device__ __forceinline__ void locate(double xd, int n, double inv_h, int& i, double& w) {
    const double s = xd * inv_h;
    const double f = floor(s);
    int ii = (int)f;
    if (ii > n - 1) ii = n - 1;
    if (ii < 0) ii = 0;
    i = ii;
    w = s - (double)ii;
}

__device__ __forceinline__ double wrap(double xn, double L) {
    if (xn >= L) xn = xn - L;
    if (xn < 0.0) xn = xn + L;
    if (xn >= L) xn = 0.0;
    return xn;
}

__device__ __forceinline__ uint32_t key_of(double x, double y, double z, int n, double inv_h) {
    int ix, iy, iz;
    double w;
    locate(x, n, inv_h, ix, w);
    locate(y, n, inv_h, iy, w);
    locate(z, n, inv_h, iz, w);
    return (uint32_t)(((uint64_t)iz * n + iy) * n + ix);
}

}  // namespace pic
