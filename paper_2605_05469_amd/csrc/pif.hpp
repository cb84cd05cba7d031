// pif.hpp -- Particle-in-Fourier field solve (internal).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "solver_state.hpp"

namespace pic {

struct PifState;

// Window width for a NUFFT tolerance (the exponential-of-semicircle rule);
// 0 if the tolerance is outside what the kernels are built for.
int pif_width(double tol);
// Buffers and plans for n modes per axis on the box [0, L)^3 (oversampled
// grid of 2n points per axis).  Returns 0 on success, -3 out of memory.
int pif_create(PifState** out, int n, double L, double tol);
void pif_destroy(PifState* p);
size_t pif_bytes(int n);
const char* pif_last_error();

// Spread (the type-1 NUFFT's first step) of np cell-sorted particles of
// charge q onto the oversampled grid (cell_start over the n^3 cells of the
// particle grid).
int pif_spread(PifState* p, int64_t np, const double* x, const double* y, const double* z,
               const uint32_t* cell_start, double q, hipStream_t s);
// The rest of the type-1 NUFFT, the mode-wise Poisson solve and the type-2
// transform up to the field grids that pif_interp evaluates; st->wx receives
// W_x = (1/2) int Ex^2 (Parseval).
int pif_fields(PifState* p, DevState* st, double* partials, hipStream_t s);

// Type-2 evaluation of the field at the particles (tiles of cells as in the
// spread; the particles must still match cell_start):
//   mode 0: store E (ex, ey, ez are per-particle outputs);
//   mode 1: leapfrog push v += coef E, x = wrap(x + dt v), key of the new x;
//   mode 2: half kick v += coef E.
int pif_interp(PifState* p, int mode, int64_t np, double* x, double* y, double* z, double* vx,
               double* vy, double* vz, double* ex, double* ey, double* ez, uint32_t* key,
               const uint32_t* cell_start, double coef, double dt, hipStream_t s);

}  // namespace pic
