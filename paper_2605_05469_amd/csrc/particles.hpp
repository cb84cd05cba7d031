// particles.hpp -- launchers of the particle kernels and the cell sort (internal).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "solver_state.hpp"

namespace pic {

hipError_t launch_keys(int64_t np, const double* x, const double* y, const double* z,
                       uint32_t* key, int n, double inv_h, hipStream_t s);
// With rec non-NULL the pushed state goes to 64-byte records rec[4p..4p+3]
// = (x, y), (z, vx), (vy, vz), padding instead of back into x..vz (which
// are then only read); launch_sort_cells takes such records as its source.
hipError_t launch_gather_push(int64_t np, double* x, double* y, double* z, double* vx, double* vy,
                              double* vz, const double* ex, const double* ey, const double* ez,
                              uint32_t* key, double2* rec, int n, double inv_h, double L,
                              double dt, double coef, hipStream_t s);
hipError_t launch_half_kick(int64_t np, const double* x, const double* y, const double* z,
                            double* vx, double* vy, double* vz, const double* ex,
                            const double* ey, const double* ez, int n, double inv_h, double coef,
                            hipStream_t s);
// Deposit + background + zero-mean projection; st->bb receives ||b||^2.
// part must hold 2 * deposit_partials() doubles.
int deposit_partials();
// With cs (sorted particles) the four n^3 FP64 scratch arrays T hold the
// per-cell-row partial sums between the two passes.
hipError_t launch_deposit(int64_t np, const double* x, const double* y, const double* z,
                          const uint32_t* cs, double* rho, int n, double inv_h, double qh3,
                          double rho_bg, DevState* st, double* part, double* const T[4],
                          hipStream_t s);

// Stable LSD radix sort of cell keys (internal scratch sized by sort_scratch_bytes).
struct SortScratch {
    uint32_t* key[2];
    uint32_t* idx[2];
    uint32_t* hist;     // radix * tiles (+ scan sums)
    uint32_t* sums;
    double2* rec;       // 4 * cap: particle records (x, y | z, vx | vy, vz | pad)
    int64_t cap;        // particles
};
size_t sort_scratch_bytes(int64_t np_max);
// The particle records (64 bytes each), a separate allocation made on the
// first sort.
size_t sort_rec_bytes(int64_t np_max);
void sort_scratch_carve(void* base, int64_t np_max, SortScratch* s);
// Sorts key[0..np) (values < n^3); writes the permutation (source index of
// each sorted slot) to perm_out (may be NULL), cell_start[0..n^3], and the
// six permuted particle arrays dst.  The source is sc->rec as filled by
// launch_gather_push when src is NULL, else the six arrays src (packed into
// sc->rec first).
hipError_t launch_sort_cells(int64_t np, int n, const uint32_t* key,
                             const double* const src[6], double* const dst[6],
                             uint32_t* cell_start, uint32_t* perm_out, SortScratch* sc,
                             hipStream_t s);

}  // namespace pic
