// solver_state.hpp -- device-resident scalars of the iterative solvers and the
// launch interface of the field kernels (internal).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pic {

// CG progress states (device).
enum : int32_t {
    CG_RUNNING = 0,
    CG_CANDIDATE = 1,   // recursive residual passed the test; verify it
    CG_CONVERGED = 2,
    CG_MAXIT = 3,
    CG_BREAKDOWN = 4,   // non-finite or non-positive curvature
    CG_ZERO_RHS = 5
};

struct CgScalars {
    double rz;        // r . M^{-1} r of the current residual
    double alpha;
    double beta;
    double rr;        // last recursive r . r
    double nb;        // ||b||
    double tol;       // stop threshold on ||r||
    double true_rn;   // last true residual norm
    double pq;        // last p . A p
    double rz_prev;   // r . M^{-1} r of the residual the last direction was built from
    int64_t iter;
    int64_t max_iter;
    int32_t state;
    int32_t restart;  // next direction = M^{-1} r (ignore the old direction)
    int32_t replacements;
    int32_t xpend;      // single-reduction FP64 sweep: x lacks alpha_pend * p[pend_slot]
    double alpha_pend;
    int32_t pend_slot;  // which of the two direction buffers holds that direction
    int32_t pad;
};

// s-step Jacobi-PCG: iterations per outer step (Gram sweep + update sweep).
constexpr int kSstepS = 3;
constexpr int kSstepNV = 2 * kSstepS + 1;  // basis vectors

struct DevState {
    CgScalars cg;      // the FP64 solve, or the inner FP32 solve of the mixed form
    double out_nr;     // mixed: ||b - A x|| of the current outer step
    double out_sc;     // mixed: 1 / out_nr
    double mean;       // mean(phi) for the gauge fix
    double wx;         // (1/2) h^3 sum Ex^2
    double bb;         // ||b||^2
    double sum;        // generic reduction result
    double flex_zq;    // learned: z . q
    double flex_zr;    // learned: z . r
    double flex_pq;    // learned: p . A p
    double flex_rr;    // learned: r . r
    double prev_nr;    // mixed: ||r|| of the previous outer step (reliable updates)
    int32_t outer_state;
    int32_t gap_restarts;  // mixed: carried directions the residual-gap test refused
    uint32_t tickets[8];
    // s-step form: coefficients of the new p and r and of the x increment on
    // the basis of the last Gram sweep; whether that outer step ended the
    // solve (1: candidate, 2: iteration limit) or a restart follows; its
    // iterations
    double ss_cp[kSstepNV];
    double ss_cr[kSstepNV];
    double ss_cx[kSstepNV];
    int32_t ss_final;
    int32_t ss_restart;
    int32_t ss_steps;
    int32_t ss_pad;
};

// Geometry of a z-marching stencil sweep: the caller sets n; the launcher
// fills in the tiling (tiles in x and y, blocks per column in z).
struct SweepGeo {
    int32_t n;   // grid points per axis
    int32_t bc;  // neighbours outside the grid: 0 periodic, 1 zero, 2 mirrored
    uint32_t nbx, nby, nbz, nb;
};

SweepGeo make_geo(int n, int bc);

// Host launchers (stream-ordered, asynchronous).  All return hipError_t.
// FP64 Jacobi-PCG pieces.
hipError_t launch_residual64(const SweepGeo& g, const double* b, const double* x, double* r,
                             double minv, double inv_h2, int init, double rtol, int64_t max_iter,
                             DevState* st, double* partials, hipStream_t s);
hipError_t launch_dir64(const SweepGeo& g, const double* r, const double* p_old, double* p_new,
                        double minv, double inv_h2, DevState* st, double* partials, hipStream_t s);
hipError_t launch_upd64(const SweepGeo& g, const double* p_new, double* x, double* r,
                        double minv, double inv_h2, DevState* st, double* partials, hipStream_t s);
// Single-reduction (Chronopoulos-Gear) Jacobi-PCG, periodic box: the start
// reduction after a (re)computed residual, then one sweep per iteration
// (r_in/r_out and p_in/p_out alternate between two buffers; x in place).
bool cg1_supported(const SweepGeo& g);
hipError_t launch_cg1_start(const SweepGeo& g, const double* r, double minv, double inv_h2,
                            DevState* st, double* partials, hipStream_t s);
// xm: 0 = x updated by every sweep; 1 / 2 alternate (x updated every other
// sweep, the odd sweep's step pending in the state; pslot: index of p_out
// among the two direction buffers); launch_cg1_flush applies a pending step.
hipError_t launch_cg1(const SweepGeo& g, const double* r_in, double* r_out, const double* p_in,
                      double* p_out, double* x, double minv, double inv_h2, DevState* st,
                      double* partials, int xm, int pslot, hipStream_t s);
hipError_t launch_cg1_flush(int64_t n3, const double* p0, const double* p1, double* x,
                            DevState* st, hipStream_t s);
// s-step form (periodic box): mode 0 = Gram sweep of (r_in, p_in) -- with
// cg.restart set p is taken as M^{-1} r -- whose last workgroup leaves the
// coefficients in the state; mode 1 = update sweep writing p_out, r_out and
// x.  npartials: doubles available in partials.
bool sstep_supported(const SweepGeo& g);
hipError_t launch_sstep(const SweepGeo& g, int mode, const double* r_in, const double* p_in,
                        double* r_out, double* p_out, double* x, double minv, DevState* st,
                        double* partials, int npartials, hipStream_t s);
// The same in FP32 for the inner solve of the mixed form (d: the inner
// solution); pgiven: p_in already holds this step's direction (a direction
// sweep formed it and its curvature: the continued first step).
hipError_t launch_cg1_start32(const SweepGeo& g, const float* r, float minvf, float inv_h2f,
                              DevState* st, double* partials, hipStream_t s);
hipError_t launch_cg1_32(const SweepGeo& g, const float* r_in, float* r_out, const float* p_in,
                         float* p_out, float* d, float minvf, float inv_h2f, int pgiven,
                         DevState* st, double* partials, int xm, int pslot, hipStream_t s);
hipError_t launch_cg1_flush32(int64_t n3, const float* p0, const float* p1, float* d,
                              DevState* st, hipStream_t s);
// Mixed-precision pieces.
hipError_t launch_outer_resid(const SweepGeo& g, const double* b, const double* x, double* r,
                              double inv_h2, DevState* st, double* partials, double tol,
                              hipStream_t s);
hipError_t launch_convert32(int64_t n3, const double* r, float* r32, float* d32, float minvf, int reliable,
                            double inner_rtol, int64_t max_inner, DevState* st,
                            double* partials, hipStream_t s);
hipError_t launch_dir32(const SweepGeo& g, const float* r, const float* p_old, float* p_new,
                        float minvf, float inv_h2f, DevState* st, double* partials, hipStream_t s);
hipError_t launch_upd32(const SweepGeo& g, const float* p_new, float* d, float* r, float minvf,
                        float inv_h2f, DevState* st, double* partials, hipStream_t s);
hipError_t launch_update_x(int64_t n3, double* x, const float* d, DevState* st, hipStream_t s);
// Field.
hipError_t launch_sum(int64_t n3, const double* v, DevState* st, double* partials, int what,
                      hipStream_t s);
hipError_t launch_field(const SweepGeo& g, double* phi, double* ex, double* ey, double* ez,
                        double ehalf, double h3, DevState* st, double* partials, hipStream_t s);
hipError_t launch_fill(int64_t n, double* v, double val, hipStream_t s);
// a = b + s c (n < 2^40), one element per thread, non-temporal stores.
hipError_t launch_triad(int64_t n, const double* b, const double* c, double* a, double s,
                        hipStream_t st);
// r = b - A x and st->out_nr = ||r|| (no state change).
hipError_t launch_resid_norm(const SweepGeo& g, const double* b, const double* x, double* r,
                             double inv_h2, DevState* st, double* partials, hipStream_t s);
// Flexible CG pieces (learned preconditioner): q = A p with p.q -> flex_pq;
// x += a p, r -= a q with r.r -> flex_rr; z.r, z.q -> flex_zr, flex_zq;
// p = z + b p; w = x + z; dst = src.
bool ssor_fused_supported(int n, int inner);
hipError_t launch_ssor_fused(int n, int bounded, int inner, int dir, const double* src,
                             const double* add, const double* rdot, double* dst, double s0,
                             double c, double oscale, DevState* st, double* partials,
                             hipStream_t s);
hipError_t launch_ssor_half(const SweepGeo& g, const double* src, const double* base,
                            const double* add, const double* rdot, double* dst, double c,
                            double bscale, double sscale, double oscale, int dir, DevState* st,
                            double* partials, hipStream_t s);
hipError_t launch_aqz(const SweepGeo& g, const double* z, const double* p_old, double* p_new,
                      double* q, double beta, int restart, double inv_h2, DevState* st,
                      double* partials, hipStream_t s);
hipError_t launch_updp(const SweepGeo& g, const double* p, double* x, double* r, double alpha,
                       double inv_h2, DevState* st, double* partials, hipStream_t s);
hipError_t launch_aq(const SweepGeo& g, const double* p, double* q, double inv_h2, DevState* st,
                     double* partials, hipStream_t s);
hipError_t launch_fcg_update(int64_t n3, double* x, double* r, const double* p, const double* q,
                             double a, DevState* st, double* partials, hipStream_t s);
hipError_t launch_fcg_dots(int64_t n3, const double* z, const double* r, const double* q,
                           DevState* st, double* partials, hipStream_t s);
hipError_t launch_xpby(int64_t n3, const double* z, double* p, double b, hipStream_t s);
hipError_t launch_axpy_copy(int64_t n3, const double* x, const double* z, double* w, hipStream_t s);
hipError_t launch_copy(int64_t n3, const double* src, double* dst, hipStream_t s);

// Upper bound on the workgroups of one sweep (size of the partials array).
int max_sweep_blocks();

}  // namespace pic
