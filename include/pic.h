/*
 * pic.h -- C ABI of the MI355X (gfx950) electrostatic PIC hot path.
 *
 * The operations are those of the PIC loop of "A Comparison of Massively
 * Parallel Performance Portable Particle-in-Cell schemes for electrostatic
 * kinetic plasma simulations" (PASC'26), Sec. 2, Fig. pic-loop:
 *   scatter (CIC deposit) -> solve (matrix-free FD PCG, Sec. 3.2)
 *   -> gather (CIC) -> push (Eq. eom),
 * on the periodic Landau-damping box of Sec. 2.1.
 *
 * Conventions (every entry point):
 *   - Grid: N points per axis, vertex-centred (value i at x = i*h, h = L/N),
 *     periodic, FP64 arrays of N^3 values laid out [iz][iy][ix], ix fastest.
 *   - Particles: structure of arrays, FP64 x, y, z, vx, vy, vz, positions in
 *     [0, L).  All macro-particles carry the same charge q.
 *   - Every array argument is a DEVICE pointer owned by the caller; the library
 *     never frees it and keeps no reference after the call returns.  Host
 *     pointers are marked "host".
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Calls are asynchronous on that stream unless an argument marked "host
 *     out" is non-NULL, in which case the call synchronises `stream` once
 *     before returning.
 *   - Return value: PIC_OK (0); PIC_NOT_CONVERGED (+1, not fatal: outputs hold
 *     the last iterate); or a negative error code with a message available
 *     from pic_last_error().  No exception or abort crosses the ABI.
 *   - One context per stream; a context is not safe for concurrent use.
 *   - Requirements checked on entry: N a multiple of 32, 32 <= N <= 1024,
 *     N^3 < 2^32, 0 <= np <= np_max, non-NULL required pointers, 8-byte
 *     aligned arrays.  Violations return PIC_ERR_INVALID and launch nothing.
 */
#ifndef PIC_H
#define PIC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    PIC_OK = 0,
    PIC_NOT_CONVERGED = 1,
    PIC_ERR_INVALID = -1,
    PIC_ERR_HIP = -2,
    PIC_ERR_NOMEM = -3,
    PIC_ERR_STATE = -4
};

/* Poisson solver forms selectable in pic_params.solver. */
enum {
    PIC_SOLVER_PCG_FP64 = 0,   /* Jacobi-PCG in FP64 (Sec. 3.2)                */
    PIC_SOLVER_PCG_MIXED = 1,  /* FP32 inner PCG inside FP64 refinement        */
    PIC_SOLVER_FCG_LEARNED = 2, /* flexible PCG, U-Net warm start/precond.     */
    PIC_SOLVER_PCG_SSOR = 3,    /* FP64 PCG with the SSOR preconditioner of the
                                   paper's runs (Sec. 4.1), see ssor_* below  */
    PIC_SOLVER_FFT = 4,         /* FFT solve (the paper's comparison solver,
                                   Sec. 3.1): the 7-point operator's
                                   eigenvalues, or with PIC_FLAG_FFT_SPECTRAL
                                   the pseudo-spectral 1/|k|^2 and E = -ik phi */
    PIC_SOLVER_PIF = 5          /* Particle-in-Fourier (Sec. 3.4): no grid
                                   solve; pic_init/pic_step and pic_pif_field
                                   (below) couple the particles to N^3 Fourier
                                   modes by NUFFTs */
};

/* pic_params.bc: boundary kind of the box (Sec. 3.2: the PCG solver takes
 * periodic, Dirichlet and Neumann boundaries; the same kind on all six faces,
 * homogeneous).  The discretisation of the bounded boxes is a reading (the
 * paper gives none):
 *   PIC_BC_PERIODIC   the PIC loop's periodic cube [0, L)^3, h = L/N.
 *   PIC_BC_DIRICHLET  phi = 0 on the boundary of [0, L]^3; the N^3 unknowns
 *                     are the interior vertices x_i = (i+1) h, h = L/(N+1); a
 *                     neighbour on the boundary contributes 0.  A is
 *                     nonsingular: rho needs no mean projection and phi is
 *                     not gauge-shifted.
 *   PIC_BC_NEUMANN    zero normal derivative; the unknowns sit at the cell
 *                     centres x_i = (i+1/2) h, h = L/N; the value across a
 *                     face mirrors the value inside.  Constants are in A's
 *                     kernel: rho must have zero mean, phi is gauge-fixed.
 * Bounded boxes take the solver forms PCG_FP64, PCG_MIXED and PCG_SSOR; the
 * Jacobi scaling stays (h^2/6) I (diag(A)^-1 for Dirichlet; the interior
 * rows' diagonal for Neumann), and SSOR's D is the same scalar with L, U the
 * couplings between unknowns.  Only pic_poisson_pcg and pic_efield accept a
 * bounded context; the particle phases need the periodic box. */
#define PIC_BC_PERIODIC 0
#define PIC_BC_DIRICHLET 1
#define PIC_BC_NEUMANN 2

/* Problem statement (Sec. 2 and 2.1; tolerance as in Sec. 4). */
/* pic_params.flags */
#define PIC_FLAG_NO_WARM_START 1   /* learned form: no network warm start */
#define PIC_FLAG_WARM_START_ONLY 2 /* learned form: warm start, then Jacobi-PCG
                                      (no flexible preconditioning) */
#define PIC_FLAG_MIXED_RELIABLE 4  /* mixed form: keep the inner direction across
                                      refinements (reliable updates) instead of
                                      restarting each inner solve */
#define PIC_FLAG_LEARNED_MIXED 8   /* learned form: the solve after the warm start
                                      (PIC_FLAG_WARM_START_ONLY) or after a
                                      fallback is the mixed form, not FP64 PCG */
#define PIC_FLAG_FFT_SPECTRAL 16   /* FFT form: pseudo-spectral symbol |k|^2 and
                                      E = -i k phi_hat (three more inverse
                                      transforms) instead of the 7-point
                                      eigenvalues and central differences */
#define PIC_FLAG_SSOR_UNFUSED 32   /* SSOR form: run every inner Jacobi step as a
                                      sweep of its own instead of one fused
                                      z-march per triangular solve (same
                                      arithmetic; for comparison) */
#define PIC_FLAG_PCG_TWO_SWEEP 64  /* Jacobi-PCG on the periodic box (the FP64
                                      solve and the mixed form's FP32 inner
                                      solves): one direction sweep and one
                                      update sweep per iteration (two
                                      reductions; 64 bytes per grid point in
                                      FP64).  Bounded boxes always take this
                                      form. */
#define PIC_FLAG_PCG_SINGLE_SWEEP 128 /* FP64 Jacobi-PCG on the periodic box:
                                      one single-reduction sweep per
                                      iteration (the Chronopoulos-Gear
                                      arrangement; 40 bytes per grid point)
                                      instead of the default s-step form (per
                                      three iterations one Gram sweep over a
                                      Chebyshev basis of p and r and one
                                      update sweep: 64 bytes per grid point).
                                      All three forms give the textbook
                                      iterates up to rounding.  The mixed
                                      form's FP32 inner solves take the
                                      single-reduction sweep unless
                                      PIC_FLAG_PCG_TWO_SWEEP is set. */

typedef struct pic_params {
    int32_t n;            /* grid points per axis N                         */
    int32_t ppc;          /* particles per cell (informational)             */
    int64_t np_max;       /* largest particle count any call will pass      */
    double length;        /* box side L of the periodic cube [0, L)^3       */
    double charge;        /* charge q of one macro-particle                 */
    double qm;            /* charge / mass                                  */
    double rho_bg;        /* uniform neutralising background density        */
    double dt;            /* time step                                      */
    double rtol;          /* stop when ||b - A phi||_2 <= rtol * ||b||_2    */
    int64_t max_iter;     /* iteration cap (all CG iterations of a solve)   */
    int32_t solver;       /* PIC_SOLVER_*                                   */
    int32_t check_every;  /* iterations launched between host checks (>=1) */
    double inner_rtol;    /* mixed: inner relative tolerance                */
    int64_t max_inner;    /* mixed: inner iteration cap per refinement step */
    int64_t max_outer;    /* mixed: refinement step cap                     */
    int32_t fcg_window;   /* learned: stall window (iterations)             */
    int32_t flags;        /* PIC_FLAG_* bits (above) */
    /* SSOR form (Sec. 4.1: four inner, two outer iterations, damping pi/2).
     * One application: z = w(2-w) (D + wU)^-1 D (D + wL)^-1 r with each cyclic
     * "triangular" solve replaced by ssor_inner Jacobi steps (L, U = backward,
     * forward neighbours); ssor_outer stationary steps z += SSOR(r - A z).
     * 0 selects the paper's values (w = pi/2, 4, 2). */
    double ssor_omega;    /* damping w in (0, 2)                            */
    int32_t ssor_inner;   /* Jacobi steps per triangular solve (>= 1)        */
    int32_t ssor_outer;   /* stationary SSOR steps per application (>= 1)    */
    int32_t bc;           /* PIC_BC_* (above); 0 = the periodic box          */
    double pif_tol;       /* PIF form: NUFFT tolerance in [1e-7, 1e-2]
                             (0: 1e-4, the paper's, Sec. 4)                 */
} pic_params;

/* Host-side result of one Poisson solve. */
typedef struct pic_solve_info {
    int64_t iterations;        /* CG iterations (inner ones for mixed)           */
    int64_t outer_iterations;  /* mixed: refinement steps; others: 0            */
    int64_t flex_iterations;   /* learned: iterations with the net, else 0      */
    double rel_res;            /* true ||b - A phi|| / ||b|| at exit            */
    double norm_b;             /* ||b||_2                                       */
    double wx;                 /* (1/2) h^3 sum Ex^2 if the field was computed  */
    int32_t converged;         /* 1 if rel_res <= rtol                          */
    int32_t replacements;      /* residual replacements performed               */
    int32_t fell_back;         /* learned: switched to Jacobi-PCG; mixed: the
                                  progress stop handed the solve to FP64
                                  Jacobi-PCG (3 refinements in a row without
                                  bringing the true residual below 0.9 times
                                  the smallest so far)                        */
    int32_t warm_start_used;   /* learned: network warm start accepted          */
    int32_t gap_restarts;      /* mixed, reliable form: refinements whose
                                  carried direction the residual-gap test
                                  refused (true reduction more than 4 times
                                  the inner solve's recursive one)            */
    int32_t reserved;
    int64_t fp64_iterations;   /* mixed: FP64 PCG iterations after the progress
                                  stop (included in `iterations`)            */
} pic_solve_info;

typedef struct pic_particle_arrays {
    double *x, *y, *z, *vx, *vy, *vz;
} pic_particle_arrays;

/* Particles for pic_step / pic_init: `cur` holds the state; `alt` is a
 * second set of the same size that the cell sort writes into, after which
 * the two sets are swapped in this struct (host memory).                    */
typedef struct pic_particles {
    pic_particle_arrays cur;
    pic_particle_arrays alt;
    int64_t np;
    uint32_t *key;        /* np cell keys                                    */
    uint32_t *cell_start; /* N^3 + 1 entries                                 */
} pic_particles;

typedef struct pic_fields {
    double *rho; /* zero-mean right-hand side b (N^3)                          */
    double *phi; /* potential: in = previous step's solution, out = new one    */
    double *ex, *ey, *ez;
} pic_fields;

typedef struct pic_step_info {
    pic_solve_info solve;
    double ms_push, ms_sort, ms_deposit, ms_solve, ms_field; /* event times */
} pic_step_info;

typedef struct pic_ctx pic_ctx;

/* ---- context ----------------------------------------------------------- */

/* Validate `params` and allocate all scratch (solver vectors, sort buffers,
 * reduction partials) on the current HIP device.  No later call allocates. */
int pic_create(const pic_params *params, pic_ctx **out);
int pic_destroy(pic_ctx *ctx);
/* Device bytes pic_create would allocate for `params`. */
size_t pic_workspace_bytes(const pic_params *params);
/* Message of the last error on this thread ("" if none). */
const char *pic_last_error(void);
/* Change the solver form (allocates the extra scratch it needs, once). */
int pic_set_solver(pic_ctx *ctx, int32_t solver);
/* Replace pic_params.flags. */
int pic_set_flags(pic_ctx *ctx, int32_t flags);
/* Library ABI version. */
int pic_abi_version(void);

/* ---- the hot path ------------------------------------------------------ */

/* Cell key of each particle: (iz*N + iy)*N + ix with i_d = floor(x_d*N/L)
 * clamped to [0, N-1] (Sec. 2, CIC shape; cells are the grid's cells). */
int pic_cell_keys(pic_ctx *ctx, int64_t np, const double *x, const double *y,
                  const double *z, uint32_t *key, void *stream);

/* Stable sort of particles by cell key (equal keys keep input order).
 * src[0..5] = x, y, z, vx, vy, vz (read), dst[0..5] (written; must not alias
 * src).  cell_start (N^3 + 1 entries) receives the first sorted index of each
 * cell; perm (nullable) receives the source index of each sorted slot.     */
int pic_sort_cells(pic_ctx *ctx, int64_t np, const uint32_t *key,
                   const double *const src[6], double *const dst[6],
                   uint32_t *cell_start, uint32_t *perm, void *stream);

/* Scatter (Sec. 2, Fig. pic-loop): CIC charge deposit of np particles of
 * charge q, plus the neutralising background rho_bg (Sec. 2), projected to
 * zero mean (the periodic problem's solvability condition):
 *   rho[v] = (q/h^3) sum_p W_p(v) + rho_bg - mean(...).
 * With cell_start (particles sorted by pic_sort_cells) the sum is formed per
 * vertex in a fixed order (deterministic); with cell_start == NULL particles
 * may be in any order and FP64 atomics are used (order not deterministic).
 * norm_b (host out, nullable) receives ||rho||_2.                          */
int pic_deposit_cic(pic_ctx *ctx, int64_t np, const double *x, const double *y,
                    const double *z, const uint32_t *cell_start, double *rho,
                    double *norm_b, void *stream);

/* No-allocation deposit, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): pic_deposit_cic without a context.  The scratch (four n^3 FP64
 * row-sum arrays, reduction partials and state, about 8.1 MiB) is a static
 * device array of the library sized for n <= PIC_NOALLOC_MAX_N, held by every
 * GPU the library runs on until the process ends; the call allocates nothing.
 * `params` supplies n, length, charge, rho_bg and bc (periodic only); the
 * other fields are ignored.  Arguments, layout, ownership and results as in
 * pic_deposit_cic (the same kernels: the same bits).  n > PIC_NOALLOC_MAX_N,
 * a bounded box, np outside [0, 2^32) or NULL/misaligned arrays return
 * PIC_ERR_INVALID and launch nothing.  All calls on one GPU share the scratch:
 * calls that overlap in time on one GPU (other streams, other threads) race
 * and must be serialised by the caller.  norm_b: host out (synchronises). */
#define PIC_NOALLOC_MAX_N 64
int pic_deposit_cic_noalloc(const pic_params *params, int64_t np, const double *x,
                            const double *y, const double *z, const uint32_t *cell_start,
                            double *rho, double *norm_b, void *stream);

/* Solve (Sec. 3.2): A phi = rho with A = -Lap_h, the 7-point second-order
 * operator on the context's box (periodic unless pic_params.bc says
 * otherwise), by the solver form selected in the context, starting from the
 * phi passed in (the previous step's solution, Sec. 4.1), to
 * ||rho - A phi|| <= rtol ||rho||.  FP64 Jacobi-PCG on the periodic box runs
 * in s-step form: per three iterations a Gram sweep and an update sweep,
 * the iteration count exact (the stop test runs after every iteration on
 * the Gram matrix); the same iterates as the textbook recurrences in exact
 * arithmetic (see PIC_FLAG_PCG_SINGLE_SWEEP, PIC_FLAG_PCG_TWO_SWEEP for the
 * other arrangements).  Every candidate that meets the tolerance by its
 * recursive residual is verified by the true residual, which replaces the
 * recursive one when it does not.  rho must have zero mean (not so on a
 * Dirichlet box).  If ex, ey, ez are all non-NULL, the field is computed as
 * pic_efield does (Sec. 2, Eq. poisson).  info: host out. */
int pic_poisson_pcg(pic_ctx *ctx, const double *rho, double *phi, double *ex,
                    double *ey, double *ez, pic_solve_info *info, void *stream);

/* Gather + push (Sec. 2, Eq. eom without external fields), leapfrog:
 *   v <- v + (dt*qm) * E_cic(x);  x <- periodic wrap of x + dt*v;
 * key_out (nullable) receives the new cell keys.  Arithmetic is bit-identical
 * to the CPU oracle (no contraction; fixed summation order).                */
int pic_gather_push(pic_ctx *ctx, int64_t np, double *x, double *y, double *z,
                    double *vx, double *vy, double *vz, const double *ex,
                    const double *ey, const double *ez, uint32_t *key_out,
                    void *stream);

/* Leapfrog start: v <- v - (dt/2)*qm * E_cic(x); positions unchanged. */
int pic_half_kick(pic_ctx *ctx, int64_t np, const double *x, const double *y,
                  const double *z, double *vx, double *vy, double *vz,
                  const double *ex, const double *ey, const double *ez, void *stream);

/* E = -grad_h phi by central differences after gauge-fixing phi to zero
 * mean (a Dirichlet potential is left as it is; a neighbour outside a
 * bounded box follows the box's boundary rule); wx (host out, nullable) =
 * (1/2) h^3 sum Ex^2, the x-field energy of Fig. correctness_landau. */
int pic_efield(pic_ctx *ctx, double *phi, double *ex, double *ey, double *ez,
               double *wx, void *stream);

/* Initial state: keys + sort (cur -> alt, swapped), deposit, t = 0 solve,
 * field, half kick.  info: host out (nullable).                            */
int pic_init(pic_ctx *ctx, pic_particles *parts, pic_fields *fields,
             pic_step_info *info, void *stream);

/* One PIC step (Fig. pic-loop): gather+push -> stable cell sort (cur -> alt,
 * swapped) -> deposit -> solve (warm start from fields->phi) -> field.
 * info: host out (nullable; when set, per-phase event times are recorded).
 * With PIC_SOLVER_PIF the step is push (field of the previous step's modes,
 * evaluated by the type-2 NUFFT) -> sort -> spread -> transforms and the
 * mode-wise solve; the grid fields in `fields` are not used and W_x comes
 * from the modes (Parseval). */
int pic_step(pic_ctx *ctx, pic_particles *parts, pic_fields *fields,
             pic_step_info *info, void *stream);

/* Particle-in-Fourier field at the particles (Sec. 3.4; NUFFT appendix):
 *   rho_hat(k) = sum_j q exp(-i k.x_j)        (type-1 NUFFT, q = charge)
 *   E_hat(k)   = -i k rho_hat(k) / |k|^2      (k = 0 dropped)
 *   E(x_j)     = Re (1/L^3) sum_k E_hat(k) exp(i k.x_j)   (type-2 NUFFT)
 * over k in (2 pi / L) {-N/2 .. N/2-1}^3, to the tolerance pic_params.pif_tol
 * (window: exponential of semicircle, width ceil(log10(1/tol)) + 1, on a
 * 2N-per-axis oversampled grid).  The particles must be cell-sorted with
 * cell_start from pic_sort_cells; ex, ey, ez (np each) receive E at them;
 * wx (host out, nullable) = (1/2) int Ex^2.  The context's solver must be
 * PIC_SOLVER_PIF (N <= 512).  The spread sums with FP64 atomics (summation
 * order not deterministic). */
int pic_pif_field(pic_ctx *ctx, int64_t np, const double *x, const double *y,
                  const double *z, const uint32_t *cell_start, double *ex, double *ey,
                  double *ez, double *wx, void *stream);

/* Average duration (ms) of the most recent solve's dominant kernel launches,
 * measured with HIP events on the solve's stream when timing is enabled by
 * pic_set_kernel_timing(ctx, 1); kernel_id: 0 = direction/stencil kernel,
 * 1 = update kernel, 2 / 3 = the SSOR preconditioner's forward / backward
 * fused triangular solve (of its last outer step; SSOR-PCG only).  Host
 * out; an id outside 0..3 gives PIC_ERR_INVALID.                           */
int pic_set_kernel_timing(pic_ctx *ctx, int32_t enable);
int pic_kernel_time(pic_ctx *ctx, int32_t kernel_id, double *avg_ms, int64_t *count);

/* Measurement aid (no context): the STREAM triad a = b + scalar * c over n
 * FP64 values (device arrays, n in [1, 2^40)), two consecutive elements per
 * thread as 16-byte accesses when the arrays allow (else one), run
 * once untimed and then `reps` times between two HIP events on `stream`;
 * avg_ms (host out; synchronises) receives the average time per launch.
 * 24 bytes per element over avg_ms is the achievable HBM bandwidth that the
 * stencil sweeps are measured against beside the nominal peak. */
int pic_stream_triad(int64_t n, const double *b, const double *c, double *a, double scalar,
                     int32_t reps, double *avg_ms, void *stream);

/* ---- learned warm start / preconditioner -------------------------------
 * Not in the paper: this library's extension of the PCG solve of Sec. 3.2.
 * A three-level 3-D convolutional U-Net (channels 16-32-64, 3^3 periodic
 * convolutions, 2x2x2 average pooling, nearest up-sampling, additive skips;
 * BF16 weights and activations, FP32 accumulation on the matrix cores) maps a
 * residual r to z = s * NN(h^2 r / s) - mean(.), s = rms(h^2 r), an
 * approximation of A^{-1} r.  PIC_SOLVER_FCG_LEARNED uses it as warm start
 * (kept only if it lowers ||b - A phi||) and as the preconditioner of
 * flexible PCG, falling back to Jacobi-PCG when the flexible iteration stalls.
 * Parameters: FP32, canonical order per layer (e1a 1->16, e1b 16->16,
 * e2a 16->32, e2b 32->32, b3a 32->64, b3b 64->32, d2a 32->32, d2b 32->16,
 * d1a 16->16, out 16->1): weights [cout][cin][3][3][3] (taps dz, dy, dx in
 * -1..1, dx fastest) followed by the bias [cout].                          */

/* Number of FP32 parameters of the network. */
int64_t pic_unet_param_count(void);
/* Load parameters (device, FP32, canonical order) into the context; allocates
 * the context's network buffers on first use (not per call afterwards).     */
int pic_set_unet(pic_ctx *ctx, const float *params, void *stream);
/* z = M(r) on the context's grid (device FP64 arrays of N^3). */
int pic_unet_precondition(pic_ctx *ctx, const double *r, double *z, void *stream);

/* A standalone network on an n^3 grid (n a multiple of 16), for training and
 * for single-network use.  training != 0 adds gradient and Adam buffers.    */
typedef struct pic_net pic_net;
int pic_net_create(int32_t n, int32_t training, pic_net **out);
int pic_net_destroy(pic_net *net);
int pic_net_set_params(pic_net *net, const float *params, void *stream);
int pic_net_get_params(pic_net *net, float *params, void *stream);
/* out = NN(x): x, out device FP32 n^3 (x is rounded to BF16 on entry). */
int pic_net_forward(pic_net *net, const float *x, float *out, void *stream);
/* grads (device FP32, canonical order) of sum(out * dout) at the last
 * forward's input; dout is rounded to BF16 like every convolution output's
 * gradient.  Requires training != 0.                                        */
int pic_net_backward(pic_net *net, const float *dout, float *grads, void *stream);
/* One Adam step (beta 0.9/0.999, eps 1e-8, FP32 master weights) on
 *   L = ||NN(rhs) - target||^2/||target||^2 + lam ||A1 NN(rhs) - rhs||^2/||rhs||^2
 * (A1: unit-spacing periodic 7-point operator); rhs, target device FP32 n^3.
 * loss (host out, nullable) receives L before the step.                    */
int pic_net_train_step(pic_net *net, const float *rhs, const float *target, double lam,
                       double lr, double *loss, void *stream);
/* z = s NN(h^2 r / s) - mean on the network's grid (r, z device FP64). */
int pic_net_precondition(pic_net *net, const double *r, double h, double *z, void *stream);
/* The loss above at (rhs, target) without an update (training != 0); loss:
 * host out. */
int pic_net_loss(pic_net *net, const float *rhs, const float *target, double lam, double *loss,
                 void *stream);
/* A training pair in the network's scale-free form from a solved step:
 * u = h^2 rho (or h^2 (rho - rho_prev)), e = phi (or phi - phi_prev), and with
 * s = rms(u): rhs = u / s, target = e / s (device FP32, n^3 each; rho, phi and
 * the nullable pair rho_prev, phi_prev device FP64).  By linearity of A a step
 * difference is an exact pair too.  scale (host out, nullable) receives s.  */
int pic_net_make_pair(pic_net *net, const double *rho, const double *phi,
                      const double *rho_prev, const double *phi_prev, double h, float *rhs,
                      float *target, double *scale, void *stream);

/* ---- single-layer primitives (3^3 periodic convolution, channels-last) ---
 * x, y, gy: BF16 bit patterns (uint16_t), [z][y][x][C]; gx FP32; weights FP32
 * [co][ci][27] + bias [co].  ci, co in {16, 32, 64} pairs used by the network:
 * (16,16) (16,32) (32,32) (32,64) (64,32) (32,16).                         */
size_t pic_conv3d_frag_elems(int32_t ci, int32_t co);
/* Pack BF16 MFMA fragments: forward (frag_elems(ci, co)) and backward-data
 * (frag_elems(co, ci)) layouts.                                             */
int pic_conv3d_pack(int32_t ci, int32_t co, const float *w, uint16_t *frag_fwd,
                    uint16_t *frag_bwd, void *stream);
/* y = relu?(conv(x) + bias (+ skip)) as BF16. */
int pic_conv3d_fwd(int32_t n, int32_t ci, int32_t co, const uint16_t *x, const uint16_t *frag_fwd,
                   const float *bias, const uint16_t *skip, int32_t relu, uint16_t *y,
                   void *stream);
/* gx (+)= conv^T(gy) in FP32. */
int pic_conv3d_bwd_data(int32_t n, int32_t ci, int32_t co, const uint16_t *gy,
                        const uint16_t *frag_bwd, float *gx, int32_t accumulate, void *stream);
/* grad[co][ci][27] + grad_bias[co] = sum over points (FP32; scratch of
 * pic_conv3d_wgrad_scratch_elems floats).                                   */
size_t pic_conv3d_wgrad_scratch_elems(int32_t n, int32_t ci, int32_t co);
int pic_conv3d_bwd_weight(int32_t n, int32_t ci, int32_t co, const uint16_t *x, const uint16_t *gy,
                          float *scratch, float *grad, void *stream);
/* Adam (Kingma & Ba 2015) on len FP32 parameters, bias-corrected, step >= 1. */
int pic_adam_step(int64_t len, float *theta, float *m, float *v, const float *g, double lr,
                  double beta1, double beta2, double eps, int32_t step, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* PIC_H */
