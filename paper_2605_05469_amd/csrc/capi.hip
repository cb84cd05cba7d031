// capi.hip -- the C ABI declared in include/pic.h: context, validation, and
// the host drivers of the solvers and of the PIC step.
//
// Host drivers only enqueue kernels; every arithmetic step runs on the GPU.
// The CG scalars live in device memory (DevState); the host reads them back
// once every `check_every` iterations to decide whether to launch more.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/pic.h"
#include "net.hpp"
#include "particles.hpp"
#include "fft.hpp"
#include "pif.hpp"
#include "solver_state.hpp"

using namespace pic;

static thread_local std::string g_err;

static int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
static int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

extern "C" int pic_set_error_(int code, const char* msg) { return fail(code, "%s", msg); }

#define HIPCHK(expr)                                                                   \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess)                                                          \
            return fail(PIC_ERR_HIP, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), \
                        __FILE__, __LINE__);                                           \
    } while (0)

#define RETCHK(expr)              \
    do {                          \
        int rc_ = (expr);         \
        if (rc_ < 0) return rc_;  \
    } while (0)

struct pic_ctx {
    pic_params p;
    int device = 0;
    SweepGeo geo;      // the operator A (boundary kind of the box)
    SweepGeo geo_tri;  // SSOR's triangular factors
    int64_t n3 = 0;
    double L = 0, inv_h = 0, inv_h2 = 0, minv = 0, h = 0, h3 = 0, ehalf = 0, qh3 = 0;
    double coef_push = 0, coef_kick = 0;
    float inv_h2f = 0, minvf = 0;
    // device memory
    DevState* st = nullptr;
    DevState* st_host = nullptr;  // pinned mirror
    double* partials = nullptr;
    int npartials = 0;
    double* r = nullptr;
    double* p2[2] = {nullptr, nullptr};
    double* t3 = nullptr;  // 4th scratch vector; r, p2[0], p2[1], t3 also serve the deposit
    float* r32 = nullptr;
    float* d32 = nullptr;
    float* p32[2] = {nullptr, nullptr};
    void* sort_pool = nullptr;
    SortScratch sort{};
    net::Net* net = nullptr;       // learned preconditioner (inference buffers at n)
    double* fz = nullptr;          // flexible CG: z = M(r)
    double* fq = nullptr;          //              q = A p
    double* fw = nullptr;          //              warm-start trial / true residual
    double* sv[6] = {};            // SSOR form: z, q, two forward, one backward, r - A z
    FftPlans* fft = nullptr;       // FFT form: rocFFT plans
    PifState* pif = nullptr;       // PIF form: oversampled grids, spectra, plans
    double2* fspec[2] = {};        //           half spectra (phi_hat, a derivative)
    std::vector<void*> allocs;
    // kernel timing
    bool timing = false;
    std::vector<hipEvent_t> ev;
    double t_sum[4] = {0, 0, 0, 0};  // 0, 1: sweeps; 2, 3: SSOR triangular solves
    int64_t t_cnt[4] = {0, 0, 0, 0};
};

// ------------------------------------------------------------------ helpers --

static bool aligned8(const void* p) { return ((uintptr_t)p & 7u) == 0; }

constexpr int32_t kKnownFlags = PIC_FLAG_NO_WARM_START | PIC_FLAG_WARM_START_ONLY |
                                 PIC_FLAG_MIXED_RELIABLE | PIC_FLAG_LEARNED_MIXED |
                                 PIC_FLAG_FFT_SPECTRAL | PIC_FLAG_SSOR_UNFUSED |
                                 PIC_FLAG_PCG_TWO_SWEEP | PIC_FLAG_PCG_SINGLE_SWEEP;

// The solver forms that take a bounded box: the matrix-free stencil ones.
// The FFT form and the network (periodic convolutions) need the periodic box.
static bool bounded_solver(int32_t solver) {
    return solver == PIC_SOLVER_PCG_FP64 || solver == PIC_SOLVER_PCG_MIXED ||
           solver == PIC_SOLVER_PCG_SSOR;
}

// PIF: the oversampled grid has 2n points per axis; n = 512 takes ~41 GB.
constexpr int kPifMaxModes = 512;

static int validate_params(const pic_params* p) {
    if (!p) return fail(PIC_ERR_INVALID, "params is NULL");
    if (p->n < 32 || p->n > 1024 || (p->n % 32) != 0)
        return fail(PIC_ERR_INVALID, "n = %d: must be a multiple of 32 in [32, 1024]", p->n);
    if (!(p->length > 0.0) || !std::isfinite(p->length))
        return fail(PIC_ERR_INVALID, "length must be positive and finite");
    if (p->np_max < 0 || p->np_max >= ((int64_t)1 << 32))
        return fail(PIC_ERR_INVALID, "np_max must be in [0, 2^32)");
    if (!(p->rtol > 0.0) || !std::isfinite(p->rtol)) return fail(PIC_ERR_INVALID, "rtol must be > 0");
    if (p->max_iter < 0) return fail(PIC_ERR_INVALID, "max_iter must be >= 0");
    if (p->max_inner < 1 || p->max_outer < 0)
        return fail(PIC_ERR_INVALID, "max_inner must be >= 1 and max_outer >= 0");
    if (p->solver < PIC_SOLVER_PCG_FP64 || p->solver > PIC_SOLVER_PIF)
        return fail(PIC_ERR_INVALID, "unknown solver %d", p->solver);
    if (p->pif_tol != 0.0 && pif_width(p->pif_tol) == 0)
        return fail(PIC_ERR_INVALID, "pif_tol must be in [1e-7, 1e-2] (0: default 1e-4)");
    if (p->solver == PIC_SOLVER_PIF && p->n > kPifMaxModes)
        return fail(PIC_ERR_INVALID, "PIF: at most %d modes per axis", kPifMaxModes);
    if (!(p->ssor_omega >= 0.0 && p->ssor_omega < 2.0) || p->ssor_inner < 0 || p->ssor_outer < 0)
        return fail(PIC_ERR_INVALID, "ssor_omega must be in (0, 2) (0: default), "
                                     "ssor_inner and ssor_outer >= 0 (0: default)");
    if (!std::isfinite(p->charge) || !std::isfinite(p->qm) || !std::isfinite(p->dt) ||
        !std::isfinite(p->rho_bg))
        return fail(PIC_ERR_INVALID, "charge, qm, dt and rho_bg must be finite");
    if (p->flags & ~kKnownFlags) return fail(PIC_ERR_INVALID, "unknown flags 0x%x", p->flags);
    if (p->bc < PIC_BC_PERIODIC || p->bc > PIC_BC_NEUMANN)
        return fail(PIC_ERR_INVALID, "unknown boundary kind %d", p->bc);
    if (p->bc != PIC_BC_PERIODIC && !bounded_solver(p->solver))
        return fail(PIC_ERR_INVALID, "solver %d needs the periodic box (bounded boxes: "
                                     "PCG_FP64, PCG_MIXED, PCG_SSOR)", p->solver);
    return PIC_OK;
}

static size_t vec_bytes(int64_t n3, size_t elem) { return ((size_t)n3 * elem + 255) & ~(size_t)255; }

static size_t base_bytes(const pic_params* p) {
    const int64_t n3 = (int64_t)p->n * p->n * p->n;
    int np = max_sweep_blocks();
    if (np < 2 * deposit_partials()) np = 2 * deposit_partials();
    size_t b = 0;
    b += 4096;                               // DevState
    b += (size_t)4 * np * sizeof(double);    // partials
    b += 4 * vec_bytes(n3, 8);               // r, p[2], t3
    return b;
}

static size_t mixed_bytes(const pic_params* p) {
    const int64_t n3 = (int64_t)p->n * p->n * p->n;
    return 4 * vec_bytes(n3, 4);
}

static int dev_alloc(pic_ctx* c, void** out, size_t bytes) {
    void* ptr = nullptr;
    hipError_t e = hipMalloc(&ptr, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(PIC_ERR_NOMEM, "hipMalloc(%zu bytes) failed: %s", bytes, hipGetErrorString(e));
    }
    c->allocs.push_back(ptr);
    *out = ptr;
    return PIC_OK;
}

// The sort's particle records (64 bytes per particle) are allocated by the
// first call that sorts (a context that only deposits and solves never
// needs them).
static int ensure_rec(pic_ctx* c) {
    if (c->sort.rec || c->p.np_max <= 0) return PIC_OK;
    void* m = nullptr;
    RETCHK(dev_alloc(c, &m, sort_rec_bytes(c->p.np_max)));
    c->sort.rec = (double2*)m;
    return PIC_OK;
}

static int ensure_mixed(pic_ctx* c) {
    if (c->r32) return PIC_OK;
    void* m = nullptr;
    RETCHK(dev_alloc(c, &m, mixed_bytes(&c->p)));
    char* q = (char*)m;
    const size_t vb = vec_bytes(c->n3, 4);
    c->r32 = (float*)q;
    c->d32 = (float*)(q + vb);
    c->p32[0] = (float*)(q + 2 * vb);
    c->p32[1] = (float*)(q + 3 * vb);
    return PIC_OK;
}

static size_t learned_bytes(const pic_params* p) {
    const int64_t n3 = (int64_t)p->n * p->n * p->n;
    return 3 * vec_bytes(n3, 8);
}

static int ensure_learned(pic_ctx* c) {
    if (c->fz) return PIC_OK;
    void* m = nullptr;
    RETCHK(dev_alloc(c, &m, learned_bytes(&c->p)));
    const size_t vb = vec_bytes(c->n3, 8);
    c->fz = (double*)m;
    c->fq = (double*)((char*)m + vb);
    c->fw = (double*)((char*)m + 2 * vb);
    return PIC_OK;
}

static size_t ssor_bytes(const pic_params* p) {
    const int64_t n3 = (int64_t)p->n * p->n * p->n;
    return 6 * vec_bytes(n3, 8);
}

static int ensure_ssor(pic_ctx* c) {
    if (c->sv[0]) return PIC_OK;
    void* m = nullptr;
    RETCHK(dev_alloc(c, &m, ssor_bytes(&c->p)));
    const size_t vb = vec_bytes(c->n3, 8);
    for (int i = 0; i < 6; ++i) c->sv[i] = (double*)((char*)m + i * vb);
    return PIC_OK;
}

// FFT form: two half spectra (the transforms' own work buffer is rocFFT's).
static size_t fft_bytes(const pic_params* p) {
    const int64_t nspec = (int64_t)(p->n / 2 + 1) * p->n * p->n;
    return 2 * vec_bytes(nspec, 16);
}

// PIF form: oversampled grids, spectra and plans of its own (pif.hip).
static int ensure_pif(pic_ctx* c) {
    if (c->pif) return PIC_OK;
    const int rc = pif_create(&c->pif, c->p.n, c->L, c->p.pif_tol);
    if (rc) {
        c->pif = nullptr;
        return fail(rc == -3 ? PIC_ERR_NOMEM : PIC_ERR_HIP, "PIF buffers: %s", pif_last_error());
    }
    return PIC_OK;
}

static int ensure_fft(pic_ctx* c) {
    if (c->fft) return PIC_OK;
    void* m = nullptr;
    RETCHK(dev_alloc(c, &m, fft_bytes(&c->p)));
    const int64_t nspec = (int64_t)(c->p.n / 2 + 1) * c->p.n * c->p.n;
    c->fspec[0] = (double2*)m;
    c->fspec[1] = (double2*)((char*)m + vec_bytes(nspec, 16));
    if (fft_create(&c->fft, c->p.n)) {
        c->fft = nullptr;
        return fail(PIC_ERR_HIP, "FFT plans: %s", fft_last_error());
    }
    return PIC_OK;
}

// The deposit's four n^3 scratch arrays: the solver vectors, free between solves.
struct DepScratch {
    double* t[4];
    operator double* const*() const { return t; }
};
static DepScratch dep_scratch(pic_ctx* c) { return DepScratch{{c->r, c->p2[0], c->p2[1], c->t3}}; }

static int read_state(pic_ctx* c, hipStream_t s) {
    HIPCHK(hipMemcpyAsync(c->st_host, c->st, sizeof(DevState), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return PIC_OK;
}

// ---------------------------------------------------------------- kernels --

__global__ void state_init_kernel(DevState* st, int32_t outer_state) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        st->outer_state = outer_state;
        st->gap_restarts = 0;
        st->cg.state = CG_RUNNING;
        st->cg.iter = 0;
        st->cg.replacements = 0;
    }
}

// --------------------------------------------------------------- timing ----

static void timing_reset(pic_ctx* c) {
    for (int j = 0; j < 4; ++j) {
        c->t_sum[j] = 0;
        c->t_cnt[j] = 0;
    }
}

static int timing_events(pic_ctx* c, size_t need) {
    while (c->ev.size() < need) {
        hipEvent_t e;
        HIPCHK(hipEventCreate(&e));
        c->ev.push_back(e);
    }
    return PIC_OK;
}

// Kernel timing samples every kTimeStride-th iteration of a batch (events
// between every launch would perturb what they measure).
constexpr int kTimeStride = 4;
static bool timed_iter(const pic_ctx* c, int k) { return c->timing && (k % kTimeStride) == 0; }

// Accumulate the sampled pairs among the first `valid` iterations of a batch.
static int timing_collect(pic_ctx* c, int launched, int64_t valid) {
    for (int k = 0; k < launched && k < valid; k += kTimeStride) {
        for (int j = 0; j < 2; ++j) {
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, c->ev[4 * k + 2 * j], c->ev[4 * k + 2 * j + 1]));
            c->t_sum[j] += ms;
            c->t_cnt[j] += 1;
        }
    }
    return PIC_OK;
}

// ------------------------------------------------------------- FP64 PCG ----

static bool use_cg1(const pic_ctx* c) {
    return !(c->p.flags & PIC_FLAG_PCG_TWO_SWEEP) && cg1_supported(c->geo);
}

// Single-reduction form: batches of one sweep per iteration.  The residual
// and the direction alternate between two buffers each (a sweep never writes
// what neighbouring workgroups read as halo); sweeps queued after the state
// left RUNNING return at once, and every (re)computed residual lands in c->r
// and restarts the recurrence, so the host's buffer parity only matters while
// RUNNING.  Timing samples go to slot 0.
// x is updated every other sweep (xm 1 / 2 alternate, starting with 1 after
// every (re)start); a step left pending when the state leaves RUNNING is
// applied (launch_cg1_flush) before x is used: the true residual of a
// candidate, or the caller's iterate.  Timing samples the two sweeps of a
// pair alike (k mod 4 = 0 and 1), so their average is the mean sweep.
static int pcg64_iterate_cg1(pic_ctx* c, const double* b, double* x, hipStream_t s) {
    const SweepGeo& g = c->geo;
    const int K = c->p.check_every > 0 ? c->p.check_every : 16;
    double* rb[2] = {c->r, c->t3};
    int rcur = 0, pcur = 0, xm = 1;
    auto timed = [c](int k) { return c->timing && (k % kTimeStride) < 2; };
    if (c->timing) RETCHK(timing_events(c, (size_t)4 * K));
    HIPCHK(launch_cg1_start(g, c->r, c->minv, c->inv_h2, c->st, c->partials, s));
    for (;;) {
        CgScalars& cg = c->st_host->cg;
        if (cg.state == CG_RUNNING) {
            const int64_t it0 = cg.iter;
            for (int k = 0; k < K; ++k) {
                if (timed(k)) HIPCHK(hipEventRecord(c->ev[4 * k + 0], s));
                HIPCHK(launch_cg1(g, rb[rcur], rb[rcur ^ 1], c->p2[pcur], c->p2[pcur ^ 1], x,
                                  c->minv, c->inv_h2, c->st, c->partials, xm, pcur ^ 1, s));
                if (timed(k)) HIPCHK(hipEventRecord(c->ev[4 * k + 1], s));
                rcur ^= 1;
                pcur ^= 1;
                xm = xm == 1 ? 2 : 1;
            }
            RETCHK(read_state(c, s));
            if (c->timing) {
                const int64_t valid = c->st_host->cg.iter - it0;
                for (int k = 0; k < K && k < valid; ++k) {
                    if (!timed(k)) continue;
                    float ms = 0.f;
                    HIPCHK(hipEventElapsedTime(&ms, c->ev[4 * k], c->ev[4 * k + 1]));
                    c->t_sum[0] += ms;
                    c->t_cnt[0] += 1;
                }
            }
            if (c->st_host->cg.state == CG_RUNNING && c->st_host->cg.iter == it0)
                return fail(PIC_ERR_STATE, "solver made no progress (iteration %lld)",
                            (long long)it0);
            continue;
        }
        if (cg.xpend) HIPCHK(launch_cg1_flush(c->n3, c->p2[0], c->p2[1], x, c->st, s));
        if (cg.state == CG_CANDIDATE) {
            HIPCHK(launch_residual64(g, b, x, c->r, c->minv, c->inv_h2, 0, c->p.rtol, c->p.max_iter,
                                     c->st, c->partials, s));
            HIPCHK(launch_cg1_start(g, c->r, c->minv, c->inv_h2, c->st, c->partials, s));
            rcur = 0;
            xm = 1;
            RETCHK(read_state(c, s));
            continue;
        }
        if (cg.xpend) RETCHK(read_state(c, s));
        return PIC_OK;  // CONVERGED, MAXIT, BREAKDOWN, ZERO_RHS
    }
}

// s-step form: batches of (Gram sweep, update sweep) pairs, each pair up to
// kSstepS iterations; p and r alternate between two buffers each (the
// update sweep reads both as halos while writing the new ones).  Every
// (re)computed residual lands in c->r with the restart flag set, which makes
// the next Gram sweep take p = M^{-1} r.  Timing: slot 0 Gram, slot 1 update.
static bool use_sstep(const pic_ctx* c) {
    return !(c->p.flags & (PIC_FLAG_PCG_TWO_SWEEP | PIC_FLAG_PCG_SINGLE_SWEEP)) &&
           sstep_supported(c->geo);
}

static int pcg64_iterate_sstep(pic_ctx* c, const double* b, double* x, hipStream_t s) {
    const SweepGeo& g = c->geo;
    const int K = c->p.check_every > 0 ? (c->p.check_every + kSstepS - 1) / kSstepS : 8;
    double* rb[2] = {c->r, c->t3};
    const int npart = 4 * c->npartials;
    int cur = 0;
    if (c->timing) RETCHK(timing_events(c, (size_t)4 * K));
    for (;;) {
        CgScalars& cg = c->st_host->cg;
        if (cg.state == CG_RUNNING) {
            const int64_t it0 = cg.iter;
            for (int k = 0; k < K; ++k) {
                const bool tm = timed_iter(c, k);
                if (tm) HIPCHK(hipEventRecord(c->ev[4 * k + 0], s));
                HIPCHK(launch_sstep(g, 0, rb[cur], c->p2[cur], nullptr, nullptr, x, c->minv,
                                    c->st, c->partials, npart, s));
                if (tm) HIPCHK(hipEventRecord(c->ev[4 * k + 1], s));
                if (tm) HIPCHK(hipEventRecord(c->ev[4 * k + 2], s));
                HIPCHK(launch_sstep(g, 1, rb[cur], c->p2[cur], rb[cur ^ 1], c->p2[cur ^ 1], x,
                                    c->minv, c->st, c->partials, npart, s));
                if (tm) HIPCHK(hipEventRecord(c->ev[4 * k + 3], s));
                cur ^= 1;
            }
            RETCHK(read_state(c, s));
            if (c->timing) RETCHK(timing_collect(c, K, (c->st_host->cg.iter - it0 + kSstepS - 1) / kSstepS));
            // (a batch may end on an outer step that only set up a restart)
            if (c->st_host->cg.state == CG_RUNNING && c->st_host->cg.iter == it0 &&
                !c->st_host->cg.restart)
                return fail(PIC_ERR_STATE, "solver made no progress (iteration %lld)",
                            (long long)it0);
            continue;
        }
        if (cg.state == CG_CANDIDATE) {
            HIPCHK(launch_residual64(g, b, x, c->r, c->minv, c->inv_h2, 0, c->p.rtol, c->p.max_iter,
                                     c->st, c->partials, s));
            cur = 0;
            RETCHK(read_state(c, s));
            continue;
        }
        return PIC_OK;  // CONVERGED, MAXIT, BREAKDOWN, ZERO_RHS
    }
}

// Runs batches of (direction, update) sweeps until the device state leaves
// RUNNING; handles candidate verification (residual replacement).
static int pcg64_iterate(pic_ctx* c, const double* b, double* x, hipStream_t s) {
    if (use_sstep(c)) return pcg64_iterate_sstep(c, b, x, s);
    if (use_cg1(c)) return pcg64_iterate_cg1(c, b, x, s);
    const SweepGeo& g = c->geo;
    const int K = c->p.check_every > 0 ? c->p.check_every : 16;
    int cur = 0;
    if (c->timing) RETCHK(timing_events(c, (size_t)4 * K));
    for (;;) {
        CgScalars& cg = c->st_host->cg;
        if (cg.state == CG_RUNNING) {
            const int64_t it0 = cg.iter;
            for (int k = 0; k < K; ++k) {
                if (timed_iter(c, k)) HIPCHK(hipEventRecord(c->ev[4 * k + 0], s));
                HIPCHK(launch_dir64(g, c->r, c->p2[cur], c->p2[cur ^ 1], c->minv, c->inv_h2, c->st,
                                    c->partials, s));
                if (timed_iter(c, k)) HIPCHK(hipEventRecord(c->ev[4 * k + 1], s));
                if (timed_iter(c, k)) HIPCHK(hipEventRecord(c->ev[4 * k + 2], s));
                HIPCHK(launch_upd64(g, c->p2[cur ^ 1], x, c->r, c->minv, c->inv_h2, c->st,
                                    c->partials, s));
                if (timed_iter(c, k)) HIPCHK(hipEventRecord(c->ev[4 * k + 3], s));
                cur ^= 1;
            }
            RETCHK(read_state(c, s));
            if (c->timing) RETCHK(timing_collect(c, K, c->st_host->cg.iter - it0));
            if (c->st_host->cg.state == CG_RUNNING && c->st_host->cg.iter == it0)
                return fail(PIC_ERR_STATE, "solver made no progress (iteration %lld)",
                            (long long)it0);
            continue;
        }
        if (cg.state == CG_CANDIDATE) {
            HIPCHK(launch_residual64(g, b, x, c->r, c->minv, c->inv_h2, 0, c->p.rtol, c->p.max_iter,
                                     c->st, c->partials, s));
            RETCHK(read_state(c, s));
            continue;
        }
        return PIC_OK;  // CONVERGED, MAXIT, BREAKDOWN, ZERO_RHS
    }
}

static int solve_fp64(pic_ctx* c, const double* b, double* x, pic_solve_info* out, hipStream_t s,
                      int64_t max_iter = -1) {
    const SweepGeo& g = c->geo;
    if (max_iter < 0) max_iter = c->p.max_iter;
    HIPCHK(launch_residual64(g, b, x, c->r, c->minv, c->inv_h2, 1, c->p.rtol, max_iter, c->st,
                             c->partials, s));
    RETCHK(read_state(c, s));
    if (c->st_host->cg.state == CG_ZERO_RHS) {
        HIPCHK(launch_fill(c->n3, x, 0.0, s));
    } else {
        RETCHK(pcg64_iterate(c, b, x, s));
    }
    const CgScalars& cg = c->st_host->cg;
    out->iterations = cg.iter;
    out->replacements = cg.replacements;
    out->norm_b = cg.nb;
    if (cg.state == CG_CONVERGED || cg.state == CG_ZERO_RHS) {
        out->converged = 1;
        out->rel_res = cg.nb > 0 ? cg.true_rn / cg.nb : 0.0;
    } else {
        // report the true residual of the last iterate (2 = report only)
        HIPCHK(launch_residual64(g, b, x, c->r, c->minv, c->inv_h2, 2, c->p.rtol, c->p.max_iter,
                                 c->st, c->partials, s));
        RETCHK(read_state(c, s));
        out->converged = 0;
        out->rel_res = c->st_host->cg.true_rn / c->st_host->cg.nb;
    }
    return PIC_OK;
}

// ---------------------------------------------------------- mixed form -----
// FP32 inner Jacobi-PCG inside FP64 iterative refinement (not in the paper).
// The refinement loop ends when the FP64 true residual meets the tolerance,
// after max_outer refinements, or when kMixedStall refinements in a row fail
// to bring it below kMixedProgress times the smallest so far; FP64 Jacobi-PCG
// (max_iter iterations) then finishes from the current iterate.
constexpr int kMixedStall = 3;
constexpr double kMixedProgress = 0.9;

static int solve_mixed(pic_ctx* c, const double* b, double* x, pic_solve_info* out, hipStream_t s) {
    RETCHK(ensure_mixed(c));
    const SweepGeo& g = c->geo;
    const bool one = use_cg1(c);
    const int K = c->p.check_every > 0 ? c->p.check_every : 16;
    HIPCHK(launch_sum(c->n3, b, c->st, c->partials, 1, s));
    hipLaunchKernelGGL(state_init_kernel, dim3(1), dim3(64), 0, s, c->st, (int32_t)CG_RUNNING);
    HIPCHK(hipGetLastError());
    RETCHK(read_state(c, s));
    const double nb = std::sqrt(c->st_host->bb);
    out->norm_b = nb;
    if (nb == 0.0) {
        HIPCHK(launch_fill(c->n3, x, 0.0, s));
        out->converged = 1;
        out->rel_res = 0.0;
        return PIC_OK;
    }
    const double tol = c->p.rtol * nb;
    int64_t outer = 0, inner_total = 0;
    int cur = 0;
    // progress stop: a refinement makes progress when its true residual falls
    // below kMixedProgress times the smallest so far; after kMixedStall
    // refinements in a row without progress FP64 Jacobi-PCG finishes the solve
    double best = 0.0;
    int stall = 0;
    bool switched = false;
    if (c->timing) RETCHK(timing_events(c, (size_t)4 * K));
    for (;;) {
        if (outer > 0) HIPCHK(launch_update_x(c->n3, x, c->d32, c->st, s));
        HIPCHK(launch_outer_resid(g, b, x, c->r, c->inv_h2, c->st, c->partials, tol, s));
        RETCHK(read_state(c, s));
        const double nr = c->st_host->out_nr;
        if (!std::isfinite(nr)) break;
        if (nr <= tol) {
            out->converged = 1;
            break;
        }
        if (outer == 0 || nr < kMixedProgress * best) {
            best = nr;
            stall = 0;
        } else if (++stall >= kMixedStall) {
            switched = true;
            break;
        }
        if (outer >= c->p.max_outer) break;
        ++outer;
        HIPCHK(launch_convert32(c->n3, c->r, c->r32, c->d32, c->minvf,
                                (c->p.flags & PIC_FLAG_MIXED_RELIABLE) ? 1 : 0, c->p.inner_rtol,
                                c->p.max_inner, c->st, c->partials, s));
        RETCHK(read_state(c, s));
        // single-reduction inner sweeps: the residual alternates between r32
        // and the (here unused) FP64 scratch vector viewed as FP32; a fresh
        // inner solve starts with the start reduction, a continued one with
        // a direction sweep (the carried direction and its exact curvature)
        float* rb32[2] = {c->r32, (float*)c->t3};
        int rcur = 0, pgiven = 0;
        if (one && c->st_host->cg.state == CG_RUNNING) {
            if (c->st_host->cg.restart) {
                HIPCHK(launch_cg1_start32(g, c->r32, c->minvf, c->inv_h2f, c->st, c->partials, s));
            } else {
                HIPCHK(launch_dir32(g, c->r32, c->p32[cur], c->p32[cur ^ 1], c->minvf, c->inv_h2f,
                                    c->st, c->partials, s));
                cur ^= 1;
                pgiven = 1;
            }
        }
        const int cur0 = cur;
        // single-reduction inner sweeps update d every other iteration (as the
        // FP64 solve updates x); both sweeps of a pair are timing samples
        int xm = 1;
        auto timed1 = [c](int k) { return c->timing && (k % kTimeStride) < 2; };
        while (c->st_host->cg.state == CG_RUNNING) {
            const int64_t it0 = c->st_host->cg.iter;
            for (int k = 0; k < K; ++k) {
                if (one) {
                    if (timed1(k)) HIPCHK(hipEventRecord(c->ev[4 * k + 0], s));
                    HIPCHK(launch_cg1_32(g, rb32[rcur], rb32[rcur ^ 1], c->p32[cur], c->p32[cur ^ 1],
                                         c->d32, c->minvf, c->inv_h2f, pgiven, c->st, c->partials,
                                         xm, cur ^ 1, s));
                    if (timed1(k)) HIPCHK(hipEventRecord(c->ev[4 * k + 1], s));
                    pgiven = 0;
                    rcur ^= 1;
                    cur ^= 1;
                    xm = xm == 1 ? 2 : 1;
                    continue;
                }
                if (timed_iter(c, k)) HIPCHK(hipEventRecord(c->ev[4 * k + 0], s));
                HIPCHK(launch_dir32(g, c->r32, c->p32[cur], c->p32[cur ^ 1], c->minvf, c->inv_h2f,
                                    c->st, c->partials, s));
                if (timed_iter(c, k)) HIPCHK(hipEventRecord(c->ev[4 * k + 1], s));
                if (timed_iter(c, k)) HIPCHK(hipEventRecord(c->ev[4 * k + 2], s));
                HIPCHK(launch_upd32(g, c->p32[cur ^ 1], c->d32, c->r32, c->minvf, c->inv_h2f, c->st,
                                    c->partials, s));
                if (timed_iter(c, k)) HIPCHK(hipEventRecord(c->ev[4 * k + 3], s));
                cur ^= 1;
            }
            RETCHK(read_state(c, s));
            if (c->timing) {
                const int64_t valid = c->st_host->cg.iter - it0;
                if (one) {
                    for (int k = 0; k < K && k < valid; ++k) {
                        if (!timed1(k)) continue;
                        float ms = 0.f;
                        HIPCHK(hipEventElapsedTime(&ms, c->ev[4 * k], c->ev[4 * k + 1]));
                        c->t_sum[0] += ms;
                        c->t_cnt[0] += 1;
                    }
                } else {
                    RETCHK(timing_collect(c, K, valid));
                }
            }
            if (c->st_host->cg.state == CG_RUNNING && c->st_host->cg.iter == it0)
                return fail(PIC_ERR_STATE, "inner solver made no progress");
        }
        // the last odd sweep's step, if pending, before d is used
        if (one && c->st_host->cg.xpend)
            HIPCHK(launch_cg1_flush32(c->n3, c->p32[0], c->p32[1], c->d32, c->st, s));
        inner_total += c->st_host->cg.iter;
        // the last direction written (the next inner solve may continue it):
        // each active iteration's direction sweep (or single sweep) wrote
        // p32[cur ^ 1]
        cur = cur0 ^ (int)(c->st_host->cg.iter & 1);
        if (c->st_host->cg.state == CG_BREAKDOWN) {
            // an FP32 breakdown still leaves a usable correction; the next outer
            // residual decides, and the step cap bounds the loop
        }
    }
    out->iterations = inner_total;
    out->outer_iterations = outer;
    out->rel_res = c->st_host->out_nr / nb;
    out->gap_restarts = c->st_host->gap_restarts;
    if (switched) {
        pic_solve_info pi;
        std::memset(&pi, 0, sizeof pi);
        RETCHK(solve_fp64(c, b, x, &pi, s));
        out->fell_back = 1;
        out->fp64_iterations = pi.iterations;
        out->iterations = inner_total + pi.iterations;
        out->replacements += pi.replacements;
        out->rel_res = pi.rel_res;
        out->converged = pi.converged;
    }
    return PIC_OK;
}

// -------------------------------------------------- learned (flexible) ----
// Flexible PCG (Notay 2000; Golub & Ye 1999) with the network preconditioner
// z = M(r) = s NN(h^2 r / s) - mean, an optional network warm start, and a
// permanent switch to Jacobi-PCG from the current iterate when the flexible
// iteration stalls: (z.r) <= 0, anything non-finite, or no 1% improvement of
// the best ||r|| over `fcg_window` iterations.  The PCG residual test decides
// convergence either way.
static int fcg_precond(pic_ctx* c, const double* r, double* z, hipStream_t s) {
    if (!c->net) return fail(PIC_ERR_STATE, "no network loaded (pic_set_unet)");
    const int rc = net::precondition(c->net, r, c->h * c->h, z, s);
    if (rc) return fail(PIC_ERR_HIP, "network: %s", net::last_error());
    return PIC_OK;
}

// The non-learned solve the learned form hands over to (after the warm start
// with PIC_FLAG_WARM_START_ONLY, or on fallback): Jacobi-PCG, or the mixed
// form with PIC_FLAG_LEARNED_MIXED (its step cap is max_outer x max_inner).
static int continue_plain(pic_ctx* c, const double* b, double* x, pic_solve_info* out,
                          hipStream_t s, int64_t max_iter) {
    if (c->p.flags & PIC_FLAG_LEARNED_MIXED) return solve_mixed(c, b, x, out, s);
    return solve_fp64(c, b, x, out, s, max_iter);
}

static int solve_learned(pic_ctx* c, const double* b, double* x, pic_solve_info* out,
                         hipStream_t s) {
    RETCHK(ensure_learned(c));
    if (!c->net) return fail(PIC_ERR_STATE, "no network loaded (pic_set_unet)");
    const SweepGeo& g = c->geo;
    const int64_t n3 = c->n3;
    // r = b - A x, ||b||, threshold (the residual kernel's init mode)
    HIPCHK(launch_residual64(g, b, x, c->r, c->minv, c->inv_h2, 1, c->p.rtol, c->p.max_iter, c->st,
                             c->partials, s));
    RETCHK(read_state(c, s));
    const double nb = c->st_host->cg.nb, tol = c->st_host->cg.tol;
    out->norm_b = nb;
    if (c->st_host->cg.state == CG_ZERO_RHS) {
        HIPCHK(launch_fill(n3, x, 0.0, s));
        out->converged = 1;
        return PIC_OK;
    }
    double rn = c->st_host->cg.true_rn;
    if (rn <= tol) {
        out->converged = 1;
        out->rel_res = rn / nb;
        return PIC_OK;
    }
    // warm start: x + M(r), kept only if it lowers the true residual
    if (!(c->p.flags & PIC_FLAG_NO_WARM_START)) {
        RETCHK(fcg_precond(c, c->r, c->fz, s));
        HIPCHK(launch_axpy_copy(n3, x, c->fz, c->fw, s));
        HIPCHK(launch_resid_norm(g, b, c->fw, c->fq, c->inv_h2, c->st, c->partials, s));
        RETCHK(read_state(c, s));
        const double rw = c->st_host->out_nr;
        if (std::isfinite(rw) && rw < rn) {
            HIPCHK(launch_copy(n3, c->fw, x, s));
            HIPCHK(launch_copy(n3, c->fq, c->r, s));
            rn = rw;
            out->warm_start_used = 1;
            if (rn <= tol) {
                out->converged = 1;
                out->rel_res = rn / nb;
                return PIC_OK;
            }
        }
    }
    if (c->p.flags & PIC_FLAG_WARM_START_ONLY) {
        // warm start only: Jacobi-PCG (or the mixed form) from the iterate
        pic_solve_info pi;
        std::memset(&pi, 0, sizeof pi);
        RETCHK(continue_plain(c, b, x, &pi, s, c->p.max_iter));
        out->iterations = pi.iterations;
        out->outer_iterations = pi.outer_iterations;
        out->replacements += pi.replacements;
        out->rel_res = pi.rel_res;
        out->converged = pi.converged;
        return PIC_OK;
    }
    double* p = c->p2[0];
    int64_t it = 0;
    bool flexible = true;
    double best = rn;
    int since = 0;
    RETCHK(fcg_precond(c, c->r, c->fz, s));
    HIPCHK(launch_fcg_dots(n3, c->fz, c->r, c->r, c->st, c->partials, s));
    RETCHK(read_state(c, s));
    double rz = c->st_host->flex_zr;
    if (!(rz > 0.0) || !std::isfinite(rz)) flexible = false;
    if (flexible) HIPCHK(launch_copy(n3, c->fz, p, s));
    while (flexible && it < c->p.max_iter) {
        HIPCHK(launch_aq(g, p, c->fq, c->inv_h2, c->st, c->partials, s));
        RETCHK(read_state(c, s));
        const double pq = c->st_host->flex_pq;
        const double alpha = rz / pq;
        if (!std::isfinite(alpha) || !(pq > 0.0)) {
            flexible = false;
            break;
        }
        HIPCHK(launch_fcg_update(n3, x, c->r, p, c->fq, alpha, c->st, c->partials, s));
        RETCHK(read_state(c, s));
        ++it;
        double rr = std::sqrt(c->st_host->flex_rr);
        if (!std::isfinite(rr)) {
            flexible = false;
            break;
        }
        if (rr <= tol) {
            // verify with the true residual (into fw); replace r if it fails
            HIPCHK(launch_resid_norm(g, b, x, c->fw, c->inv_h2, c->st, c->partials, s));
            RETCHK(read_state(c, s));
            if (c->st_host->out_nr <= tol) {
                out->converged = 1;
                out->iterations = it;
                out->flex_iterations = it;
                out->rel_res = c->st_host->out_nr / nb;
                return PIC_OK;
            }
            HIPCHK(launch_copy(n3, c->fw, c->r, s));
            rr = c->st_host->out_nr;
            out->replacements += 1;
        }
        if (rr < 0.99 * best) {
            best = rr;
            since = 0;
        } else if (++since >= c->p.fcg_window) {
            flexible = false;
            break;
        }
        RETCHK(fcg_precond(c, c->r, c->fz, s));
        HIPCHK(launch_fcg_dots(n3, c->fz, c->r, c->fq, c->st, c->partials, s));
        RETCHK(read_state(c, s));
        const double zr = c->st_host->flex_zr, zq = c->st_host->flex_zq;
        if (!(zr > 0.0) || !std::isfinite(zr) || !std::isfinite(zq)) {
            flexible = false;
            break;
        }
        HIPCHK(launch_xpby(n3, c->fz, p, -zq / pq, s));
        rz = zr;
    }
    out->flex_iterations = it;
    if (it >= c->p.max_iter) {
        HIPCHK(launch_resid_norm(g, b, x, c->fw, c->inv_h2, c->st, c->partials, s));
        RETCHK(read_state(c, s));
        out->iterations = it;
        out->rel_res = c->st_host->out_nr / nb;
        out->converged = out->rel_res <= c->p.rtol;
        return PIC_OK;
    }
    // fallback: Jacobi-PCG (or the mixed form) from the current iterate
    out->fell_back = 1;
    pic_solve_info pi;
    std::memset(&pi, 0, sizeof pi);
    RETCHK(continue_plain(c, b, x, &pi, s, c->p.max_iter - it));
    out->iterations = it + pi.iterations;
    out->outer_iterations = pi.outer_iterations;
    out->replacements += pi.replacements;
    out->rel_res = pi.rel_res;
    out->converged = pi.converged;
    return PIC_OK;
}

// ------------------------------------------------------------- SSOR form --
// The paper's preconditioner (Sec. 4.1: SSOR, four inner and two outer
// iterations, damping pi/2), matrix-free: one application is
//   y_0 = D^-1 r,  y_{j+1} = D^-1 r + (w/6) (y_j[i-ex] + y_j[i-ey] + y_j[i-ez]),
//   z_0 = y,       z_{j+1} = y + (w/6) (z_j[i+ex] + z_j[i+ey] + z_j[i+ez]),
//   z = w (2 - w) z_inner,
// j < inner (Jacobi steps for the cyclic triangular solves), each step one
// z-marching half-stencil sweep; `outer` stationary steps add SSOR(r - A z).
// The last sweep of the application reduces r . z for PCG.  By default each
// triangular solve (all its inner steps) is one fused z-march; with
// PIC_FLAG_SSOR_UNFUSED every step is a sweep of its own (same values of z).
// Buffers: sv[2], sv[3] forward ping-pong, sv[4] backward, sv[5] = r - A z.
static int ssor_once(pic_ctx* c, const double* rhs, double* out, const double* add,
                     const double* rdot, hipStream_t s, bool timed = false) {
    const SweepGeo& g = c->geo_tri;
    const int bounded = c->p.bc != PIC_BC_PERIODIC;
    const int k = c->p.ssor_inner;
    const double w = c->p.ssor_omega;
    const double cc = w / 6.0, dinv = c->minv, sc = w * (2.0 - w);
    if (!(c->p.flags & PIC_FLAG_SSOR_UNFUSED) && ssor_fused_supported(c->p.n, k)) {
        // timed: events 4..7 around the two solves (read by ssor_timing_collect)
        if (timed) HIPCHK(hipEventRecord(c->ev[4], s));
        HIPCHK(launch_ssor_fused(c->p.n, bounded, k, 0, rhs, nullptr, nullptr, c->sv[2], dinv, cc,
                                 1.0, c->st, c->partials, s));
        if (timed) HIPCHK(hipEventRecord(c->ev[5], s));
        if (timed) HIPCHK(hipEventRecord(c->ev[6], s));
        HIPCHK(launch_ssor_fused(c->p.n, bounded, k, 1, c->sv[2], add, rdot, out, 1.0, cc, sc,
                                 c->st, c->partials, s));
        if (timed) HIPCHK(hipEventRecord(c->ev[7], s));
        return PIC_OK;
    }
    double* ya = c->sv[2];
    double* yb = c->sv[3];
    const double* stage = rhs;
    double sscale = dinv;
    double* dst = ya;
    for (int j = 0; j < k; ++j) {
        dst = (j & 1) ? yb : ya;
        HIPCHK(launch_ssor_half(g, stage, rhs, nullptr, nullptr, dst, cc, dinv, sscale, 1.0, 0,
                                c->st, c->partials, s));
        stage = dst;
        sscale = 1.0;
    }
    double* Y = dst;                       // y_inner
    double* other = (Y == ya) ? yb : ya;   // free forward buffer
    double* zb[2] = {c->sv[4], other};
    stage = Y;
    for (int j = 0; j < k; ++j) {
        const bool last = j + 1 == k;
        double* d = last ? out : zb[j & 1];
        HIPCHK(launch_ssor_half(g, stage, Y, last ? add : nullptr, last ? rdot : nullptr, d, cc, 1.0,
                                1.0, last ? sc : 1.0, 1, c->st, c->partials, s));
        stage = d;
    }
    return PIC_OK;
}

// z = SSOR^outer(r); r . z into st->flex_zr.  timed: the last outer step's
// two fused triangular solves are timed (timing slots 2 and 3, collected by
// ssor_timing_collect once the stream has passed them).
static int ssor_apply(pic_ctx* c, const double* r, double* z, hipStream_t s, bool timed = false) {
    const int o = c->p.ssor_outer;
    RETCHK(ssor_once(c, r, z, nullptr, o == 1 ? r : nullptr, s, timed && o == 1));
    for (int i = 1; i < o; ++i) {
        HIPCHK(launch_resid_norm(c->geo, r, z, c->sv[5], c->inv_h2, c->st, c->partials, s));
        RETCHK(ssor_once(c, c->sv[5], z, z, i + 1 == o ? r : nullptr, s, timed && i + 1 == o));
    }
    return PIC_OK;
}

static int ssor_timing_collect(pic_ctx* c) {
    for (int j = 0; j < 2; ++j) {
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, c->ev[4 + 2 * j], c->ev[5 + 2 * j]));
        c->t_sum[2 + j] += ms;
        c->t_cnt[2 + j] += 1;
    }
    return PIC_OK;
}

// PCG with the SSOR preconditioner; iteration and stopping rule of the FP64
// form (recursive residual, then the true residual, one replacement on a
// failed check).
static int solve_ssor(pic_ctx* c, const double* b, double* x, pic_solve_info* out,
                      hipStream_t s) {
    RETCHK(ensure_ssor(c));
    const SweepGeo& g = c->geo;
    const int64_t n3 = c->n3;
    double* z = c->sv[0];
    HIPCHK(launch_residual64(g, b, x, c->r, c->minv, c->inv_h2, 1, c->p.rtol, c->p.max_iter, c->st,
                             c->partials, s));
    RETCHK(read_state(c, s));
    const double nb = c->st_host->cg.nb, tol = c->st_host->cg.tol;
    out->norm_b = nb;
    if (c->st_host->cg.state == CG_ZERO_RHS) {
        HIPCHK(launch_fill(n3, x, 0.0, s));
        out->converged = 1;
        return PIC_OK;
    }
    double rn = c->st_host->cg.true_rn;
    out->rel_res = rn / nb;
    if (rn <= tol) {
        out->converged = 1;
        return PIC_OK;
    }
    RETCHK(ssor_apply(c, c->r, z, s));
    RETCHK(read_state(c, s));
    double rz = c->st_host->flex_zr, beta = 0.0;
    int restart = 1;  // p = z (no previous direction)
    int cur = 0;      // p2[cur] holds the current direction
    int64_t it = 0;
    // kernel timing: every kTimeStride-th iteration, the direction sweep
    // (slot 0), the update sweep (slot 1) and, with the fused triangular
    // solves, the forward and backward solve of the preconditioner's last
    // outer step (slots 2, 3); the state is read back after each, so the
    // events have completed when they are read
    if (c->timing) RETCHK(timing_events(c, 8));
    const bool fused =
        !(c->p.flags & PIC_FLAG_SSOR_UNFUSED) && ssor_fused_supported(c->p.n, c->p.ssor_inner);
    while (it < c->p.max_iter) {
        const bool timed = c->timing && (it % kTimeStride) == 0;
        // p_new = z + beta p and p_new . A p_new (A p_new not stored)
        if (timed) HIPCHK(hipEventRecord(c->ev[0], s));
        HIPCHK(launch_aqz(g, z, c->p2[cur], c->p2[cur ^ 1], nullptr, beta, restart, c->inv_h2,
                          c->st, c->partials, s));
        if (timed) HIPCHK(hipEventRecord(c->ev[1], s));
        cur ^= 1;
        double* p = c->p2[cur];
        RETCHK(read_state(c, s));
        const double pq = c->st_host->flex_pq;
        const double alpha = rz / pq;
        if (!std::isfinite(alpha) || !(pq > 0.0)) break;
        // x += alpha p, r -= alpha A p (A p recomputed), r . r
        if (timed) HIPCHK(hipEventRecord(c->ev[2], s));
        HIPCHK(launch_updp(g, p, x, c->r, alpha, c->inv_h2, c->st, c->partials, s));
        if (timed) HIPCHK(hipEventRecord(c->ev[3], s));
        RETCHK(read_state(c, s));
        if (timed) RETCHK(timing_collect(c, 1, 1));
        ++it;
        rn = std::sqrt(c->st_host->flex_rr);
        out->rel_res = rn / nb;
        if (!std::isfinite(rn)) break;
        if (rn <= tol) {
            double* res = c->fw ? c->fw : c->sv[5];
            HIPCHK(launch_resid_norm(g, b, x, res, c->inv_h2, c->st, c->partials, s));
            RETCHK(read_state(c, s));
            const double tn = c->st_host->out_nr;
            out->rel_res = tn / nb;
            if (tn <= tol) {
                out->converged = 1;
                break;
            }
            // residual replacement: r = b - A x, the direction restarts
            HIPCHK(launch_copy(n3, res, c->r, s));
            RETCHK(ssor_apply(c, c->r, z, s));
            RETCHK(read_state(c, s));
            rz = c->st_host->flex_zr;
            restart = 1;
            out->replacements += 1;
            continue;
        }
        RETCHK(ssor_apply(c, c->r, z, s, timed && fused));
        RETCHK(read_state(c, s));
        if (timed && fused) RETCHK(ssor_timing_collect(c));
        const double rz_new = c->st_host->flex_zr;
        beta = rz_new / rz;
        rz = rz_new;
        restart = 0;
    }
    out->iterations = it;
    if (!out->converged) {
        HIPCHK(launch_resid_norm(g, b, x, c->sv[5], c->inv_h2, c->st, c->partials, s));
        RETCHK(read_state(c, s));
        out->rel_res = c->st_host->out_nr / nb;
    }
    return PIC_OK;
}

// -------------------------------------------------------------- FFT form --
// phi = IFFT(FFT(b) / symbol) with the zero mode removed; with
// PIC_FLAG_FFT_SPECTRAL and E requested, E_d = IFFT(-i k_d phi_hat) as well
// (then *e_done is set).  The residual reported is the 7-point operator's
// (round-off for the discrete symbol; the O(h^2) operator difference for the
// spectral one).
static bool fft_spectral(const pic_ctx* c) {
    return (c->p.flags & PIC_FLAG_FFT_SPECTRAL) != 0;
}

static int solve_fft(pic_ctx* c, const double* b, double* x, pic_solve_info* out, hipStream_t s,
                     double* ex, double* ey, double* ez, bool* e_done) {
    RETCHK(ensure_fft(c));
    const int n = c->p.n;
    const int64_t nspec = (int64_t)(n / 2 + 1) * n * n;
    const bool spec = fft_spectral(c);
    const double kf = 2.0 * M_PI / c->L;
    *e_done = false;
    // rocFFT may overwrite a transform's input: b goes through scratch
    HIPCHK(launch_copy(c->n3, b, c->r, s));
    if (fft_forward(c->fft, c->r, c->fspec[0], s)) return fail(PIC_ERR_HIP, "%s", fft_last_error());
    HIPCHK(launch_fft_divide(nspec, n, c->inv_h2, kf, spec ? 1 : 0, 1.0 / (double)c->n3,
                             c->fspec[0], s));
    if (spec && ex && ey && ez) {
        double* E[3] = {ex, ey, ez};
        for (int d = 0; d < 3; ++d) {
            HIPCHK(launch_fft_grad(nspec, n, kf, d, c->fspec[0], c->fspec[1], s));
            if (fft_inverse(c->fft, c->fspec[1], E[d], s))
                return fail(PIC_ERR_HIP, "%s", fft_last_error());
        }
        *e_done = true;
    }
    if (fft_inverse(c->fft, c->fspec[0], x, s)) return fail(PIC_ERR_HIP, "%s", fft_last_error());
    HIPCHK(launch_resid_norm(c->geo, b, x, c->r, c->inv_h2, c->st, c->partials, s));
    HIPCHK(launch_sum(c->n3, b, c->st, c->partials, 1, s));
    RETCHK(read_state(c, s));
    const double nb = std::sqrt(c->st_host->bb);
    out->norm_b = nb;
    out->rel_res = nb > 0 ? c->st_host->out_nr / nb : 0.0;
    out->converged = 1;
    return PIC_OK;
}

// W_x of a spectral field (the field sweep computes it otherwise).
static int spectral_wx(pic_ctx* c, const double* ex, hipStream_t s, double* wx) {
    HIPCHK(launch_sum(c->n3, ex, c->st, c->partials, 1, s));
    RETCHK(read_state(c, s));
    *wx = 0.5 * c->h3 * c->st_host->bb;
    return PIC_OK;
}

// ------------------------------------------------------------------ field --

static int field(pic_ctx* c, double* phi, double* ex, double* ey, double* ez, hipStream_t s) {
    // the gauge (mean of phi) where constants are in A's kernel; a Dirichlet
    // potential is unique and kept as it is
    if (c->p.bc != PIC_BC_DIRICHLET) HIPCHK(launch_sum(c->n3, phi, c->st, c->partials, 0, s));
    HIPCHK(launch_field(c->geo, phi, ex, ey, ez, c->ehalf, c->h3, c->st, c->partials, s));
    return PIC_OK;
}

// ====================================================================== ABI ==

extern "C" {

int pic_abi_version(void) { return 3; }

const char* pic_last_error(void) { return g_err.c_str(); }

size_t pic_workspace_bytes(const pic_params* p) {
    if (validate_params(p) != PIC_OK) return 0;
    size_t b = base_bytes(p);
    if (p->np_max > 0) b += sort_scratch_bytes(p->np_max) + sort_rec_bytes(p->np_max);
    if (p->solver == PIC_SOLVER_PCG_MIXED) b += mixed_bytes(p);
    if (p->solver == PIC_SOLVER_FCG_LEARNED) b += learned_bytes(p);
    if (p->solver == PIC_SOLVER_PCG_SSOR) b += ssor_bytes(p);
    if (p->solver == PIC_SOLVER_FFT) b += fft_bytes(p);
    if (p->solver == PIC_SOLVER_PIF) b += pif_bytes(p->n);
    return b;
}

int pic_create(const pic_params* params, pic_ctx** out) {
    g_err.clear();
    if (!out) return fail(PIC_ERR_INVALID, "out is NULL");
    *out = nullptr;
    RETCHK(validate_params(params));
    pic_ctx* c = new (std::nothrow) pic_ctx();
    if (!c) return fail(PIC_ERR_NOMEM, "host allocation failed");
    c->p = *params;
    if (c->p.check_every <= 0) c->p.check_every = 16;
    if (c->p.max_outer <= 0) c->p.max_outer = 50;
    if (c->p.max_inner <= 0) c->p.max_inner = 20000;
    if (!(c->p.inner_rtol > 0.0)) c->p.inner_rtol = 1e-3;
    if (c->p.fcg_window <= 0) c->p.fcg_window = 10;
    if (c->p.ssor_omega == 0.0) c->p.ssor_omega = 1.5707963267948966;  // pi / 2
    if (c->p.ssor_inner == 0) c->p.ssor_inner = 4;
    if (c->p.ssor_outer == 0) c->p.ssor_outer = 2;
    if (c->p.pif_tol == 0.0) c->p.pif_tol = 1e-4;  // the paper's NUFFT tolerance (Sec. 4)
    const int n = c->p.n;
    c->n3 = (int64_t)n * n * n;
    const int bc = c->p.bc;
    c->geo = make_geo(n, bc);
    // SSOR's triangular factors couple unknowns only: no neighbour across a
    // bounded face (zero ghosts), cyclic on the periodic box
    c->geo_tri = make_geo(n, bc == PIC_BC_PERIODIC ? 0 : 1);
    c->L = c->p.length;
    // the same formulas, in the same order, as the CPU definition; a
    // Dirichlet box has N interior vertices, so h = L / (N + 1)
    const int cells = bc == PIC_BC_DIRICHLET ? n + 1 : n;
    c->inv_h = (double)cells / c->L;
    c->inv_h2 = c->inv_h * c->inv_h;
    c->minv = 1.0 / (6.0 * (c->inv_h * c->inv_h));
    c->h = c->L / (double)cells;
    c->h3 = c->h * c->h * c->h;
    c->ehalf = 0.5 * c->inv_h;
    c->qh3 = c->p.charge * (c->inv_h * c->inv_h * c->inv_h);
    c->coef_push = c->p.dt * c->p.qm;
    c->coef_kick = (-0.5 * c->p.dt) * c->p.qm;
    c->inv_h2f = (float)(c->inv_h * c->inv_h);
    c->minvf = (float)(1.0 / (6.0 * (c->inv_h * c->inv_h)));
    if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        return fail(PIC_ERR_HIP, "no HIP device");
    }
    int rc = PIC_OK;
    do {
        void* m = nullptr;
        if ((rc = dev_alloc(c, &m, base_bytes(&c->p))) != PIC_OK) break;
        char* q = (char*)m;
        c->st = (DevState*)q;
        q += 4096;
        c->npartials = max_sweep_blocks() < 2 * deposit_partials() ? 2 * deposit_partials()
                                                                    : max_sweep_blocks();
        c->partials = (double*)q;
        q += (size_t)4 * c->npartials * sizeof(double);
        q = (char*)(((uintptr_t)q + 255) & ~(uintptr_t)255);
        const size_t vb = vec_bytes(c->n3, 8);
        c->r = (double*)q;
        c->p2[0] = (double*)(q + vb);
        c->p2[1] = (double*)(q + 2 * vb);
        c->t3 = (double*)(q + 3 * vb);
        if (hipHostMalloc((void**)&c->st_host, sizeof(DevState), hipHostMallocDefault) != hipSuccess) {
            rc = fail(PIC_ERR_NOMEM, "pinned host allocation failed");
            break;
        }
        std::memset(c->st_host, 0, sizeof(DevState));
        if (hipMemcpy(c->st, c->st_host, sizeof(DevState), hipMemcpyHostToDevice) != hipSuccess) {
            rc = fail(PIC_ERR_HIP, "state upload failed");
            break;
        }
        if (c->p.np_max > 0) {
            if ((rc = dev_alloc(c, &c->sort_pool, sort_scratch_bytes(c->p.np_max))) != PIC_OK) break;
            sort_scratch_carve(c->sort_pool, c->p.np_max, &c->sort);
        }
        if (c->p.solver == PIC_SOLVER_PCG_MIXED && (rc = ensure_mixed(c)) != PIC_OK) break;
        if (c->p.solver == PIC_SOLVER_FCG_LEARNED && (rc = ensure_learned(c)) != PIC_OK) break;
        if (c->p.solver == PIC_SOLVER_PCG_SSOR && (rc = ensure_ssor(c)) != PIC_OK) break;
        if (c->p.solver == PIC_SOLVER_FFT && (rc = ensure_fft(c)) != PIC_OK) break;
        if (c->p.solver == PIC_SOLVER_PIF && (rc = ensure_pif(c)) != PIC_OK) break;
    } while (0);
    if (rc != PIC_OK) {
        std::string keep = g_err;
        pic_destroy(c);
        g_err = keep;
        return rc;
    }
    *out = c;
    return PIC_OK;
}

int pic_destroy(pic_ctx* c) {
    if (!c) return PIC_OK;
    (void)hipDeviceSynchronize();
    for (void* a : c->allocs) (void)hipFree(a);
    if (c->st_host) (void)hipHostFree(c->st_host);
    for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
    if (c->net) net::destroy(c->net);
    if (c->fft) fft_destroy(c->fft);
    if (c->pif) pif_destroy(c->pif);
    delete c;
    return PIC_OK;
}

int pic_set_solver(pic_ctx* c, int32_t solver) {
    if (!c) return fail(PIC_ERR_INVALID, "ctx is NULL");
    if (solver < PIC_SOLVER_PCG_FP64 || solver > PIC_SOLVER_PIF)
        return fail(PIC_ERR_INVALID, "unknown solver %d", solver);
    if (solver == PIC_SOLVER_PIF && c->p.n > kPifMaxModes)
        return fail(PIC_ERR_INVALID, "PIF: at most %d modes per axis", kPifMaxModes);
    if (c->p.bc != PIC_BC_PERIODIC && !bounded_solver(solver))
        return fail(PIC_ERR_INVALID, "solver %d needs the periodic box", solver);
    if (solver == PIC_SOLVER_PCG_SSOR) RETCHK(ensure_ssor(c));
    if (solver == PIC_SOLVER_FFT) RETCHK(ensure_fft(c));
    if (solver == PIC_SOLVER_PIF) RETCHK(ensure_pif(c));
    if (solver == PIC_SOLVER_PCG_MIXED) RETCHK(ensure_mixed(c));
    if (solver == PIC_SOLVER_FCG_LEARNED) RETCHK(ensure_learned(c));
    c->p.solver = solver;
    return PIC_OK;
}

int pic_set_flags(pic_ctx* c, int32_t flags) {
    if (!c) return fail(PIC_ERR_INVALID, "ctx is NULL");
    if (flags & ~kKnownFlags) return fail(PIC_ERR_INVALID, "unknown flags 0x%x", flags);
    c->p.flags = flags;
    return PIC_OK;
}

int pic_set_kernel_timing(pic_ctx* c, int32_t enable) {
    if (!c) return fail(PIC_ERR_INVALID, "ctx is NULL");
    c->timing = enable != 0;
    timing_reset(c);
    return PIC_OK;
}

int pic_stream_triad(int64_t n, const double* b, const double* cv, double* a, double scalar,
                     int32_t reps, double* avg_ms, void* stream) {
    if (n < 1 || n >= ((int64_t)1 << 40) || reps < 1 || !b || !cv || !a || !avg_ms)
        return fail(PIC_ERR_INVALID, "pic_stream_triad: n in [1, 2^40), reps >= 1, non-NULL arrays");
    if (!aligned8(b) || !aligned8(cv) || !aligned8(a))
        return fail(PIC_ERR_INVALID, "pic_stream_triad: arrays must be 8-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e[2] = {nullptr, nullptr};
    HIPCHK(hipEventCreate(&e[0]));
    hipError_t err = hipEventCreate(&e[1]);
    if (err == hipSuccess) err = launch_triad(n, b, cv, a, scalar, s);  // untimed first launch
    if (err == hipSuccess) err = hipEventRecord(e[0], s);
    for (int32_t k = 0; k < reps && err == hipSuccess; ++k) err = launch_triad(n, b, cv, a, scalar, s);
    if (err == hipSuccess) err = hipEventRecord(e[1], s);
    if (err == hipSuccess) err = hipEventSynchronize(e[1]);
    float ms = 0.f;
    if (err == hipSuccess) err = hipEventElapsedTime(&ms, e[0], e[1]);
    (void)hipEventDestroy(e[0]);
    if (e[1]) (void)hipEventDestroy(e[1]);
    if (err != hipSuccess) return fail(PIC_ERR_HIP, "pic_stream_triad: %s", hipGetErrorString(err));
    *avg_ms = (double)ms / reps;
    return PIC_OK;
}

int pic_kernel_time(pic_ctx* c, int32_t id, double* avg_ms, int64_t* count) {
    if (!c || !avg_ms || !count || id < 0 || id > 3)
        return fail(PIC_ERR_INVALID, "bad arguments to pic_kernel_time");
    *count = c->t_cnt[id];
    *avg_ms = c->t_cnt[id] ? c->t_sum[id] / (double)c->t_cnt[id] : 0.0;
    return PIC_OK;
}

#define NEED(ptr, what)                                                   \
    do {                                                                  \
        if (!(ptr)) return fail(PIC_ERR_INVALID, "%s is NULL", what);     \
        if (!aligned8(ptr)) return fail(PIC_ERR_INVALID, "%s is not 8-byte aligned", what); \
    } while (0)

static int check_np(pic_ctx* c, int64_t np) {
    if (!c) return fail(PIC_ERR_INVALID, "ctx is NULL");
    if (np < 0 || np > c->p.np_max)
        return fail(PIC_ERR_INVALID, "np = %lld outside [0, np_max = %lld]", (long long)np,
                    (long long)c->p.np_max);
    return PIC_OK;
}

// Particles live in the periodic cube: the particle phases refuse a context
// made for a bounded box (only its solve and field are built).
static int check_periodic(pic_ctx* c) {
    if (c->p.bc != PIC_BC_PERIODIC)
        return fail(PIC_ERR_INVALID, "particle phases need the periodic box (bc = %d)", c->p.bc);
    return PIC_OK;
}

int pic_cell_keys(pic_ctx* c, int64_t np, const double* x, const double* y, const double* z,
                  uint32_t* key, void* stream) {
    RETCHK(check_np(c, np));
    RETCHK(check_periodic(c));
    if (np == 0) return PIC_OK;
    NEED(x, "x"); NEED(y, "y"); NEED(z, "z");
    if (!key) return fail(PIC_ERR_INVALID, "key is NULL");
    HIPCHK(launch_keys(np, x, y, z, key, c->p.n, c->inv_h, (hipStream_t)stream));
    return PIC_OK;
}

int pic_sort_cells(pic_ctx* c, int64_t np, const uint32_t* key, const double* const src[6],
                   double* const dst[6], uint32_t* cell_start, uint32_t* perm, void* stream) {
    RETCHK(check_np(c, np));
    if (!src || !dst) return fail(PIC_ERR_INVALID, "src/dst is NULL");
    if (!cell_start) return fail(PIC_ERR_INVALID, "cell_start is NULL");
    if (np > 0) {
        if (!key) return fail(PIC_ERR_INVALID, "key is NULL");
        for (int i = 0; i < 6; ++i) {
            NEED(src[i], "src[i]");
            NEED(dst[i], "dst[i]");
            for (int j = 0; j < 6; ++j)
                if ((const void*)src[i] == (const void*)dst[j])
                    return fail(PIC_ERR_INVALID, "dst must not alias src");
        }
    }
    RETCHK(ensure_rec(c));
    HIPCHK(launch_sort_cells(np, c->p.n, key, src, dst, cell_start, perm, &c->sort,
                             (hipStream_t)stream));
    return PIC_OK;
}

int pic_deposit_cic(pic_ctx* c, int64_t np, const double* x, const double* y, const double* z,
                    const uint32_t* cell_start, double* rho, double* norm_b, void* stream) {
    RETCHK(check_np(c, np));
    RETCHK(check_periodic(c));
    NEED(rho, "rho");
    if (np > 0) { NEED(x, "x"); NEED(y, "y"); NEED(z, "z"); }
    hipStream_t s = (hipStream_t)stream;
    HIPCHK(launch_deposit(np, x, y, z, np > 0 ? cell_start : nullptr, rho, c->p.n, c->inv_h,
                          c->qh3, c->p.rho_bg, c->st, c->partials, dep_scratch(c), s));
    if (norm_b) {
        RETCHK(read_state(c, s));
        *norm_b = std::sqrt(c->st_host->bb);
    }
    return PIC_OK;
}

int pic_efield(pic_ctx* c, double* phi, double* ex, double* ey, double* ez, double* wx,
               void* stream) {
    if (!c) return fail(PIC_ERR_INVALID, "ctx is NULL");
    NEED(phi, "phi"); NEED(ex, "ex"); NEED(ey, "ey"); NEED(ez, "ez");
    hipStream_t s = (hipStream_t)stream;
    RETCHK(field(c, phi, ex, ey, ez, s));
    if (wx) {
        RETCHK(read_state(c, s));
        *wx = c->st_host->wx;
    }
    return PIC_OK;
}

int pic_poisson_pcg(pic_ctx* c, const double* rho, double* phi, double* ex, double* ey,
                    double* ez, pic_solve_info* info, void* stream) {
    if (!c) return fail(PIC_ERR_INVALID, "ctx is NULL");
    NEED(rho, "rho");
    NEED(phi, "phi");
    const bool want_e = ex && ey && ez;
    if (want_e) { NEED(ex, "ex"); NEED(ey, "ey"); NEED(ez, "ez"); }
    hipStream_t s = (hipStream_t)stream;
    pic_solve_info si;
    std::memset(&si, 0, sizeof si);
    if (c->timing) timing_reset(c);
    bool e_done = false;
    if (c->p.solver == PIC_SOLVER_PIF)
        return fail(PIC_ERR_INVALID, "the PIF form has no grid solve (pic_pif_field, pic_step)");
    switch (c->p.solver) {
        case PIC_SOLVER_PCG_FP64: RETCHK(solve_fp64(c, rho, phi, &si, s)); break;
        case PIC_SOLVER_PCG_MIXED: RETCHK(solve_mixed(c, rho, phi, &si, s)); break;
        case PIC_SOLVER_PCG_SSOR: RETCHK(solve_ssor(c, rho, phi, &si, s)); break;
        case PIC_SOLVER_FFT:
            RETCHK(solve_fft(c, rho, phi, &si, s, want_e ? ex : nullptr, ey, ez, &e_done));
            break;
        default: RETCHK(solve_learned(c, rho, phi, &si, s)); break;
    }
    if (want_e && e_done) {
        RETCHK(spectral_wx(c, ex, s, &si.wx));
    } else if (want_e) {
        RETCHK(field(c, phi, ex, ey, ez, s));
        RETCHK(read_state(c, s));
        si.wx = c->st_host->wx;
    }
    if (info) *info = si;
    return si.converged ? PIC_OK : PIC_NOT_CONVERGED;
}

int pic_pif_field(pic_ctx* c, int64_t np, const double* x, const double* y, const double* z,
                  const uint32_t* cell_start, double* ex, double* ey, double* ez, double* wx,
                  void* stream) {
    RETCHK(check_np(c, np));
    RETCHK(check_periodic(c));
    if (c->p.solver != PIC_SOLVER_PIF) return fail(PIC_ERR_INVALID, "solver is not PIF");
    NEED(cell_start, "cell_start");
    if (np > 0) {
        NEED(x, "x"); NEED(y, "y"); NEED(z, "z"); NEED(ex, "ex"); NEED(ey, "ey"); NEED(ez, "ez");
    }
    RETCHK(ensure_pif(c));
    hipStream_t s = (hipStream_t)stream;
    if (pif_spread(c->pif, np, x, y, z, cell_start, c->p.charge, s) ||
        pif_fields(c->pif, c->st, c->partials, s))
        return fail(PIC_ERR_HIP, "PIF field: %s", pif_last_error());
    if (pif_interp(c->pif, 0, np, const_cast<double*>(x), const_cast<double*>(y),
                   const_cast<double*>(z), nullptr, nullptr, nullptr, ex, ey, ez, nullptr,
                   cell_start, 0.0, 0.0, s))
        return fail(PIC_ERR_HIP, "PIF field: %s", pif_last_error());
    if (wx) {
        RETCHK(read_state(c, s));
        *wx = c->st_host->wx;
    }
    return PIC_OK;
}

int pic_set_unet(pic_ctx* c, const float* params, void* stream) {
    if (!c) return fail(PIC_ERR_INVALID, "ctx is NULL");
    if (!params) return fail(PIC_ERR_INVALID, "params is NULL");
    if (!c->net) {
        const int rc = net::create(&c->net, c->p.n, false);
        if (rc) {
            c->net = nullptr;
            return fail(rc == -3 ? PIC_ERR_NOMEM : PIC_ERR_HIP, "network buffers: %s", net::last_error());
        }
    }
    if (net::set_params(c->net, params, (hipStream_t)stream))
        return fail(PIC_ERR_HIP, "network parameters: %s", net::last_error());
    return PIC_OK;
}

int pic_unet_precondition(pic_ctx* c, const double* r, double* z, void* stream) {
    if (!c) return fail(PIC_ERR_INVALID, "ctx is NULL");
    if (c->p.bc != PIC_BC_PERIODIC)
        return fail(PIC_ERR_INVALID, "the network's convolutions need the periodic box");
    NEED(r, "r");
    NEED(z, "z");
    return fcg_precond(c, r, z, (hipStream_t)stream);
}

int pic_gather_push(pic_ctx* c, int64_t np, double* x, double* y, double* z, double* vx,
                    double* vy, double* vz, const double* ex, const double* ey, const double* ez,
                    uint32_t* key_out, void* stream) {
    RETCHK(check_np(c, np));
    RETCHK(check_periodic(c));
    if (np == 0) return PIC_OK;
    NEED(x, "x"); NEED(y, "y"); NEED(z, "z"); NEED(vx, "vx"); NEED(vy, "vy"); NEED(vz, "vz");
    NEED(ex, "ex"); NEED(ey, "ey"); NEED(ez, "ez");
    HIPCHK(launch_gather_push(np, x, y, z, vx, vy, vz, ex, ey, ez, key_out, nullptr, c->p.n,
                              c->inv_h, c->L, c->p.dt, c->coef_push, (hipStream_t)stream));
    return PIC_OK;
}

int pic_half_kick(pic_ctx* c, int64_t np, const double* x, const double* y, const double* z,
                  double* vx, double* vy, double* vz, const double* ex, const double* ey,
                  const double* ez, void* stream) {
    RETCHK(check_np(c, np));
    RETCHK(check_periodic(c));
    if (np == 0) return PIC_OK;
    NEED(x, "x"); NEED(y, "y"); NEED(z, "z"); NEED(vx, "vx"); NEED(vy, "vy"); NEED(vz, "vz");
    NEED(ex, "ex"); NEED(ey, "ey"); NEED(ez, "ez");
    HIPCHK(launch_half_kick(np, x, y, z, vx, vy, vz, ex, ey, ez, c->p.n, c->inv_h, c->coef_kick,
                            (hipStream_t)stream));
    return PIC_OK;
}

static int check_parts(pic_ctx* c, pic_particles* P, pic_fields* F) {
    if (!P || !F) return fail(PIC_ERR_INVALID, "particles/fields is NULL");
    RETCHK(check_np(c, P->np));
    RETCHK(check_periodic(c));
    NEED(F->rho, "rho"); NEED(F->phi, "phi"); NEED(F->ex, "ex"); NEED(F->ey, "ey"); NEED(F->ez, "ez");
    if (!P->cell_start) return fail(PIC_ERR_INVALID, "cell_start is NULL");
    if (P->np > 0) {
        if (!P->key) return fail(PIC_ERR_INVALID, "key is NULL");
        double* a[12] = {P->cur.x, P->cur.y, P->cur.z, P->cur.vx, P->cur.vy, P->cur.vz,
                         P->alt.x, P->alt.y, P->alt.z, P->alt.vx, P->alt.vy, P->alt.vz};
        for (int i = 0; i < 12; ++i) NEED(a[i], "particle array");
    }
    return PIC_OK;
}

// Sort into the second set of arrays and swap; from_rec: the push left the
// particles in the sort's record array (the current arrays are stale).
static int sort_swap(pic_ctx* c, pic_particles* P, hipStream_t s, bool from_rec = false) {
    RETCHK(ensure_rec(c));
    const double* src[6] = {P->cur.x, P->cur.y, P->cur.z, P->cur.vx, P->cur.vy, P->cur.vz};
    double* dst[6] = {P->alt.x, P->alt.y, P->alt.z, P->alt.vx, P->alt.vy, P->alt.vz};
    HIPCHK(launch_sort_cells(P->np, c->p.n, P->key, from_rec ? nullptr : src, dst, P->cell_start,
                             nullptr, &c->sort, s));
    pic_particle_arrays t = P->cur;
    P->cur = P->alt;
    P->alt = t;
    return PIC_OK;
}

struct PhaseTimer {
    bool on = false;
    hipEvent_t e[6];
    int init(bool enable) {
        on = enable;
        if (!on) return PIC_OK;
        for (auto& x : e) HIPCHK(hipEventCreate(&x));
        return PIC_OK;
    }
    int mark(int i, hipStream_t s) {
        if (on) HIPCHK(hipEventRecord(e[i], s));
        return PIC_OK;
    }
    double ms(int a, int b) {
        float t = 0.f;
        if (on) (void)hipEventElapsedTime(&t, e[a], e[b]);
        return t;
    }
    ~PhaseTimer() {
        if (on)
            for (auto& x : e) (void)hipEventDestroy(x);
    }
};

// The PIF form's field: spread of the sorted particles, transforms and the
// mode-wise solve (the field grids stay in the PIF state for the next push).
static int pif_field_phase(pic_ctx* c, pic_particles* P, hipStream_t s, bool spread) {
    if (spread && pif_spread(c->pif, P->np, P->cur.x, P->cur.y, P->cur.z, P->cell_start,
                             c->p.charge, s))
        return fail(PIC_ERR_HIP, "PIF spread: %s", pif_last_error());
    if (!spread && pif_fields(c->pif, c->st, c->partials, s))
        return fail(PIC_ERR_HIP, "PIF field: %s", pif_last_error());
    return PIC_OK;
}

static int pif_info(pic_ctx* c, hipStream_t s, pic_solve_info* si) {
    std::memset(si, 0, sizeof *si);
    RETCHK(read_state(c, s));
    si->wx = c->st_host->wx;
    si->converged = 1;
    return PIC_OK;
}

int pic_init(pic_ctx* c, pic_particles* P, pic_fields* F, pic_step_info* info, void* stream) {
    RETCHK(check_parts(c, P, F));
    hipStream_t s = (hipStream_t)stream;
    if (P->np > 0) HIPCHK(launch_keys(P->np, P->cur.x, P->cur.y, P->cur.z, P->key, c->p.n, c->inv_h, s));
    RETCHK(sort_swap(c, P, s));
    if (c->p.solver == PIC_SOLVER_PIF) {
        RETCHK(ensure_pif(c));
        RETCHK(pif_field_phase(c, P, s, true));
        RETCHK(pif_field_phase(c, P, s, false));
        if (pif_interp(c->pif, 2, P->np, P->cur.x, P->cur.y, P->cur.z, P->cur.vx, P->cur.vy,
                       P->cur.vz, nullptr, nullptr, nullptr, nullptr, P->cell_start, c->coef_kick,
                       0.0, s))
            return fail(PIC_ERR_HIP, "PIF half kick: %s", pif_last_error());
        if (info) {
            std::memset(info, 0, sizeof *info);
            RETCHK(pif_info(c, s, &info->solve));
        }
        return PIC_OK;
    }
    HIPCHK(launch_deposit(P->np, P->cur.x, P->cur.y, P->cur.z, P->np > 0 ? P->cell_start : nullptr,
                          F->rho, c->p.n, c->inv_h, c->qh3, c->p.rho_bg, c->st, c->partials, dep_scratch(c), s));
    pic_solve_info si;
    int rc = pic_poisson_pcg(c, F->rho, F->phi, F->ex, F->ey, F->ez, &si, stream);
    if (rc < 0) return rc;
    HIPCHK(launch_half_kick(P->np, P->cur.x, P->cur.y, P->cur.z, P->cur.vx, P->cur.vy, P->cur.vz,
                            F->ex, F->ey, F->ez, c->p.n, c->inv_h, c->coef_kick, s));
    if (info) {
        std::memset(info, 0, sizeof *info);
        info->solve = si;
        HIPCHK(hipStreamSynchronize(s));
    }
    return rc;
}

int pic_step(pic_ctx* c, pic_particles* P, pic_fields* F, pic_step_info* info, void* stream) {
    RETCHK(check_parts(c, P, F));
    hipStream_t s = (hipStream_t)stream;
    PhaseTimer T;
    RETCHK(T.init(info != nullptr));
    RETCHK(T.mark(0, s));
    if (c->p.solver == PIC_SOLVER_PIF) {
        // push with the field of the previous solve, sort, spread, solve
        RETCHK(ensure_pif(c));
        if (pif_interp(c->pif, 1, P->np, P->cur.x, P->cur.y, P->cur.z, P->cur.vx, P->cur.vy,
                       P->cur.vz, nullptr, nullptr, nullptr, P->key, P->cell_start, c->coef_push,
                       c->p.dt, s))
            return fail(PIC_ERR_HIP, "PIF push: %s", pif_last_error());
        RETCHK(T.mark(1, s));
        RETCHK(sort_swap(c, P, s));
        RETCHK(T.mark(2, s));
        RETCHK(pif_field_phase(c, P, s, true));
        RETCHK(T.mark(3, s));
        RETCHK(pif_field_phase(c, P, s, false));
        RETCHK(T.mark(4, s));
        RETCHK(T.mark(5, s));
        if (info) {
            RETCHK(pif_info(c, s, &info->solve));
            info->ms_push = T.ms(0, 1);
            info->ms_sort = T.ms(1, 2);
            info->ms_deposit = T.ms(2, 3);
            info->ms_solve = T.ms(3, 4);
            info->ms_field = T.ms(4, 5);
        }
        return PIC_OK;
    }
    RETCHK(ensure_rec(c));
    HIPCHK(launch_gather_push(P->np, P->cur.x, P->cur.y, P->cur.z, P->cur.vx, P->cur.vy, P->cur.vz,
                              F->ex, F->ey, F->ez, P->key, c->sort.rec, c->p.n, c->inv_h, c->L,
                              c->p.dt, c->coef_push, s));
    RETCHK(T.mark(1, s));
    RETCHK(sort_swap(c, P, s, true));
    RETCHK(T.mark(2, s));
    HIPCHK(launch_deposit(P->np, P->cur.x, P->cur.y, P->cur.z, P->np > 0 ? P->cell_start : nullptr,
                          F->rho, c->p.n, c->inv_h, c->qh3, c->p.rho_bg, c->st, c->partials, dep_scratch(c), s));
    RETCHK(T.mark(3, s));
    pic_solve_info si;
    std::memset(&si, 0, sizeof si);
    int rc;
    bool e_done = false;
    switch (c->p.solver) {
        case PIC_SOLVER_PCG_FP64: rc = solve_fp64(c, F->rho, F->phi, &si, s); break;
        case PIC_SOLVER_PCG_MIXED: rc = solve_mixed(c, F->rho, F->phi, &si, s); break;
        case PIC_SOLVER_PCG_SSOR: rc = solve_ssor(c, F->rho, F->phi, &si, s); break;
        case PIC_SOLVER_FFT:
            rc = solve_fft(c, F->rho, F->phi, &si, s, F->ex, F->ey, F->ez, &e_done);
            break;
        default: rc = solve_learned(c, F->rho, F->phi, &si, s);
    }
    if (rc < 0) return rc;
    RETCHK(T.mark(4, s));
    double wx_spec = 0.0;
    if (e_done) RETCHK(spectral_wx(c, F->ex, s, &wx_spec));
    else RETCHK(field(c, F->phi, F->ex, F->ey, F->ez, s));
    RETCHK(T.mark(5, s));
    if (info) {
        RETCHK(read_state(c, s));
        si.wx = e_done ? wx_spec : c->st_host->wx;
        info->solve = si;
        info->ms_push = T.ms(0, 1);
        info->ms_sort = T.ms(1, 2);
        info->ms_deposit = T.ms(2, 3);
        info->ms_solve = T.ms(3, 4);
        info->ms_field = T.ms(4, 5);
    }
    return si.converged ? PIC_OK : PIC_NOT_CONVERGED;
}

}  // extern "C"
