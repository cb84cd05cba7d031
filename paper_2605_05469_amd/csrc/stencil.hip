// stencil.hip -- matrix-free periodic 7-point sweeps of the PCG solver
// (Sec. 3.2: second-order central differences, action of A only) and of the
// field E = -grad phi (Sec. 2, Eq. poisson).
//
// Design (MI355X / gfx950):
//  * FP64 Jacobi-PCG on the periodic box runs by default in s-step form
//    (sstep.hip: a Gram sweep and an update sweep per three iterations).
//    Here: the single-reduction sweep (the mixed form's FP32 inner solves,
//    and FP64 with PIC_FLAG_PCG_SINGLE_SWEEP), ONE sweep per iteration
//    (cg1_kernel, the single-reduction arrangement of the same iteration):
//    a 512-thread workgroup owns a 64 x 32 (x, y) tile (128 x 16 for the
//    mixed form's FP32 inner sweeps) and an equal share of its column's
//    z-planes.  From r_k, p_{k-1}, x_k it forms p_k, x_{k+1} and r_{k+1} and
//    reduces the five dot products that give the next beta and alpha, so it
//    streams r, p and x once each: 48 bytes per grid point in FP64 (24 in
//    FP32); with x updated every other sweep (XM 1 / 2) 40 on average (20).  A r_{k+1} on the tile needs r_{k+1} on a one-point ring, which
//    needs p_k on a two-point ring: every stage is evaluated on the 68 x 36
//    region; each thread keeps the z-neighbours of its region points in
//    registers and in-plane neighbours pass through two double-buffered LDS
//    planes (one barrier per plane).  Each wave takes 64 aligned columns of
//    one region row, so loads and stores are whole 128-byte lines.
//  * The textbook two-sweep pair (bounded boxes, PIC_FLAG_PCG_TWO_SWEEP, and
//    the SSOR form's PCG sweeps): a 256-thread workgroup owns a 64 x 32 tile,
//    LDS holds two planes with their one-point halo, the z-1 neighbour stays
//    in registers.  The direction sweep forms p_new = M^{-1} r + beta p_old
//    while staging and reduces p.(A p) (24 B/point); the update sweep
//    recomputes A p from p_new (no q vector), updates x and r and reduces
//    r.r and r.M^{-1} r (40 B/point): 64 bytes per grid point per iteration.
//  * Dot products are deterministic: wave tree + fixed-order block sum, one
//    partial per block, summed in index order by the last block, which also
//    advances the CG scalars held in device memory (alpha, beta, state).  The
//    host polls the state only every few iterations; once the state leaves
//    RUNNING the remaining queued sweeps return immediately.
//  * Workgroup ids are remapped so that neighbouring tiles run on one XCD and
//    share its L2 for their halos; own-point streams are non-temporal.
//
// Arithmetic order matches the CPU oracle's definition (neighbour sum
// ((xm+xp)+(ym+yp))+(zm+zp), no contraction) so that A p is bit-identical;
// only the summation order of the dot products differs.
#include "common.hpp"
#include "solver_state.hpp"

namespace pic {

constexpr int kNT = 256;
#ifndef PIC_TY
#define PIC_TY 32
#endif
#ifndef PIC_NT
#define PIC_NT 1
#endif
constexpr int kTY = PIC_TY;  // tile rows in y

// Own-point operands (read or written by exactly one workgroup, never staged
// as a halo) may bypass L2 retention so the halo rows stay cached.
template <class T>
__device__ __forceinline__ T ld_own(const T* p) {
    if constexpr (PIC_NT) return __builtin_nontemporal_load(p);
    else return *p;
}
template <class T>
__device__ __forceinline__ void st_own(T v, T* p) {
    if constexpr (PIC_NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}
constexpr int kMaxSweepBlocks = 8192;

// --------------------------------------------------------------------------
// Generic sweep.  A sweep never writes the array it stages into LDS:
// neighbouring workgroups read that array as their halo at any time.
//
// Neighbours outside the grid follow g.bc: the periodic image (0), zero (1:
// Dirichlet, and the triangular factors of a bounded box), or the mirrored
// value inside the face (2: Neumann).  Ghost entries are loaded from the
// clamped index (always in bounds) and replaced by zero for bc 1.
//
// LDS holds two planes (z and z+1, each with its halo); the z-1 neighbour of
// each thread's own points is kept in registers from the previous plane.  The
// loads for plane z+2 (halo plane) and for the own-point operands of plane z+1
// are issued one plane ahead, so their latency overlaps the arithmetic and the
// barriers of the current plane.
//
// Op provides:
//   using T, In, Own;  static constexpr int NACC;
//   bool active() const;  void prepare();            // reads device scalars
//   In  fetch(size_t g) const;                        // loads for a staged value
//   T   make(const In&, size_t g, bool own) const;    // staged value (may store)
//   Own pre(size_t g) const;                          // loads at an own point
//   void out(const Own&, size_t g, T c, T xm, T xp, T ym, T yp, T zm, T zp,
//            double (&acc)[NACC]) const;
//   void finish(double (&tot)[NACC]) const;           // thread 0 of last block
//   uint32_t* ticket() const;  double* partials() const;
template <class Op, int TX, int BC>
__global__ __launch_bounds__(kNT) void sweep_kernel(Op op_in, SweepGeo g) {
    using T = typename Op::T;
    using In = typename Op::In;
    using Own = typename Op::Own;
    constexpr int NACC = Op::NACC;
    constexpr int PX = TX + 2;
    constexpr int PY = kTY + 2;
    constexpr int PLANE = PX * PY;
    // staged entries per thread (whole-row dealing for 64-wide tiles, below)
    constexpr int NE = TX == kWave
                           ? (PY + (2 * PY + kWave - 1) / kWave + kNT / kWave - 1) / (kNT / kWave)
                           : (PLANE + kNT - 1) / kNT;
    constexpr int RPT = kNT / TX;                // thread rows
    constexpr int PPT = kTY / RPT;               // own points per thread per plane
    __shared__ T buf[2][PLANE];
    __shared__ double red[NACC * (kNT / kWave)];
    __shared__ int lflag;

    Op op = op_in;
    if (!op.active()) return;
    op.prepare();

    const int n = g.n;
    const uint32_t lb = remap_xcd(blockIdx.x, g.nb);
    const uint32_t bx = lb % g.nbx;
    const uint32_t t1 = lb / g.nbx;
    const uint32_t by = t1 % g.nby;
    const uint32_t bz = t1 / g.nby;
    // this block's z-range: the columns' planes are split evenly over nbz blocks
    const int x0 = (int)bx * TX, y0 = (int)by * kTY;
    const int z0 = (int)(((int64_t)bz * n) / g.nbz);
    const int zc = (int)((((int64_t)bz + 1) * n) / g.nbz) - z0;
    const size_t nn = (size_t)n * n;
    const int tid = threadIdx.x;
    const int lx = tid % TX, ly0 = tid / TX;

    // in-plane offsets of this thread's staged entries (fixed for the block)
    constexpr int bc = BC;  // g.bc, fixed at compile time
    auto gmap = [n](int v) {
        if (v >= 0 && v < n) return v;
        if (bc == 0) return v < 0 ? v + n : v - n;
        return v < 0 ? 0 : n - 1;
    };
    // With 64-wide tiles each wave stages the 64 tile columns of one plane
    // row (whole cache lines) and the spare waves of the last slot the two
    // halo columns; otherwise entries are dealt out in row-major order.
    uint32_t eoff[NE];
    int eidx[NE];  // LDS index of entry j in the staged plane, -1: none
    uint32_t eown = 0, ezero = 0;
#pragma unroll
    for (int j = 0; j < NE; ++j) {
        int ly = -1, lxx = 0;
        if constexpr (TX == kWave) {
            const int unit = j * (kNT / kWave) + tid / kWave, lane = tid % kWave;
            if (unit < PY) {
                ly = unit;
                lxx = 1 + lane;
            } else {
                const int e2 = (unit - PY) * kWave + lane;
                if (e2 < 2 * PY) {
                    ly = e2 >> 1;
                    lxx = (e2 & 1) ? TX + 1 : 0;
                }
            }
        } else {
            const int e = tid + j * kNT;
            if (e < PLANE) {
                ly = e / PX;
                lxx = e - ly * PX;
            }
        }
        eidx[j] = -1;
        eoff[j] = 0;
        if (ly < 0) continue;
        eidx[j] = ly * PX + lxx;
        const int rx = x0 + lxx - 1, ry = y0 + ly - 1;
        const int gx = gmap(rx), gy = gmap(ry);
        eoff[j] = (uint32_t)gy * (uint32_t)n + (uint32_t)gx;
        if (lxx >= 1 && lxx <= TX && ly >= 1 && ly <= kTY) eown |= 1u << j;
        if (bc == 1 && (rx != gx || ry != gy)) ezero |= 1u << j;
    }
    auto zwrap = [&gmap](int z) { return gmap(z); };
    auto zzero = [n](int z) { return bc == 1 && (z < 0 || z >= n); };
    auto own_index = [&](int z, int k) {
        return (size_t)z * nn + (size_t)(y0 + ly0 + k * RPT) * n + (size_t)(x0 + lx);
    };

    In fin[NE];
    Own fown[PPT];
    T zm[PPT];
    double acc[NACC];
#pragma unroll
    for (int k = 0; k < NACC; ++k) acc[k] = 0.0;

    auto fetch_plane = [&](int gz) {
        const size_t zo = (size_t)gz * nn;
#pragma unroll
        for (int j = 0; j < NE; ++j)
            if (eidx[j] >= 0) fin[j] = op.fetch(zo + eoff[j]);
    };
    // zr: the plane's coordinate before the boundary rule
    auto commit_plane = [&](T* dst, int zr, bool ownz) {
        const size_t zo = (size_t)zwrap(zr) * nn;
        const uint32_t zmask = zzero(zr) ? ~0u : ezero;
#pragma unroll
        for (int j = 0; j < NE; ++j) {
            const int e = eidx[j];
            if (e >= 0)
                dst[e] = ((zmask >> j) & 1u) ? T(0)
                                             : op.make(fin[j], zo + eoff[j], ownz && ((eown >> j) & 1u));
        }
    };

    // prologue: z-1 values of the own points, planes z0 and z0+1, prefetches
    {
        const int zb = zwrap(z0 - 1);
        const bool zero = zzero(z0 - 1);
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            const size_t gi = own_index(zb, k);
            zm[k] = zero ? T(0) : op.make(op.fetch(gi), gi, false);
        }
    }
    fetch_plane(z0);
    commit_plane(buf[0], z0, true);
    fetch_plane(zwrap(z0 + 1));
    commit_plane(buf[1], z0 + 1, zc > 1);
    if (zc >= 2) fetch_plane(zwrap(z0 + 2));
#pragma unroll
    for (int k = 0; k < PPT; ++k) fown[k] = op.pre(own_index(z0, k));
    __syncthreads();

    int cur = 0;
    for (int i = 0; i < zc; ++i) {
        const int z = z0 + i;
        const T* C = buf[cur];
        const T* Nx = buf[cur ^ 1];
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            const int e = (ly0 + k * RPT + 1) * PX + lx + 1;
            const T c = C[e];
            op.out(fown[k], own_index(z, k), c, C[e - 1], C[e + 1], C[e - PX], C[e + PX], zm[k],
                   Nx[e], acc);
            zm[k] = c;
        }
        if (i + 1 < zc) {
#pragma unroll
            for (int k = 0; k < PPT; ++k) fown[k] = op.pre(own_index(z + 1, k));
        }
        __syncthreads();
        if (i + 2 <= zc) commit_plane(buf[cur], z + 2, i + 2 < zc);
        if (i + 3 <= zc) fetch_plane(zwrap(z + 3));
        __syncthreads();
        cur ^= 1;
    }

    block_sum<kNT, NACC>(acc, red);
    double* part = op.partials();
    if (tid == 0) {
#pragma unroll
        for (int k = 0; k < NACC; ++k) part[(size_t)k * g.nb + lb] = acc[k];
    }
    if (last_block(op.ticket(), g.nb, &lflag)) {
        double tot[NACC];
        sum_partials<kNT, NACC>(part, (int)g.nb, tot, red);
        if (tid == 0) op.finish(tot);
    }
}

struct Nothing {};

// --------------------------------------------------------------------------
// The operator at one point, in the oracle's order.
template <class T>
__device__ __forceinline__ T apply_A(T c, T xm, T xp, T ym, T yp, T zm, T zp, T inv_h2) {
    T t = ((xm + xp) + (ym + yp)) + (zm + zp);
    return (T(6) * c - t) * inv_h2;
}

// r = b - A x with norms.  init != 0: first residual of a solve (also forms
// ||b|| and the stop threshold); otherwise the check of a candidate.
struct OpResidual64 {
    using T = double;
    using In = double;
    using Own = double;
    static constexpr int NACC = 3;
    const double* b;
    const double* x;
    double* r;
    double minv, inv_h2, rtol;
    int64_t max_iter;
    int init;
    DevState* st;
    double* part;
    __device__ bool active() const {
        return init ? true : st->cg.state == CG_CANDIDATE;
    }  // init: 1 = first residual of a solve, 0 = verify a candidate, 2 = report only
    __device__ void prepare() {}
    __device__ double fetch(size_t g) const { return x[g]; }
    __device__ double make(double v, size_t, bool) const { return v; }
    __device__ double pre(size_t g) const { return ld_own(b + g); }
    __device__ void out(double bv, size_t g, double c, double xm, double xp, double ym, double yp,
                        double zm, double zp, double (&acc)[3]) const {
        const double rv = bv - apply_A<double>(c, xm, xp, ym, yp, zm, zp, inv_h2);
        st_own(rv, r + g);
        acc[0] += bv * bv;
        acc[1] += rv * rv;
        acc[2] += rv * (minv * rv);
    }
    __device__ void finish(double (&t)[3]) const {
        CgScalars& cg = st->cg;
        if (init == 2) {
            cg.true_rn = sqrt(t[1]);
            return;
        }
        cg.xpend = 0;  // a residual of x: no step of x is pending (the host flushed it)
        if (init) {
            st->bb = t[0];
            cg.nb = sqrt(t[0]);
            cg.tol = rtol * cg.nb;
            cg.iter = 0;
            cg.max_iter = max_iter;
            cg.replacements = 0;
            cg.restart = 1;
            cg.alpha = 0.0;
            cg.beta = 0.0;
        }
        const double rn = sqrt(t[1]);
        cg.true_rn = rn;
        cg.rr = t[1];
        cg.rz = t[2];
        cg.restart = 1;
        if (init && cg.nb == 0.0) {
            cg.state = CG_ZERO_RHS;
        } else if (!isfinite(rn)) {
            cg.state = CG_BREAKDOWN;
        } else if (rn <= cg.tol) {
            cg.state = CG_CONVERGED;
        } else {
            if (!init) cg.replacements += 1;
            cg.state = cg.iter >= cg.max_iter ? CG_MAXIT : CG_RUNNING;
        }
    }
    __device__ uint32_t* ticket() const { return &st->tickets[0]; }
    __device__ double* partials() const { return part; }
};

// Direction sweep: p_new = M^{-1} r + beta p_old (filled into LDS and stored
// at own points), reduce p_new . A p_new; the last block forms alpha.
// beta and the restart flag are read from the device state at kernel start.
template <class V>
struct OpDir {
    using T = V;
    struct In {
        V r, p;
    };
    using Own = Nothing;
    static constexpr int NACC = 1;
    const V* r;
    const V* p_old;
    V* p_new;
    V minv, inv_h2;
    DevState* st;
    double* part;
    V beta;
    int restart;
    __device__ bool active() const { return st->cg.state == CG_RUNNING; }
    __device__ void prepare() {
        restart = st->cg.restart;
        beta = (V)st->cg.beta;
    }
    __device__ In fetch(size_t g) const {
        In v;
        v.r = r[g];
        v.p = restart ? V(0) : p_old[g];
        return v;
    }
    __device__ V make(const In& v, size_t g, bool own) const {
        V pn = minv * v.r;
        if (!restart) pn = pn + beta * v.p;
        if (own) st_own(pn, p_new + g);
        return pn;
    }
    __device__ Nothing pre(size_t) const { return Nothing{}; }
    __device__ void out(const Nothing&, size_t, V c, V xm, V xp, V ym, V yp, V zm, V zp,
                        double (&acc)[1]) const {
        const V q = apply_A<V>(c, xm, xp, ym, yp, zm, zp, inv_h2);
        acc[0] += (double)c * (double)q;
    }
    __device__ void finish(double (&t)[1]) const {
        CgScalars& cg = st->cg;
        cg.pq = t[0];
        const double a = cg.rz / t[0];
        cg.alpha = a;
        cg.restart = 0;
        if (!isfinite(a) || !(t[0] > 0.0)) cg.state = CG_BREAKDOWN;
    }
    __device__ uint32_t* ticket() const { return &st->tickets[1]; }
    __device__ double* partials() const { return part; }
};

// Update sweep: x += alpha p, r -= alpha A p; reduce r.r and r.M^{-1} r; the
// last block advances the iteration (stop test on ||r||, then beta).  For the
// FP32 inner solve of the mixed form the same test uses the inner threshold
// and CG_CANDIDATE just ends the inner solve.
template <class V>
struct OpUpd {
    using T = V;
    using In = V;
    struct Own {
        V x, r;
    };
    static constexpr int NACC = 2;
    const V* p;
    V* x;
    V* r;
    V minv, inv_h2;
    DevState* st;
    double* part;
    V alpha;
    __device__ bool active() const { return st->cg.state == CG_RUNNING; }
    __device__ void prepare() { alpha = (V)st->cg.alpha; }
    __device__ V fetch(size_t g) const { return p[g]; }
    __device__ V make(V v, size_t, bool) const { return v; }
    __device__ Own pre(size_t g) const {
        Own o;
        o.x = ld_own(x + g);
        o.r = ld_own(r + g);
        return o;
    }
    __device__ void out(const Own& o, size_t g, V c, V xm, V xp, V ym, V yp, V zm, V zp,
                        double (&acc)[2]) const {
        const V q = apply_A<V>(c, xm, xp, ym, yp, zm, zp, inv_h2);
        const V xv = o.x + alpha * c;
        const V rv = o.r - alpha * q;
        st_own(xv, x + g);
        st_own(rv, r + g);
        acc[0] += (double)rv * (double)rv;
        acc[1] += (double)rv * (double)(minv * rv);
    }
    __device__ void finish(double (&t)[2]) const {
        CgScalars& cg = st->cg;
        cg.rz_prev = cg.rz;
        cg.iter += 1;
        cg.rr = t[0];
        const double rn = sqrt(t[0]);
        if (!isfinite(rn)) {
            cg.state = CG_BREAKDOWN;
            return;
        }
        if (rn <= cg.tol) {
            cg.state = CG_CANDIDATE;
            return;
        }
        cg.beta = t[1] / cg.rz;
        cg.rz = t[1];
        if (cg.iter >= cg.max_iter) cg.state = CG_MAXIT;
    }
    __device__ uint32_t* ticket() const { return &st->tickets[2]; }
    __device__ double* partials() const { return part; }
};

// Start of the single-reduction form after a (re)computed residual: reduce
// r.r, gamma = r.M^{-1} r and delta = (M^{-1} r).A (M^{-1} r) with the same
// expressions as the single-reduction sweep; the first step takes
// p = M^{-1} r and alpha = gamma / delta.
template <class V>
struct OpCg1Start {
    using T = V;
    using In = V;
    using Own = Nothing;
    static constexpr int NACC = 3;
    const V* r;
    V minv, inv_h2;
    DevState* st;
    double* part;
    __device__ bool active() const { return st->cg.state == CG_RUNNING && st->cg.restart; }
    __device__ void prepare() {}
    __device__ V fetch(size_t g) const { return r[g]; }
    __device__ V make(V v, size_t, bool) const { return v; }
    __device__ Nothing pre(size_t) const { return Nothing{}; }
    __device__ void out(const Nothing&, size_t, V rv, V xm, V xp, V ym, V yp, V zm, V zp,
                        double (&acc)[3]) const {
        const V ar = apply_A<V>(rv, xm, xp, ym, yp, zm, zp, inv_h2);
        const V u = minv * rv;
        acc[0] += (double)rv * (double)rv;
        acc[1] += (double)rv * (double)u;
        acc[2] += (double)u * (double)(minv * ar);
    }
    __device__ void finish(double (&t)[3]) const {
        CgScalars& cg = st->cg;
        cg.rz = t[1];
        cg.pq = t[2];
        cg.alpha = t[1] / t[2];
        cg.beta = 0.0;
        cg.restart = 1;
        cg.xpend = 0;
        if (!(t[2] > 0.0) || !isfinite(cg.alpha)) cg.state = CG_BREAKDOWN;
    }
    __device__ uint32_t* ticket() const { return &st->tickets[1]; }
    __device__ double* partials() const { return part; }
};

// Mixed form, outer step: r = b - A x in FP64; reduce r.r; the last block
// decides.  (The correction x += ||r_prev|| d is a separate pass before it:
// a sweep never writes the array it stages, because neighbouring workgroups
// read that array as their halo.)
struct OpOuterResid {
    using T = double;
    using In = double;
    using Own = double;
    static constexpr int NACC = 1;
    const double* b;
    const double* x;
    double* r;
    double inv_h2;
    double tol;  // outer stop threshold rtol * ||b||
    int gate;    // 1: run only while the outer state is RUNNING and update it
    DevState* st;
    double* part;
    __device__ bool active() const { return !gate || st->outer_state == CG_RUNNING; }
    __device__ void prepare() {}
    __device__ double fetch(size_t g) const { return x[g]; }
    __device__ double make(double v, size_t, bool) const { return v; }
    __device__ double pre(size_t g) const { return ld_own(b + g); }
    __device__ void out(double bv, size_t g, double c, double xm, double xp, double ym, double yp,
                        double zm, double zp, double (&acc)[1]) const {
        const double rv = bv - apply_A<double>(c, xm, xp, ym, yp, zm, zp, inv_h2);
        st_own(rv, r + g);
        acc[0] += rv * rv;
    }
    __device__ void finish(double (&t)[1]) const {
        const double nr = sqrt(t[0]);
        st->out_nr = nr;
        st->out_sc = 1.0 / nr;
        if (!gate) return;
        st->cg.true_rn = nr;
        if (!isfinite(nr)) st->outer_state = CG_BREAKDOWN;
        else if (nr <= tol) st->outer_state = CG_CONVERGED;
    }
    __device__ uint32_t* ticket() const { return &st->tickets[3]; }
    __device__ double* partials() const { return part; }
};

// Flexible CG: q = A p (stored), reduce p . q.
// p_new = z + beta p_old (p_new = z on a restart), q = A p_new (stored when
// q is not null); reduce p_new . q into st->flex_pq.  The direction update
// of a PCG with a general preconditioner, fused into its product sweep.
struct OpAqZ {
    using T = double;
    struct In {
        double z, p;
    };
    using Own = Nothing;
    static constexpr int NACC = 1;
    const double* z;
    const double* p_old;
    double* p_new;
    double* q;
    double beta;
    int restart;
    double inv_h2;
    DevState* st;
    double* part;
    __device__ bool active() const { return true; }
    __device__ void prepare() {}
    __device__ In fetch(size_t g) const {
        In v;
        v.z = z[g];
        v.p = restart ? 0.0 : p_old[g];
        return v;
    }
    __device__ double make(const In& v, size_t g, bool own) const {
        const double pn = restart ? v.z : v.z + beta * v.p;
        if (own) st_own(pn, p_new + g);
        return pn;
    }
    __device__ Nothing pre(size_t) const { return Nothing{}; }
    __device__ void out(const Nothing&, size_t g, double c, double xm, double xp, double ym,
                        double yp, double zm, double zp, double (&acc)[1]) const {
        const double qv = apply_A<double>(c, xm, xp, ym, yp, zm, zp, inv_h2);
        if (q) st_own(qv, q + g);
        acc[0] += c * qv;
    }
    __device__ void finish(double (&t)[1]) const { st->flex_pq = t[0]; }
    __device__ uint32_t* ticket() const { return &st->tickets[1]; }
    __device__ double* partials() const { return part; }
};

// x += alpha p, r -= alpha A p (A p recomputed from the staged p, so q is
// never stored); reduce r . r into st->flex_rr.
struct OpUpdP {
    using T = double;
    using In = double;
    struct Own {
        double x, r;
    };
    static constexpr int NACC = 1;
    const double* p;
    double* x;
    double* r;
    double alpha, inv_h2;
    DevState* st;
    double* part;
    __device__ bool active() const { return true; }
    __device__ void prepare() {}
    __device__ double fetch(size_t g) const { return p[g]; }
    __device__ double make(double v, size_t, bool) const { return v; }
    __device__ Own pre(size_t g) const {
        Own o;
        o.x = ld_own(x + g);
        o.r = ld_own(r + g);
        return o;
    }
    __device__ void out(const Own& o, size_t g, double c, double xm, double xp, double ym,
                        double yp, double zm, double zp, double (&acc)[1]) const {
        const double q = apply_A<double>(c, xm, xp, ym, yp, zm, zp, inv_h2);
        st_own(o.x + alpha * c, x + g);
        const double rv = o.r - alpha * q;
        st_own(rv, r + g);
        acc[0] += rv * rv;
    }
    __device__ void finish(double (&t)[1]) const { st->flex_rr = t[0]; }
    __device__ uint32_t* ticket() const { return &st->tickets[2]; }
    __device__ double* partials() const { return part; }
};

struct OpAq {
    using T = double;
    using In = double;
    using Own = Nothing;
    static constexpr int NACC = 1;
    const double* p;
    double* q;
    double inv_h2;
    DevState* st;
    double* part;
    __device__ bool active() const { return true; }
    __device__ void prepare() {}
    __device__ double fetch(size_t g) const { return p[g]; }
    __device__ double make(double v, size_t, bool) const { return v; }
    __device__ Nothing pre(size_t) const { return Nothing{}; }
    __device__ void out(const Nothing&, size_t g, double c, double xm, double xp, double ym,
                        double yp, double zm, double zp, double (&acc)[1]) const {
        const double qv = apply_A<double>(c, xm, xp, ym, yp, zm, zp, inv_h2);
        st_own(qv, q + g);
        acc[0] += c * qv;
    }
    __device__ void finish(double (&t)[1]) const { st->flex_pq = t[0]; }
    __device__ uint32_t* ticket() const { return &st->tickets[1]; }
    __device__ double* partials() const { return part; }
};

// SSOR preconditioner, one half-sweep (a Jacobi step of an approximate
// triangular solve, Sec. 4.1's SSOR on the periodic grid):
//   out = oscale * (bscale * base + c * ((s_x + s_y) + s_z)) (+ add)
// with s the staged array's backward (dir 0: x-1, y-1, z-1) or forward
// (dir 1: x+1, y+1, z+1) neighbours, staged values scaled by sscale.
// Optionally reduces r . out into st->flex_zr (the preconditioned dot of
// PCG).  Summation order as in the oracle.
struct OpSsorHalf {
    using T = double;
    using In = double;
    struct Own {
        double base, add, r;
    };
    static constexpr int NACC = 1;
    const double* src;
    const double* base;
    const double* add;   // nullable
    const double* rdot;  // nullable: reduce rdot . out
    double* dst;
    double c, bscale, sscale, oscale;
    int dir;
    DevState* st;
    double* part;
    __device__ bool active() const { return true; }
    __device__ void prepare() {}
    __device__ double fetch(size_t g) const { return src[g]; }
    __device__ double make(double v, size_t, bool) const { return sscale == 1.0 ? v : sscale * v; }
    __device__ Own pre(size_t g) const {
        Own o;
        o.base = ld_own(base + g);
        o.add = add ? ld_own(add + g) : 0.0;
        o.r = rdot ? ld_own(rdot + g) : 0.0;
        return o;
    }
    __device__ void out(const Own& o, size_t g, double, double xm, double xp, double ym, double yp,
                        double zm, double zp, double (&acc)[1]) const {
        const double sn = dir == 0 ? (xm + ym) + zm : (xp + yp) + zp;
        double v = (bscale == 1.0 ? o.base : bscale * o.base) + c * sn;
        if (oscale != 1.0) v = oscale * v;
        if (add) v = v + o.add;
        st_own(v, dst + g);
        acc[0] += o.r * v;
    }
    __device__ void finish(double (&t)[1]) const {
        if (rdot) st->flex_zr = t[0];
    }
    __device__ uint32_t* ticket() const { return &st->tickets[4]; }
    __device__ double* partials() const { return part; }
};

// SSOR, one whole approximate triangular solve in one z-march (temporal
// blocking of its K Jacobi steps).  Forward (DIR 0, backward neighbours):
//   y_0 = s0 * src,  y_l = y_0 + c ((y_{l-1}[x-1] + y_{l-1}[y-1]) + y_{l-1}[z-1]),
// backward (DIR 1) the same with forward neighbours and s0 = 1; the output is
// oscale * y_K (+ add), optionally reducing rdot . out into st->flex_zr.
// Level l at plane z needs level l-1 at planes z and z-1 at the neighbours on
// one side, so each level is computed on the TX x TY tile widened by K - l
// points on that side, and each level keeps its previous plane in LDS: the
// block marches its z range (upward for DIR 0, downward for DIR 1) starting K
// planes early, after which every level is valid.  The arithmetic and its
// order are those of K separate half-sweeps (identical results); the bytes
// moved are one read of src (with a K-point halo) and one write per point.
// Every level is computed on the whole (TX + K) x (TY + K) region of level 0
// (values outside a level's own region are not needed by any output and are
// simply not used), so each thread owns the same NP0 region points at every
// level and plane: its level-0 value (the B term) and each level's value of
// the previous plane (the z neighbour) stay in its registers, and only the
// in-plane upwind neighbours go through LDS -- one padded plane per level
// (a zero row and column on the upwind side keep the edge reads in bounds).
template <int K, int DIR, int TX, int TY>
__global__ __launch_bounds__(kNT) void ssor_fused_kernel(int n, int bounded, int nbx, int nby,
                                                         int zlen,
                                                         const double* __restrict__ src,
                                                         const double* add,  // may be dst
                                                         const double* __restrict__ rdot,
                                                         double* dst, double s0,
                                                         double c, double oscale, DevState* st,
                                                         double* part) {
    constexpr int W0 = TX + K, H0 = TY + K;
    constexpr int WP = W0 + 1, HP = H0 + 1;  // padded plane
    constexpr int PLANE = WP * HP;
    // Region points per thread: TX consecutive lanes take the TX tile columns
    // of one region row (whole cache lines for the loads and the stores); the
    // spare lane groups of the last slot take the K halo columns.
    constexpr int GPS = kNT / TX;  // row groups per slot
    constexpr int NP0 = (H0 + (K * H0 + TX - 1) / TX + GPS - 1) / GPS;
    __shared__ double lds[K][PLANE];
    __shared__ double red[kNT / kWave];
    __shared__ int lflag;
    const int tid = threadIdx.x;
    const uint32_t lb = remap_xcd(blockIdx.x, gridDim.x);
    const int bx = (int)(lb % nbx), by = (int)((lb / nbx) % nby), bz = (int)(lb / (nbx * nby));
    const int x0 = bx * TX, y0 = by * TY;
    const int z0 = bz * zlen, z1 = z0 + zlen;
    const size_t nn = (size_t)n * n;
    // region origin: widened towards -x, -y (DIR 0) or +x, +y (DIR 1)
    const int ax = DIR == 0 ? x0 - K : x0, ay = DIR == 0 ? y0 - K : y0;
    // padded offset of region point (lx, ly): the pad is the row/column before
    // the region (DIR 0) or after it (DIR 1)
    constexpr int PO = DIR == 0 ? WP + 1 : 0;
    auto outside = [n](int v) { return v < 0 || v >= n; };
    auto gmap = [n, bounded](int v) {
        if (v >= 0 && v < n) return v;
        if (!bounded) return v < 0 ? v + n : v - n;
        return v < 0 ? 0 : n - 1;
    };
    // this thread's region points (fixed for all levels and planes)
    int pofs[NP0];            // padded LDS offset, -1: no point
    uint32_t goff[NP0];       // in-plane global offset of the (mapped) point
    uint32_t outm = 0;        // bit k: point k is an output point
    uint32_t zerom = 0;       // bit k: point k lies outside a bounded grid
#pragma unroll
    for (int k = 0; k < NP0; ++k) {
        const int unit = k * GPS + tid / TX, lane = tid % TX;
        int lx = -1, ly = -1;
        if (unit < H0) {
            lx = (DIR == 0 ? K : 0) + lane;  // the tile's columns
            ly = unit;
        } else {
            const int e = (unit - H0) * TX + lane;  // halo column entry
            if (e < K * H0) {
                lx = (DIR == 0 ? 0 : TX) + e % K;
                ly = e / K;
            }
        }
        pofs[k] = -1;
        goff[k] = 0;
        if (ly >= 0) {
            const int rx = ax + lx, ry = ay + ly;
            pofs[k] = PO + ly * WP + lx;
            goff[k] = (uint32_t)gmap(ry) * (uint32_t)n + (uint32_t)gmap(rx);
            const bool in_tile = rx >= x0 && rx < x0 + TX && ry >= y0 && ry < y0 + TY;
            if (in_tile) outm |= 1u << k;
            if (bounded && (outside(rx) || outside(ry))) zerom |= 1u << k;
        }
    }
    for (int i = tid; i < K * PLANE; i += kNT) (&lds[0][0])[i] = 0.0;
    double acc[1] = {0.0};
    double stg[NP0];          // level 0 of the next plane (prefetched)
    double prev[K][NP0];      // levels 0..K-1 at the previous plane
#pragma unroll
    for (int l = 0; l < K; ++l)
#pragma unroll
        for (int k = 0; k < NP0; ++k) prev[l][k] = 0.0;
    const int nsteps = zlen + K;  // planes in march order: z0 - K .. z1 - 1 (DIR 0)
    auto zof = [&](int p) { return DIR == 0 ? z0 - K + p : z1 - 1 + K - p; };
    auto fetch0 = [&](int p) {
        const int zr = zof(p);
        const bool zout = bounded && outside(zr);
        const size_t zo = (size_t)gmap(zr) * nn;
#pragma unroll
        for (int k = 0; k < NP0; ++k) {
            const double v = pofs[k] >= 0 ? src[zo + goff[k]] : 0.0;
            stg[k] = (zout || ((zerom >> k) & 1u)) ? 0.0 : v;
        }
    };
    __syncthreads();
    fetch0(0);
    for (int t = 0; t < nsteps; ++t) {
        const int z = zof(t);
        const bool zout = bounded && outside(z);
        const bool out_plane = DIR == 0 ? (z >= z0) : (z < z1);
        double cur[NP0];
#pragma unroll
        for (int k = 0; k < NP0; ++k) {
            cur[k] = s0 == 1.0 ? stg[k] : s0 * stg[k];
            if (pofs[k] >= 0) lds[0][pofs[k]] = cur[k];
        }
        double B[NP0];
#pragma unroll
        for (int k = 0; k < NP0; ++k) B[k] = cur[k];
        if (t + 1 < nsteps) fetch0(t + 1);
        __syncthreads();
#pragma unroll
        for (int l = 1; l <= K; ++l) {
            const double* P = lds[l - 1];
            double nxt[NP0];
#pragma unroll
            for (int k = 0; k < NP0; ++k) {
                nxt[k] = 0.0;
                if (pofs[k] < 0) continue;
                const int pi = pofs[k];
                const double sn = DIR == 0 ? (P[pi - 1] + P[pi - WP]) + prev[l - 1][k]
                                           : (P[pi + 1] + P[pi + WP]) + prev[l - 1][k];
                double v = B[k] + c * sn;
                if (bounded && (zout || ((zerom >> k) & 1u))) v = 0.0;
                nxt[k] = v;
            }
            // the previous plane's level l-1 values are consumed: keep this plane's
#pragma unroll
            for (int k = 0; k < NP0; ++k) prev[l - 1][k] = cur[k];
            if (l < K) {
                // level l's plane was last read by level l+1 of the previous
                // plane, before the end-of-plane barrier
#pragma unroll
                for (int k = 0; k < NP0; ++k)
                    if (pofs[k] >= 0) lds[l][pofs[k]] = nxt[k];
                __syncthreads();
#pragma unroll
                for (int k = 0; k < NP0; ++k) cur[k] = nxt[k];
            } else if (out_plane) {
#pragma unroll
                for (int k = 0; k < NP0; ++k) {
                    if (!((outm >> k) & 1u)) continue;
                    const size_t g = (size_t)z * nn + goff[k];
                    double o = oscale == 1.0 ? nxt[k] : oscale * nxt[k];
                    if (add) o = o + add[g];
                    dst[g] = o;
                    if (rdot) acc[0] += rdot[g] * o;
                }
            }
        }
        __syncthreads();  // level K's reads of level K-1 done before the next plane
    }
    block_sum<kNT, 1>(acc, red);
    if (tid == 0) part[lb] = acc[0];
    if (last_block(&st->tickets[4], gridDim.x, &lflag)) {
        double tot[1];
        sum_partials<kNT, 1>(part, (int)gridDim.x, tot, red);
        if (tid == 0 && rdot) st->flex_zr = tot[0];
    }
}

// --------------------------------------------------------------------------
// Single-reduction Jacobi-PCG sweep: the arrangement of Chronopoulos and
// Gear, which produces the same iterates as the direction + update pair in
// exact arithmetic but needs one reduction per iteration.  From r_k, p_{k-1},
// x_k and the scalars alpha_k, beta_k one sweep forms
//   p_k = M^{-1} r_k + beta_k p_{k-1},  x_{k+1} = x_k + alpha_k p_k,
//   r_{k+1} = r_k - alpha_k A p_k,
// and reduces, with u = M^{-1} r_{k+1} and q = A p_k,
//   r.r,  gamma = r.u,  delta = u.A u,  sigma = u.q,  pi = p_k.q;
// the last block forms beta_{k+1} = gamma_{k+1} / gamma_k and
//   alpha_{k+1} = gamma_{k+1} / p_{k+1}.A p_{k+1},
//   p_{k+1}.A p_{k+1} = delta + 2 beta sigma + beta^2 pi
// (the expansion of p_{k+1} = u + beta p_k; Chronopoulos and Gear shorten it
// to delta - beta gamma / alpha_k by the orthogonality of the residuals,
// which a continued inner solve of the mixed form does not keep exactly).
// Each of r, p, x is read once and written once: 48 bytes per grid point and
// iteration against 64 for the pair.
//
// Tiling: a TX x TY tile of (x, y) marches over its share of the z planes.
// A r_{k+1} at the tile needs r_{k+1} on a one-point ring, which needs p_k on
// a two-point ring; every stage is evaluated on the whole (TX+4) x (TY+4)
// region (the outer values are never used), so each thread owns the same
// region points at every stage and plane, keeps their z neighbours in
// registers and passes only in-plane neighbours through LDS.  At step j the
// block forms p_k(j) (staged two planes ahead), r_{k+1}(j), and the outputs
// of plane j-1.  Two LDS slots per stage leave one barrier per plane.  The
// padded border of each LDS plane is never written (zero), which keeps the
// region edge's reads in bounds.  Periodic box only: r_in and p_in are read
// as halos by neighbouring blocks and are never written here.
// V = double: the FP64 solve; V = float: the inner solve of the mixed form
// (dot products accumulated in FP64 as in the two-sweep form).  pgiven: p_in
// already holds p_k (formed, with its exact p.A p, by a direction sweep: the
// first step of an inner solve that continues the previous direction).
//
// XM: how the sweep treats x.  0: x_{k+1} = x_k + alpha_k p_k at every sweep
// (48 B/point).  1 and 2 alternate (FP64 solve): x is not updated by an odd
// (XM = 1) sweep, which records alpha_k and the buffer holding p_k as a
// pending update; the next (XM = 2) sweep reads p_k as its p_in anyway and
// applies x = (x + alpha_k p_k) + alpha_{k+1} p_{k+1}, the same two updates
// in the same order (bit-identical x), so x is read and written every other
// iteration: 32 and 48 B/point, 40 on average.  A pending update left when
// the state leaves RUNNING is applied by cg1_flush_kernel before x is used.
template <class V, int TX, int TY, int NT, int XM>
__global__ __launch_bounds__(NT) void cg1_kernel(int n, int nbx, int nby, int nbz,
                                                  const V* __restrict__ r_in,
                                                  V* __restrict__ r_out,
                                                  const V* __restrict__ p_in,
                                                  V* __restrict__ p_out, V* x, V minv, V inv_h2,
                                                  DevState* st, double* part, int pgiven,
                                                  int pslot) {
    constexpr int W0 = TX + 4, H0 = TY + 4;
    constexpr int WP = W0 + 2, HP = H0 + 2;
    constexpr int PLANE = WP * HP;
    // Region points per thread.  With tiles a multiple of 64 wide each wave
    // takes 64 aligned columns of one row of the tile (whole cache lines for
    // the loads and the stores) and the spare waves of the last slot take the
    // four halo columns; otherwise points are dealt out in row-major order.
    constexpr bool ROWS = TX % kWave == 0;
    constexpr int NW = NT / kWave;
    constexpr int SEG = TX / kWave;  // wave segments per row
    constexpr int NP = ROWS ? (H0 * SEG + (4 * H0 + kWave - 1) / kWave + NW - 1) / NW
                            : (W0 * H0 + NT - 1) / NT;
    __shared__ V lp[2][PLANE];
    __shared__ V lr[2][PLANE];
    __shared__ double red[5 * (NT / kWave)];
    __shared__ int lflag;
    if (st->cg.state != CG_RUNNING) return;
    const int restart = st->cg.restart;
    const V alpha = (V)st->cg.alpha;
    const V beta = (V)st->cg.beta;
    const V alpha_p = XM == 2 ? (V)st->cg.alpha_pend : V(0);

    const int tid = threadIdx.x;
    const uint32_t nb = (uint32_t)(nbx * nby * nbz);
    const uint32_t lb = remap_xcd(blockIdx.x, nb);
    const int bx = (int)(lb % nbx), by = (int)((lb / nbx) % nby), bz = (int)(lb / (nbx * nby));
    const int x0 = bx * TX, y0 = by * TY;
    const int z0 = (int)(((int64_t)bz * n) / nbz);
    const int z1 = (int)((((int64_t)bz + 1) * n) / nbz);
    const size_t nn = (size_t)n * n;
    auto wrap = [n](int v) { return v < 0 ? v + n : (v >= n ? v - n : v); };

    int pofs[NP];       // padded LDS offset of region point k, -1: none
    uint32_t goff[NP];  // its in-plane global offset (periodic image)
    uint32_t ownm = 0;  // bit k: point k is in the tile
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        int lx = -1, ly = -1;
        if constexpr (ROWS) {
            const int unit = k * NW + tid / kWave, lane = tid % kWave;
            if (unit < H0 * SEG) {
                lx = 2 + (unit % SEG) * kWave + lane;
                ly = unit / SEG;
            } else {
                const int e = (unit - H0 * SEG) * kWave + lane;  // halo column entry
                if (e < 4 * H0) {
                    const int c = e & 3;
                    lx = c < 2 ? c : TX + c;  // columns 0, 1, TX+2, TX+3
                    ly = e >> 2;
                }
            }
        } else {
            const int e = tid + k * NT;
            if (e < W0 * H0) {
                lx = e % W0;
                ly = e / W0;
            }
        }
        pofs[k] = -1;
        goff[k] = 0;
        if (ly >= 0) {
            pofs[k] = (ly + 1) * WP + lx + 1;
            goff[k] = (uint32_t)wrap(y0 - 2 + ly) * (uint32_t)n + (uint32_t)wrap(x0 - 2 + lx);
            if (lx >= 2 && lx < TX + 2 && ly >= 2 && ly < TY + 2) ownm |= 1u << k;
        }
    }
    for (int i = tid; i < 2 * PLANE; i += NT) {
        (&lp[0][0])[i] = V(0);
        (&lr[0][0])[i] = V(0);
    }

    V ldr[NP], ldp[NP];  // r_k, p_{k-1} (p_k if pgiven) of the plane being staged
    auto fetch = [&](int zr) {
        const size_t zo = (size_t)wrap(zr) * nn;
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            ldr[k] = V(0);
            ldp[k] = V(0);
            if (pofs[k] < 0) continue;
            ldr[k] = r_in[zo + goff[k]];
            // XM 2: p_in is the pending direction, needed for x even on a restart
            if (!restart || XM == 2) ldp[k] = p_in[zo + goff[k]];
        }
    };
    // p_k from the staged loads, in the direction sweep's order
    auto dir = [&](int k) {
        if (pgiven) return ldp[k];
        V v = minv * ldr[k];
        if (!restart) v = v + beta * ldp[k];
        return v;
    };
    V pm[NP], pc[NP], pn[NP];  // p_k at planes j-1, j, j+1
    V rc[NP], rn[NP];          // r_k at planes j, j+1
    V s2[NP], s1[NP];          // r_{k+1} at planes j-2, j-1
    V xo[NP], xn[NP];          // x_k at planes j-1, j (tile points)
    V qm[NP];                  // A p_k at plane j-1
    V om[XM == 2 ? NP : 1], oc[XM == 2 ? NP : 1], on[XM == 2 ? NP : 1];  // pending p, j-1..j+1
    fetch(z0 - 2);
#pragma unroll
    for (int k = 0; k < NP; ++k) pm[k] = dir(k);
    if constexpr (XM == 2) {
#pragma unroll
        for (int k = 0; k < NP; ++k) om[k] = ldp[k];
    }
    fetch(z0 - 1);
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        pc[k] = dir(k);
        rc[k] = ldr[k];
    }
    if constexpr (XM == 2) {
#pragma unroll
        for (int k = 0; k < NP; ++k) oc[k] = ldp[k];
    }
    fetch(z0);
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        pn[k] = dir(k);
        rn[k] = ldr[k];
        s2[k] = s1[k] = xo[k] = xn[k] = qm[k] = V(0);
    }
    if constexpr (XM == 2) {
#pragma unroll
        for (int k = 0; k < NP; ++k) on[k] = ldp[k];
    }
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    __syncthreads();  // LDS cleared before the first stores

    const int nsteps = z1 - z0 + 2;  // j = z0 - 1 .. z1
    for (int s = 0; s < nsteps; ++s) {
        const int j = z0 - 1 + s;
        const int slot = s & 1;
        V* LP = lp[slot];
        V* LR = lr[slot];
        const V* LRo = lr[slot ^ 1];
#pragma unroll
        for (int k = 0; k < NP; ++k)
            if (pofs[k] >= 0) LP[pofs[k]] = pc[k];
        if (j + 2 <= z1 + 1) fetch(j + 2);
        if (XM != 1 && j >= z0 && j < z1) {
            const size_t zo = (size_t)j * nn;
#pragma unroll
            for (int k = 0; k < NP; ++k)
                if ((ownm >> k) & 1u) xn[k] = ld_own(x + zo + goff[k]);
        }
        __syncthreads();
        // r_{k+1}(j) on the region
        V r1[NP], q1[NP];
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            r1[k] = q1[k] = V(0);
            if (pofs[k] < 0) continue;
            const int pi = pofs[k];
            q1[k] = apply_A<V>(pc[k], LP[pi - 1], LP[pi + 1], LP[pi - WP], LP[pi + WP], pm[k],
                               pn[k], inv_h2);
            r1[k] = rc[k] - alpha * q1[k];
            LR[pi] = r1[k];
        }
        // outputs of plane j-1 (its in-plane r_{k+1} neighbours were stored
        // in the previous step, before this step's barrier)
        if (j - 1 >= z0 && j - 1 < z1) {
            const size_t zo = (size_t)(j - 1) * nn;
#pragma unroll
            for (int k = 0; k < NP; ++k) {
                if (!((ownm >> k) & 1u)) continue;
                const int pi = pofs[k];
                const V rv = s1[k];
                const V ar = apply_A<V>(rv, LRo[pi - 1], LRo[pi + 1], LRo[pi - WP], LRo[pi + WP],
                                        s2[k], r1[k], inv_h2);
                const V u = minv * rv;
                acc[0] += (double)rv * (double)rv;
                acc[1] += (double)rv * (double)u;
                acc[2] += (double)u * (double)(minv * ar);
                acc[3] += (double)u * (double)qm[k];
                acc[4] += (double)pm[k] * (double)qm[k];
                const size_t g = zo + goff[k];
                if constexpr (XM == 0) st_own(xo[k] + alpha * pm[k], x + g);
                if constexpr (XM == 2) st_own((xo[k] + alpha_p * om[k]) + alpha * pm[k], x + g);
                st_own(rv, r_out + g);
                st_own(pm[k], p_out + g);
            }
        }
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            s2[k] = s1[k];
            s1[k] = r1[k];
            qm[k] = q1[k];
            pm[k] = pc[k];
            pc[k] = pn[k];
            rc[k] = rn[k];
            xo[k] = xn[k];
            pn[k] = dir(k);
            rn[k] = ldr[k];
        }
        if constexpr (XM == 2) {
#pragma unroll
            for (int k = 0; k < NP; ++k) {
                om[k] = oc[k];
                oc[k] = on[k];
                on[k] = ldp[k];
            }
        }
    }

    block_sum<NT, 5>(acc, red);
    if (tid == 0) {
#pragma unroll
        for (int k = 0; k < 5; ++k) part[(size_t)k * nb + lb] = acc[k];
    }
    if (last_block(&st->tickets[2], nb, &lflag)) {
        double t[5];
        sum_partials<NT, 5>(part, (int)nb, t, red);
        if (tid == 0) {
            CgScalars& cg = st->cg;
            if (XM == 1) {
                cg.alpha_pend = cg.alpha;  // this sweep's step, not yet in x
                cg.pend_slot = pslot;
            }
            cg.xpend = XM == 1 ? 1 : 0;
            cg.rz_prev = cg.rz;
            cg.iter += 1;
            cg.rr = t[0];
            const double rn2 = sqrt(t[0]);
            if (!isfinite(rn2)) {
                cg.state = CG_BREAKDOWN;
                return;
            }
            if (rn2 <= cg.tol) {
                cg.state = CG_CANDIDATE;
                return;
            }
            const double b = t[1] / cg.rz;
            const double den = t[2] + 2.0 * b * t[3] + b * b * t[4];
            if (den > 0.0 && isfinite(den)) {
                cg.beta = b;
                cg.alpha = t[1] / den;
                cg.pq = den;
                cg.restart = 0;
            } else {
                // p.A p lost to cancellation: restart from p = M^{-1} r
                // (its curvature is delta)
                cg.beta = 0.0;
                cg.alpha = t[1] / t[2];
                cg.pq = t[2];
                cg.restart = 1;
                if (!(t[2] > 0.0) || !isfinite(cg.alpha)) cg.state = CG_BREAKDOWN;
            }
            cg.rz = t[1];
            if (cg.state == CG_RUNNING && cg.iter >= cg.max_iter) cg.state = CG_MAXIT;
        }
    }
}

// Field: E = -grad (phi - mean) from the gauge-fixed values, W_x =
// (1/2) h^3 sum Ex^2.  phi itself is shifted by a separate pass afterwards.
struct OpField {
    using T = double;
    using In = double;
    using Own = Nothing;
    static constexpr int NACC = 1;
    const double* phi;
    double* ex;
    double* ey;
    double* ez;
    double ehalf, h3, mean;
    int gauge;  // 0: phi as it is (Dirichlet box)
    DevState* st;
    double* part;
    __device__ bool active() const { return true; }
    __device__ void prepare() { mean = gauge ? st->mean : 0.0; }
    __device__ double fetch(size_t g) const { return phi[g]; }
    __device__ double make(double v, size_t, bool) const { return v - mean; }
    __device__ Nothing pre(size_t) const { return Nothing{}; }
    __device__ void out(const Nothing&, size_t g, double, double xm, double xp, double ym,
                        double yp, double zm, double zp, double (&acc)[1]) const {
        const double exv = -(xp - xm) * ehalf;
        st_own(exv, ex + g);
        st_own(-(yp - ym) * ehalf, ey + g);
        st_own(-(zp - zm) * ehalf, ez + g);
        acc[0] += exv * exv;
    }
    __device__ void finish(double (&t)[1]) const { st->wx = 0.5 * t[0] * h3; }
    __device__ uint32_t* ticket() const { return &st->tickets[4]; }
    __device__ double* partials() const { return part; }
};

// --------------------------------------------------------------------------
// Streaming (non-stencil) kernels.
constexpr int kStreamBlocks = 2048;

// r32 = (float)(r * (1/||r||)), d = 0; reduce r32.r32 and r32.(minv r32); the
// last block starts the inner solve.
// Reliable form (`reliable`): when the previous inner solve ended at its
// tolerance or step cap, its last direction p_j carries over instead of a
// restart: p~' = M r~' + beta~ p~_j with beta~ = (nr' / nr) (r~'.M r~') /
// (r~_j.M r~_j) in the scaled variables (CG's recurrence with the residual
// replaced by b - A x; nr, nr' the outer residual norms before and after).
__global__ __launch_bounds__(kNT) void convert32_kernel(int64_t n3, const double* __restrict__ r,
                                                        float* __restrict__ r32,
                                                        float* __restrict__ d32, float minvf,
                                                        int reliable, double inner_rtol,
                                                        int64_t max_inner, DevState* st,
                                                        double* part) {
    __shared__ double red[2 * (kNT / kWave)];
    __shared__ int lflag;
    if (st->outer_state != CG_RUNNING) return;
    const double sc = st->out_sc;
    double acc[2] = {0.0, 0.0};
    for (int64_t i = (int64_t)blockIdx.x * kNT + threadIdx.x; i < n3; i += (int64_t)gridDim.x * kNT) {
        const float v = (float)(r[i] * sc);
        r32[i] = v;
        d32[i] = 0.0f;
        acc[0] += (double)v * (double)v;
        acc[1] += (double)v * (double)(minvf * v);
    }
    block_sum<kNT, 2>(acc, red);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = acc[0];
        part[gridDim.x + blockIdx.x] = acc[1];
    }
    if (last_block(&st->tickets[5], gridDim.x, &lflag)) {
        double tot[2];
        sum_partials<kNT, 2>(part, gridDim.x, tot, red);
        if (threadIdx.x == 0) {
            CgScalars& cg = st->cg;
            const double n0 = sqrt(tot[0]);
            // carry the direction only while the refinement's true reduction
            // stays within a factor 4 of the last inner solve's recursive one
            // (FP32 drift of about eps32 kappa makes the replaced residual
            // inconsistent with the recursion at tight inner tolerances): a
            // residual-gap test, the gap between the true and the recursive
            // residual being at least out_nr - rec * prev_nr
            const double rec = sqrt(cg.rr) / cg.nb;
            const bool ended = reliable && (cg.state == CG_CANDIDATE || cg.state == CG_MAXIT) &&
                               st->prev_nr > 0.0;
            const bool cont = ended && st->out_nr <= 4.0 * rec * st->prev_nr;
            if (ended && !cont) st->gap_restarts += 1;
            const double bt = cont ? (st->out_nr / st->prev_nr) * (tot[1] / cg.rz_prev) : 0.0;
            cg.nb = n0;
            cg.tol = inner_rtol * n0;
            cg.rz = tot[1];
            cg.rr = tot[0];
            cg.iter = 0;
            cg.max_iter = max_inner;
            cg.restart = (cont && isfinite(bt)) ? 0 : 1;
            cg.beta = cg.restart ? 0.0 : bt;
            cg.xpend = 0;
            cg.state = (n0 == 0.0 || !isfinite(n0)) ? CG_BREAKDOWN : CG_RUNNING;
        }
    }
}

// x += ||r|| * d: the refinement step's correction, before the next residual
// (which overwrites out_nr; its value is kept as prev_nr).
__global__ __launch_bounds__(kNT) void update_x_kernel(int64_t n3, double* __restrict__ x,
                                                       const float* __restrict__ d,
                                                       DevState* st) {
    const double s = st->out_nr;
    if (blockIdx.x == 0 && threadIdx.x == 0) st->prev_nr = s;
    for (int64_t i = (int64_t)blockIdx.x * kNT + threadIdx.x; i < n3; i += (int64_t)gridDim.x * kNT)
        x[i] = x[i] + s * (double)d[i];
}

// sum of v (what = 0: st->mean = sum/n3; what = 1: st->bb = sum v^2).
__global__ __launch_bounds__(kNT) void sum_kernel(int64_t n3, const double* __restrict__ v,
                                                  DevState* st, double* part, int what) {
    __shared__ double red[kNT / kWave];
    __shared__ int lflag;
    double acc[1] = {0.0};
    for (int64_t i = (int64_t)blockIdx.x * kNT + threadIdx.x; i < n3; i += (int64_t)gridDim.x * kNT) {
        const double a = v[i];
        acc[0] += what ? a * a : a;
    }
    block_sum<kNT, 1>(acc, red);
    if (threadIdx.x == 0) part[blockIdx.x] = acc[0];
    if (last_block(&st->tickets[6], gridDim.x, &lflag)) {
        double tot[1];
        sum_partials<kNT, 1>(part, gridDim.x, tot, red);
        if (threadIdx.x == 0) {
            if (what == 0) st->mean = tot[0] / (double)n3;
            else st->bb = tot[0];
            st->sum = tot[0];
        }
    }
}

// a = b + s c (24 bytes per element): the achievable-bandwidth reference the
// sweeps are compared with.  Two consecutive elements per thread as 16-byte
// loads and stores (arrays 16-byte aligned, n even), else one.
typedef double triad_v2 __attribute__((ext_vector_type(2)));
__global__ __launch_bounds__(256) void triad2_kernel(int64_t n2, const triad_v2* __restrict__ b,
                                                     const triad_v2* __restrict__ c,
                                                     triad_v2* __restrict__ a, double s) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n2) {
        const triad_v2 x = b[i], y = c[i];
        triad_v2 r;
        r.x = x.x + s * y.x;
        r.y = x.y + s * y.y;
        __builtin_nontemporal_store(r, a + i);
    }
}
__global__ __launch_bounds__(256) void triad1_kernel(int64_t n, const double* __restrict__ b,
                                                     const double* __restrict__ c,
                                                     double* __restrict__ a, double s) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) __builtin_nontemporal_store(b[i] + s * c[i], a + i);
}

hipError_t launch_triad(int64_t n, const double* b, const double* c, double* a, double s,
                        hipStream_t st) {
    if ((n % 2) == 0 && (((uintptr_t)a | (uintptr_t)b | (uintptr_t)c) & 15u) == 0)
        hipLaunchKernelGGL(triad2_kernel, dim3((uint32_t)((n / 2 + 255) / 256)), dim3(256), 0, st,
                           n / 2, (const triad_v2*)b, (const triad_v2*)c, (triad_v2*)a, s);
    else
        hipLaunchKernelGGL(triad1_kernel, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, st, n,
                           b, c, a, s);
    return hipGetLastError();
}

__global__ __launch_bounds__(kNT) void fill_kernel(int64_t n, double* __restrict__ v, double val) {
    for (int64_t i = (int64_t)blockIdx.x * kNT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kNT)
        v[i] = val;
}

// --------------------------------------------------------------------------
// Host side.
SweepGeo make_geo(int n, int bc) {
    SweepGeo g;
    g.n = n;
    g.bc = bc;
    g.nbx = g.nby = g.nbz = g.nb = 0;
    return g;
}

int max_sweep_blocks() { return kMaxSweepBlocks; }

// Launch one wave of resident workgroups: every (x, y) tile column gets the
// same number of blocks (nbz), each marching an equal share of the z planes,
// so all blocks finish together and the z-halo overhead is 2 planes per share.
template <class Op, int TX, int BC>
static hipError_t launch_sweep_tx(const Op& op, const SweepGeo& gin, hipStream_t s) {
    static int occ = 0, cus = 0;
    if (occ == 0) {
        int o = 0, c = 0, dev = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&o, sweep_kernel<Op, TX, BC>, kNT, 0) !=
                hipSuccess || o < 1)
            o = 1;
        (void)hipGetDevice(&dev);
        if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            c < 1)
            c = 1;
        cus = c;
        occ = o;
    }
    const int n = gin.n;
    SweepGeo g = gin;
    g.nbx = (uint32_t)(n / TX);
    g.nby = (uint32_t)(n / kTY);
    const uint32_t tiles = g.nbx * g.nby;
    uint32_t nbz = (uint32_t)(occ * cus) / tiles;
    const uint32_t cap = (uint32_t)kMaxSweepBlocks / tiles;
    if (nbz > cap) nbz = cap;
    if (nbz > (uint32_t)(n / 2)) nbz = (uint32_t)(n / 2);
    if (nbz < 1) nbz = 1;
    g.nbz = nbz;
    g.nb = tiles * nbz;
    hipLaunchKernelGGL((sweep_kernel<Op, TX, BC>), dim3(g.nb), dim3(kNT), 0, s, op, g);
    return hipGetLastError();
}

template <class Op, int BC>
static hipError_t launch_sweep_bc(const Op& op, const SweepGeo& g, hipStream_t s) {
    if (g.n % 64 == 0) return launch_sweep_tx<Op, 64, BC>(op, g, s);
    return launch_sweep_tx<Op, 32, BC>(op, g, s);
}

template <class Op>
static hipError_t launch_sweep(const Op& op, const SweepGeo& g, hipStream_t s) {
    if (g.bc == 1) return launch_sweep_bc<Op, 1>(op, g, s);
    if (g.bc == 2) return launch_sweep_bc<Op, 2>(op, g, s);
    return launch_sweep_bc<Op, 0>(op, g, s);
}

hipError_t launch_residual64(const SweepGeo& g, const double* b, const double* x, double* r,
                             double minv, double inv_h2, int init, double rtol, int64_t max_iter,
                             DevState* st, double* partials, hipStream_t s) {
    OpResidual64 op{b, x, r, minv, inv_h2, rtol, max_iter, init, st, partials};
    return launch_sweep(op, g, s);
}

hipError_t launch_dir64(const SweepGeo& g, const double* r, const double* p_old, double* p_new,
                        double minv, double inv_h2, DevState* st, double* partials, hipStream_t s) {
    OpDir<double> op{r, p_old, p_new, minv, inv_h2, st, partials, 0.0, 0};
    return launch_sweep(op, g, s);
}

hipError_t launch_upd64(const SweepGeo& g, const double* p_new, double* x, double* r, double minv,
                        double inv_h2, DevState* st, double* partials, hipStream_t s) {
    OpUpd<double> op{p_new, x, r, minv, inv_h2, st, partials, 0.0};
    return launch_sweep(op, g, s);
}

bool cg1_supported(const SweepGeo& g) { return g.bc == 0 && g.n % 32 == 0 && g.n >= 32; }

hipError_t launch_cg1_start(const SweepGeo& g, const double* r, double minv, double inv_h2,
                            DevState* st, double* partials, hipStream_t s) {
    OpCg1Start<double> op{r, minv, inv_h2, st, partials};
    return launch_sweep(op, g, s);
}

hipError_t launch_cg1_start32(const SweepGeo& g, const float* r, float minvf, float inv_h2f,
                              DevState* st, double* partials, hipStream_t s) {
    OpCg1Start<float> op{r, minvf, inv_h2f, st, partials};
    return launch_sweep(op, g, s);
}

// One resident wave of workgroups: TX x TY tiles, the z planes of each tile
// column split evenly over nbz blocks.  Shapes measured at 512^3 (FP64):
// 64 x 32 tiles of 512 threads and 128 x 16 x 512 alike (one workgroup per
// CU, 2 waves per SIMD, halo ring 1.2-1.3x the tile), 8% faster than
// 64 x 16 x 256, which beats 64 x 16 x 512 and 64 x 32 x 1024 by 6% and
// 32 x 16 x 256 and 64 x 8 x 256 by 20%; FP32: 128 x 16 x 512 4% faster than
// 64 x 32 x 1024, which beats 64 x 16 x 256 by 5% and 64 x 32 x 512 by 12%
// (these with points dealt out in row-major order; with whole rows per wave
// 64 x 32 x 1024 and 128 x 16 x 512 are within 1%).
template <class V, int TX, int TY, int NT, int XM = 0>
static hipError_t cg1_t(int n, const V* r_in, V* r_out, const V* p_in, V* p_out, V* x, V minv,
                        V inv_h2, DevState* st, double* partials, int pgiven, hipStream_t s,
                        int pslot = 0) {
    static int occ = 0, cus = 0;
    if (occ == 0) {
        int o = 0, c = 0, dev = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&o, cg1_kernel<V, TX, TY, NT, XM>, NT, 0) !=
                hipSuccess || o < 1)
            o = 1;
        (void)hipGetDevice(&dev);
        if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            c < 1)
            c = 1;
        cus = c;
        occ = o;
    }
    const int nbx = n / TX, nby = n / TY;
    const int tiles = nbx * nby;
    int nbz = occ * cus / tiles;
    // five partials per block in the partials array (4 x kMaxSweepBlocks)
    constexpr int kMaxBlocks = 4 * kMaxSweepBlocks / 5;
    if (nbz > kMaxBlocks / tiles) nbz = kMaxBlocks / tiles;
    if (nbz > n / 4) nbz = n / 4;
    if (nbz < 1) nbz = 1;
    const int nb = tiles * nbz;
    if (nb > kMaxBlocks) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL((cg1_kernel<V, TX, TY, NT, XM>), dim3(nb), dim3(NT), 0, s, n, nbx, nby,
                       nbz, r_in, r_out, p_in, p_out, x, minv, inv_h2, st, partials, pgiven, pslot);
    return hipGetLastError();
}

template <class V, int TX, int TY, int NT>
static hipError_t cg1_xm(int xm, int n, const V* r_in, V* r_out, const V* p_in, V* p_out, V* x,
                         V minv, V inv_h2, DevState* st, double* partials, int pgiven, int pslot,
                         hipStream_t s) {
    if (xm == 1)
        return cg1_t<V, TX, TY, NT, 1>(n, r_in, r_out, p_in, p_out, x, minv, inv_h2, st, partials,
                                       pgiven, s, pslot);
    if (xm == 2)
        return cg1_t<V, TX, TY, NT, 2>(n, r_in, r_out, p_in, p_out, x, minv, inv_h2, st, partials,
                                       pgiven, s, pslot);
    return cg1_t<V, TX, TY, NT, 0>(n, r_in, r_out, p_in, p_out, x, minv, inv_h2, st, partials,
                                   pgiven, s, pslot);
}

hipError_t launch_cg1(const SweepGeo& g, const double* r_in, double* r_out, const double* p_in,
                      double* p_out, double* x, double minv, double inv_h2, DevState* st,
                      double* partials, int xm, int pslot, hipStream_t s) {
    if (!cg1_supported(g) || xm < 0 || xm > 2) return hipErrorInvalidValue;
    // 1024^3 (measured, 200 sweeps): 128 x 16 tiles 9.14 ms per sweep = 5.64 TB/s
    // against 10.4 ms for 64 x 32 (9.65 ms with the z column split in two);
    // at 512^3 the two shapes are within 1% (1.077 / 1.086 ms)
    if (g.n >= 1024 && g.n % 128 == 0)
        return cg1_xm<double, 128, 16, 512>(xm, g.n, r_in, r_out, p_in, p_out, x, minv, inv_h2, st,
                                            partials, 0, pslot, s);
    if (g.n % 64 == 0)
        return cg1_xm<double, 64, 32, 512>(xm, g.n, r_in, r_out, p_in, p_out, x, minv, inv_h2, st,
                                           partials, 0, pslot, s);
    return cg1_xm<double, 32, 16, 256>(xm, g.n, r_in, r_out, p_in, p_out, x, minv, inv_h2, st,
                                       partials, 0, pslot, s);
}

static int stream_blocks(int64_t n);

// x += alpha_pend p[pend_slot] when an odd sweep left its update pending;
// the flag is cleared by a second launch (blocks of this one still read it).
__global__ __launch_bounds__(kNT) void cg1_flush_kernel(int64_t n3, const double* __restrict__ p0,
                                                        const double* __restrict__ p1,
                                                        double* __restrict__ x,
                                                        const DevState* st) {
    if (!st->cg.xpend) return;
    const double a = st->cg.alpha_pend;
    const double* __restrict__ p = st->cg.pend_slot ? p1 : p0;
    for (int64_t i = (int64_t)blockIdx.x * kNT + threadIdx.x; i < n3; i += (int64_t)gridDim.x * kNT)
        x[i] = x[i] + a * p[i];
}
__global__ void cg1_flush_done_kernel(DevState* st) {
    if (threadIdx.x == 0 && blockIdx.x == 0) st->cg.xpend = 0;
}

hipError_t launch_cg1_flush(int64_t n3, const double* p0, const double* p1, double* x,
                            DevState* st, hipStream_t s) {
    hipLaunchKernelGGL(cg1_flush_kernel, dim3(stream_blocks(n3)), dim3(kNT), 0, s, n3, p0, p1, x,
                       (const DevState*)st);
    hipLaunchKernelGGL(cg1_flush_done_kernel, dim3(1), dim3(64), 0, s, st);
    return hipGetLastError();
}

hipError_t launch_cg1_32(const SweepGeo& g, const float* r_in, float* r_out, const float* p_in,
                         float* p_out, float* d, float minvf, float inv_h2f, int pgiven,
                         DevState* st, double* partials, int xm, int pslot, hipStream_t s) {
    if (!cg1_supported(g) || xm < 0 || xm > 2) return hipErrorInvalidValue;
    if (g.n % 128 == 0)
        return cg1_xm<float, 128, 16, 512>(xm, g.n, r_in, r_out, p_in, p_out, d, minvf, inv_h2f,
                                           st, partials, pgiven, pslot, s);
    if (g.n % 64 == 0)
        return cg1_xm<float, 64, 32, 1024>(xm, g.n, r_in, r_out, p_in, p_out, d, minvf, inv_h2f,
                                           st, partials, pgiven, pslot, s);
    return cg1_xm<float, 32, 16, 256>(xm, g.n, r_in, r_out, p_in, p_out, d, minvf, inv_h2f, st,
                                      partials, pgiven, pslot, s);
}

// d += (float)alpha_pend p[pend_slot]: the FP32 inner solve's pending step.
__global__ __launch_bounds__(kNT) void cg1_flush32_kernel(int64_t n3, const float* __restrict__ p0,
                                                          const float* __restrict__ p1,
                                                          float* __restrict__ d,
                                                          const DevState* st) {
    if (!st->cg.xpend) return;
    const float a = (float)st->cg.alpha_pend;
    const float* __restrict__ p = st->cg.pend_slot ? p1 : p0;
    for (int64_t i = (int64_t)blockIdx.x * kNT + threadIdx.x; i < n3; i += (int64_t)gridDim.x * kNT)
        d[i] = d[i] + a * p[i];
}

hipError_t launch_cg1_flush32(int64_t n3, const float* p0, const float* p1, float* d,
                              DevState* st, hipStream_t s) {
    hipLaunchKernelGGL(cg1_flush32_kernel, dim3(stream_blocks(n3)), dim3(kNT), 0, s, n3, p0, p1, d,
                       (const DevState*)st);
    hipLaunchKernelGGL(cg1_flush_done_kernel, dim3(1), dim3(64), 0, s, st);
    return hipGetLastError();
}

hipError_t launch_dir32(const SweepGeo& g, const float* r, const float* p_old, float* p_new,
                        float minvf, float inv_h2f, DevState* st, double* partials, hipStream_t s) {
    OpDir<float> op{r, p_old, p_new, minvf, inv_h2f, st, partials, 0.0f, 0};
    return launch_sweep(op, g, s);
}

hipError_t launch_upd32(const SweepGeo& g, const float* p_new, float* d, float* r, float minvf,
                        float inv_h2f, DevState* st, double* partials, hipStream_t s) {
    OpUpd<float> op{p_new, d, r, minvf, inv_h2f, st, partials, 0.0f};
    return launch_sweep(op, g, s);
}

hipError_t launch_outer_resid(const SweepGeo& g, const double* b, const double* x, double* r,
                              double inv_h2, DevState* st, double* partials, double tol,
                              hipStream_t s) {
    OpOuterResid op{b, x, r, inv_h2, tol, 1, st, partials};
    return launch_sweep(op, g, s);
}

hipError_t launch_resid_norm(const SweepGeo& g, const double* b, const double* x, double* r,
                             double inv_h2, DevState* st, double* partials, hipStream_t s) {
    OpOuterResid op{b, x, r, inv_h2, 0.0, 0, st, partials};
    return launch_sweep(op, g, s);
}

// phi -= st->mean (the gauge fix, after the field sweep has read phi).
__global__ __launch_bounds__(kNT) void shift_kernel(int64_t n3, double* __restrict__ v,
                                                    const DevState* st) {
    const double m = st->mean;
    for (int64_t i = (int64_t)blockIdx.x * kNT + threadIdx.x; i < n3; i += (int64_t)gridDim.x * kNT)
        v[i] = v[i] - m;
}

hipError_t launch_field(const SweepGeo& g, double* phi, double* ex, double* ey, double* ez,
                        double ehalf, double h3, DevState* st, double* partials, hipStream_t s) {
    const int gauge = g.bc != 1;
    OpField op{phi, ex, ey, ez, ehalf, h3, 0.0, gauge, st, partials};
    hipError_t e = launch_sweep(op, g, s);
    if (e != hipSuccess || !gauge) return e;
    const int64_t n3 = (int64_t)g.n * g.n * g.n;
    hipLaunchKernelGGL(shift_kernel, dim3(stream_blocks(n3)), dim3(kNT), 0, s, n3, phi,
                       (const DevState*)st);
    return hipGetLastError();
}

static int stream_blocks(int64_t n) {
    int64_t b = (n + kNT - 1) / kNT;
    return (int)(b < kStreamBlocks ? (b < 1 ? 1 : b) : kStreamBlocks);
}

hipError_t launch_convert32(int64_t n3, const double* r, float* r32, float* d32, float minvf,
                            int reliable, double inner_rtol, int64_t max_inner, DevState* st,
                            double* partials, hipStream_t s) {
    hipLaunchKernelGGL(convert32_kernel, dim3(stream_blocks(n3)), dim3(kNT), 0, s, n3, r, r32, d32,
                       minvf, reliable, inner_rtol, max_inner, st, partials);
    return hipGetLastError();
}

hipError_t launch_update_x(int64_t n3, double* x, const float* d, DevState* st, hipStream_t s) {
    hipLaunchKernelGGL(update_x_kernel, dim3(stream_blocks(n3)), dim3(kNT), 0, s, n3, x, d, st);
    return hipGetLastError();
}

hipError_t launch_sum(int64_t n3, const double* v, DevState* st, double* partials, int what,
                      hipStream_t s) {
    hipLaunchKernelGGL(sum_kernel, dim3(stream_blocks(n3)), dim3(kNT), 0, s, n3, v, st, partials,
                       what);
    return hipGetLastError();
}

hipError_t launch_fill(int64_t n, double* v, double val, hipStream_t s) {
    hipLaunchKernelGGL(fill_kernel, dim3(stream_blocks(n)), dim3(kNT), 0, s, n, v, val);
    return hipGetLastError();
}

// ------------------------------------------------- flexible CG streams ----
// Streaming kernels take two consecutive points per thread (16-byte loads and
// stores) when every pointer is 16-byte aligned and n3 is even; VEC = 1 is
// the one-point form.  Reductions sum each thread's points in index order.
template <int VEC>
__global__ __launch_bounds__(kNT) void fcg_update_kernel(int64_t n3, double* __restrict__ x,
                                                         double* __restrict__ r,
                                                         const double* __restrict__ p,
                                                         const double* __restrict__ q, double a,
                                                         DevState* st, double* part) {
    __shared__ double red[kNT / kWave];
    __shared__ int lflag;
    double acc[1] = {0.0};
    if (VEC == 2) {
        const int64_t n2 = n3 / 2;
        for (int64_t i = (int64_t)blockIdx.x * kNT + threadIdx.x; i < n2;
             i += (int64_t)gridDim.x * kNT) {
            const double2 xv = reinterpret_cast<const double2*>(x)[i];
            const double2 pv = reinterpret_cast<const double2*>(p)[i];
            const double2 rv = reinterpret_cast<const double2*>(r)[i];
            const double2 qv = reinterpret_cast<const double2*>(q)[i];
            const double2 xn = make_double2(xv.x + a * pv.x, xv.y + a * pv.y);
            const double2 rn = make_double2(rv.x - a * qv.x, rv.y - a * qv.y);
            reinterpret_cast<double2*>(x)[i] = xn;
            reinterpret_cast<double2*>(r)[i] = rn;
            acc[0] += rn.x * rn.x;
            acc[0] += rn.y * rn.y;
        }
    } else {
        for (int64_t i = (int64_t)blockIdx.x * kNT + threadIdx.x; i < n3;
             i += (int64_t)gridDim.x * kNT) {
            x[i] = x[i] + a * p[i];
            const double rv = r[i] - a * q[i];
            r[i] = rv;
            acc[0] += rv * rv;
        }
    }
    block_sum<kNT, 1>(acc, red);
    if (threadIdx.x == 0) part[blockIdx.x] = acc[0];
    if (last_block(&st->tickets[5], gridDim.x, &lflag)) {
        double t[1];
        sum_partials<kNT, 1>(part, gridDim.x, t, red);
        if (threadIdx.x == 0) st->flex_rr = t[0];
    }
}

__global__ __launch_bounds__(kNT) void fcg_dots_kernel(int64_t n3, const double* __restrict__ z,
                                                       const double* __restrict__ r,
                                                       const double* __restrict__ q, DevState* st,
                                                       double* part) {
    __shared__ double red[2 * (kNT / kWave)];
    __shared__ int lflag;
    double acc[2] = {0.0, 0.0};
    for (int64_t i = (int64_t)blockIdx.x * kNT + threadIdx.x; i < n3; i += (int64_t)gridDim.x * kNT) {
        const double zv = z[i];
        acc[0] += zv * r[i];
        acc[1] += zv * q[i];
    }
    block_sum<kNT, 2>(acc, red);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = acc[0];
        part[gridDim.x + blockIdx.x] = acc[1];
    }
    if (last_block(&st->tickets[5], gridDim.x, &lflag)) {
        double t[2];
        sum_partials<kNT, 2>(part, gridDim.x, t, red);
        if (threadIdx.x == 0) {
            st->flex_zr = t[0];
            st->flex_zq = t[1];
        }
    }
}

template <int VEC>
__global__ __launch_bounds__(kNT) void xpby_kernel(int64_t n3, const double* __restrict__ z,
                                                   double* __restrict__ p, double b) {
    if (VEC == 2) {
        const int64_t n2 = n3 / 2;
        for (int64_t i = (int64_t)blockIdx.x * kNT + threadIdx.x; i < n2;
             i += (int64_t)gridDim.x * kNT) {
            const double2 zv = reinterpret_cast<const double2*>(z)[i];
            const double2 pv = reinterpret_cast<const double2*>(p)[i];
            reinterpret_cast<double2*>(p)[i] = make_double2(zv.x + b * pv.x, zv.y + b * pv.y);
        }
        return;
    }
    for (int64_t i = (int64_t)blockIdx.x * kNT + threadIdx.x; i < n3; i += (int64_t)gridDim.x * kNT)
        p[i] = z[i] + b * p[i];
}

__global__ __launch_bounds__(kNT) void axpy_copy_kernel(int64_t n3, const double* __restrict__ x,
                                                        const double* __restrict__ z,
                                                        double* __restrict__ w) {
    for (int64_t i = (int64_t)blockIdx.x * kNT + threadIdx.x; i < n3; i += (int64_t)gridDim.x * kNT)
        w[i] = x[i] + z[i];
}

template <int VEC>
__global__ __launch_bounds__(kNT) void copy_kernel(int64_t n3, const double* __restrict__ a,
                                                   double* __restrict__ b) {
    if (VEC == 2) {
        const int64_t n2 = n3 / 2;
        for (int64_t i = (int64_t)blockIdx.x * kNT + threadIdx.x; i < n2;
             i += (int64_t)gridDim.x * kNT)
            reinterpret_cast<double2*>(b)[i] = reinterpret_cast<const double2*>(a)[i];
        return;
    }
    for (int64_t i = (int64_t)blockIdx.x * kNT + threadIdx.x; i < n3; i += (int64_t)gridDim.x * kNT)
        b[i] = a[i];
}

hipError_t launch_aqz(const SweepGeo& g, const double* z, const double* p_old, double* p_new,
                      double* q, double beta, int restart, double inv_h2, DevState* st,
                      double* partials, hipStream_t s) {
    OpAqZ op{z, p_old, p_new, q, beta, restart, inv_h2, st, partials};
    return launch_sweep(op, g, s);
}

hipError_t launch_updp(const SweepGeo& g, const double* p, double* x, double* r, double alpha,
                       double inv_h2, DevState* st, double* partials, hipStream_t s) {
    OpUpdP op{p, x, r, alpha, inv_h2, st, partials};
    return launch_sweep(op, g, s);
}

hipError_t launch_aq(const SweepGeo& g, const double* p, double* q, double inv_h2, DevState* st,
                     double* partials, hipStream_t s) {
    OpAq op{p, q, inv_h2, st, partials};
    return launch_sweep(op, g, s);
}
// Fused SSOR solve launcher: K = inner steps (1..4 instantiated); z split to
// about 4096 blocks.
template <int K, int DIR, int TX, int TY>
static hipError_t ssor_fused_t(int n, int bounded, const double* src, const double* add, const double* rdot,
                               double* dst, double s0, double c, double oscale, DevState* st,
                               double* partials, hipStream_t s) {
    const int nbx = n / TX, nby = n / TY;
    int nbz = 1;
    for (int z = 1; z <= n / 16; ++z)
        if (n % z == 0 && (int64_t)nbx * nby * z <= 4096) nbz = z;
    const int nb = nbx * nby * nbz;
    if (nb > kMaxSweepBlocks) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL((ssor_fused_kernel<K, DIR, TX, TY>), dim3(nb), dim3(kNT), 0, s, n, bounded,
                       nbx, nby, n / nbz, src, add, rdot, dst, s0, c, oscale, st, partials);
    return hipGetLastError();
}

template <int K, int DIR>
static hipError_t ssor_fused_k(int n, int bounded, const double* src, const double* add,
                               const double* rdot, double* dst, double s0, double c, double oscale,
                               DevState* st, double* partials, hipStream_t s) {
    // 64-wide tiles only while their LDS keeps 5+ waves per SIMD resident
    // (4 inner steps on 64 x 8 tiles: 8% slower per solve at 512^3)
    if (n % 64 == 0 && K < 3)
        return ssor_fused_t<K, DIR, 64, 8>(n, bounded, src, add, rdot, dst, s0, c, oscale, st,
                                           partials, s);
    return ssor_fused_t<K, DIR, 32, 8>(n, bounded, src, add, rdot, dst, s0, c, oscale, st,
                                       partials, s);
}

bool ssor_fused_supported(int n, int inner) { return n % 32 == 0 && inner >= 1 && inner <= 4; }

hipError_t launch_ssor_fused(int n, int bounded, int inner, int dir, const double* src,
                             const double* add, const double* rdot, double* dst, double s0,
                             double c, double oscale, DevState* st, double* partials,
                             hipStream_t s) {
#define SF(KK)                                                                                  \
    if (inner == KK)                                                                            \
        return dir == 0 ? ssor_fused_k<KK, 0>(n, bounded, src, add, rdot, dst, s0, c, oscale, st, \
                                              partials, s)                                      \
                        : ssor_fused_k<KK, 1>(n, bounded, src, add, rdot, dst, s0, c, oscale, st, \
                                              partials, s)
    SF(1);
    SF(2);
    SF(3);
    SF(4);
#undef SF
    return hipErrorInvalidValue;
}

hipError_t launch_ssor_half(const SweepGeo& g, const double* src, const double* base,
                            const double* add, const double* rdot, double* dst, double c,
                            double bscale, double sscale, double oscale, int dir, DevState* st,
                            double* partials, hipStream_t s) {
    OpSsorHalf op{src, base, add, rdot, dst, c, bscale, sscale, oscale, dir, st, partials};
    return launch_sweep(op, g, s);
}
static bool vec2_ok(int64_t n3, const void* a, const void* b, const void* c = nullptr,
                    const void* d = nullptr) {
    const uintptr_t m = (uintptr_t)a | (uintptr_t)b | (uintptr_t)c | (uintptr_t)d;
    return (n3 % 2) == 0 && (m & 15u) == 0;
}

hipError_t launch_fcg_update(int64_t n3, double* x, double* r, const double* p, const double* q,
                             double a, DevState* st, double* partials, hipStream_t s) {
    if (vec2_ok(n3, x, r, p, q))
        hipLaunchKernelGGL(fcg_update_kernel<2>, dim3(stream_blocks(n3 / 2)), dim3(kNT), 0, s, n3, x,
                           r, p, q, a, st, partials);
    else
        hipLaunchKernelGGL(fcg_update_kernel<1>, dim3(stream_blocks(n3)), dim3(kNT), 0, s, n3, x, r,
                           p, q, a, st, partials);
    return hipGetLastError();
}
hipError_t launch_fcg_dots(int64_t n3, const double* z, const double* r, const double* q,
                           DevState* st, double* partials, hipStream_t s) {
    hipLaunchKernelGGL(fcg_dots_kernel, dim3(stream_blocks(n3)), dim3(kNT), 0, s, n3, z, r, q, st,
                       partials);
    return hipGetLastError();
}
hipError_t launch_xpby(int64_t n3, const double* z, double* p, double b, hipStream_t s) {
    if (vec2_ok(n3, z, p))
        hipLaunchKernelGGL(xpby_kernel<2>, dim3(stream_blocks(n3 / 2)), dim3(kNT), 0, s, n3, z, p, b);
    else
        hipLaunchKernelGGL(xpby_kernel<1>, dim3(stream_blocks(n3)), dim3(kNT), 0, s, n3, z, p, b);
    return hipGetLastError();
}
hipError_t launch_axpy_copy(int64_t n3, const double* x, const double* z, double* w, hipStream_t s) {
    hipLaunchKernelGGL(axpy_copy_kernel, dim3(stream_blocks(n3)), dim3(kNT), 0, s, n3, x, z, w);
    return hipGetLastError();
}
hipError_t launch_copy(int64_t n3, const double* src, double* dst, hipStream_t s) {
    if (vec2_ok(n3, src, dst))
        hipLaunchKernelGGL(copy_kernel<2>, dim3(stream_blocks(n3 / 2)), dim3(kNT), 0, s, n3, src, dst);
    else
        hipLaunchKernelGGL(copy_kernel<1>, dim3(stream_blocks(n3)), dim3(kNT), 0, s, n3, src, dst);
    return hipGetLastError();
}

}  // namespace pic
