// particles.hip -- particle side of the PIC loop (Sec. 2, Fig. pic-loop):
// cell keys, CIC gather + leapfrog push (Eq. eom, electrostatic), the initial
// half kick, and the CIC charge deposit (scatter) with the neutralising
// background of Sec. 2.
//
// Bit-exactness: the whole library is compiled without floating-point
// contraction, and the per-particle arithmetic below follows the CPU oracle's
// definition operation by operation (cell index floor(x*N/L) clamped to
// [0, N-1]; weight products ((Wz*Wy)*Wx); gather summed z-offset outer, then y,
// then x; v += (dt*qm)*E; x = wrap(x + dt*v)), so keys, positions and
// velocities match the oracle bit for bit given the same field.
//
// Deposit on cell-sorted particles, without atomics: each cell's particles
// are summed in sorted order into the cell's eight corner sums, the two cells
// of a row that touch a vertex are added, and each vertex adds its four cell
// rows in increasing key order.  The result is deterministic and every term
// is the oracle's (the same weight products), but the association differs
// from a sequential scatter over the sorted particles: the two agree within
// 2 gamma(n_v) of the vertex's weight sum (n_v particles in the eight cells
// around the vertex, gamma(n) = n u / (1 - n u)), not bit for bit.
#include "common.hpp"
#include "particles.hpp"
#include "particle_math.hpp"
#include "solver_state.hpp"

namespace pic {

constexpr int kPT = 256;

// CIC gather of (Ex, Ey, Ez) at one particle.  The two x corners of a
// vertex row are adjacent in memory unless the row wraps (i0 = n - 1), so
// each row's pair is one 16-byte load (8-byte aligned); the wrapping lanes
// take their second corner from the start of the row.  Values and summation
// order are those of the eight separate loads.
typedef double pair_u __attribute__((ext_vector_type(2), aligned(8)));
__device__ __forceinline__ void gather3(double px, double py, double pz, int n, double inv_h,
                                        const double* __restrict__ ex,
                                        const double* __restrict__ ey,
                                        const double* __restrict__ ez, double& sx, double& sy,
                                        double& sz) {
    int i0, i1, i2;
    double w0, w1, w2;
    locate(px, n, inv_h, i0, w0);
    locate(py, n, inv_h, i1, w1);
    locate(pz, n, inv_h, i2, w2);
    sx = 0.0;
    sy = 0.0;
    sz = 0.0;
    // the pair starts at i0, or at n - 2 for the wrapping corner (grids
    // have n >= 32)
    const bool wraps = i0 == n - 1;
    const int xs = wraps ? n - 2 : i0;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const double wz = c ? w2 : 1.0 - w2;
        int vz = i2 + c;
        vz = vz == n ? 0 : vz;
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const double wy = b ? w1 : 1.0 - w1;
            int vy = i1 + b;
            vy = vy == n ? 0 : vy;
            const size_t row = ((size_t)vz * n + vy) * n;
            const pair_u px2 = *(const pair_u*)(ex + row + xs);
            const pair_u py2 = *(const pair_u*)(ey + row + xs);
            const pair_u pz2 = *(const pair_u*)(ez + row + xs);
            double ex0 = px2.x, ex1 = px2.y, ey0 = py2.x, ey1 = py2.y, ez0 = pz2.x, ez1 = pz2.y;
            if (wraps) {
                ex0 = ex1; ey0 = ey1; ez0 = ez1;
                ex1 = ex[row]; ey1 = ey[row]; ez1 = ez[row];
            }
            const double W0 = (wz * wy) * (1.0 - w0);
            const double W1 = (wz * wy) * w0;
            sx = sx + W0 * ex0;
            sy = sy + W0 * ey0;
            sz = sz + W0 * ez0;
            sx = sx + W1 * ex1;
            sy = sy + W1 * ey1;
            sz = sz + W1 * ez1;
        }
    }
}

__global__ __launch_bounds__(kPT) void keys_kernel(int64_t np, const double* __restrict__ x,
                                                   const double* __restrict__ y,
                                                   const double* __restrict__ z,
                                                   uint32_t* __restrict__ key, int n, double inv_h) {
    for (int64_t p = (int64_t)blockIdx.x * kPT + threadIdx.x; p < np; p += (int64_t)gridDim.x * kPT)
        key[p] = key_of(x[p], y[p], z[p], n, inv_h);
}

// Each thread takes kPushK particles per trip (kPT apart, so every load and
// store of a wave stays one contiguous run) and issues the loads of all of
// them before the first gather: 6 kPushK streaming loads in flight per
// thread instead of 6.  The outputs are written once and not read again by
// this kernel, so they bypass L2 retention.
//
// With a record array (the PIC step, before the cell sort) the new state
// goes to 64-byte records (x, y | z, vx | vy, vz | padding) in the input
// order instead of back into the six arrays: the sort then gathers one
// record per sorted slot rather than six scattered 8-byte values.
constexpr int kPushK = 4;
template <bool REC>
__global__ __launch_bounds__(kPT) void gather_push_kernel(
    int64_t np, double* __restrict__ x, double* __restrict__ y, double* __restrict__ z,
    double* __restrict__ vx, double* __restrict__ vy, double* __restrict__ vz,
    const double* __restrict__ ex, const double* __restrict__ ey, const double* __restrict__ ez,
    uint32_t* __restrict__ key, double2* __restrict__ rec, int n, double inv_h, double L,
    double dt, double coef) {
    // records: each wave puts its 64 particles' records in its own 4 KB of
    // LDS, then stores them as four runs of 1 KB (consecutive lanes,
    // consecutive 16-byte parts)
    __shared__ double2 srec[REC ? kPT * 4 : 1];
    const int lane = threadIdx.x & (kWave - 1);
    double2* wrec = srec + (REC ? (threadIdx.x - lane) * 4 : 0);
    const int64_t stride = (int64_t)gridDim.x * kPT * kPushK;
    // the trip count is uniform over the workgroup (particles past np idle)
    for (int64_t b0 = (int64_t)blockIdx.x * kPT * kPushK; b0 < np; b0 += stride) {
        const int64_t p0 = b0 + threadIdx.x;
        double px[kPushK], py[kPushK], pz[kPushK], qx[kPushK], qy[kPushK], qz[kPushK];
#pragma unroll
        for (int k = 0; k < kPushK; ++k) {
            const int64_t p = p0 + (int64_t)kPT * k;
            const bool ok = p < np;
            px[k] = ok ? x[p] : 0.0;
            py[k] = ok ? y[p] : 0.0;
            pz[k] = ok ? z[p] : 0.0;
            qx[k] = ok ? vx[p] : 0.0;
            qy[k] = ok ? vy[p] : 0.0;
            qz[k] = ok ? vz[p] : 0.0;
        }
#pragma unroll
        for (int k = 0; k < kPushK; ++k) {
            const int64_t p = p0 + (int64_t)kPT * k;
            if (!REC && p >= np) break;
            double sx, sy, sz;
            gather3(px[k], py[k], pz[k], n, inv_h, ex, ey, ez, sx, sy, sz);
            const double ux = qx[k] + coef * sx;
            const double uy = qy[k] + coef * sy;
            const double uz = qz[k] + coef * sz;
            const double nx = wrap(px[k] + dt * ux, L);
            const double ny = wrap(py[k] + dt * uy, L);
            const double nz = wrap(pz[k] + dt * uz, L);
            if (REC) {
                wrec[4 * lane] = make_double2(nx, ny);
                wrec[4 * lane + 1] = make_double2(nz, ux);
                wrec[4 * lane + 2] = make_double2(uy, uz);
                wrec[4 * lane + 3] = make_double2(0.0, 0.0);
                __builtin_amdgcn_wave_barrier();
                const int64_t pb = p - lane;  // the wave's first particle
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int c = q * kWave + lane;  // part c % 4 of record c / 4
                    if (pb + c / 4 < np) __builtin_nontemporal_store(wrec[c].x, &rec[4 * pb + c].x),
                                             __builtin_nontemporal_store(wrec[c].y, &rec[4 * pb + c].y);
                }
                __builtin_amdgcn_wave_barrier();
                if (key && p < np) __builtin_nontemporal_store(key_of(nx, ny, nz, n, inv_h), key + p);
            } else {
                __builtin_nontemporal_store(ux, vx + p);
                __builtin_nontemporal_store(uy, vy + p);
                __builtin_nontemporal_store(uz, vz + p);
                __builtin_nontemporal_store(nx, x + p);
                __builtin_nontemporal_store(ny, y + p);
                __builtin_nontemporal_store(nz, z + p);
                if (key) __builtin_nontemporal_store(key_of(nx, ny, nz, n, inv_h), key + p);
            }
        }
    }
}

__global__ __launch_bounds__(kPT) void half_kick_kernel(
    int64_t np, const double* __restrict__ x, const double* __restrict__ y,
    const double* __restrict__ z, double* __restrict__ vx, double* __restrict__ vy,
    double* __restrict__ vz, const double* __restrict__ ex, const double* __restrict__ ey,
    const double* __restrict__ ez, int n, double inv_h, double coef) {
    for (int64_t p = (int64_t)blockIdx.x * kPT + threadIdx.x; p < np; p += (int64_t)gridDim.x * kPT) {
        double sx, sy, sz;
        gather3(x[p], y[p], z[p], n, inv_h, ex, ey, ez, sx, sy, sz);
        vx[p] = vx[p] + coef * sx;
        vy[p] = vy[p] + coef * sy;
        vz[p] = vz[p] + coef * sz;
    }
}

// Deterministic deposit on sorted particles, two passes.
// Pass 1, one lane per cell, one wave per 63 cells of a row (lane 0 takes
// the cell before the segment): each lane sums its cell's particles in sorted
// order into the eight CIC corner sums S[a][b][c]; lanes then combine the two
// cells of a row that touch vertex x (cell x-1 with a = 1, cell x with a = 0)
// and store T[2c+b][(z, y) row][x]: the contribution of cell row (y, z) to
// vertex (x, y+b, z+c).  Every particle is read once: the cells of a segment
// hold one contiguous run of sorted particles, which the wave stages through
// LDS in chunks of kDepCh with whole-line loads (a lane reading its own
// cell's particles touches a new line per particle, and the lines a wave
// needs outlive their stay in L2), and each lane then takes its cell's part
// of the chunk in order.
constexpr int kDepCh = 256;  // particles per staged chunk

// LDS written by some lanes of a wave and then read by others
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__global__ __launch_bounds__(kPT) void deposit_cells_kernel(
    const double* __restrict__ x, const double* __restrict__ y, const double* __restrict__ z,
    const uint32_t* __restrict__ cs, int n, double inv_h, double* __restrict__ T0,
    double* __restrict__ T1, double* __restrict__ T2, double* __restrict__ T3) {
    __shared__ double sp[kPT / kWave][3][kDepCh];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t wid = ((int64_t)blockIdx.x * kPT + threadIdx.x) >> 6;
    const int segs = (n + 62) / 63;
    const int64_t rows = (int64_t)n * n;
    if (wid >= rows * segs) return;  // uniform per wave
    const int64_t row = wid / segs;
    const int x0 = (int)(wid % segs) * 63;
    const int xl = x0 + lane - 1;  // this lane's cell x (lane 0: x0 - 1)
    const bool active = xl < n;
    const int cx = xl < 0 ? n - 1 : xl;
    double s[2][2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int c = 0; c < 2; ++c) s[a][b][c] = 0.0;
    uint32_t pb = 0, pe = 0;  // this lane's particles
    if (active) {
        const size_t cell = (size_t)row * n + cx;
        pb = cs[cell];
        pe = cs[cell + 1];
    }
    // particles [rb, re) through LDS; lanes lo..hi take theirs
    auto run = [&](uint32_t rb, uint32_t re, int lo, int hi) {
        for (uint32_t c0 = rb; c0 < re; c0 += kDepCh) {
            const uint32_t cn = re - c0 < (uint32_t)kDepCh ? re - c0 : (uint32_t)kDepCh;
            for (uint32_t q = lane; q < cn; q += kWave) {
                sp[wv][0][q] = x[c0 + q];
                sp[wv][1][q] = y[c0 + q];
                sp[wv][2][q] = z[c0 + q];
            }
            wave_lds_sync();
            if (active && lane >= lo && lane <= hi) {
                const uint32_t p0 = pb > c0 ? pb : c0;
                const uint32_t p1 = pe < c0 + cn ? pe : c0 + cn;
                for (uint32_t p = p0; p < p1; ++p) {
                    int i0;
                    double w0, w1, w2;
                    locate(sp[wv][0][p - c0], n, inv_h, i0, w0);
                    locate(sp[wv][1][p - c0], n, inv_h, i0, w1);
                    locate(sp[wv][2][p - c0], n, inv_h, i0, w2);
#pragma unroll
                    for (int c = 0; c < 2; ++c) {
                        const double wz = c ? w2 : 1.0 - w2;
#pragma unroll
                        for (int b = 0; b < 2; ++b) {
                            const double wy = b ? w1 : 1.0 - w1;
                            s[0][b][c] += (wz * wy) * (1.0 - w0);
                            s[1][b][c] += (wz * wy) * w0;
                        }
                    }
                }
            }
            wave_lds_sync();  // the chunk is consumed before the next overwrites it
        }
    };
    // cells x0 - 1 .. x0 + last - 1 of the row (lanes 0..last) hold one run,
    // except in the first segment, whose lane 0 takes the row's last cell
    const int last = n - x0 < 63 ? n - x0 : 63;
    const uint32_t b0 = __shfl(pb, 0, 64), e0 = __shfl(pe, 0, 64);
    const uint32_t b1 = __shfl(pb, 1, 64), e1 = __shfl(pe, last, 64);
    if (x0 > 0) {
        run(b0, e1, 0, 63);
    } else {
        run(b0, e0, 0, 0);
        run(b1, e1, 1, 63);
    }
    double* T[4] = {T0, T1, T2, T3};
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const double left = __shfl_up(s[1][b][c], 1, 64);  // cell x-1, a = 1
            if (lane >= 1 && active) T[2 * c + b][(size_t)row * n + xl] = left + s[0][b][c];
        }
}

// Pass 2, one thread per vertex: rho[v] = (sum of the four cell-row
// contributions, rows in increasing key order) * (q/h^3) + rho_bg; partial
// sums of rho for the mean.
__global__ __launch_bounds__(kPT) void deposit_vertices_kernel(
    const double* __restrict__ T0, const double* __restrict__ T1, const double* __restrict__ T2,
    const double* __restrict__ T3, double* __restrict__ rho, int n, double qh3, double rho_bg,
    double* part, DevState* st) {
    __shared__ double red[kPT / kWave];
    __shared__ int lflag;
    const double* T[4] = {T0, T1, T2, T3};
    const int64_t n3 = (int64_t)n * n * n;
    double acc[1] = {0.0};
    for (int64_t v = (int64_t)blockIdx.x * kPT + threadIdx.x; v < n3; v += (int64_t)gridDim.x * kPT) {
        const int ix = (int)(v % n);
        const int iy = (int)((v / n) % n);
        const int iz = (int)(v / ((int64_t)n * n));
        double sum = 0.0;
        for (int kc = 0; kc < 2; ++kc) {
            const int c = (iz == 0) ? kc : 1 - kc;
            const int cz = iz - c < 0 ? n - 1 : iz - c;
            for (int kb = 0; kb < 2; ++kb) {
                const int b = (iy == 0) ? kb : 1 - kb;
                const int cy = iy - b < 0 ? n - 1 : iy - b;
                sum += T[2 * c + b][((size_t)cz * n + cy) * n + ix];
            }
        }
        const double rv = sum * qh3 + rho_bg;
        rho[v] = rv;
        acc[0] += rv;
    }
    block_sum<kPT, 1>(acc, red);
    if (threadIdx.x == 0) part[blockIdx.x] = acc[0];
    if (last_block(&st->tickets[7], gridDim.x, &lflag)) {
        double t[1];
        sum_partials<kPT, 1>(part, gridDim.x, t, red);
        if (threadIdx.x == 0) st->mean = t[0] / (double)n3;
    }
}

// Unsorted deposit: FP64 atomics into acc (zeroed), one thread per particle.
__global__ __launch_bounds__(kPT) void deposit_atomic_kernel(int64_t np,
                                                             const double* __restrict__ x,
                                                             const double* __restrict__ y,
                                                             const double* __restrict__ z,
                                                             double* acc, int n, double inv_h) {
    for (int64_t p = (int64_t)blockIdx.x * kPT + threadIdx.x; p < np; p += (int64_t)gridDim.x * kPT) {
        int i0, i1, i2;
        double w0, w1, w2;
        locate(x[p], n, inv_h, i0, w0);
        locate(y[p], n, inv_h, i1, w1);
        locate(z[p], n, inv_h, i2, w2);
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const double wz = c ? w2 : 1.0 - w2;
            const int vz = i2 + c == n ? 0 : i2 + c;
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                const double wy = b ? w1 : 1.0 - w1;
                const int vy = i1 + b == n ? 0 : i1 + b;
#pragma unroll
                for (int a = 0; a < 2; ++a) {
                    const double wx = a ? w0 : 1.0 - w0;
                    const int vx = i0 + a == n ? 0 : i0 + a;
                    unsafeAtomicAdd(acc + (((size_t)vz * n + vy) * n + vx), (wz * wy) * wx);
                }
            }
        }
    }
}

// rho = acc * (q/h^3) + rho_bg in place; partial sums of rho.
__global__ __launch_bounds__(kPT) void deposit_scale_kernel(int64_t n3, double* __restrict__ rho,
                                                            double qh3, double rho_bg,
                                                            double* part, DevState* st) {
    __shared__ double red[kPT / kWave];
    double acc[1] = {0.0};
    for (int64_t v = (int64_t)blockIdx.x * kPT + threadIdx.x; v < n3; v += (int64_t)gridDim.x * kPT) {
        const double rv = rho[v] * qh3 + rho_bg;
        rho[v] = rv;
        acc[0] += rv;
    }
    block_sum<kPT, 1>(acc, red);
    if (threadIdx.x == 0) part[blockIdx.x] = acc[0];
    __shared__ int lflag;
    if (last_block(&st->tickets[7], gridDim.x, &lflag)) {
        double t[1];
        sum_partials<kPT, 1>(part, gridDim.x, t, red);
        if (threadIdx.x == 0) st->mean = t[0] / (double)n3;
    }
}

// b = rho - mean(rho) (mean formed by the previous kernel), partial sums of
// b^2; the last block stores ||b||^2.
__global__ __launch_bounds__(kPT) void project_kernel(int64_t n3, double* __restrict__ rho,
                                                      double* part, DevState* st) {
    __shared__ double red[kPT / kWave];
    __shared__ int lflag;
    const double mean = st->mean;
    double acc[1] = {0.0};
    for (int64_t v = (int64_t)blockIdx.x * kPT + threadIdx.x; v < n3; v += (int64_t)gridDim.x * kPT) {
        const double bv = rho[v] - mean;
        rho[v] = bv;
        acc[0] += bv * bv;
    }
    block_sum<kPT, 1>(acc, red);
    if (threadIdx.x == 0) part[blockIdx.x] = acc[0];
    if (last_block(&st->tickets[6], gridDim.x, &lflag)) {
        double t[1];
        sum_partials<kPT, 1>(part, gridDim.x, t, red);
        if (threadIdx.x == 0) st->bb = t[0];
    }
}

// --------------------------------------------------------------------------
static int pblocks(int64_t n, int cap = 8192) {
    int64_t b = (n + kPT - 1) / kPT;
    if (b < 1) b = 1;
    return (int)(b < cap ? b : cap);
}

hipError_t launch_keys(int64_t np, const double* x, const double* y, const double* z,
                       uint32_t* key, int n, double inv_h, hipStream_t s) {
    if (np == 0) return hipSuccess;
    hipLaunchKernelGGL(keys_kernel, dim3(pblocks(np)), dim3(kPT), 0, s, np, x, y, z, key, n, inv_h);
    return hipGetLastError();
}

hipError_t launch_gather_push(int64_t np, double* x, double* y, double* z, double* vx, double* vy,
                              double* vz, const double* ex, const double* ey, const double* ez,
                              uint32_t* key, double2* rec, int n, double inv_h, double L,
                              double dt, double coef, hipStream_t s) {
    if (np == 0) return hipSuccess;
    const int64_t groups = (np + kPushK - 1) / kPushK;
    if (rec)
        hipLaunchKernelGGL(gather_push_kernel<true>, dim3(pblocks(groups, 4096)), dim3(kPT), 0, s,
                           np, x, y, z, vx, vy, vz, ex, ey, ez, key, rec, n, inv_h, L, dt, coef);
    else
        hipLaunchKernelGGL(gather_push_kernel<false>, dim3(pblocks(groups, 4096)), dim3(kPT), 0, s,
                           np, x, y, z, vx, vy, vz, ex, ey, ez, key, rec, n, inv_h, L, dt, coef);
    return hipGetLastError();
}

hipError_t launch_half_kick(int64_t np, const double* x, const double* y, const double* z,
                            double* vx, double* vy, double* vz, const double* ex,
                            const double* ey, const double* ez, int n, double inv_h, double coef,
                            hipStream_t s) {
    if (np == 0) return hipSuccess;
    hipLaunchKernelGGL(half_kick_kernel, dim3(pblocks(np, 16384)), dim3(kPT), 0, s, np, x, y, z,
                       vx, vy, vz, ex, ey, ez, n, inv_h, coef);
    return hipGetLastError();
}

int deposit_partials() { return 4096; }

hipError_t launch_deposit(int64_t np, const double* x, const double* y, const double* z,
                          const uint32_t* cs, double* rho, int n, double inv_h, double qh3,
                          double rho_bg, DevState* st, double* part, double* const T[4],
                          hipStream_t s) {
    const int64_t n3 = (int64_t)n * n * n;
    const int nb = pblocks(n3, deposit_partials());
    if (cs) {
        const int64_t waves = (int64_t)n * n * ((n + 62) / 63);
        const int64_t blocks = (waves * 64 + kPT - 1) / kPT;
        hipLaunchKernelGGL(deposit_cells_kernel, dim3((uint32_t)blocks), dim3(kPT), 0, s, x, y, z, cs,
                           n, inv_h, T[0], T[1], T[2], T[3]);
        hipLaunchKernelGGL(deposit_vertices_kernel, dim3(nb), dim3(kPT), 0, s, (const double*)T[0],
                           (const double*)T[1], (const double*)T[2], (const double*)T[3], rho, n, qh3,
                           rho_bg, part, st);
    } else {
        hipError_t e = launch_fill(n3, rho, 0.0, s);
        if (e != hipSuccess) return e;
        if (np > 0)
            hipLaunchKernelGGL(deposit_atomic_kernel, dim3(pblocks(np, 16384)), dim3(kPT), 0, s, np,
                               x, y, z, rho, n, inv_h);
        hipLaunchKernelGGL(deposit_scale_kernel, dim3(nb), dim3(kPT), 0, s, n3, rho, qh3, rho_bg,
                           part, st);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(project_kernel, dim3(nb), dim3(kPT), 0, s, n3, rho, part, st);
    return hipGetLastError();
}

}  // namespace pic
