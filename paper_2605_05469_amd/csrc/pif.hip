// pif.hip -- Particle-in-Fourier field (Sec. 3.4; NUFFT steps of the
// appendix, Eqs. type1nufft and type2nufft).
//
//   rho_hat(k) = sum_j q exp(-i k.x_j)            type-1 NUFFT, k in K_N
//   E_hat(k)   = -i k rho_hat(k) / |k|^2         (k = 0 dropped; eps0 = 1)
//   E(x_j)     = Re (1/L^3) sum_k E_hat(k) exp(i k.x_j)   type-2 NUFFT
//
// with K_N = (2 pi / L) {-n/2 .. n/2-1}^3 and an oversampled grid of m = 2n
// points per axis (spacing h = L/m).  Window: the exponential of semicircle
// phi(z) = exp(beta (sqrt(1 - z^2) - 1)), |z| <= 1 (Barnett, Magland and
// af Klinteberg, SIAM J. Sci. Comput. 41, 2019), over w points with
// w = ceil(log10(1/tol)) + 1 and beta = 2.30 w; a coordinate s = x/h touches
// the points i0 .. i0+w-1, i0 = ceil(s - w/2), at offsets z = (i - s)/(w/2).
//
// GPU layout.  Particles are cell-sorted on the n^3 particle grid; a block
// owns a tile of T^3 cells, whose particles touch (2T + w)^3 points of the
// oversampled grid (one cell spans two points per axis).  The spread sums a
// tile's particles into that region in LDS and adds the region into the
// grid with FP64 atomics; the field evaluation stages the region of the
// three field grids in LDS and evaluates every particle of the tile from
// there.  Between them: one real-to-complex transform of the grid, and per
// field component one pass over the half spectrum (selection of K_N, both
// window deconvolutions, -i k / |k|^2, 1/L^3, and the Hermitian symmetrisation
// that makes the type-2 sum's real part a complex-to-real transform) and one
// complex-to-real transform.
#include <cmath>
#include <string>
#include <vector>

#include "common.hpp"
#include "fft.hpp"
#include "particle_math.hpp"
#include "pif.hpp"

namespace pic {

constexpr int kPifT = 4;      // cells per tile edge
constexpr int kPifNT = 256;   // threads per block
constexpr int kPifWMin = 3, kPifWMax = 8;

struct PifState {
    int n = 0, m = 0, w = 0;
    double L = 0, h = 0, inv_h = 0, beta = 0, kf = 0;
    FftPlans* fft = nullptr;
    void* mem = nullptr;
    double* grid = nullptr;   // spread target, then the x field
    double* fy = nullptr;
    double* fz = nullptr;
    double2* G = nullptr;     // spectrum of the spread grid
    double2* F = nullptr;     // one field component's spectrum
    double* corr = nullptr;   // h / psi_hat(2 pi j / L), j = -n/2 .. n/2
};

static std::string g_pif_err;
const char* pif_last_error() { return g_pif_err.c_str(); }

int pif_width(double tol) {
    if (!(tol > 0.0) || !(tol < 1.0)) return 0;
    const int w = (int)std::ceil(std::log10(1.0 / tol)) + 1;
    return (w >= kPifWMin && w <= kPifWMax) ? w : 0;
}

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

size_t pif_bytes(int n) {
    const size_t m = 2 * (size_t)n;
    const size_t real = align256(m * m * m * sizeof(double));
    const size_t half = align256(m * m * (m / 2 + 1) * sizeof(double2));
    return 3 * real + 2 * half + align256((size_t)(n + 1) * sizeof(double));
}

// Gauss-Legendre nodes and weights on [-1, 1]: Newton's method on P_q from
// the usual cosine estimates, P_q and P_q' by Bonnet's recurrence.
static void gauss_legendre(int q, std::vector<double>& x, std::vector<double>& wt) {
    x.assign(q, 0.0);
    wt.assign(q, 0.0);
    const double pi = 3.14159265358979323846;
    for (int i = 0; i < q; ++i) {
        double t = std::cos(pi * (i + 0.75) / (q + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = t;
            for (int k = 1; k < q; ++k) {
                const double p2 = ((2.0 * k + 1.0) * t * p1 - k * p0) / (k + 1.0);
                p0 = p1;
                p1 = p2;
            }
            dp = q * (t * p1 - p0) / (t * t - 1.0);
            const double dt = p1 / dp;
            t -= dt;
            if (std::fabs(dt) < 1e-16) break;
        }
        x[i] = t;
        wt[i] = 2.0 / ((1.0 - t * t) * dp * dp);
    }
}

// psi_hat(k) of psi(x) = phi(x / a), a = w h / 2:
//   a int_{-pi/2}^{pi/2} exp(beta (cos th - 1)) cos(k a sin th) cos th dth
// (t = sin th removes the square-root endpoint behaviour of the window).
static double window_ft(double k, double a, double beta, const std::vector<double>& g,
                        const std::vector<double>& gw) {
    const double hp = 1.57079632679489661923;
    double s = 0.0;
    for (size_t i = 0; i < g.size(); ++i) {
        const double th = hp * g[i];
        s += (hp * gw[i]) * std::exp(beta * (std::cos(th) - 1.0)) * std::cos(k * a * std::sin(th)) *
             std::cos(th);
    }
    return a * s;
}

int pif_create(PifState** out, int n, double L, double tol) {
    *out = nullptr;
    const int w = pif_width(tol);
    if (w == 0 || n % kPifT != 0) {
        g_pif_err = "tolerance outside [1e-7, 1e-2] or n not a multiple of the tile";
        return -1;
    }
    PifState* p = new PifState();
    p->n = n;
    p->m = 2 * n;
    p->w = w;
    p->L = L;
    p->h = L / (double)p->m;
    p->inv_h = (double)p->m / L;
    p->beta = 2.30 * w;
    p->kf = 2.0 * 3.14159265358979323846 / L;
    const size_t m = (size_t)p->m;
    if (hipMalloc(&p->mem, pif_bytes(n)) != hipSuccess) {
        (void)hipGetLastError();
        g_pif_err = "device allocation failed";
        delete p;
        return -3;
    }
    char* b = (char*)p->mem;
    const size_t real = align256(m * m * m * sizeof(double));
    const size_t half = align256(m * m * (m / 2 + 1) * sizeof(double2));
    p->grid = (double*)b;
    p->fy = (double*)(b + real);
    p->fz = (double*)(b + 2 * real);
    p->G = (double2*)(b + 3 * real);
    p->F = (double2*)(b + 3 * real + half);
    p->corr = (double*)(b + 3 * real + 2 * half);
    if (fft_create(&p->fft, p->m) != 0) {
        g_pif_err = std::string("FFT plans: ") + fft_last_error();
        pif_destroy(p);
        return -1;
    }
    std::vector<double> g, gw;
    gauss_legendre(100, g, gw);
    std::vector<double> c(n + 1);
    const double a = 0.5 * w * p->h;
    for (int j = -n / 2; j <= n / 2; ++j) c[j + n / 2] = p->h / window_ft(p->kf * j, a, p->beta, g, gw);
    if (hipMemcpy(p->corr, c.data(), c.size() * sizeof(double), hipMemcpyHostToDevice) !=
        hipSuccess) {
        g_pif_err = "copy of the deconvolution table failed";
        pif_destroy(p);
        return -1;
    }
    *out = p;
    return 0;
}

void pif_destroy(PifState* p) {
    if (!p) return;
    if (p->fft) fft_destroy(p->fft);
    if (p->mem) (void)hipFree(p->mem);
    delete p;
}

// ------------------------------------------------------------ kernels ----

__device__ __forceinline__ double es_window(double z, double beta) {
    const double t = 1.0 - z * z;
    return t >= 0.0 ? exp(beta * (sqrt(t) - 1.0)) : 0.0;
}

// One axis of a particle: local start (clamped into the tile's region) and
// the W window values.
template <int W>
__device__ __forceinline__ int axis_weights(double s, int lo, double beta, double (&wv)[W]) {
    const int i0 = (int)ceil(s - 0.5 * W);
    int l = i0 - lo;
    l = l < 0 ? 0 : (l > 2 * kPifT ? 2 * kPifT : l);
#pragma unroll
    for (int a = 0; a < W; ++a) wv[a] = es_window(((double)(i0 + a) - s) / (0.5 * W), beta);
    return l;
}

// The particles of a tile: T^2 runs of T consecutive cells (x rows).
struct TileRuns {
    uint32_t start[kPifT * kPifT];
    uint32_t off[kPifT * kPifT + 1];
};

__device__ __forceinline__ void tile_runs(TileRuns& tr, const uint32_t* __restrict__ cs, int n,
                                          int cx0, int cy0, int cz0) {
    if (threadIdx.x == 0) {
        uint32_t acc = 0;
        for (int r = 0; r < kPifT * kPifT; ++r) {
            const size_t c0 = ((size_t)(cz0 + r / kPifT) * n + (cy0 + r % kPifT)) * n + cx0;
            const uint32_t a = cs[c0], e = cs[c0 + kPifT];
            tr.start[r] = a;
            tr.off[r] = acc;
            acc += e - a;
        }
        tr.off[kPifT * kPifT] = acc;
    }
    __syncthreads();
}

__device__ __forceinline__ uint32_t tile_particle(const TileRuns& tr, uint32_t j) {
    int r = 0;
    while (r + 1 < kPifT * kPifT && tr.off[r + 1] <= j) ++r;
    return tr.start[r] + (j - tr.off[r]);
}

__device__ __forceinline__ void tile_origin(int n, int& cx0, int& cy0, int& cz0) {
    const uint32_t nt = (uint32_t)(n / kPifT);
    const uint32_t b = remap_xcd(blockIdx.x, gridDim.x);
    cx0 = (int)(b % nt) * kPifT;
    cy0 = (int)((b / nt) % nt) * kPifT;
    cz0 = (int)(b / (nt * nt)) * kPifT;
}

template <int W>
__global__ __launch_bounds__(kPifNT) void pif_spread_kernel(
    int n, int m, const double* __restrict__ x, const double* __restrict__ y,
    const double* __restrict__ z, const uint32_t* __restrict__ cs, double q, double inv_h,
    double beta, double* __restrict__ grid) {
    constexpr int R = 2 * kPifT + W;
    __shared__ double acc[R * R * R];
    __shared__ TileRuns tr;
    int cx0, cy0, cz0;
    tile_origin(n, cx0, cy0, cz0);
    for (int e = threadIdx.x; e < R * R * R; e += kPifNT) acc[e] = 0.0;
    tile_runs(tr, cs, n, cx0, cy0, cz0);
    const int lox = 2 * cx0 - W / 2, loy = 2 * cy0 - W / 2, loz = 2 * cz0 - W / 2;
    const uint32_t cnt = tr.off[kPifT * kPifT];
    for (uint32_t j = threadIdx.x; j < cnt; j += kPifNT) {
        const uint32_t p = tile_particle(tr, j);
        double wx[W], wy[W], wz[W];
        const int lx = axis_weights<W>(x[p] * inv_h, lox, beta, wx);
        const int ly = axis_weights<W>(y[p] * inv_h, loy, beta, wy);
        const int lz = axis_weights<W>(z[p] * inv_h, loz, beta, wz);
#pragma unroll
        for (int c = 0; c < W; ++c) {
#pragma unroll
            for (int b = 0; b < W; ++b) {
                const double qzy = q * (wz[c] * wy[b]);
                double* row = acc + ((lz + c) * R + (ly + b)) * R + lx;
#pragma unroll
                for (int a = 0; a < W; ++a) atomicAdd(row + a, qzy * wx[a]);
            }
        }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < R * R * R; e += kPifNT) {
        const double v = acc[e];
        if (v == 0.0) continue;
        int gx = lox + e % R, gy = loy + (e / R) % R, gz = loz + e / (R * R);
        gx = gx < 0 ? gx + m : (gx >= m ? gx - m : gx);
        gy = gy < 0 ? gy + m : (gy >= m ? gy - m : gy);
        gz = gz < 0 ? gz + m : (gz >= m ? gz - m : gz);
        atomicAdd(grid + ((size_t)gz * m + gy) * m + gx, v);
    }
}

__global__ __launch_bounds__(kPifNT) void pif_zero_kernel(int64_t cnt, double* __restrict__ a) {
    for (int64_t i = (int64_t)blockIdx.x * kPifNT + threadIdx.x; i < cnt;
         i += (int64_t)gridDim.x * kPifNT)
        a[i] = 0.0;
}

// One field component's half spectrum from the grid's: entry (kz, ky, kx),
// kx = 0 .. m/2, signed ky, kz.  Modes in K_N and in -K_N each contribute
// half (the Hermitian part of the type-2 sum), both window deconvolutions
// corr(kx) corr(ky) corr(kz) squared, -i k_d / |k|^2 and 1/L^3.  With
// want_wx, W_x = (1 / (2 L^3)) sum over the full spectrum of |E_hat_x|^2
// (a kx > 0 entry stands for its conjugate partner too).
__global__ __launch_bounds__(kPifNT) void pif_modes_kernel(
    int n, int m, double kf, double inv_l3, int dir, const double* __restrict__ corr,
    const double2* __restrict__ G, double2* __restrict__ F, int want_wx, DevState* st,
    double* part) {
    __shared__ double red[kPifNT / kWave];
    __shared__ int lflag;
    const int mh = m / 2 + 1;
    const int64_t total = (int64_t)m * m * mh;
    double acc[1] = {0.0};
    for (int64_t e = (int64_t)blockIdx.x * kPifNT + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * kPifNT) {
        const int ix = (int)(e % mh);
        const int iy = (int)((e / mh) % m);
        const int iz = (int)(e / ((int64_t)mh * m));
        const int jx = ix, jy = iy < m / 2 ? iy : iy - m, jz = iz < m / 2 ? iz : iz - m;
        const int lo = -n / 2, hi = n / 2 - 1;
        const bool in_k = jx <= hi && jy >= lo && jy <= hi && jz >= lo && jz <= hi;
        const bool in_neg = jx <= -lo && jy >= -hi && jy <= -lo && jz >= -hi && jz <= -lo;
        double2 o = make_double2(0.0, 0.0);
        if ((in_k || in_neg) && (jx | jy | jz) != 0) {
            const double wgt = 0.5 * ((in_k ? 1.0 : 0.0) + (in_neg ? 1.0 : 0.0));
            const double kx = kf * jx, ky = kf * jy, kz = kf * jz;
            const double k2 = (kx * kx + ky * ky) + kz * kz;
            const double c = (corr[jx + n / 2] * corr[jy + n / 2]) * corr[jz + n / 2];
            const double kd = dir == 0 ? kx : (dir == 1 ? ky : kz);
            const double2 g = G[e];
            // E_hat = -i k_d rho_hat / |k|^2, rho_hat = c G
            const double s = wgt * c / k2;
            const double er = kd * (s * g.y), ei = -kd * (s * g.x);
            if (want_wx) acc[0] += (ix == 0 ? 1.0 : 2.0) * (er * er + ei * ei);
            o = make_double2(er * (c * inv_l3), ei * (c * inv_l3));
        }
        F[e] = o;
    }
    if (!want_wx) return;
    block_sum<kPifNT, 1>(acc, red);
    if (threadIdx.x == 0) part[blockIdx.x] = acc[0];
    if (last_block(&st->tickets[5], gridDim.x, &lflag)) {
        double tot[1];
        sum_partials<kPifNT, 1>(part, (int)gridDim.x, tot, red);
        if (threadIdx.x == 0) st->wx = 0.5 * tot[0] * inv_l3;
    }
}

template <int W, int MODE>
__global__ __launch_bounds__(kPifNT) void pif_interp_kernel(
    int n, int m, double* __restrict__ x, double* __restrict__ y, double* __restrict__ z,
    double* __restrict__ vx, double* __restrict__ vy, double* __restrict__ vz,
    double* __restrict__ ex, double* __restrict__ ey, double* __restrict__ ez,
    uint32_t* __restrict__ key, const uint32_t* __restrict__ cs, const double* __restrict__ fx,
    const double* __restrict__ fy, const double* __restrict__ fz, double inv_h, double beta,
    double coef, double dt, double L, double inv_hn) {
    constexpr int R = 2 * kPifT + W;
    constexpr int R3 = R * R * R;
    __shared__ double reg[3 * R3];
    __shared__ TileRuns tr;
    int cx0, cy0, cz0;
    tile_origin(n, cx0, cy0, cz0);
    const int lox = 2 * cx0 - W / 2, loy = 2 * cy0 - W / 2, loz = 2 * cz0 - W / 2;
    for (int e = threadIdx.x; e < R3; e += kPifNT) {
        int gx = lox + e % R, gy = loy + (e / R) % R, gz = loz + e / (R * R);
        gx = gx < 0 ? gx + m : (gx >= m ? gx - m : gx);
        gy = gy < 0 ? gy + m : (gy >= m ? gy - m : gy);
        gz = gz < 0 ? gz + m : (gz >= m ? gz - m : gz);
        const size_t g = ((size_t)gz * m + gy) * m + gx;
        reg[e] = fx[g];
        reg[R3 + e] = fy[g];
        reg[2 * R3 + e] = fz[g];
    }
    tile_runs(tr, cs, n, cx0, cy0, cz0);
    const uint32_t cnt = tr.off[kPifT * kPifT];
    for (uint32_t j = threadIdx.x; j < cnt; j += kPifNT) {
        const uint32_t p = tile_particle(tr, j);
        const double px = x[p], py = y[p], pz = z[p];
        double wx[W], wy[W], wz[W];
        const int lx = axis_weights<W>(px * inv_h, lox, beta, wx);
        const int ly = axis_weights<W>(py * inv_h, loy, beta, wy);
        const int lz = axis_weights<W>(pz * inv_h, loz, beta, wz);
        double sx = 0.0, sy = 0.0, sz = 0.0;
#pragma unroll
        for (int c = 0; c < W; ++c) {
#pragma unroll
            for (int b = 0; b < W; ++b) {
                const double wzy = wz[c] * wy[b];
                const int row = ((lz + c) * R + (ly + b)) * R + lx;
#pragma unroll
                for (int a = 0; a < W; ++a) {
                    const double wt = wzy * wx[a];
                    sx += wt * reg[row + a];
                    sy += wt * reg[R3 + row + a];
                    sz += wt * reg[2 * R3 + row + a];
                }
            }
        }
        if (MODE == 0) {
            ex[p] = sx;
            ey[p] = sy;
            ez[p] = sz;
        } else {
            const double ux = vx[p] + coef * sx;
            const double uy = vy[p] + coef * sy;
            const double uz = vz[p] + coef * sz;
            vx[p] = ux;
            vy[p] = uy;
            vz[p] = uz;
            if (MODE == 1) {
                const double nx = wrap(px + dt * ux, L);
                const double ny = wrap(py + dt * uy, L);
                const double nz = wrap(pz + dt * uz, L);
                x[p] = nx;
                y[p] = ny;
                z[p] = nz;
                key[p] = key_of(nx, ny, nz, n, inv_hn);
            }
        }
    }
}

// ----------------------------------------------------------- launchers ----

static int hip_fail(const char* what, hipError_t e) {
    g_pif_err = std::string(what) + ": " + hipGetErrorString(e);
    return -2;
}

template <int W>
static hipError_t spread_w(PifState* p, const double* x, const double* y, const double* z,
                           const uint32_t* cs, double q, hipStream_t s) {
    const int nt = p->n / kPifT;
    hipLaunchKernelGGL(pif_spread_kernel<W>, dim3(nt * nt * nt), dim3(kPifNT), 0, s, p->n, p->m, x,
                       y, z, cs, q, p->inv_h, p->beta, p->grid);
    return hipGetLastError();
}

static hipError_t spread(PifState* p, const double* x, const double* y, const double* z,
                         const uint32_t* cs, double q, hipStream_t s) {
    switch (p->w) {
        case 3: return spread_w<3>(p, x, y, z, cs, q, s);
        case 4: return spread_w<4>(p, x, y, z, cs, q, s);
        case 5: return spread_w<5>(p, x, y, z, cs, q, s);
        case 6: return spread_w<6>(p, x, y, z, cs, q, s);
        case 7: return spread_w<7>(p, x, y, z, cs, q, s);
        case 8: return spread_w<8>(p, x, y, z, cs, q, s);
        default: return hipErrorInvalidValue;
    }
}

int pif_spread(PifState* p, int64_t np, const double* x, const double* y, const double* z,
               const uint32_t* cell_start, double q, hipStream_t s) {
    const int64_t m3 = (int64_t)p->m * p->m * p->m;
    hipError_t e;
    hipLaunchKernelGGL(pif_zero_kernel, dim3(4096), dim3(kPifNT), 0, s, m3, p->grid);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail("zero", e);
    if (np > 0 && (e = spread(p, x, y, z, cell_start, q, s)) != hipSuccess)
        return hip_fail("spread", e);
    return 0;
}

int pif_fields(PifState* p, DevState* st, double* partials, hipStream_t s) {
    hipError_t e;
    if (fft_forward(p->fft, p->grid, p->G, s) != 0) {
        g_pif_err = std::string("forward transform: ") + fft_last_error();
        return -2;
    }
    double* out[3] = {p->grid, p->fy, p->fz};
    const double inv_l3 = 1.0 / (p->L * p->L * p->L);
    for (int d = 0; d < 3; ++d) {
        hipLaunchKernelGGL(pif_modes_kernel, dim3(2048), dim3(kPifNT), 0, s, p->n, p->m, p->kf,
                           inv_l3, d, p->corr, p->G, p->F, d == 0 ? 1 : 0, st, partials);
        if ((e = hipGetLastError()) != hipSuccess) return hip_fail("modes", e);
        if (fft_inverse(p->fft, p->F, out[d], s) != 0) {
            g_pif_err = std::string("inverse transform: ") + fft_last_error();
            return -2;
        }
    }
    return 0;
}

template <int W, int MODE>
static hipError_t interp_wm(PifState* p, int64_t, double* x, double* y, double* z, double* vx,
                            double* vy, double* vz, double* ex, double* ey, double* ez,
                            uint32_t* key, const uint32_t* cs, double coef, double dt,
                            hipStream_t s) {
    const int nt = p->n / kPifT;
    hipLaunchKernelGGL((pif_interp_kernel<W, MODE>), dim3(nt * nt * nt), dim3(kPifNT), 0, s, p->n,
                       p->m, x, y, z, vx, vy, vz, ex, ey, ez, key, cs, p->grid, p->fy, p->fz,
                       p->inv_h, p->beta, coef, dt, p->L, (double)p->n / p->L);
    return hipGetLastError();
}

template <int MODE>
static hipError_t interp_m(PifState* p, int64_t np, double* x, double* y, double* z, double* vx,
                           double* vy, double* vz, double* ex, double* ey, double* ez,
                           uint32_t* key, const uint32_t* cs, double coef, double dt,
                           hipStream_t s) {
#define PIF_W(WW)                                                                             \
    case WW:                                                                                  \
        return interp_wm<WW, MODE>(p, np, x, y, z, vx, vy, vz, ex, ey, ez, key, cs, coef, dt, s)
    switch (p->w) {
        PIF_W(3);
        PIF_W(4);
        PIF_W(5);
        PIF_W(6);
        PIF_W(7);
        PIF_W(8);
        default: return hipErrorInvalidValue;
    }
#undef PIF_W
}

int pif_interp(PifState* p, int mode, int64_t np, double* x, double* y, double* z, double* vx,
               double* vy, double* vz, double* ex, double* ey, double* ez, uint32_t* key,
               const uint32_t* cell_start, double coef, double dt, hipStream_t s) {
    if (np == 0) return 0;
    hipError_t e;
    if (mode == 0)
        e = interp_m<0>(p, np, x, y, z, vx, vy, vz, ex, ey, ez, key, cell_start, coef, dt, s);
    else if (mode == 1)
        e = interp_m<1>(p, np, x, y, z, vx, vy, vz, ex, ey, ez, key, cell_start, coef, dt, s);
    else
        e = interp_m<2>(p, np, x, y, z, vx, vy, vz, ex, ey, ez, key, cell_start, coef, dt, s);
    return e == hipSuccess ? 0 : hip_fail("field at the particles", e);
}

}  // namespace pic
