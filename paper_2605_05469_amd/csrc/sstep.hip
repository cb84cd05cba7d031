// sstep.hip -- Jacobi-PCG on the periodic box in s-step form (Sec. 3.2's
// PCG with the scalar Jacobi preconditioner; the iterates are those of the
// textbook recurrence up to rounding).
//
// With M^{-1} = c I (c = h^2 / 6), PCG is CG on Ahat = c A with the scaled
// residual z = c r.  One outer step covers S iterations: the vectors the
// next S iterations combine lie in the span of the basis
//   Y = [T_0(p) .. T_S(p), T_0(r) .. T_{S-1}(r)],  T_j Chebyshev polynomials
// of Ahat - I = -N / 6 (N: sum of the six neighbours; the spectrum of
// Ahat - I lies in [-1, 1], where the T_j stay bounded, so the basis is well
// conditioned), T_0(v) = v, T_1(v) = -N v / 6, T_{j+1}(v) = -N T_j(v) / 3 -
// T_{j-1}(v).  Two sweeps per outer step:
//   * Gram sweep: forms Y at every point from p and r (a z-march with the
//     levels T_j staggered by one plane each; in-plane neighbours through
//     one LDS plane per level that feeds another; a level only where some
//     point of the work unit needs it) and reduces the 6S inner products
//     that fix G = Y^T Y (ss_gram).
//     The last workgroup runs the S iterations on coordinate vectors of
//     length 2S + 1 (alpha, beta and ||r|| from G; Ahat acts on coordinates
//     through the Chebyshev three-term relation) and leaves the coefficients
//     of the new p, r and the x increment in the device state.
//   * update sweep: forms Y again and writes p = Y c_p, r = Y c_r and
//     x += Y c_x.
// Bytes per grid point per outer step: 16 (Gram: p, r read) + 48 (update:
// p, r, x read, p, r, x written) = 64 for S iterations; against 40 per
// iteration for the single-reduction sweep.  The S-fold temporal blocking
// costs a halo of S points around the tile and 2S - 1 neighbour sums per
// point per sweep.
//
// The stop test uses ||r|| = sqrt(z^T G z) / c after every iteration, so the
// iteration count is exact; a step that passes it ends the outer step early
// (the update sweep then applies x only) and the true residual decides, as
// in the single-reduction form.
#include <type_traits>
#include <utility>

#include "common.hpp"
#include "solver_state.hpp"

namespace pic {

// The s-step sweeps are not compared bit for bit with anything (only their
// iterates, up to rounding), so products and sums may contract into FMAs.
#pragma clang fp contract(fast)

__device__ __forceinline__ double ld_nt(const double* p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ void st_nt(double v, double* p) { __builtin_nontemporal_store(v, p); }
// The element at byte offset o of a plane: the plane's base is uniform and
// the lane offset 32-bit (plane offsets stay below 2^32 bytes), so loads and
// stores take the scalar-base addressing form.
template <class T>
__device__ __forceinline__ T* ss_at(T* base, uint32_t o) {
    return (T*)((char*)base + o);
}
template <class T>
__device__ __forceinline__ const T* ss_at(const T* base, uint32_t o) {
    return (const T*)((const char*)base + o);
}

// ring of planes kept per level: chain 0 = p (levels 0..S), 1 = r (0..S-1)
__host__ __device__ constexpr int ss_qsz(int chain, int m, int S) {
    const int top = chain == 0 ? S : S - 1;
    if (m == top) return chain == 0 ? 1 : 2;
    const int h = S - m + 1;
    return h < 3 ? 3 : h;
}
__host__ __device__ constexpr int ss_base(int chain, int m, int S) {
    int b = 0;
    if (chain == 1)
        for (int i = 0; i <= S; ++i) b += ss_qsz(0, i, S);
    for (int i = 0; i < m; ++i) b += ss_qsz(chain, i, S);
    return b;
}
__host__ __device__ constexpr int ss_total(int S) { return ss_base(1, S, S); }
// Ring entry of level m holding the value pushed at phase ph (ph may be
// negative: pushes of the previous period).
__host__ __device__ constexpr int ss_slot(int chain, int m, int ph, int S) {
    const int q = ss_qsz(chain, m, S);
    return ss_base(chain, m, S) + ((ph % q) + q) % q;
}
__host__ __device__ constexpr int ss_gcd(int a, int b) { return b == 0 ? a : ss_gcd(b, a % b); }
// Phases after which every ring is back at its first entry (the least
// common multiple of the ring sizes).
__host__ __device__ constexpr int ss_period(int S) {
    int l = 1;
    for (int ch = 0; ch < 2; ++ch)
        for (int m = 0; m <= (ch == 0 ? S : S - 1); ++m) {
            const int q = ss_qsz(ch, m, S);
            l = l / ss_gcd(l, q) * q;
        }
    return l;
}
template <class F, int... I>
__device__ __forceinline__ void ss_unroll(F&& f, std::integer_sequence<int, I...>) {
    (f(std::integral_constant<int, I>{}), ...);
}

// Work units of a workgroup's (TX + 2S) x (TY + 2S) region: RU units of two
// region rows' TX tile columns (whole cache lines), HU units of 64 halo-column
// points taken row by row (2S points per row: short contiguous runs), then
// units with no point; unit k * NW + w is slot k of wave w.  A point at
// distance d from the tile (the larger of its x and y distances) needs
// p-level m only for d <= S - m and r-level m only for d <= S - 1 - m, so a
// unit need not form the levels that none of its points needs (the outer
// row pairs form p-level 1 only, the halo-column units no top level).
template <int S, int TX, int TY, int NT>
struct SsUnits {
    static constexpr int H0 = TY + 2 * S, NW = NT / kWave, RU = (H0 + 1) / 2;
    static constexpr int NH = 2 * S * H0;  // halo-column points
    static constexpr int HU = (NH + kWave - 1) / kWave;
    static constexpr int NU = (RU + HU + NW - 1) / NW * NW;
    int dmin[NU];  // distance of the unit's nearest point (S + 1: no point)
    static constexpr int dist(int l, int t) { return l < S ? S - l : (l >= t + S ? l - t - S + 1 : 0); }
    // halo-column entry e: region column and row
    static constexpr int halo_lx(int e) {
        const int cc = e % (2 * S);
        return cc < S ? cc : TX + cc;
    }
    static constexpr int halo_ly(int e) { return e / (2 * S); }
    constexpr SsUnits() : dmin() {
        for (int u = 0; u < NU; ++u) {
            int d = S + 1;
            if (u < RU) {
                for (int ly = 2 * u; ly < 2 * u + 2 && ly < H0; ++ly)
                    d = dist(ly, TY) < d ? dist(ly, TY) : d;
            } else if (u < RU + HU) {
                for (int e = (u - RU) * kWave; e < (u - RU + 1) * kWave && e < NH; ++e) {
                    const int dx = dist(halo_lx(e), TX), dy = dist(halo_ly(e), TY);
                    const int de = dx > dy ? dx : dy;
                    d = de < d ? de : d;
                }
            }
            dmin[u] = d;
        }
    }
};

// The Gram matrix from 6S inner products.  The T_j are Chebyshev
// polynomials of one symmetric operator, so T_i T_j = (T_{i+j} + T_{|i-j|})/2
// and (T_i u, T_j v) = (m_{i+j} + m_{|i-j|}) / 2 with the moments m_k =
// (u, T_k v); the moments up to 2S come from (u, T_k v) for small k and
// from products with the top level, (T_a u, T_b v) = (m_{a+b} + m_{|a-b|})/2
// solved for m_{a+b}.  Input order: (p, T_k p) k = 0..S; (T_S p, T_j p)
// j = 1..S; (r, T_k r) k = 0..S-1; (T_{S-1} r, T_j r) j = 1..S-1;
// (p, T_k r) k = 0..S-1; (T_i p, T_{S-1} r) i = 1..S.  Output: packed
// upper triangle of G over [T_0 p .. T_S p, T_0 r .. T_{S-1} r].
template <int S>
__device__ void ss_gram(const double* a, double* Gp) {
    constexpr int NV = 2 * S + 1;
    double mp[2 * S + 1], mr[2 * S - 1], mx[2 * S];
    int o = 0;
    for (int k = 0; k <= S; ++k) mp[k] = a[o++];
    for (int j = 1; j <= S; ++j) mp[S + j] = 2.0 * a[o++] - mp[S - j];
    for (int k = 0; k < S; ++k) mr[k] = a[o++];
    for (int j = 1; j < S; ++j) mr[S - 1 + j] = 2.0 * a[o++] - mr[S - 1 - j];
    for (int k = 0; k < S; ++k) mx[k] = a[o++];
    for (int i = 1; i <= S; ++i) {
        const int d = i - (S - 1);
        mx[i + S - 1] = 2.0 * a[o++] - mx[d < 0 ? -d : d];
    }
    int k = 0;
    for (int i = 0; i < NV; ++i)
        for (int j = i; j < NV; ++j) {
            double v;
            if (j <= S) {  // p, p
                v = 0.5 * (mp[i + j] + mp[j - i]);
            } else if (i > S) {  // r, r
                const int a2 = i - S - 1, b2 = j - S - 1;
                v = 0.5 * (mr[a2 + b2] + mr[b2 - a2]);
            } else {  // p, r
                const int b2 = j - S - 1, d = i - b2;
                v = 0.5 * (mx[i + b2] + mx[d < 0 ? -d : d]);
            }
            Gp[k++] = v;
        }
}

// Tile of a workgroup.  Workgroups are dealt to the eight XCDs in turn and
// (one per CU) run in rounds of 256 when the grid has more tiles than CUs
// (1024^3: 1024 tiles).  With tiles in rows of a multiple of 16 and one
// workgroup per tile column, each round takes a 16 x 16 block of tiles and
// each XCD two adjacent tile rows of it, so the halo rows a workgroup reads
// belong to tiles running at the same time on the same XCD or the next (in
// its L2, or read once more); otherwise the generic XCD-contiguous order.
__device__ __forceinline__ void ss_tile(uint32_t bid, int nbx, int nby, int nbz, int& bx, int& by,
                                        int& bz) {
    if (nbz == 1 && nbx % 16 == 0 && nby % 16 == 0) {
        const uint32_t group = bid >> 8, w = bid & 255u;
        const uint32_t xcd = w & 7u, k = w >> 3;  // k-th workgroup of this XCD in the round
        const uint32_t gpr = (uint32_t)nbx / 16u;  // 16 x 16 blocks per block row
        by = (int)((group / gpr) * 16u + 2u * xcd + (k >> 4));
        bx = (int)((group % gpr) * 16u + (k & 15u));
        bz = 0;
        return;
    }
    const uint32_t nb = (uint32_t)(nbx * nby * nbz);
    const uint32_t lb = remap_xcd(bid, nb);
    bx = (int)(lb % nbx);
    by = (int)((lb / nbx) % nby);
    bz = (int)(lb / (nbx * nby));
}

// Coefficient step (one thread): G packed upper triangle of Y^T Y (r-world
// basis), c = M^{-1} scalar.  Runs up to S iterations of CG on coordinates.
template <int S>
__device__ void ss_coefficients(const double* Gp, double c, DevState* st) {
    constexpr int NV = 2 * S + 1;
    CgScalars& cg = st->cg;
    double G[NV][NV];
    {
        int k = 0;
        for (int i = 0; i < NV; ++i)
            for (int j = i; j < NV; ++j) {
                const double di = i > S ? c : 1.0, dj = j > S ? c : 1.0;
                G[i][j] = G[j][i] = di * dj * Gp[k++];
            }
    }
    // Ahat on coordinates: Ahat T_0 = T_0 + T_1, Ahat T_j = T_j + (T_{j+1} + T_{j-1}) / 2
    auto bmul = [&](const double* w, double* o) {
        for (int i = 0; i < NV; ++i) o[i] = 0.0;
        for (int ch = 0; ch < 2; ++ch) {
            const int b0 = ch == 0 ? 0 : S + 1, top = ch == 0 ? S : S - 1;
            for (int j = 0; j <= top; ++j) {
                const double v = w[b0 + j];
                if (v == 0.0) continue;
                o[b0 + j] += v;
                if (j == 0) {
                    if (top >= 1) o[b0 + 1] += v;
                } else {
                    if (j + 1 <= top) o[b0 + j + 1] += 0.5 * v;
                    o[b0 + j - 1] += 0.5 * v;
                }
            }
        }
    };
    auto quad = [&](const double* a, const double* b) {
        double s = 0.0;
        for (int i = 0; i < NV; ++i) {
            double t = 0.0;
            for (int j = 0; j < NV; ++j) t += G[i][j] * b[j];
            s += a[i] * t;
        }
        return s;
    };
    double pp[NV], zz[NV], xx[NV], w[NV];
    for (int i = 0; i < NV; ++i) pp[i] = zz[i] = xx[i] = 0.0;
    pp[0] = 1.0;
    zz[S + 1] = 1.0;
    double mu = quad(zz, zz);
    int final = 0, rst = 0, steps = 0;
    for (int j = 0; j < S; ++j) {
        bmul(pp, w);
        const double nu = quad(pp, w);
        if (!(nu > 0.0) || !isfinite(nu) || !isfinite(mu)) {
            // p . A p lost to cancellation (the residual at the rounding
            // floor): keep the steps made and restart from p = M^{-1} r; a
            // restarted direction without positive curvature is a breakdown
            if (j == 0 && (cg.restart || !isfinite(nu) || !isfinite(mu))) {
                cg.state = CG_BREAKDOWN;
                return;
            }
            rst = 1;
            break;
        }
        const double alpha = mu / nu;
        for (int i = 0; i < NV; ++i) {
            xx[i] += alpha * pp[i];
            zz[i] -= alpha * w[i];
        }
        const double mu2 = quad(zz, zz);
        ++steps;
        cg.iter += 1;
        const double rn = sqrt(mu2 > 0.0 ? mu2 : 0.0) / c;
        cg.rr = rn * rn;
        if (!isfinite(mu2)) {
            cg.state = CG_BREAKDOWN;
            return;
        }
        if (rn <= cg.tol) {
            final = 1;
            break;
        }
        if (cg.iter >= cg.max_iter) {
            final = 2;
            break;
        }
        const double beta = mu2 / mu;
        for (int i = 0; i < NV; ++i) pp[i] = zz[i] + beta * pp[i];
        mu = mu2;
    }
    // r-world coefficients: p = Y_z pp, r = Y_z zz / c, x += Y_z xx, where
    // the r-chain vectors of Y_z are c times those of Y
    for (int i = 0; i < NV; ++i) {
        const bool rch = i > S;
        st->ss_cp[i] = rch ? c * pp[i] : pp[i];
        st->ss_cr[i] = rch ? zz[i] : zz[i] / c;
        st->ss_cx[i] = rch ? c * xx[i] : xx[i];
    }
    st->ss_final = final;
    st->ss_restart = rst;
    st->ss_steps = steps;
}

// MODE 0: Gram sweep; MODE 1: update sweep.
template <int S, int TX, int TY, int NT, int MODE>
__global__ __launch_bounds__(NT) void sstep_kernel(int n, int nbx, int nby, int nbz,
                                                   const double* __restrict__ r_in,
                                                   const double* __restrict__ p_in,
                                                   double* __restrict__ r_out,
                                                   double* __restrict__ p_out, double* x, double c,
                                                   DevState* st, double* part) {
    constexpr int NV = 2 * S + 1;
    constexpr int NG = NV * (NV + 1) / 2;
    constexpr int NM = 6 * S;  // Gram sweep: moments reduced per point
    constexpr int W0 = TX + 2 * S, H0 = TY + 2 * S;
    constexpr int WP = W0 + 2, HP = H0 + 2;
    // two rows past the padded region: the LDS entries of the slots that
    // hold no region point (their writes land there and are never read)
    constexpr int PLANE = WP * (HP + 2);
    // Region points per thread.  Each wave takes two region rows' 32 tile
    // columns (whole cache lines for every load and store of the tile
    // columns); the spare waves take the 2S halo columns of every row.
    static_assert(TX == 32, "row-aligned dealing assumes 32-wide tiles");
    constexpr int NW = NT / kWave;
    constexpr int RU = (H0 + 1) / 2;                          // row units
    constexpr int HU = (2 * S * H0 + kWave - 1) / kWave;      // halo-column units
    constexpr int NP = (RU + HU + NW - 1) / NW;
    constexpr int NF = 2 * S - 1;  // feeding levels: p-chain 0..S-1, r-chain 0..S-2
    constexpr int TOT = ss_total(S);
    __shared__ double lds[2][NF][PLANE];  // double-buffered: one barrier per plane
    __shared__ double red[(MODE == 0 ? NM : 1) * (NT / kWave)];
    __shared__ int lflag;
    if (st->cg.state != CG_RUNNING) return;
    const int restart = st->cg.restart;

    const int tid = threadIdx.x;
    const uint32_t nb = (uint32_t)(nbx * nby * nbz);
    const uint32_t lb = blockIdx.x;  // partials slot
    int bx, by, bz;
    ss_tile(blockIdx.x, nbx, nby, nbz, bx, by, bz);
    const int x0 = bx * TX, y0 = by * TY;
    const int z0 = (int)(((int64_t)bz * n) / nbz);
    const int z1 = (int)((((int64_t)bz + 1) * n) / nbz);
    const size_t nn = (size_t)n * n;
    auto wrap = [n](int v) { return v < 0 ? v + n : (v >= n ? v - n : v); };

    // Gram sweep: skip the levels no point of a unit needs (13% off the
    // sweep at 512^3, and the registers this frees let its rings be
    // phase-indexed too); update sweep: form every level at every point
    constexpr bool SKIP = MODE == 0;
    using Units = SsUnits<S, TX, TY, NT>;
    static_assert(Units::NU == NP * NW, "one unit per slot");
    constexpr Units units{};
    int pofs[NP];       // padded LDS offset of region point k
    uint32_t gofb[NP];  // its in-plane global offset in bytes (periodic image)
    uint32_t ownm = 0;  // bit k: point k is in the tile
    uint32_t ldpm = 0, ldrm = 0;  // bit k: point k loads p / r
    int dmn[NP];        // nearest distance of slot k's unit (uniform)
    // slots past the region (no point) compute on a spare LDS row, so no
    // slot needs a validity branch and none writes a region point's entry
    const int wv = __builtin_amdgcn_readfirstlane(tid / kWave);
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        const int unit = k * NW + wv, lane = tid % kWave;
        dmn[k] = units.dmin[unit];
        int lx = S, ly = 0;  // no point: a tile-column point for the global offset
        bool real = false;
        if (unit < RU) {
            ly = 2 * unit + (lane >> 5);
            lx = S + (lane & 31);
            real = ly < H0;
            if (!real) ly = H0 - 1;
        } else {
            const int e = (unit - RU) * kWave + lane;  // halo column entry
            if (e < Units::NH) {
                lx = Units::halo_lx(e);
                ly = Units::halo_ly(e);
                real = true;
            }
        }
        pofs[k] = real ? (ly + 1) * WP + lx + 1 : HP * WP + 1 + lane % (WP - 2);
        gofb[k] = ((uint32_t)wrap(y0 - S + ly) * (uint32_t)n + (uint32_t)wrap(x0 - S + lx)) * 8u;
        if (real && lx >= S && lx < TX + S && ly >= S && ly < TY + S) ownm |= 1u << k;
        const int dx = Units::dist(lx, TX), dy = Units::dist(ly, TY), d = dx > dy ? dx : dy;
        // p (level 0 of the p chain) to distance S; r to S - 1, or to S when
        // the direction restarts as M^{-1} r
        if (real) ldpm |= 1u << k;
        if (real && (!SKIP || d <= S - 1 || restart)) ldrm |= 1u << k;
    }
    // the p- or r-chain level m is formed in slot k (and its plane kept in LDS)
    auto lvl_on = [&](int k, int ch, int m) {
        return !SKIP || dmn[k] <= (ch == 0 ? S - m : S - 1 - m);
    };
    for (int i = tid; i < 2 * NF * PLANE; i += NT) (&lds[0][0][0])[i] = 0.0;

    double cp[NV], cr[NV], cx[NV];
    if constexpr (MODE == 1) {
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            cp[i] = st->ss_cp[i];
            cr[i] = st->ss_cr[i];
            cx[i] = st->ss_cx[i];
        }
    }

    double ring[TOT][NP];
#pragma unroll
    for (int i = 0; i < TOT; ++i)
#pragma unroll
        for (int k = 0; k < NP; ++k) ring[i][k] = 0.0;
    double ldp[NP], ldr[NP];  // level 0 of the next plane (loads in flight)
    double xn[MODE == 1 ? NP : 1];  // update sweep: x of the next output plane
#pragma unroll
    for (int k = 0; k < (MODE == 1 ? NP : 1); ++k) xn[k] = 0.0;
    auto fetch = [&](int zr) {
        const size_t zo = (size_t)wrap(zr) * nn;
        const double* rz = r_in + zo;
        const double* pz = p_in + zo;
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            ldr[k] = ((ldrm >> k) & 1u) ? *ss_at(rz, gofb[k]) : 0.0;
            ldp[k] = (restart || !((ldpm >> k) & 1u)) ? 0.0 : *ss_at(pz, gofb[k]);
        }
    };
    double acc[MODE == 0 ? NM : 1];
#pragma unroll
    for (int i = 0; i < (MODE == 0 ? NM : 1); ++i) acc[i] = 0.0;

    const int t0 = z0 - S, t1 = z1 + S;  // level 0 planes t0 .. t1 - 1
    fetch(t0);
    __syncthreads();  // LDS cleared
    // Each level keeps its last q planes in registers, in a ring indexed by
    // the phase PH = (t - t0) mod ss_period(S); the march is unrolled over
    // one period, so every ring index is a compile-time constant and pushing
    // a plane moves no value between registers.
    constexpr int PER = ss_period(S);
    auto step = [&](auto phc, int t) __attribute__((always_inline)) {
        constexpr int PH = decltype(phc)::value;
        // ring entry of level m holding the plane pushed `age` pushes before
        // the newest (before this step's push of that level: pre)
        auto rix = [](int ch, int m, int age, bool pre) {
            return ss_slot(ch, m, PH - age - (pre ? 1 : 0), S);
        };
        auto push = [&](int ch, int m, int k, double v) __attribute__((always_inline)) {
            ring[ss_slot(ch, m, PH, S)][k] = v;
        };
        double(*lb2)[PLANE] = lds[t & 1];
        // LDS: each feeding level's plane before this step (level m: t - 1 - m)
#pragma unroll
        for (int ch = 0; ch < 2; ++ch) {
#pragma unroll
            for (int m = 0; m < (ch == 0 ? S : S - 1); ++m) {
                const int slot = ch == 0 ? m : S + m;
                const int e = rix(ch, m, 0, true);
#pragma unroll
                for (int k = 0; k < NP; ++k)
                    if (lvl_on(k, ch, m)) lb2[slot][pofs[k]] = ring[e][k];
            }
        }
        // level 0 at plane t
        double l0p[NP], l0r[NP];
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            l0r[k] = ldr[k];
            l0p[k] = restart ? c * ldr[k] : ldp[k];
        }
        if (t + 1 < t1) fetch(t + 1);
        const int zo = t - S;  // output plane of this step
        const bool outp = zo >= z0 && zo < z1;
        // x of this step's output plane was loaded one step ahead; load the next
        double xv[NP];
        if constexpr (MODE == 1) {
#pragma unroll
            for (int k = 0; k < NP; ++k) xv[k] = xn[k];
            if (zo + 1 >= z0 && zo + 1 < z1) {
                const double* xz = x + (size_t)(zo + 1) * nn;
#pragma unroll
                for (int k = 0; k < NP; ++k)
                    xn[k] = ((ownm >> k) & 1u) ? ld_nt(ss_at(xz, gofb[k])) : 0.0;
            }
        }
        __syncthreads();
        // push level 0, then levels 1.. in increasing order (each reads its
        // parent's newest three planes and the parent's LDS plane)
#pragma unroll
        for (int ch = 0; ch < 2; ++ch) {
            const int top = ch == 0 ? S : S - 1;
#pragma unroll
            for (int k = 0; k < NP; ++k) push(ch, 0, k, ch == 0 ? l0p[k] : l0r[k]);
#pragma unroll
            for (int m = 1; m <= top; ++m) {
                const int slot = ch == 0 ? m - 1 : S + m - 1;
                // parent planes t - m + 1 (newest) and t - m - 1
                const int pn = rix(ch, m - 1, 0, false), po = rix(ch, m - 1, 2, false);
#pragma unroll
                for (int k = 0; k < NP; ++k) {
                    if (!lvl_on(k, ch, m)) continue;
                    double v;
                    const int pi = pofs[k];
                    const double* L = lb2[slot];
                    const double nsum = ((L[pi - 1] + L[pi + 1]) + (L[pi - WP] + L[pi + WP])) +
                                        (ring[po][k] + ring[pn][k]);
                    if (m == 1) {
                        v = nsum * (-1.0 / 6.0);
                    } else {  // grandparent plane t - m
                        v = nsum * (-1.0 / 3.0) - ring[rix(ch, m - 2, 2, false)][k];
                    }
                    push(ch, m, k, v);
                }
            }
        }
        // outputs of plane t - S at the tile points (level m: S - m pushes ago)
        if (outp) {
            const size_t zb = (size_t)zo * nn;
#pragma unroll
            for (int k = 0; k < NP; ++k) {
                if (!((ownm >> k) & 1u)) continue;
                double y[NV];
#pragma unroll
                for (int m = 0; m <= S; ++m) y[m] = ring[rix(0, m, S - m, false)][k];
#pragma unroll
                for (int m = 0; m < S; ++m) y[S + 1 + m] = ring[rix(1, m, S - m, false)][k];
                if constexpr (MODE == 0) {
                    // the products ss_gram() turns into G (y[0..S] = T_i p,
                    // y[S+1+j] = T_j r)
                    int a = 0;
#pragma unroll
                    for (int k = 0; k <= S; ++k) acc[a++] += y[0] * y[k];          // (p, T_k p)
#pragma unroll
                    for (int j = 1; j <= S; ++j) acc[a++] += y[S] * y[j];          // (T_S p, T_j p)
#pragma unroll
                    for (int k = 0; k < S; ++k) acc[a++] += y[S + 1] * y[S + 1 + k];  // (r, T_k r)
#pragma unroll
                    for (int j = 1; j < S; ++j) acc[a++] += y[2 * S] * y[S + 1 + j];  // (T_{S-1} r, T_j r)
#pragma unroll
                    for (int k = 0; k < S; ++k) acc[a++] += y[0] * y[S + 1 + k];      // (p, T_k r)
#pragma unroll
                    for (int i = 1; i <= S; ++i) acc[a++] += y[i] * y[2 * S];        // (T_i p, T_{S-1} r)
                } else {
                    double pv = 0.0, rv = 0.0, dx = 0.0;
#pragma unroll
                    for (int i = 0; i < NV; ++i) {
                        pv += cp[i] * y[i];
                        rv += cr[i] * y[i];
                        dx += cx[i] * y[i];
                    }
                    st_nt(pv, ss_at(p_out + zb, gofb[k]));
                    st_nt(rv, ss_at(r_out + zb, gofb[k]));
                    st_nt(xv[k] + dx, ss_at(x + zb, gofb[k]));
                }
            }
        }
    };
    for (int t = t0; t < t1; t += PER)
        ss_unroll(
            [&](auto phc) __attribute__((always_inline)) {
                if (t + decltype(phc)::value < t1) step(phc, t + decltype(phc)::value);
            },
            std::make_integer_sequence<int, PER>{});

    if constexpr (MODE == 0) {
        block_sum<NT, NM>(acc, red);
        if (tid == 0) {
#pragma unroll
            for (int k = 0; k < NM; ++k) part[(size_t)k * nb + lb] = acc[k];
        }
        if (last_block(&st->tickets[3], nb, &lflag)) {
            double tot[NM];
            sum_partials<NT, NM>(part, (int)nb, tot, red);
            if (tid == 0) {
                double Gp[NG];
                ss_gram<S>(tot, Gp);
                ss_coefficients<S>(Gp, c, st);
            }
        }
    } else {
        if (last_block(&st->tickets[4], nb, &lflag) && tid == 0) {
            CgScalars& cg = st->cg;
            cg.xpend = 0;
            cg.restart = st->ss_restart;
            if (st->ss_final == 1) cg.state = CG_CANDIDATE;
            else if (st->ss_final == 2) cg.state = CG_MAXIT;
        }
    }
}

// Launch shape: tiles of TX x TY, one z range per workgroup; as many
// workgroups as are resident at once (or fewer z splits when the grid has
// enough tiles).
template <int S, int TX, int TY, int NT, int MODE>
static hipError_t ss_launch(int n, const double* r_in, const double* p_in, double* r_out,
                            double* p_out, double* x, double c, DevState* st, double* part,
                            int max_blocks, hipStream_t s) {
    static int occ = 0, cus = 0;
    if (occ == 0) {
        int o = 0, cu = 0, dev = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&o, sstep_kernel<S, TX, TY, NT, MODE>, NT,
                                                         0) != hipSuccess || o < 1)
            o = 1;
        (void)hipGetDevice(&dev);
        if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            cu < 1)
            cu = 1;
        cus = cu;
        occ = o;
    }
    const int nbx = n / TX, nby = n / TY;
    const int tiles = nbx * nby;
    int nbz = occ * cus / tiles;
    if (nbz > max_blocks / tiles) nbz = max_blocks / tiles;
    if (nbz > n / 2) nbz = n / 2;  // at least two output planes per workgroup
    if (nbz < 1) nbz = 1;
    const int nb = tiles * nbz;
    if (nb > max_blocks) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL((sstep_kernel<S, TX, TY, NT, MODE>), dim3(nb), dim3(NT), 0, s, n, nbx, nby,
                       nbz, r_in, p_in, r_out, p_out, x, c, st, part);
    return hipGetLastError();
}

bool sstep_supported(const SweepGeo& g) { return g.bc == 0 && g.n % 32 == 0 && g.n >= 32; }

hipError_t launch_sstep(const SweepGeo& g, int mode, const double* r_in, const double* p_in,
                        double* r_out, double* p_out, double* x, double minv, DevState* st,
                        double* partials, int npartials, hipStream_t s) {
    constexpr int S = kSstepS;
    if (!sstep_supported(g)) return hipErrorInvalidValue;
    const int maxb = npartials / (6 * S);
    if (mode == 0)
        return ss_launch<S, 32, 32, 768, 0>(g.n, r_in, p_in, r_out, p_out, x, minv, st, partials,
                                            maxb, s);
    return ss_launch<S, 32, 32, 768, 1>(g.n, r_in, p_in, r_out, p_out, x, minv, st, partials, maxb,
                                        s);
}

}  // namespace pic
