// net_kernels.hip -- kernels of the learned warm start / preconditioner's
// network (this project's extension of the PCG solve; not in the paper).
//
// Layout: activations channels-last, BF16, [z][y][x][C]; gradients FP32 in
// the same layout until they are rounded to BF16 at a convolution's output.
// Weights: FP32 master copy in the canonical order [co][ci][27] per layer
// (tap t = 9*(dz+1) + 3*(dy+1) + (dx+1)), packed to BF16 MFMA fragments.
//
// 3^3 periodic convolutions with >= 16 channels on both sides run on the
// matrix cores as a transposed implicit GEMM,
//     D[co][pt] = sum_k W[co][k] * X^T[k][pt],  k = (tap, ci),
// with v_mfma_f32_16x16x32_bf16 (FP32 accumulation): the A fragments are the
// packed weights (staged in LDS), the B fragments are 8 consecutive channels
// of a neighbour point (one 16-byte load), and each lane's accumulator holds 4
// consecutive output channels of one point, stored as one 8-byte (BF16) or
// 16-byte (FP32) write.  The backward-data pass is the same kernel on the
// flipped, transposed weights.  The weight gradient is a GEMM over points:
// tiles of 32 points are gathered per tap into LDS transposed ([ch][pt]) so
// both MFMA operands are 16-byte LDS reads.  Layers with one channel (the
// input and output layers) are tiny contractions done on the vector ALUs.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "common.hpp"
#include "net.hpp"

namespace pic {
namespace net {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kNT = 256;

__device__ __forceinline__ uint16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

struct Pt {
    int x, y, z;
};
__device__ __forceinline__ Pt decomp(int64_t p, int n) {
    Pt r;
    r.x = (int)(p % n);
    const int64_t q = p / n;
    r.y = (int)(q % n);
    r.z = (int)(q / n);
    return r;
}
__device__ __forceinline__ int wrapi(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }
__device__ __forceinline__ int64_t nbr(const Pt& p, int t, int n) {
    const int dz = t / 9 - 1, dy = (t / 3) % 3 - 1, dx = t % 3 - 1;
    return ((int64_t)wrapi(p.z + dz, n) * n + wrapi(p.y + dy, n)) * n + wrapi(p.x + dx, n);
}

// ----------------------------------------------------------- weight pack ---
// Forward fragments: for K-chunk s and output block cb, lane l holds
// A[co = 16 cb + l%16][k = 32 s + 8 (l/16) + i], k = t*CI + ci.
// Backward-data fragments: the transposed convolution gathers dY[p - d_t]:
// as a gather over taps t' = 26 - t it has input channels co and outputs ci:
// A[ci = 16 cb + l%16][k' = t'*CO + co] = W[co][ci][t].
__global__ void pack_kernel(const float* __restrict__ W, int ci_n, int co_n, int bwd,
                            uint16_t* __restrict__ frag) {
    const int cin = bwd ? co_n : ci_n;   // gathered channels
    const int cout = bwd ? ci_n : co_n;  // produced channels
    const int kch = (27 * cin + 31) / 32;
    const int nfrag = kch * (cout / 16) * 64 * 8;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < nfrag; e += gridDim.x * blockDim.x) {
        const int i = e & 7;
        const int lane = (e >> 3) & 63;
        const int f = e >> 9;  // fragment index = s * (cout/16) + cb
        const int cb = f % (cout / 16);
        const int s = f / (cout / 16);
        const int m = cb * 16 + (lane & 15);
        const int k = 32 * s + 8 * (lane >> 4) + i;
        float v = 0.f;
        if (k < 27 * cin) {
            const int t = k / cin, c = k % cin;
            if (!bwd) v = W[((size_t)m * ci_n + c) * 27 + t];          // W[co=m][ci=c][t]
            else v = W[((size_t)c * ci_n + m) * 27 + (26 - t)];        // W[co=c][ci=m][26-t]
        }
        frag[e] = f2bf(v);
    }
}

// Plane-major fragments of the z-marching kernel: for tap plane dzi (the
// input plane z + dzi - 1), K-chunk s of that plane and output block cb,
// lane l holds A[m = 16 cb + l%16][k = 32 s + 8 (l/16) + i], k = u*cin + c
// over the 9 in-plane taps u = 3 (dy+1) + (dx+1), zero-padded to whole
// chunks.  Same transposition as above for the backward-data weights.
__global__ void pack_zm_kernel(const float* __restrict__ W, int ci_n, int co_n, int bwd,
                               uint16_t* __restrict__ frag) {
    const int cin = bwd ? co_n : ci_n;
    const int cout = bwd ? ci_n : co_n;
    const int ksp = (9 * cin + 31) / 32;
    const int ncb = cout / 16;
    const int nfrag = 3 * ksp * ncb * 64 * 8;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < nfrag; e += gridDim.x * blockDim.x) {
        const int i = e & 7;
        const int lane = (e >> 3) & 63;
        const int f = e >> 9;  // ((dzi * ksp + s) * ncb + cb)
        const int cb = f % ncb;
        const int s = (f / ncb) % ksp;
        const int dzi = f / (ncb * ksp);
        const int m = cb * 16 + (lane & 15);
        const int k = 32 * s + 8 * (lane >> 4) + i;
        float v = 0.f;
        if (k < 9 * cin) {
            const int t = 9 * dzi + k / cin, c = k % cin;
            if (!bwd) v = W[((size_t)m * ci_n + c) * 27 + t];
            else v = W[((size_t)c * ci_n + m) * 27 + (26 - t)];
        }
        frag[e] = f2bf(v);
    }
}

// ------------------------------------------------------- MFMA conv (gather) --
// MODE 0: forward, Y = relu?(acc + bias (+ skip)) in BF16.
// MODE 1: backward data, Yf = acc (+ Yf if accumulate) in FP32.
// Launch: grid.x blocks over point tiles, grid.y = output-block groups of NG.
template <int CI, int CO, int NG, int MODE>
__global__ __launch_bounds__(kNT) void conv_mfma_kernel(int n, const uint16_t* __restrict__ X,
                                                        const uint16_t* __restrict__ frag,
                                                        const float* __restrict__ bias,
                                                        const uint16_t* __restrict__ skip, int relu,
                                                        uint16_t* __restrict__ Yb,
                                                        float* __restrict__ Yf, int accumulate) {
    constexpr int KCH = (27 * CI + 31) / 32;
    constexpr int NCB = CO / 16;
    constexpr int PT = 4;  // point tiles per wave per pass
    __shared__ bf16x8 wl[KCH * NG * 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int m = lane & 15, g = lane >> 4;
    const int cg = blockIdx.y;  // output-block group
    const bf16x8* fr = reinterpret_cast<const bf16x8*>(frag);
    for (int i = threadIdx.x; i < KCH * NG * 64; i += kNT) {
        const int l = i & 63, f = i >> 6;
        const int s = f / NG, c = f % NG;
        wl[i] = fr[(s * NCB + cg * NG + c) * 64 + l];
    }
    __syncthreads();
    const int64_t n3 = (int64_t)n * n * n;
    const int64_t ntiles = n3 / 16;
    for (int64_t t0 = ((int64_t)blockIdx.x * 4 + wave) * PT; t0 < ntiles;
         t0 += (int64_t)gridDim.x * 4 * PT) {
        f32x4 acc[PT][NG];
        Pt pp[PT];
#pragma unroll
        for (int j = 0; j < PT; ++j) {
            pp[j] = decomp((t0 + j < ntiles ? t0 + j : t0) * 16 + m, n);
#pragma unroll
            for (int c = 0; c < NG; ++c) acc[j][c] = f32x4{0.f, 0.f, 0.f, 0.f};
        }
        for (int s = 0; s < KCH; ++s) {
            const int k0 = 32 * s + 8 * g;
            const int t = k0 / CI, ci0 = k0 - (k0 / CI) * CI;
            bf16x8 b[PT];
#pragma unroll
            for (int j = 0; j < PT; ++j) {
                if (t < 27) {
                    const int64_t q = nbr(pp[j], t, n);
                    b[j] = *reinterpret_cast<const bf16x8*>(X + q * CI + ci0);
                } else {
                    b[j] = bf16x8{};
                }
            }
#pragma unroll
            for (int c = 0; c < NG; ++c) {
                const bf16x8 a = wl[(s * NG + c) * 64 + lane];
#pragma unroll
                for (int j = 0; j < PT; ++j)
                    acc[j][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b[j], acc[j][c], 0, 0, 0);
            }
        }
        // lane holds D[co = 16 cb + 4 g + i][pt = m]
#pragma unroll
        for (int j = 0; j < PT; ++j) {
            if (t0 + j >= ntiles) continue;
            const int64_t p = (t0 + j) * 16 + m;
#pragma unroll
            for (int c = 0; c < NG; ++c) {
                const int co0 = (cg * NG + c) * 16 + 4 * g;
                if constexpr (MODE == 0) {
                    float y[4];
                    uint2 sk = make_uint2(0u, 0u);
                    if (skip) sk = *reinterpret_cast<const uint2*>(skip + p * CO + co0);
                    const uint16_t* sh = reinterpret_cast<const uint16_t*>(&sk);
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        y[i] = acc[j][c][i] + bias[co0 + i];
                        if (skip) y[i] += bf2f(sh[i]);
                        if (relu) y[i] = y[i] > 0.f ? y[i] : 0.f;
                    }
                    uint2 o;
                    o.x = (uint32_t)f2bf(y[0]) | ((uint32_t)f2bf(y[1]) << 16);
                    o.y = (uint32_t)f2bf(y[2]) | ((uint32_t)f2bf(y[3]) << 16);
                    *reinterpret_cast<uint2*>(Yb + p * CO + co0) = o;
                } else {
                    float4 o = make_float4(acc[j][c][0], acc[j][c][1], acc[j][c][2], acc[j][c][3]);
                    float4* dst = reinterpret_cast<float4*>(Yf + p * CO + co0);
                    if (accumulate) {
                        const float4 prev = *dst;
                        o.x += prev.x;
                        o.y += prev.y;
                        o.z += prev.z;
                        o.w += prev.w;
                    }
                    *dst = o;
                }
            }
        }
    }
}

// ------------------------------------------------ MFMA conv (z-marching) --
// Same contraction as above, organised for reuse.  A block owns a 64 x TY
// column of output points over a z range [zb, zb + zlen) and marches up it
// one input plane at a time.  Each input plane (with a one-point periodic
// halo in x and y) is staged once into LDS as [channel group][y][x] 16-byte
// records, so the B fragment of a 16-point row and 8 channels is one
// conflict-free 16-byte LDS read per lane; the next plane is loaded into
// registers while the current one is consumed.  Every B fragment feeds the
// three output planes it touches (taps dz = -1, 0, +1) through three rolling
// accumulator sets, and each wave keeps all 27 taps of its output block's
// weights in registers, so the only LDS traffic is one read per fragment.
// Output plane z is complete (and stored, with the MODE 0/1 epilogue of the
// gather kernel) once input plane z + 1 has been consumed.
// Wave w computes output block w % NCB for the point tiles q, q + WQ, ... of
// the plane (q = w / NCB, WQ = 4 / NCB).  Requires n % 64 == 0, n % TY == 0.
// UP: X is given on the n/2 grid and nearest-neighbour up-sampled while it is
// staged (the decoder's up-sampling never materialises).  SK: a skip input is
// added before the ReLU.  PL: the 2x2x2 average pool of the (BF16-rounded)
// output is formed in registers and written to Yp as well (x pairs are
// neighbouring lanes, y pairs are tiles j and j + NCB of the same wave, z
// pairs are consecutive planes; requires an even zlen).
template <int CI, int CO, int TY, int MODE, bool UP = false, bool SK = false, bool PL = false>
__global__ __launch_bounds__(kNT, (CI == 16 && MODE == 0) ? 2 : 1) void conv_zm_kernel(int n, int zlen, const uint16_t* __restrict__ X,
                                                      const uint16_t* __restrict__ fragz,
                                                      const float* __restrict__ bias,
                                                      const uint16_t* __restrict__ skip, int relu,
                                                      uint16_t* __restrict__ Yb,
                                                      float* __restrict__ Yf, int accumulate,
                                                      uint16_t* __restrict__ Yp) {
    constexpr int TX = 64, SX = TX + 2, SY = TY + 2;
    constexpr int CG = CI / 8;
    constexpr int KSP = (9 * CI + 31) / 32;
    constexpr int NCB = CO / 16;
    static_assert(NCB == 1 || NCB == 2 || NCB == 4, "output blocks per block");
    constexpr int WQ = 4 / NCB;
    constexpr int NTILE = 4 * TY;
    constexpr int PW = NTILE / WQ;
    constexpr int NCH = SY * SX * CG;  // 16-byte records per staged plane
    constexpr int NPT = (NCH + kNT - 1) / kNT;
    __shared__ bf16x8 lds[2 * NCH];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int m = lane & 15, g = lane >> 4;
    const int cb = wave % NCB, q = wave / NCB;
    const int ntx = n / TX;
    const int ncol = ntx * (n / TY);
    const int bid = (int)remap_xcd(blockIdx.x, gridDim.x);
    const int col = bid % ncol;
    const int zb = (bid / ncol) * zlen, ze = zb + zlen;
    const int x0 = (col % ntx) * TX, y0 = (col / ntx) * TY;

    bf16x8 w[3][KSP];
    const bf16x8* fz = reinterpret_cast<const bf16x8*>(fragz);
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int s = 0; s < KSP; ++s) w[d][s] = fz[((d * KSP + s) * NCB + cb) * 64 + lane];
    // LDS offset (in records, within a plane buffer) of this lane's B row
    // for each K-chunk, before the tile offset
    int boff[KSP];
#pragma unroll
    for (int s = 0; s < KSP; ++s) {
        const int k0 = 32 * s + 8 * g;
        const int u = k0 / CI, c0 = k0 - u * CI;
        // padded K entries (u >= 9) have zero weights: read any valid record
        boff[s] = u < 9 ? ((c0 / 8) * SY + u / 3) * SX + (u % 3) + m : m;
    }
    float bv[4] = {0.f, 0.f, 0.f, 0.f};
    if constexpr (MODE == 0) {
#pragma unroll
        for (int i = 0; i < 4; ++i) bv[i] = bias[16 * cb + 4 * g + i];
    }

    bf16x8 stg[NPT];
    const int ns = UP ? n / 2 : n;  // grid of X
    auto load_plane = [&](int zp) {
        int zz = zp < 0 ? zp + n : (zp >= n ? zp - n : zp);
        if constexpr (UP) zz >>= 1;
#pragma unroll
        for (int i = 0; i < NPT; ++i) {
            const int c = threadIdx.x + kNT * i;
            if (c < NCH) {
                const int cg = c % CG, pt = c / CG;
                const int xx = pt % SX, yy = pt / SX;
                int x = wrapi(x0 - 1 + xx, n), y = wrapi(y0 - 1 + yy, n);
                if constexpr (UP) {
                    x >>= 1;
                    y >>= 1;
                }
                stg[i] = *reinterpret_cast<const bf16x8*>(
                    X + (((int64_t)zz * ns + y) * ns + x) * CI + cg * 8);
            }
        }
    };
    auto store_plane = [&](int b) {
#pragma unroll
        for (int i = 0; i < NPT; ++i) {
            const int c = threadIdx.x + kNT * i;
            if (c < NCH) {
                const int cg = c % CG, pt = c / CG;
                const int xx = pt % SX, yy = pt / SX;
                lds[b * NCH + (cg * SY + yy) * SX + xx] = stg[i];
            }
        }
    };

    f32x4 acc[3][PW];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int j = 0; j < PW; ++j) acc[a][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    f32x4 rv[PL ? PW : 1];      // rounded outputs of the plane (PL)
    f32x4 pz[PL ? PW / 2 : 1];  // pooled partial sums of the even plane (PL)

    // acc[0], acc[1], acc[2] hold output planes zp - 1, zp, zp + 1 while input
    // plane zp is consumed; the partial sums of the two planes below zb and
    // of plane ze are computed and dropped (no branches around the MFMAs).
    load_plane(zb - 1);
    store_plane(0);
    __syncthreads();
    int buf = 0;
    for (int zp = zb - 1; zp <= ze; ++zp) {
        if (zp < ze) load_plane(zp + 1);
        // the skip input of output plane zp - 1, loaded before the MFMAs
        uint2 skv[PW];
        if constexpr (MODE == 0 && SK) {
            if (zp - 1 >= zb) {
#pragma unroll
                for (int j = 0; j < PW; ++j) {
                    const int T = q + WQ * j;
                    const int64_t p =
                        ((int64_t)(zp - 1) * n + y0 + (T >> 2)) * n + x0 + 16 * (T & 3) + m;
                    skv[j] = *reinterpret_cast<const uint2*>(skip + p * CO + 16 * cb + 4 * g);
                }
            }
        }
        const bf16x8* L = lds + buf * NCH;
#pragma unroll
        for (int j = 0; j < PW; ++j) {
            const int T = q + WQ * j;
            const int toff = (T >> 2) * SX + 16 * (T & 3);
#pragma unroll
            for (int s = 0; s < KSP; ++s) {
                const bf16x8 b = L[boff[s] + toff];
                acc[2][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w[0][s], b, acc[2][j], 0, 0, 0);
                acc[1][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w[1][s], b, acc[1][j], 0, 0, 0);
                acc[0][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w[2][s], b, acc[0][j], 0, 0, 0);
            }
        }
        if (zp - 1 >= zb) {
            const int z = zp - 1;
#pragma unroll
            for (int j = 0; j < PW; ++j) {
                const int T = q + WQ * j;
                const int64_t p = ((int64_t)z * n + y0 + (T >> 2)) * n + x0 + 16 * (T & 3) + m;
                const int co0 = 16 * cb + 4 * g;
                if constexpr (MODE == 0) {
                    float y[4];
                    const uint16_t* sh = reinterpret_cast<const uint16_t*>(&skv[j]);
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        y[i] = acc[0][j][i] + bv[i];
                        if constexpr (SK) y[i] += bf2f(sh[i]);
                        if (relu) y[i] = y[i] > 0.f ? y[i] : 0.f;
                    }
                    uint2 o;
                    o.x = (uint32_t)f2bf(y[0]) | ((uint32_t)f2bf(y[1]) << 16);
                    o.y = (uint32_t)f2bf(y[2]) | ((uint32_t)f2bf(y[3]) << 16);
                    *reinterpret_cast<uint2*>(Yb + p * CO + co0) = o;
                    if constexpr (PL) {
#pragma unroll
                        for (int i = 0; i < 4; ++i) rv[j][i] = bf2f(f2bf(y[i]));
                    }
                } else {
                    float4 o = make_float4(acc[0][j][0], acc[0][j][1], acc[0][j][2], acc[0][j][3]);
                    float4* dst = reinterpret_cast<float4*>(Yf + p * CO + co0);
                    if (accumulate) {
                        const float4 prev = *dst;
                        o.x += prev.x;
                        o.y += prev.y;
                        o.z += prev.z;
                        o.w += prev.w;
                    }
                    *dst = o;
                }
            }
        }
        if constexpr (MODE == 0 && PL) {
            if (zp - 1 >= zb) {
                const int z = zp - 1;
#pragma unroll
                for (int jp = 0; jp < PW / 2; ++jp) {
                    const int j0 = (jp / NCB) * 2 * NCB + (jp % NCB), j1 = j0 + NCB;
                    f32x4 sxy;
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const float a0 = rv[j0][i] + __shfl_xor(rv[j0][i], 1);
                        const float a1 = rv[j1][i] + __shfl_xor(rv[j1][i], 1);
                        sxy[i] = a0 + a1;
                    }
                    if ((z & 1) == 0) {
                        pz[jp] = sxy;
                    } else if ((m & 1) == 0) {
                        const int T = q + WQ * j0;
                        const int nh = n >> 1;
                        const int64_t P = ((int64_t)(z >> 1) * nh + ((y0 + (T >> 2)) >> 1)) * nh +
                                          ((x0 + 16 * (T & 3) + m) >> 1);
                        uint2 o;
                        o.x = (uint32_t)f2bf((pz[jp][0] + sxy[0]) * 0.125f) |
                              ((uint32_t)f2bf((pz[jp][1] + sxy[1]) * 0.125f) << 16);
                        o.y = (uint32_t)f2bf((pz[jp][2] + sxy[2]) * 0.125f) |
                              ((uint32_t)f2bf((pz[jp][3] + sxy[3]) * 0.125f) << 16);
                        *reinterpret_cast<uint2*>(Yp + P * CO + 16 * cb + 4 * g) = o;
                    }
                }
            }
        }
#pragma unroll
        for (int j = 0; j < PW; ++j) {
            acc[0][j] = acc[1][j];
            acc[1][j] = acc[2][j];
            acc[2][j] = f32x4{0.f, 0.f, 0.f, 0.f};
        }
        if (zp < ze) store_plane(buf ^ 1);
        __syncthreads();
        buf ^= 1;
    }
}

// ------------------------------------------------- MFMA weight gradient ----
// dW[co][ci][t] = sum_p X[p + d_t][ci] * G[p][co]  and  db[co] = sum_p G[p][co].
// Block y handles accumulator tiles [64 y, 64 y + 64) of the list
// (t, ci-block, co-block), t-major.  Each wave owns every 4th tile.  Per
// 32-point chunk the needed taps of X and the G tile are staged in LDS as
// [channel][point] so operands are 16-byte LDS reads.  Partial sums per block
// go to part[block][...] (canonical layout, bias last); a second kernel sums
// them over blocks in a fixed order.
template <int CI, int CO>
__global__ __launch_bounds__(kNT) void dw_mfma_kernel(int n, const uint16_t* __restrict__ X,
                                                      const uint16_t* __restrict__ G,
                                                      float* __restrict__ part, int nparts_x) {
    constexpr int CIB = CI / 16, COB = CO / 16;
    constexpr int PER_TAP = CIB * COB;
    constexpr int J = 27 * PER_TAP;
    constexpr int JG = 64;                       // tiles per block
    constexpr int TPW = JG / 4;                  // tiles per wave
    constexpr int TAPS_G = (JG + PER_TAP - 1) / PER_TAP + 1;  // taps touched by a group (bound)
    constexpr int NTAP = TAPS_G < 27 ? TAPS_G : 27;
    constexpr int CH = 32;                       // points per chunk
    __shared__ __attribute__((aligned(16))) uint16_t xs[NTAP][CI][CH];
    __shared__ __attribute__((aligned(16))) uint16_t gs[CO][CH];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int m = lane & 15, g = lane >> 4;
    const int j0 = blockIdx.y * JG;
    const int t_first = j0 / PER_TAP;
    const int j1 = (j0 + JG < J ? j0 + JG : J);
    const int t_last = (j1 - 1) / PER_TAP;
    const int ntap = t_last - t_first + 1;
    f32x4 acc[TPW];
#pragma unroll
    for (int i = 0; i < TPW; ++i) acc[i] = f32x4{0.f, 0.f, 0.f, 0.f};
    float bsum = 0.f;  // bias partial: thread tid < CO (group 0 only)
    const int64_t n3 = (int64_t)n * n * n;
    const int64_t nchunk = n3 / CH;
    for (int64_t ck = blockIdx.x; ck < nchunk; ck += gridDim.x) {
        const int64_t pbase = ck * CH;
        __syncthreads();
        // stage G tile transposed
        for (int e = threadIdx.x; e < CH * (CO / 8); e += kNT) {
            const int pt = e / (CO / 8), c8 = (e % (CO / 8)) * 8;
            const uint4 v = *reinterpret_cast<const uint4*>(G + (pbase + pt) * CO + c8);
            const uint16_t* h = reinterpret_cast<const uint16_t*>(&v);
#pragma unroll
            for (int i = 0; i < 8; ++i) gs[c8 + i][pt] = h[i];
        }
        // stage the taps this group needs, transposed
        for (int e = threadIdx.x; e < ntap * CH * (CI / 8); e += kNT) {
            const int tt = e / (CH * (CI / 8));
            const int r = e % (CH * (CI / 8));
            const int pt = r / (CI / 8), c8 = (r % (CI / 8)) * 8;
            const Pt p = decomp(pbase + pt, n);
            const int64_t q = nbr(p, t_first + tt, n);
            const uint4 v = *reinterpret_cast<const uint4*>(X + q * CI + c8);
            const uint16_t* h = reinterpret_cast<const uint16_t*>(&v);
#pragma unroll
            for (int i = 0; i < 8; ++i) xs[tt][c8 + i][pt] = h[i];
        }
        __syncthreads();
        if (blockIdx.y == 0 && threadIdx.x < CO) {
            for (int pt = 0; pt < CH; ++pt) bsum += bf2f(gs[threadIdx.x][pt]);
        }
#pragma unroll
        for (int i = 0; i < TPW; ++i) {
            const int jj = j0 + wave + 4 * i;
            if (jj >= j1) break;
            const int t = jj / PER_TAP, r = jj % PER_TAP;
            const int cib = r / COB, cob = r % COB;
            // D[ci][co] += sum_pt X[ci][pt] G[pt][co]: A = X^T rows ci, B = G cols co
            const bf16x8 a = *reinterpret_cast<const bf16x8*>(&xs[t - t_first][cib * 16 + m][8 * g]);
            const bf16x8 b = *reinterpret_cast<const bf16x8*>(&gs[cob * 16 + m][8 * g]);
            acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[i], 0, 0, 0);
        }
    }
    // write partials: lane holds D[ci = 16 cib + 4 g + e][co = 16 cob + m]
    const int64_t stride = (int64_t)27 * CI * CO + CO;
    float* out = part + ((int64_t)blockIdx.y * nparts_x + blockIdx.x) * stride;
#pragma unroll
    for (int i = 0; i < TPW; ++i) {
        const int jj = j0 + wave + 4 * i;
        if (jj >= j1) break;
        const int t = jj / PER_TAP, r = jj % PER_TAP;
        const int cib = r / COB, cob = r % COB;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int ci = cib * 16 + 4 * g + e, co = cob * 16 + m;
            out[((int64_t)co * CI + ci) * 27 + t] = acc[i][e];
        }
    }
    if (threadIdx.x < CO) out[(int64_t)27 * CI * CO + threadIdx.x] = blockIdx.y == 0 ? bsum : 0.f;
}

// Sum the partial gradients over blocks (fixed order) into grad[0..len).
// Block y of the weight-gradient kernel wrote only its own tiles; every
// group's slots are disjoint, so summing all rows adds zeros elsewhere --
// the partial buffer is cleared by the caller's fill before the launch.
__global__ void dw_reduce_kernel(const float* __restrict__ part, int64_t rows, int64_t len,
                                 float* __restrict__ grad) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len;
         i += (int64_t)gridDim.x * blockDim.x) {
        float s = 0.f;
        for (int64_t r = 0; r < rows; ++r) s += part[r * len + i];
        grad[i] = s;
    }
}

__global__ void fill_f32_kernel(int64_t n, float* __restrict__ a, float v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        a[i] = v;
}

// ------------------------------------------------ one-channel layers (VALU) --
// Weights are rounded to BF16 like the MFMA layers' (emulated in FP32).
__device__ __forceinline__ float wbf(float w) { return bf2f(f2bf(w)); }

// e1a: y[p][co] = relu(b[co] + sum_t W[co][0][t] x[p + d_t]), 16 outputs, on
// the matrix cores: the 27 taps of the single input channel (zero-padded to
// 32) are the K dimension of one v_mfma_f32_16x16x32_bf16 per 16 points;
// lane (m, g) gathers taps 8g..8g+7 of point m (cached 2-byte loads).
__global__ __launch_bounds__(kNT) void conv_in_fwd_kernel(int n, const uint16_t* __restrict__ x,
                                                          const float* __restrict__ W,
                                                          const float* __restrict__ b,
                                                          uint16_t* __restrict__ y) {
    constexpr int PT = 4;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int m = lane & 15, g = lane >> 4;
    bf16x8 a;
    uint16_t* ah = reinterpret_cast<uint16_t*>(&a);
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int t = 8 * g + i;
        ah[i] = t < 27 ? f2bf(W[m * 27 + t]) : (uint16_t)0;
    }
    float bv[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) bv[i] = b[4 * g + i];
    const int64_t ntiles = (int64_t)n * n * n / 16;
    for (int64_t t0 = ((int64_t)blockIdx.x * 4 + wave) * PT; t0 < ntiles;
         t0 += (int64_t)gridDim.x * 4 * PT) {
        bf16x8 bb[PT];
#pragma unroll
        for (int j = 0; j < PT; ++j) {
            const int64_t tile = t0 + j < ntiles ? t0 + j : t0;
            const Pt pt = decomp(tile * 16 + m, n);
            uint16_t* bh = reinterpret_cast<uint16_t*>(&bb[j]);
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int t = 8 * g + i;
                bh[i] = t < 27 ? x[nbr(pt, t, n)] : (uint16_t)0;
            }
        }
#pragma unroll
        for (int j = 0; j < PT; ++j) {
            if (t0 + j >= ntiles) continue;
            const f32x4 acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bb[j], f32x4{0.f, 0.f, 0.f, 0.f},
                                                                     0, 0, 0);
            float v[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                v[i] = acc[i] + bv[i];
                v[i] = v[i] > 0.f ? v[i] : 0.f;
            }
            uint2 o;
            o.x = (uint32_t)f2bf(v[0]) | ((uint32_t)f2bf(v[1]) << 16);
            o.y = (uint32_t)f2bf(v[2]) | ((uint32_t)f2bf(v[3]) << 16);
            *reinterpret_cast<uint2*>(y + ((t0 + j) * 16 + m) * 16 + 4 * g) = o;
        }
    }
}

// e1a, z-marching (n % 64 == 0): the single-channel input planes are staged
// in LDS (one-point halo); per input plane and 16-point tile, the 9 in-plane
// taps (zero-padded to K = 16) of v_mfma_f32_16x16x16bf16_1k feed the three
// output planes the input plane touches (weights of tap planes dz = -1, 0, +1
// in registers), with rotating accumulators as in conv_zm_kernel.  Every
// input value is read from HBM once; the kernel is bound by writing the 16
// output channels.
typedef short s16x4 __attribute__((ext_vector_type(4)));

template <int TY>
__global__ __launch_bounds__(kNT) void conv_in_zm_kernel(int n, int zlen,
                                                         const uint16_t* __restrict__ x,
                                                         const float* __restrict__ W,
                                                         const float* __restrict__ b,
                                                         uint16_t* __restrict__ y) {
    constexpr int TX = 64, SX = TX + 2, SY = TY + 2;
    constexpr int NCH = SX * SY;
    constexpr int NPT = (NCH + kNT - 1) / kNT;
    constexpr int PW = TY;  // 16-point tiles per wave per plane
    __shared__ uint16_t lds[2 * NCH];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int m = lane & 15, g = lane >> 4;
    const int ntx = n / TX;
    const int ncol = ntx * (n / TY);
    const int bid = (int)remap_xcd(blockIdx.x, gridDim.x);
    const int col = bid % ncol;
    const int zb = (bid / ncol) * zlen, ze = zb + zlen;
    const int x0 = (col % ntx) * TX, y0 = (col / ntx) * TY;

    // A: w[dzi], lane (m, g): W[co = m][tap 9 dzi + u], u = 4 g + i < 9
    s16x4 w[3];
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int u = 4 * g + i;
            w[d][i] = (short)(u < 9 ? f2bf(W[m * 27 + 9 * d + u]) : (uint16_t)0);
        }
    // LDS offsets of this lane's 4 taps (padding reads tap 0; its weight is 0)
    int toffs[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int u = 4 * g + i;
        toffs[i] = u < 9 ? (u / 3) * SX + (u % 3) + m : m;
    }
    float bv[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) bv[i] = b[4 * g + i];

    uint16_t stg[NPT];
    auto load_plane = [&](int zp) {
        const int zz = zp < 0 ? zp + n : (zp >= n ? zp - n : zp);
#pragma unroll
        for (int i = 0; i < NPT; ++i) {
            const int c = threadIdx.x + kNT * i;
            if (c < NCH) {
                const int xx = c % SX, yy = c / SX;
                stg[i] = x[((int64_t)zz * n + wrapi(y0 - 1 + yy, n)) * n + wrapi(x0 - 1 + xx, n)];
            }
        }
    };
    auto store_plane = [&](int bb) {
#pragma unroll
        for (int i = 0; i < NPT; ++i) {
            const int c = threadIdx.x + kNT * i;
            if (c < NCH) lds[bb * NCH + c] = stg[i];
        }
    };

    f32x4 acc[3][PW];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int j = 0; j < PW; ++j) acc[a][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    load_plane(zb - 1);
    store_plane(0);
    __syncthreads();
    int buf = 0;
    for (int zp = zb - 1; zp <= ze; ++zp) {
        if (zp < ze) load_plane(zp + 1);
        const uint16_t* L = lds + buf * NCH;
#pragma unroll
        for (int j = 0; j < PW; ++j) {
            const int T = wave + 4 * j;
            const int toff = (T >> 2) * SX + 16 * (T & 3);
            s16x4 bb;
#pragma unroll
            for (int i = 0; i < 4; ++i) bb[i] = (short)L[toffs[i] + toff];
            acc[2][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(w[0], bb, acc[2][j], 0, 0, 0);
            acc[1][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(w[1], bb, acc[1][j], 0, 0, 0);
            acc[0][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(w[2], bb, acc[0][j], 0, 0, 0);
        }
        if (zp - 1 >= zb) {
            const int z = zp - 1;
#pragma unroll
            for (int j = 0; j < PW; ++j) {
                const int T = wave + 4 * j;
                const int64_t p = ((int64_t)z * n + y0 + (T >> 2)) * n + x0 + 16 * (T & 3) + m;
                float v[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    v[i] = acc[0][j][i] + bv[i];
                    v[i] = v[i] > 0.f ? v[i] : 0.f;
                }
                uint2 o;
                o.x = (uint32_t)f2bf(v[0]) | ((uint32_t)f2bf(v[1]) << 16);
                o.y = (uint32_t)f2bf(v[2]) | ((uint32_t)f2bf(v[3]) << 16);
                *reinterpret_cast<uint2*>(y + p * 16 + 4 * g) = o;
            }
        }
#pragma unroll
        for (int j = 0; j < PW; ++j) {
            acc[0][j] = acc[1][j];
            acc[1][j] = acc[2][j];
            acc[2][j] = f32x4{0.f, 0.f, 0.f, 0.f};
        }
        if (zp < ze) store_plane(buf ^ 1);
        __syncthreads();
        buf ^= 1;
    }
}

// out: o[p] = b + sum_t sum_ci W[0][ci][t] a[p + d_t][ci]   (FP32 output)
__global__ __launch_bounds__(kNT) void conv_out_fwd_kernel(int n, const uint16_t* __restrict__ a,
                                                           const float* __restrict__ W,
                                                           const float* __restrict__ bptr,
                                                           float* __restrict__ o) {
    __shared__ float ws[16 * 27];
    for (int i = threadIdx.x; i < 16 * 27; i += kNT) ws[i] = wbf(W[i]);  // [ci][t]
    __syncthreads();
    const int64_t n3 = (int64_t)n * n * n;
    for (int64_t p = (int64_t)blockIdx.x * kNT + threadIdx.x; p < n3; p += (int64_t)gridDim.x * kNT) {
        const Pt pt = decomp(p, n);
        float s = 0.f;
        for (int t = 0; t < 27; ++t) {
            const uint16_t* src = a + nbr(pt, t, n) * 16;
            const uint4 v0 = *reinterpret_cast<const uint4*>(src);
            const uint4 v1 = *reinterpret_cast<const uint4*>(src + 8);
            const uint16_t* h0 = reinterpret_cast<const uint16_t*>(&v0);
            const uint16_t* h1 = reinterpret_cast<const uint16_t*>(&v1);
#pragma unroll
            for (int c = 0; c < 8; ++c) s += ws[c * 27 + t] * bf2f(h0[c]);
#pragma unroll
            for (int c = 0; c < 8; ++c) s += ws[(c + 8) * 27 + t] * bf2f(h1[c]);
        }
        o[p] = s + bptr[0];
    }
}

// out on the matrix cores, z-marching (n % 64 == 0): staging as in
// conv_zm_kernel<16, ...>; the MFMA's A operand is the staged activations
// (16 points x 32 of (in-plane tap, channel)), its B operand the weights with
// one column per output plane, so one MFMA chain per K-chunk serves all three
// output planes an input plane touches (a third of the work of a 16-output
// layer).  Column c accumulates the output planes z = c (mod 3): for input
// plane zp, column c holds tap plane dzi = (zp - c + 1) mod 3 of the weights.
// After input plane zp, output plane zp - 1 is complete in column
// (zp - 1) mod 3: its lanes add the bias, store 4 consecutive x (FP32) and
// clear that column for plane zp + 2.
template <int TY>
__global__ __launch_bounds__(kNT) void conv_out_zm_kernel(int n, int zlen,
                                                          const uint16_t* __restrict__ X,
                                                          const float* __restrict__ W,
                                                          const float* __restrict__ bptr,
                                                          float* __restrict__ o) {
    constexpr int CI = 16;
    constexpr int TX = 64, SX = TX + 2, SY = TY + 2;
    constexpr int CG = CI / 8;
    constexpr int KSP = (9 * CI + 31) / 32;
    constexpr int NTILE = 4 * TY;
    constexpr int PW = NTILE / 4;
    constexpr int NCH = SY * SX * CG;
    constexpr int NPT = (NCH + kNT - 1) / kNT;
    __shared__ bf16x8 lds[2 * NCH];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int m = lane & 15, g = lane >> 4;
    const int ntx = n / TX;
    const int ncol = ntx * (n / TY);
    const int bid = (int)remap_xcd(blockIdx.x, gridDim.x);
    const int col = bid % ncol;
    const int zb = (bid / ncol) * zlen, ze = zb + zlen;
    const int x0 = (col % ntx) * TX, y0 = (col / ntx) * TY;

    // B fragments: wf[ph][s], lane (m, g): B[k = 32 s + 8 g + i][column m]
    bf16x8 wf[3][KSP];
#pragma unroll
    for (int ph = 0; ph < 3; ++ph)
#pragma unroll
        for (int s2 = 0; s2 < KSP; ++s2) {
            uint16_t* wh = reinterpret_cast<uint16_t*>(&wf[ph][s2]);
            const int dzi = (ph - m + 1 + 3 * 16) % 3;
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int k = 32 * s2 + 8 * g + i;
                const int u = k / CI, c = k - u * CI;
                wh[i] = (m < 3 && u < 9) ? f2bf(W[c * 27 + 9 * dzi + u]) : (uint16_t)0;
            }
        }
    int boff[KSP];
#pragma unroll
    for (int s2 = 0; s2 < KSP; ++s2) {
        const int k0 = 32 * s2 + 8 * g;
        const int u = k0 / CI, c0 = k0 - u * CI;
        boff[s2] = u < 9 ? ((c0 / 8) * SY + u / 3) * SX + (u % 3) + m : m;  // padding: weight 0
    }
    const float bias = bptr[0];

    bf16x8 stg[NPT];
    auto load_plane = [&](int zp) {
        const int zz = zp < 0 ? zp + n : (zp >= n ? zp - n : zp);
#pragma unroll
        for (int i = 0; i < NPT; ++i) {
            const int c = threadIdx.x + kNT * i;
            if (c < NCH) {
                const int cg = c % CG, pt = c / CG;
                const int xx = pt % SX, yy = pt / SX;
                const int x = wrapi(x0 - 1 + xx, n), y = wrapi(y0 - 1 + yy, n);
                stg[i] = *reinterpret_cast<const bf16x8*>(
                    X + (((int64_t)zz * n + y) * n + x) * CI + cg * 8);
            }
        }
    };
    auto store_plane = [&](int b) {
#pragma unroll
        for (int i = 0; i < NPT; ++i) {
            const int c = threadIdx.x + kNT * i;
            if (c < NCH) {
                const int cg = c % CG, pt = c / CG;
                const int xx = pt % SX, yy = pt / SX;
                lds[b * NCH + (cg * SY + yy) * SX + xx] = stg[i];
            }
        }
    };

    f32x4 acc[PW];
#pragma unroll
    for (int j = 0; j < PW; ++j) acc[j] = f32x4{0.f, 0.f, 0.f, 0.f};
    load_plane(zb - 1);
    store_plane(0);
    __syncthreads();
    int buf = 0;
    for (int zp = zb - 1; zp <= ze; ++zp) {
        if (zp < ze) load_plane(zp + 1);
        const int ph = (zp + 3) % 3;
        const bf16x8* L = lds + buf * NCH;
        auto plane = [&](auto phase) {
            constexpr int PH = decltype(phase)::value;
#pragma unroll
            for (int j = 0; j < PW; ++j) {
                const int T = wave + 4 * j;
                const int toff = (T >> 2) * SX + 16 * (T & 3);
#pragma unroll
                for (int s2 = 0; s2 < KSP; ++s2) {
                    const bf16x8 av = L[boff[s2] + toff];
                    acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, wf[PH][s2], acc[j], 0, 0, 0);
                }
            }
        };
        if (ph == 0) plane(std::integral_constant<int, 0>{});
        else if (ph == 1) plane(std::integral_constant<int, 1>{});
        else plane(std::integral_constant<int, 2>{});
        const int co = (zp + 2) % 3;  // column of output plane zp - 1
        if (m == co) {
            const int z = zp - 1;
#pragma unroll
            for (int j = 0; j < PW; ++j) {
                if (z >= zb) {
                    const int T = wave + 4 * j;
                    const int64_t p = ((int64_t)z * n + y0 + (T >> 2)) * n + x0 + 16 * (T & 3) + 4 * g;
                    *reinterpret_cast<float4*>(o + p) =
                        make_float4(acc[j][0] + bias, acc[j][1] + bias, acc[j][2] + bias, acc[j][3] + bias);
                }
                acc[j] = f32x4{0.f, 0.f, 0.f, 0.f};
            }
        }
        if (zp < ze) store_plane(buf ^ 1);
        __syncthreads();
        buf ^= 1;
    }
}

// out layer, backward data: da[p][ci] (+)= sum_t W[0][ci][t] g[p - d_t]
// (g = BF16-rounded output gradient, one channel).
__global__ __launch_bounds__(kNT) void conv_out_bwd_kernel(int n, const uint16_t* __restrict__ g,
                                                           const float* __restrict__ W,
                                                           float* __restrict__ da, int accumulate) {
    __shared__ float ws[16 * 27];
    for (int i = threadIdx.x; i < 16 * 27; i += kNT) ws[i] = wbf(W[i]);
    __syncthreads();
    const int64_t n3 = (int64_t)n * n * n;
    for (int64_t p = (int64_t)blockIdx.x * kNT + threadIdx.x; p < n3; p += (int64_t)gridDim.x * kNT) {
        const Pt pt = decomp(p, n);
        float s[16];
#pragma unroll
        for (int c = 0; c < 16; ++c) s[c] = 0.f;
        for (int t = 0; t < 27; ++t) {
            const float gv = bf2f(g[nbr(pt, 26 - t, n)]);  // g[p - d_t]
#pragma unroll
            for (int c = 0; c < 16; ++c) s[c] += ws[c * 27 + t] * gv;
        }
        float4* dst = reinterpret_cast<float4*>(da + p * 16);
#pragma unroll
        for (int c = 0; c < 16; c += 4) {
            float4 v = make_float4(s[c], s[c + 1], s[c + 2], s[c + 3]);
            if (accumulate) {
                const float4 q = dst[c / 4];
                v.x += q.x;
                v.y += q.y;
                v.z += q.z;
                v.w += q.w;
            }
            dst[c / 4] = v;
        }
    }
}

// Weight gradient of a one-channel-side layer, per-block partials:
//   in layer  (CIN = 1, COUT = 16): dW[co][0][t] = sum_p x[p + d_t] G[p][co]
//   out layer (CIN = 16, COUT = 1): dW[0][ci][t] = sum_p A[p + d_t][ci] g[p]
// Per 32-point chunk the gathered operands are staged in LDS; thread i owns
// output i of the layer's canonical [co][ci][27] list (bias last) and sums
// over the chunk's points in order.
constexpr int kSmallNT = 512;
template <int CIN, int COUT>
__global__ __launch_bounds__(kSmallNT) void dw_small_kernel(int n, const uint16_t* __restrict__ X,
                                                            const uint16_t* __restrict__ G,
                                                            float* __restrict__ part) {
    constexpr int LEN = 27 * CIN * COUT + COUT;
    constexpr int CH = 32;
    static_assert(LEN <= kSmallNT, "one output per thread");
    __shared__ float xs[27][CH][CIN];
    __shared__ float gs[CH][COUT];
    const int tid = threadIdx.x;
    float acc = 0.f;
    const int64_t n3 = (int64_t)n * n * n;
    const int64_t nchunk = n3 / CH;
    for (int64_t ck = blockIdx.x; ck < nchunk; ck += gridDim.x) {
        const int64_t pb = ck * CH;
        __syncthreads();
        for (int e = tid; e < CH * COUT; e += kSmallNT) {
            const int pt = e / COUT, c = e % COUT;
            gs[pt][c] = bf2f(G[(pb + pt) * COUT + c]);
        }
        for (int e = tid; e < 27 * CH * CIN; e += kSmallNT) {
            const int t = e / (CH * CIN), r = e % (CH * CIN);
            const int pt = r / CIN, c = r % CIN;
            const Pt pp = decomp(pb + pt, n);
            xs[t][pt][c] = bf2f(X[nbr(pp, t, n) * CIN + c]);
        }
        __syncthreads();
        if (tid < 27 * CIN * COUT) {
            const int t = tid % 27, ci = (tid / 27) % CIN, co = tid / (27 * CIN);
            for (int pt = 0; pt < CH; ++pt) acc += xs[t][pt][ci] * gs[pt][co];
        } else if (tid < LEN) {
            const int co = tid - 27 * CIN * COUT;
            for (int pt = 0; pt < CH; ++pt) acc += gs[pt][co];
        }
    }
    if (tid < LEN) part[(int64_t)blockIdx.x * LEN + tid] = acc;
}

// ------------------------------------------------ pooling / up-sampling ----
// pool: y[P][c] = bf16((1/8) sum_{d in {0,1}^3} x[2P + d][c]);  m = coarse size
__global__ void pool_fwd_kernel(int m, int C, const uint16_t* __restrict__ x,
                                uint16_t* __restrict__ y) {
    const int n = 2 * m;
    const int64_t total = (int64_t)m * m * m * C;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(e % C);
        const Pt P = decomp(e / C, m);
        float s = 0.f;
#pragma unroll
        for (int d = 0; d < 8; ++d) {
            const int64_t q = ((int64_t)(2 * P.z + (d >> 2)) * n + (2 * P.y + ((d >> 1) & 1))) * n +
                              (2 * P.x + (d & 1));
            s += bf2f(x[q * C + c]);
        }
        y[e] = f2bf(s * 0.125f);
    }
}

// pool backward: gx[2P + d][c] (+)= gy[P][c] / 8      (n = fine size)
__global__ void pool_bwd_kernel(int n, int C, const float* __restrict__ gy, float* __restrict__ gx,
                                int accumulate) {
    const int m = n / 2;
    const int64_t total = (int64_t)n * n * n * C;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(e % C);
        const Pt p = decomp(e / C, n);
        const int64_t P = ((int64_t)(p.z / 2) * m + p.y / 2) * m + p.x / 2;
        const float v = gy[P * C + c] * 0.125f;
        gx[e] = accumulate ? gx[e] + v : v;
    }
}

// up: y[p][c] = x[p/2][c]   (n = fine size)
__global__ void up_fwd_kernel(int n, int C, const uint16_t* __restrict__ x, uint16_t* __restrict__ y) {
    const int m = n / 2;
    const int64_t total = (int64_t)n * n * n * C;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(e % C);
        const Pt p = decomp(e / C, n);
        const int64_t P = ((int64_t)(p.z / 2) * m + p.y / 2) * m + p.x / 2;
        y[e] = x[P * C + c];
    }
}

// up backward: gx[P][c] = sum_d gy[2P + d][c]   (m = coarse size)
__global__ void up_bwd_kernel(int m, int C, const float* __restrict__ gy, float* __restrict__ gx) {
    const int n = 2 * m;
    const int64_t total = (int64_t)m * m * m * C;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(e % C);
        const Pt P = decomp(e / C, m);
        float s = 0.f;
#pragma unroll
        for (int d = 0; d < 8; ++d) {
            const int64_t q = ((int64_t)(2 * P.z + (d >> 2)) * n + (2 * P.y + ((d >> 1) & 1))) * n +
                              (2 * P.x + (d & 1));
            s += gy[q * C + c];
        }
        gx[e] = s;
    }
}

// g_bf16 = bf16(g * (act > 0))  (act == nullptr: no mask)
__global__ void grad_round_kernel(int64_t count, const float* __restrict__ g,
                                  const uint16_t* __restrict__ act, uint16_t* __restrict__ out) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
         e += (int64_t)gridDim.x * blockDim.x) {
        float v = g[e];
        if (act && !(bf2f(act[e]) > 0.f)) v = 0.f;
        out[e] = f2bf(v);
    }
}

// ------------------------------------------------------------- the loss ----
// L = ||o - t||^2 / nt + lam ||A1 o - r||^2 / nr, A1 the unit-spacing periodic
// 7-point operator.  Pass 1: d2 = A1 o - r, partial sums of (o - t)^2 and d2^2.
// Pass 2: dL/do = 2 (o - t)/nt + 2 lam A1 d2 / nr.
__device__ __forceinline__ float a1_at(const float* u, const Pt& p, int n) {
    const int64_t c = ((int64_t)p.z * n + p.y) * n + p.x;
    const float xm = u[((int64_t)p.z * n + p.y) * n + wrapi(p.x - 1, n)];
    const float xp = u[((int64_t)p.z * n + p.y) * n + wrapi(p.x + 1, n)];
    const float ym = u[((int64_t)p.z * n + wrapi(p.y - 1, n)) * n + p.x];
    const float yp = u[((int64_t)p.z * n + wrapi(p.y + 1, n)) * n + p.x];
    const float zm = u[((int64_t)wrapi(p.z - 1, n) * n + p.y) * n + p.x];
    const float zp = u[((int64_t)wrapi(p.z + 1, n) * n + p.y) * n + p.x];
    return 6.f * u[c] - (((xm + xp) + (ym + yp)) + (zm + zp));
}

__global__ __launch_bounds__(kNT) void loss_pass1_kernel(int n, const float* __restrict__ o,
                                                         const float* __restrict__ t,
                                                         const float* __restrict__ r,
                                                         float* __restrict__ d2,
                                                         double* __restrict__ part) {
    __shared__ double red[2 * (kNT / kWave)];
    double acc[2] = {0.0, 0.0};
    const int64_t n3 = (int64_t)n * n * n;
    for (int64_t p = (int64_t)blockIdx.x * kNT + threadIdx.x; p < n3; p += (int64_t)gridDim.x * kNT) {
        const Pt pt = decomp(p, n);
        const float d = a1_at(o, pt, n) - r[p];
        d2[p] = d;
        const float e = o[p] - t[p];
        acc[0] += (double)e * e;
        acc[1] += (double)d * d;
    }
    block_sum<kNT, 2>(acc, red);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = acc[0];
        part[2 * blockIdx.x + 1] = acc[1];
    }
}

// Norms of the target and of the right-hand side (partial sums).
__global__ __launch_bounds__(kNT) void loss_norms_kernel(int64_t n3, const float* __restrict__ t,
                                                         const float* __restrict__ r,
                                                         double* __restrict__ part) {
    __shared__ double red[2 * (kNT / kWave)];
    double acc[2] = {0.0, 0.0};
    for (int64_t p = (int64_t)blockIdx.x * kNT + threadIdx.x; p < n3; p += (int64_t)gridDim.x * kNT) {
        acc[0] += (double)t[p] * t[p];
        acc[1] += (double)r[p] * r[p];
    }
    block_sum<kNT, 2>(acc, red);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = acc[0];
        part[2 * blockIdx.x + 1] = acc[1];
    }
}

// coef[0] = 2/||t||^2, coef[1] = 2 lam/||r||^2 (one block, fixed order).
__global__ __launch_bounds__(kNT) void loss_coef_kernel(const double* __restrict__ part, int nparts,
                                                        double lam, double* __restrict__ coef) {
    __shared__ double red[2 * (kNT / kWave)];
    double acc[2] = {0.0, 0.0};
    for (int i = threadIdx.x; i < nparts; i += kNT) {
        acc[0] += part[2 * i];
        acc[1] += part[2 * i + 1];
    }
    block_sum<kNT, 2>(acc, red);
    if (threadIdx.x == 0) {
        coef[0] = 2.0 / acc[0];
        coef[1] = 2.0 * lam / acc[1];
        coef[2] = acc[0];
        coef[3] = acc[1];
    }
}

__global__ __launch_bounds__(kNT) void loss_pass2_kernel(int n, const float* __restrict__ o,
                                                         const float* __restrict__ t,
                                                         const float* __restrict__ d2,
                                                         const double* __restrict__ coef,
                                                         uint16_t* __restrict__ gout) {
    const float c1 = (float)coef[0], c2 = (float)coef[1];
    const int64_t n3 = (int64_t)n * n * n;
    for (int64_t p = (int64_t)blockIdx.x * kNT + threadIdx.x; p < n3; p += (int64_t)gridDim.x * kNT) {
        const Pt pt = decomp(p, n);
        const float g = c1 * (o[p] - t[p]) + c2 * a1_at(d2, pt, n);
        gout[p] = f2bf(g);  // the output layer's gradient, rounded like every conv output's
    }
}

__global__ void add_bf16_kernel(int64_t count, const uint16_t* __restrict__ a, float* __restrict__ g) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
         e += (int64_t)gridDim.x * blockDim.x)
        g[e] += bf2f(a[e]);
}

__global__ void to_bf16_kernel(int64_t count, const float* __restrict__ a, uint16_t* __restrict__ o) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
         e += (int64_t)gridDim.x * blockDim.x)
        o[e] = f2bf(a[e]);
}

// --------------------------------------------------------------- Adam -----
__global__ void adam_kernel(int64_t len, float* __restrict__ th, float* __restrict__ mm,
                            float* __restrict__ vv, const float* __restrict__ g, float lr, float b1,
                            float b2, float eps, float bc1, float bc2) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len;
         i += (int64_t)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float m = b1 * mm[i] + (1.f - b1) * gi;
        const float v = b2 * vv[i] + (1.f - b2) * gi * gi;
        mm[i] = m;
        vv[i] = v;
        th[i] = th[i] - lr * (m / bc1) / (sqrtf(v / bc2) + eps);
    }
}

// --------------------------------------- preconditioner input / output ----
// sum of (h^2 r)^2 -> partials (double)
__global__ __launch_bounds__(kNT) void sumsq_kernel(int64_t n3, const double* __restrict__ r,
                                                    double h2, double* __restrict__ part) {
    __shared__ double red[kNT / kWave];
    double acc[1] = {0.0};
    for (int64_t p = (int64_t)blockIdx.x * kNT + threadIdx.x; p < n3; p += (int64_t)gridDim.x * kNT) {
        const double v = h2 * r[p];
        acc[0] += v * v;
    }
    block_sum<kNT, 1>(acc, red);
    if (threadIdx.x == 0) part[blockIdx.x] = acc[0];
}

// x = bf16(h^2 r / s), s from the fixed-order sum of the partials.
__global__ __launch_bounds__(kNT) void prep_kernel(int64_t n3, const double* __restrict__ r,
                                                   double h2, const double* __restrict__ part,
                                                   int nparts, double* __restrict__ s_out,
                                                   uint16_t* __restrict__ x) {
    __shared__ double red[kNT / kWave];
    __shared__ double s_sh;
    double t[1];
    sum_partials<kNT, 1>(part, nparts, t, red);
    if (threadIdx.x == 0) {
        s_sh = sqrt(t[0] / (double)n3);
        if (blockIdx.x == 0) *s_out = s_sh;
    }
    __syncthreads();
    const double s = s_sh;
    const double inv = s > 0.0 ? 1.0 / s : 0.0;
    for (int64_t p = (int64_t)blockIdx.x * kNT + threadIdx.x; p < n3; p += (int64_t)gridDim.x * kNT)
        x[p] = f2bf((float)(h2 * r[p] * inv));
}

// Training pairs in the scale-free form: u = h^2 (b - b_prev), e = phi - phi_prev
// (b_prev, phi_prev NULL: no difference); partial sums of u^2.
__global__ __launch_bounds__(kNT) void pair_sumsq_kernel(int64_t n3, const double* __restrict__ b,
                                                         const double* __restrict__ bp, double h2,
                                                         double* __restrict__ part) {
    __shared__ double red[kNT / kWave];
    double acc[1] = {0.0};
    for (int64_t p = (int64_t)blockIdx.x * kNT + threadIdx.x; p < n3; p += (int64_t)gridDim.x * kNT) {
        const double v = h2 * (bp ? b[p] - bp[p] : b[p]);
        acc[0] += v * v;
    }
    block_sum<kNT, 1>(acc, red);
    if (threadIdx.x == 0) part[blockIdx.x] = acc[0];
}

// rhs = (float)(u / s), tgt = (float)(e / s), s = rms(u) from the partials.
__global__ __launch_bounds__(kNT) void pair_kernel(int64_t n3, const double* __restrict__ b,
                                                   const double* __restrict__ bp,
                                                   const double* __restrict__ phi,
                                                   const double* __restrict__ pp, double h2,
                                                   const double* __restrict__ part, int nparts,
                                                   double* __restrict__ s_out,
                                                   float* __restrict__ rhs,
                                                   float* __restrict__ tgt) {
    __shared__ double red[kNT / kWave];
    __shared__ double s_sh;
    double t[1];
    sum_partials<kNT, 1>(part, nparts, t, red);
    if (threadIdx.x == 0) {
        s_sh = sqrt(t[0] / (double)n3);
        if (blockIdx.x == 0) *s_out = s_sh;
    }
    __syncthreads();
    const double s = s_sh;
    const double inv = s > 0.0 ? 1.0 / s : 0.0;
    for (int64_t p = (int64_t)blockIdx.x * kNT + threadIdx.x; p < n3; p += (int64_t)gridDim.x * kNT) {
        const double u = h2 * (bp ? b[p] - bp[p] : b[p]);
        const double e = pp ? phi[p] - pp[p] : phi[p];
        rhs[p] = (float)(u * inv);
        tgt[p] = (float)(e * inv);
    }
}

// z = s * o (FP64), partial sums of z for the mean.
__global__ __launch_bounds__(kNT) void post_kernel(int64_t n3, const float* __restrict__ o,
                                                   const double* __restrict__ s_in,
                                                   double* __restrict__ z, double* __restrict__ part) {
    __shared__ double red[kNT / kWave];
    const double s = *s_in;
    double acc[1] = {0.0};
    for (int64_t p = (int64_t)blockIdx.x * kNT + threadIdx.x; p < n3; p += (int64_t)gridDim.x * kNT) {
        const double v = s * (double)o[p];
        z[p] = v;
        acc[0] += v;
    }
    block_sum<kNT, 1>(acc, red);
    if (threadIdx.x == 0) part[blockIdx.x] = acc[0];
}

__global__ __launch_bounds__(kNT) void center_kernel(int64_t n3, double* __restrict__ z,
                                                     const double* __restrict__ part, int nparts) {
    __shared__ double red[kNT / kWave];
    __shared__ double m_sh;
    double t[1];
    sum_partials<kNT, 1>(part, nparts, t, red);
    if (threadIdx.x == 0) m_sh = t[0] / (double)n3;
    __syncthreads();
    const double mean = m_sh;
    for (int64_t p = (int64_t)blockIdx.x * kNT + threadIdx.x; p < n3; p += (int64_t)gridDim.x * kNT)
        z[p] = z[p] - mean;
}

// ================================================================ launchers ==

static int blocks_for(int64_t work, int per = kNT, int cap = 4096) {
    int64_t b = (work + per - 1) / per;
    if (b < 1) b = 1;
    return (int)(b < cap ? b : cap);
}

// A fragment buffer holds the gather kernel's fragments, followed (for
// 16 or 32 gathered channels) by the z-marching kernel's plane-major ones.
static size_t gather_frag_elems(int cin, int cout) {
    return (size_t)((27 * cin + 31) / 32) * (cout / 16) * 512;
}
static bool zm_channels(int cin) { return cin == 16 || cin == 32; }
static size_t zm_frag_elems(int cin, int cout) {
    return zm_channels(cin) ? (size_t)3 * ((9 * cin + 31) / 32) * (cout / 16) * 512 : 0;
}

hipError_t pack(const float* W, int ci, int co, int bwd, uint16_t* frag, hipStream_t s) {
    const int cin = bwd ? co : ci, cout = bwd ? ci : co;
    const int64_t nfrag = (int64_t)gather_frag_elems(cin, cout);
    hipLaunchKernelGGL(pack_kernel, dim3(blocks_for(nfrag)), dim3(kNT), 0, s, W, ci, co, bwd, frag);
    const int64_t nz = (int64_t)zm_frag_elems(cin, cout);
    if (nz > 0)
        hipLaunchKernelGGL(pack_zm_kernel, dim3(blocks_for(nz)), dim3(kNT), 0, s, W, ci, co, bwd,
                           frag + nfrag);
    return hipGetLastError();
}

size_t frag_elems(int cin, int cout) { return gather_frag_elems(cin, cout) + zm_frag_elems(cin, cout); }

// z-split of the z-marching kernel: the largest divisor of n that keeps at
// least 8 planes per block and gives at most 4096 blocks.
static int zm_zsplit(int n, int ncol) {
    int best = 1;
    for (int zs = 1; zs <= n / 8; ++zs)
        if (n % zs == 0 && (int64_t)ncol * zs <= 4096) best = zs;
    return best;
}

template <int CI, int CO, int TY, int MODE, bool UP = false, bool SK = false, bool PL = false>
static hipError_t zm_launch_t(int n, const uint16_t* X, const uint16_t* frag, const float* bias,
                              const uint16_t* skip, int relu, uint16_t* Yb, float* Yf, int acc,
                              hipStream_t s, uint16_t* Yp = nullptr) {
    const int ncol = (n / 64) * (n / TY);
    const int zs = zm_zsplit(n, ncol);
    const uint16_t* fz = frag + gather_frag_elems(CI, CO);
    hipLaunchKernelGGL((conv_zm_kernel<CI, CO, TY, MODE, UP, SK, PL>), dim3(ncol * zs), dim3(kNT), 0,
                       s, n, n / zs, X, fz, bias, skip, relu, Yb, Yf, acc, Yp);
    return hipGetLastError();
}

// Only the 32-channel encoder layer: at 16 channels the pooled epilogue
// needs 4-row tiles (registers), and at 512^3 the 8-row tile plus a separate
// pool pass measured faster (3.1 ms against 4.0 ms).
bool conv_pool_fused(int n, int ci, int co) {
    if (n % 64 != 0 || (n / zm_zsplit(n, (n / 64) * (n / 4))) % 2 != 0) return false;
    return ci == 32 && co == 32;
}

hipError_t conv_fwd_pool(int n, int ci, int co, const uint16_t* X, const uint16_t* frag,
                         const float* bias, uint16_t* Y, uint16_t* Yp, hipStream_t s) {
    if (!conv_pool_fused(n, ci, co)) return hipErrorInvalidValue;
    return zm_launch_t<32, 32, 4, 0, false, false, true>(n, X, frag, bias, nullptr, 1, Y, nullptr, 0,
                                                         s, Yp);
}

// With a skip input the 16-channel variants use 4-row tiles (the skip values
// are held in registers across the MFMAs).
template <int CI, int CO, int TY, int MODE, bool UP = false>
static hipError_t zm_launch(int n, const uint16_t* X, const uint16_t* frag, const float* bias,
                            const uint16_t* skip, int relu, uint16_t* Yb, float* Yf, int acc,
                            hipStream_t s) {
    if constexpr (MODE == 0) {
        if (skip) {
            constexpr int TYS = (CI == 16 && TY > 4) ? 4 : TY;
            return zm_launch_t<CI, CO, TYS, MODE, UP, true>(n, X, frag, bias, skip, relu, Yb, Yf,
                                                            acc, s);
        }
    }
    return zm_launch_t<CI, CO, TY, MODE, UP, false>(n, X, frag, bias, nullptr, relu, Yb, Yf, acc, s);
}

bool conv_up_fused(int n, int ci, int co) {
    return n % 64 == 0 && ((ci == 16 && co == 16) || (ci == 32 && co == 32));
}

hipError_t conv_fwd_up(int n, int ci, int co, const uint16_t* Xc, const uint16_t* frag,
                       const float* bias, const uint16_t* skip, int relu, uint16_t* Y,
                       hipStream_t s) {
    if (!conv_up_fused(n, ci, co)) return hipErrorInvalidValue;
    if (ci == 16) return zm_launch<16, 16, 8, 0, true>(n, Xc, frag, bias, skip, relu, Y, nullptr, 0, s);
    return zm_launch<32, 32, 4, 0, true>(n, Xc, frag, bias, skip, relu, Y, nullptr, 0, s);
}

template <int CI, int CO, int NG, int MODE>
static hipError_t conv_launch(int n, const uint16_t* X, const uint16_t* frag, const float* bias,
                              const uint16_t* skip, int relu, uint16_t* Yb, float* Yf, int acc,
                              hipStream_t s) {
    const int64_t ntiles = (int64_t)n * n * n / 16;
    const int nb = blocks_for(ntiles, 16, 2048);  // 4 waves x 4 tiles per pass
    hipLaunchKernelGGL((conv_mfma_kernel<CI, CO, NG, MODE>), dim3(nb, CO / 16 / NG), dim3(kNT), 0, s,
                       n, X, frag, bias, skip, relu, Yb, Yf, acc);
    return hipGetLastError();
}

// NG (output blocks per launch) keeps the staged weights under 64 KB of LDS.
hipError_t conv_fwd(int n, int ci, int co, const uint16_t* X, const uint16_t* frag,
                    const float* bias, const uint16_t* skip, int relu, uint16_t* Y, hipStream_t s) {
    if (n % 64 == 0) {
#define ZF(A, B, T) \
    if (ci == A && co == B) return zm_launch<A, B, T, 0>(n, X, frag, bias, skip, relu, Y, nullptr, 0, s)
        ZF(16, 16, 8);
        ZF(16, 32, 4);
        ZF(32, 32, 4);
        ZF(32, 64, 2);
        ZF(32, 16, 4);
#undef ZF
    }
#define CF(A, B, G) \
    if (ci == A && co == B) return conv_launch<A, B, G, 0>(n, X, frag, bias, skip, relu, Y, nullptr, 0, s)
    CF(16, 16, 1);
    CF(16, 32, 2);
    CF(32, 32, 2);
    CF(32, 64, 2);
    CF(64, 32, 1);
    CF(32, 16, 1);
#undef CF
    return hipErrorInvalidValue;
}

hipError_t conv_bwd_data(int n, int ci, int co, const uint16_t* G, const uint16_t* frag_bwd,
                         float* dX, int accumulate, hipStream_t s) {
    // gathers the layer's output gradient (co channels), produces ci channels
    if (n % 64 == 0) {
#define ZB(A, B, T) \
    if (ci == A && co == B) return zm_launch<B, A, T, 1>(n, G, frag_bwd, nullptr, nullptr, 0, nullptr, dX, accumulate, s)
        ZB(16, 16, 8);
        ZB(32, 16, 4);
        ZB(16, 32, 4);
        ZB(64, 32, 2);
        ZB(32, 32, 4);
#undef ZB
    }
#define CB(A, B, G2) \
    if (ci == A && co == B) return conv_launch<B, A, G2, 1>(n, G, frag_bwd, nullptr, nullptr, 0, nullptr, dX, accumulate, s)
    CB(16, 16, 1);
    CB(16, 32, 1);
    CB(32, 32, 2);
    CB(32, 64, 1);
    CB(64, 32, 2);
    CB(32, 16, 2);
#undef CB
    return hipErrorInvalidValue;
}

int dw_parts_x(int n) {
    const int64_t nchunk = (int64_t)n * n * n / 32;
    return (int)(nchunk < 512 ? nchunk : 512);
}
int dw_groups(int ci, int co) { return (27 * (ci / 16) * (co / 16) + 63) / 64; }

template <int CI, int CO>
static hipError_t dw_launch(int n, const uint16_t* X, const uint16_t* G, float* part, float* grad,
                            hipStream_t s) {
    const int px = dw_parts_x(n), gy = dw_groups(CI, CO);
    const int64_t len = (int64_t)27 * CI * CO + CO;
    const int64_t rows = (int64_t)px * gy;
    hipLaunchKernelGGL(fill_f32_kernel, dim3(blocks_for(rows * len)), dim3(kNT), 0, s, rows * len,
                       part, 0.f);
    hipLaunchKernelGGL((dw_mfma_kernel<CI, CO>), dim3(px, gy), dim3(kNT), 0, s, n, X, G, part, px);
    hipLaunchKernelGGL(dw_reduce_kernel, dim3(blocks_for(len)), dim3(kNT), 0, s, (const float*)part,
                       rows, len, grad);
    return hipGetLastError();
}

hipError_t conv_dw(int n, int ci, int co, const uint16_t* X, const uint16_t* G, float* part,
                   float* grad, hipStream_t s) {
#define CW(A, B) \
    if (ci == A && co == B) return dw_launch<A, B>(n, X, G, part, grad, s)
    CW(16, 16);
    CW(16, 32);
    CW(32, 32);
    CW(32, 64);
    CW(64, 32);
    CW(32, 16);
#undef CW
    return hipErrorInvalidValue;
}

size_t dw_part_elems(int n, int ci, int co) {
    if (ci == 1 || co == 1) return (size_t)dw_parts_x(n) * (27 * ci * co + co);
    return (size_t)dw_parts_x(n) * dw_groups(ci, co) * ((size_t)27 * ci * co + co);
}

hipError_t conv_in_fwd(int n, const uint16_t* x, const float* W, const float* b, uint16_t* y,
                       hipStream_t s) {
    if (n % 64 == 0) {
        constexpr int TY = 8;
        const int ncol = (n / 64) * (n / TY);
        const int zs = zm_zsplit(n, ncol);
        hipLaunchKernelGGL(conv_in_zm_kernel<TY>, dim3(ncol * zs), dim3(kNT), 0, s, n, n / zs, x, W,
                           b, y);
        return hipGetLastError();
    }
    const int64_t ntiles = (int64_t)n * n * n / 16;
    hipLaunchKernelGGL(conv_in_fwd_kernel, dim3(blocks_for(ntiles, 16, 8192)), dim3(kNT), 0, s, n,
                       x, W, b, y);
    return hipGetLastError();
}

hipError_t conv_out_fwd(int n, const uint16_t* a, const float* W, const float* b, float* o,
                        hipStream_t s) {
    if (n % 64 == 0) {
        constexpr int TY = 8;
        const int ncol = (n / 64) * (n / TY);
        const int zs = zm_zsplit(n, ncol);
        hipLaunchKernelGGL(conv_out_zm_kernel<TY>, dim3(ncol * zs), dim3(kNT), 0, s, n, n / zs, a, W,
                           b, o);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(conv_out_fwd_kernel, dim3(blocks_for((int64_t)n * n * n)), dim3(kNT), 0, s, n,
                       a, W, b, o);
    return hipGetLastError();
}

hipError_t conv_out_bwd(int n, const uint16_t* g, const float* W, float* da, int accumulate,
                        hipStream_t s) {
    hipLaunchKernelGGL(conv_out_bwd_kernel, dim3(blocks_for((int64_t)n * n * n)), dim3(kNT), 0, s, n,
                       g, W, da, accumulate);
    return hipGetLastError();
}

hipError_t conv_dw_small(int n, int ci, int co, const uint16_t* X, const uint16_t* G, float* part,
                         float* grad, hipStream_t s) {
    const int nb = dw_parts_x(n);
    const int64_t len = 27 * ci * co + co;
    if (ci == 1 && co == 16)
        hipLaunchKernelGGL((dw_small_kernel<1, 16>), dim3(nb), dim3(kSmallNT), 0, s, n, X, G, part);
    else if (ci == 16 && co == 1)
        hipLaunchKernelGGL((dw_small_kernel<16, 1>), dim3(nb), dim3(kSmallNT), 0, s, n, X, G, part);
    else
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(dw_reduce_kernel, dim3(blocks_for(len)), dim3(kNT), 0, s, (const float*)part,
                       (int64_t)nb, len, grad);
    return hipGetLastError();
}

hipError_t pool_fwd(int m, int C, const uint16_t* x, uint16_t* y, hipStream_t s) {
    hipLaunchKernelGGL(pool_fwd_kernel, dim3(blocks_for((int64_t)m * m * m * C)), dim3(kNT), 0, s, m,
                       C, x, y);
    return hipGetLastError();
}
hipError_t pool_bwd(int n, int C, const float* gy, float* gx, int accumulate, hipStream_t s) {
    hipLaunchKernelGGL(pool_bwd_kernel, dim3(blocks_for((int64_t)n * n * n * C)), dim3(kNT), 0, s, n,
                       C, gy, gx, accumulate);
    return hipGetLastError();
}
hipError_t up_fwd(int n, int C, const uint16_t* x, uint16_t* y, hipStream_t s) {
    hipLaunchKernelGGL(up_fwd_kernel, dim3(blocks_for((int64_t)n * n * n * C)), dim3(kNT), 0, s, n, C,
                       x, y);
    return hipGetLastError();
}
hipError_t up_bwd(int m, int C, const float* gy, float* gx, hipStream_t s) {
    hipLaunchKernelGGL(up_bwd_kernel, dim3(blocks_for((int64_t)m * m * m * C)), dim3(kNT), 0, s, m, C,
                       gy, gx);
    return hipGetLastError();
}
hipError_t grad_round(int64_t count, const float* g, const uint16_t* act, uint16_t* out,
                      hipStream_t s) {
    hipLaunchKernelGGL(grad_round_kernel, dim3(blocks_for(count)), dim3(kNT), 0, s, count, g, act, out);
    return hipGetLastError();
}

int loss_parts(int n) { return blocks_for((int64_t)n * n * n, kNT, 1024); }
hipError_t loss_pass1(int n, const float* o, const float* t, const float* r, float* d2,
                      double* part, hipStream_t s) {
    hipLaunchKernelGGL(loss_pass1_kernel, dim3(loss_parts(n)), dim3(kNT), 0, s, n, o, t, r, d2, part);
    return hipGetLastError();
}
hipError_t loss_norms(int n, const float* t, const float* r, double* part, hipStream_t s) {
    const int64_t n3 = (int64_t)n * n * n;
    hipLaunchKernelGGL(loss_norms_kernel, dim3(loss_parts(n)), dim3(kNT), 0, s, n3, t, r, part);
    return hipGetLastError();
}
// norm_part: the partials of loss_norms; its tail (from 2 * loss_parts) holds
// the four coefficients written here.
hipError_t loss_pass2(int n, const float* o, const float* t, const float* d2,
                      const double* norm_part, double lam, uint16_t* gout, hipStream_t s) {
    double* coef = const_cast<double*>(norm_part) + 2 * loss_parts(n);
    hipLaunchKernelGGL(loss_coef_kernel, dim3(1), dim3(kNT), 0, s, norm_part, loss_parts(n), lam,
                       coef);
    hipLaunchKernelGGL(loss_pass2_kernel, dim3(blocks_for((int64_t)n * n * n)), dim3(kNT), 0, s, n, o,
                       t, d2, (const double*)coef, gout);
    return hipGetLastError();
}
hipError_t add_bf16(int64_t count, const uint16_t* a, float* g, hipStream_t s) {
    hipLaunchKernelGGL(add_bf16_kernel, dim3(blocks_for(count)), dim3(kNT), 0, s, count, a, g);
    return hipGetLastError();
}
hipError_t to_bf16(int64_t count, const float* a, uint16_t* o, hipStream_t s) {
    hipLaunchKernelGGL(to_bf16_kernel, dim3(blocks_for(count)), dim3(kNT), 0, s, count, a, o);
    return hipGetLastError();
}
hipError_t adam(int64_t len, float* th, float* m, float* v, const float* g, float lr, float b1,
                float b2, float eps, int step, hipStream_t s) {
    const float bc1 = 1.f - powf(b1, (float)step), bc2 = 1.f - powf(b2, (float)step);
    hipLaunchKernelGGL(adam_kernel, dim3(blocks_for(len)), dim3(kNT), 0, s, len, th, m, v, g, lr, b1,
                       b2, eps, bc1, bc2);
    return hipGetLastError();
}

int pre_parts(int64_t n3) { return blocks_for(n3, kNT, 1024); }
hipError_t prep_input(int64_t n3, const double* r, double h2, double* part, double* s_out,
                      uint16_t* x, hipStream_t s) {
    const int nb = pre_parts(n3);
    hipLaunchKernelGGL(sumsq_kernel, dim3(nb), dim3(kNT), 0, s, n3, r, h2, part);
    hipLaunchKernelGGL(prep_kernel, dim3(nb), dim3(kNT), 0, s, n3, r, h2, (const double*)part, nb,
                       s_out, x);
    return hipGetLastError();
}
hipError_t scale_pair(int64_t n3, const double* b, const double* bp, const double* phi,
                      const double* pp, double h2, double* part, double* s_out, float* rhs,
                      float* tgt, hipStream_t s) {
    const int nb = pre_parts(n3);
    hipLaunchKernelGGL(pair_sumsq_kernel, dim3(nb), dim3(kNT), 0, s, n3, b, bp, h2, part);
    hipLaunchKernelGGL(pair_kernel, dim3(nb), dim3(kNT), 0, s, n3, b, bp, phi, pp, h2,
                       (const double*)part, nb, s_out, rhs, tgt);
    return hipGetLastError();
}
hipError_t post_output(int64_t n3, const float* o, const double* s_in, double* z, double* part,
                       hipStream_t s) {
    const int nb = pre_parts(n3);
    hipLaunchKernelGGL(post_kernel, dim3(nb), dim3(kNT), 0, s, n3, o, s_in, z, part);
    hipLaunchKernelGGL(center_kernel, dim3(nb), dim3(kNT), 0, s, n3, z, (const double*)part, nb);
    return hipGetLastError();
}

}  // namespace net
}  // namespace pic
