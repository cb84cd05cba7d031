// sort.hip -- stable sort of particles by cell key, cell_start and the payload
// permutation.
//
// The cell sort keeps every cell's particles contiguous so the deposit can
// gather them per vertex and the push streams through the field in memory
// order.  Ties keep their input order (stable), which makes the result a pure
// function of the input sequence (the oracle's counting sort gives the same
// permutation).
//
// Algorithm: LSD radix sort on digits of up to 9 bits over (key, index)
// pairs, as few passes as the largest key needs (27-bit keys of a 512^3 grid:
// three 9-bit passes).  Each pass:
//   1. tile histograms (12288 keys per tile; each wave matches equal digits
//      with ballots and its group leaders add the group sizes to
//      wave-private LDS counters),
//   2. exclusive scan of the digit-major histogram table,
//   3. stable scatter: inside a tile, keys are ranked in input order -- within
//      a wave by matching equal digits with ballots and counting lower lanes,
//      across the tile's waves with per-wave digit counts -- and the tile is
//      placed in LDS in digit order, so consecutive threads write consecutive
//      slots of each digit's output run (about 24 slots per digit and tile).
// Then cell_start from the sorted keys and a gather of the particle records.
#include "common.hpp"
#include "particles.hpp"

namespace pic {

constexpr int kSortNT = 768;                   // threads of a scatter workgroup
constexpr int kIPT = 16;                       // items per thread per tile
constexpr int kTile = kSortNT * kIPT;          // 12288
constexpr int kMaxBits = 9;
constexpr int kMaxRadix = 1 << kMaxBits;
constexpr int kHistNT = 256;
constexpr int kScanNT = 256;
constexpr int kScanIPT = 16;
constexpr int kScanTile = kScanNT * kScanIPT;  // 4096

static int64_t ntiles(int64_t np) { return (np + kTile - 1) / kTile; }

size_t sort_scratch_bytes(int64_t np_max) {
    const int64_t cap = np_max > 0 ? np_max : 1;
    const int64_t t = ntiles(cap);
    const int64_t hist = t * kMaxRadix;
    const int64_t sums = (hist + kScanTile - 1) / kScanTile + 1;
    size_t b = 0;
    b += 4 * (size_t)cap * sizeof(uint32_t);
    b += (size_t)(hist + 64) * sizeof(uint32_t);
    b += (size_t)(sums + 1088) * sizeof(uint32_t);
    return b + 1024;
}

size_t sort_rec_bytes(int64_t np_max) {
    const int64_t cap = np_max > 0 ? np_max : 1;
    return 4 * (size_t)cap * sizeof(double2);
}

void sort_scratch_carve(void* base, int64_t np_max, SortScratch* s) {
    const int64_t cap = np_max > 0 ? np_max : 1;
    const int64_t t = ntiles(cap);
    const int64_t hist = t * kMaxRadix;
    char* p = (char*)base;
    auto take = [&](size_t bytes) {
        char* r = p;
        p += (bytes + 255) & ~(size_t)255;
        return r;
    };
    s->rec = nullptr;  // sort_rec_bytes, allocated on the first sort
    s->key[0] = (uint32_t*)take((size_t)cap * 4);
    s->key[1] = (uint32_t*)take((size_t)cap * 4);
    s->idx[0] = (uint32_t*)take((size_t)cap * 4);
    s->idx[1] = (uint32_t*)take((size_t)cap * 4);
    s->hist = (uint32_t*)take((size_t)(hist + 64) * 4);
    s->sums = (uint32_t*)take((size_t)((hist + kScanTile - 1) / kScanTile + 1089) * 4);
    s->cap = cap;
}

// Lanes of the wave whose digit equals this lane's (valid lanes only).
__device__ __forceinline__ uint64_t match_digit(uint32_t d, int bits, bool valid) {
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int bit = 0; bit < kMaxBits; ++bit) {
        if (bit < bits) {
            const uint64_t bl = __ballot((d >> bit) & 1u);
            peers &= ((d >> bit) & 1u) ? bl : ~bl;
        }
    }
    return valid ? peers : 0ull;
}

// ---------------------------------------------------------------- pass 1 --
__global__ __launch_bounds__(kHistNT) void hist_kernel(int64_t np, const uint32_t* __restrict__ key,
                                                        int shift, int bits,
                                                        uint32_t* __restrict__ hist, int64_t tiles) {
    constexpr int NW = kHistNT / kWave;
    __shared__ uint32_t cnt[NW][kMaxRadix];
    const int tid = threadIdx.x, lane = tid & (kWave - 1), w = tid / kWave;
    const uint32_t radix = 1u << bits, mask = radix - 1;
    for (int d = tid; d < NW * kMaxRadix; d += kHistNT) (&cnt[0][0])[d] = 0;
    __syncthreads();
    // consecutive tiles on one XCD (their entries of each digit's row of the
    // table are adjacent and merge in that XCD's L2)
    const int64_t t = remap_xcd_any(blockIdx.x, (uint32_t)tiles);
    const int64_t base = t * kTile;
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (kWave - lane));
    // each wave counts its own contiguous quarter of the tile, loading
    // kHB rounds of keys before matching them (loads in flight together)
    constexpr int kHB = 16;
    for (int k0 = 0; k0 < kTile / kHistNT; k0 += kHB) {
        uint32_t kk[kHB];
#pragma unroll
        for (int k = 0; k < kHB; ++k) {
            const int64_t i = base + (int64_t)w * (kTile / NW) + (int64_t)(k0 + k) * kWave + lane;
            kk[k] = i < np ? key[i] : 0u;
        }
#pragma unroll
        for (int k = 0; k < kHB; ++k) {
            const int64_t i = base + (int64_t)w * (kTile / NW) + (int64_t)(k0 + k) * kWave + lane;
            const bool valid = i < np;
            const uint32_t d = (kk[k] >> shift) & mask;
            const uint64_t peers = match_digit(d, bits, valid);
            if (valid && (peers & lt) == 0) cnt[w][d] += (uint32_t)__popcll(peers);
            __builtin_amdgcn_wave_barrier();
        }
    }
    __syncthreads();
    for (uint32_t d = tid; d < radix; d += kHistNT) {
        uint32_t c = 0;
#pragma unroll
        for (int j = 0; j < NW; ++j) c += cnt[j][d];
        hist[(int64_t)d * tiles + t] = c;
    }
}

// ---------------------------------------------------------- exclusive scan --
// Block-local exclusive scan of kScanTile uint32 values; writes the block sum.
__global__ __launch_bounds__(kScanNT) void scan_tiles_kernel(uint32_t* __restrict__ a, int64_t m,
                                                              uint32_t* __restrict__ sums) {
    __shared__ uint32_t ws[kScanNT / kWave];
    const int tid = threadIdx.x, lane = tid & (kWave - 1), w = tid / kWave;
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)tid * kScanIPT;
    uint32_t v[kScanIPT];
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanIPT; ++k) {
        const int64_t i = base + k;
        v[k] = i < m ? a[i] : 0u;
        s += v[k];
    }
    // inclusive wave scan of per-thread sums
    uint32_t inc = s;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const uint32_t o = __shfl_up(inc, off, kWave);
        if (lane >= off) inc += o;
    }
    if (lane == kWave - 1) ws[w] = inc;
    __syncthreads();
    uint32_t wofs = 0;
    for (int j = 0; j < w; ++j) wofs += ws[j];
    uint32_t run = wofs + inc - s;
#pragma unroll
    for (int k = 0; k < kScanIPT; ++k) {
        const int64_t i = base + k;
        const uint32_t x = v[k];
        if (i < m) a[i] = run;
        run += x;
    }
    if (tid == kScanNT - 1) sums[blockIdx.x] = run;
}

__global__ __launch_bounds__(kScanNT) void scan_add_kernel(uint32_t* __restrict__ a, int64_t m,
                                                            const uint32_t* __restrict__ sums) {
    const uint32_t add = sums[blockIdx.x];
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    for (int k = threadIdx.x; k < kScanTile; k += kScanNT) {
        const int64_t i = base + k;
        if (i < m) a[i] += add;
    }
}

static hipError_t exclusive_scan(uint32_t* a, int64_t m, uint32_t* sums, hipStream_t s) {
    const int64_t nb = (m + kScanTile - 1) / kScanTile;
    hipLaunchKernelGGL(scan_tiles_kernel, dim3((uint32_t)nb), dim3(kScanNT), 0, s, a, m, sums);
    if (nb > 1) {
        hipError_t e = exclusive_scan(sums, nb, sums + ((nb + 63) & ~63LL), s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(scan_add_kernel, dim3((uint32_t)nb), dim3(kScanNT), 0, s, a, m,
                           (const uint32_t*)sums);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------- pass 3 --
// Stable scatter of one tile (12288 items: 64 KB of LDS, two workgroups per
// CU, so one tile's loads overlap another's ranking).  Each wave ranks its own 1024 consecutive
// items (16 rounds of 64) in input order within their digit with a
// wave-private LDS counter per digit: ballots match equal digits inside a
// round, the lowest lane of each match group reads and advances the counter,
// so no block barrier is needed while ranking.  Then the per-digit counts of
// the waves are turned into exclusive prefixes, which give each item its
// tile-local slot (digit offset + earlier waves' count + rank).  The keys are
// placed in LDS in slot order and written out by walking that copy in order
// (coalesced runs per digit); the indices follow through the same buffer.
// The tile's digit counts are differences of consecutive entries of the
// scanned, digit-major histogram table.
constexpr int kWItems = kTile / (kSortNT / kWave);  // items per wave (1024)
__global__ __launch_bounds__(kSortNT, 6) void scatter_kernel(int64_t np,
                                                           const uint32_t* __restrict__ kin,
                                                           const uint32_t* __restrict__ iin,
                                                           uint32_t* __restrict__ kout,
                                                           uint32_t* __restrict__ iout, int shift,
                                                           int bits,
                                                           const uint32_t* __restrict__ hist,
                                                           int64_t tiles) {
    constexpr int NW = kSortNT / kWave;
    constexpr int R = kWItems / kWave;  // rounds per wave (16)
    constexpr int RS = kTile / kSortNT; // slots per thread in the write-out (16)
    __shared__ uint32_t gbase[kMaxRadix];  // global first slot of each digit for this tile
    __shared__ uint32_t loff[kMaxRadix];   // tile-local first slot of each digit
    __shared__ uint16_t wcnt[NW][kMaxRadix];  // counts, then slots (< kTile)
    __shared__ uint32_t wsum[kMaxRadix / kWave];
    __shared__ uint32_t sbuf[kTile];
    const int tid = threadIdx.x, lane = tid & (kWave - 1), w = tid / kWave;
    const uint32_t radix = 1u << bits, mask = radix - 1;
    // consecutive tiles on one XCD: their runs of each digit are adjacent in
    // the output, so the partial cache lines where two runs meet merge in
    // that XCD's L2 instead of being written twice
    const int64_t t = remap_xcd_any(blockIdx.x, (uint32_t)tiles);
    const int64_t tbase = t * kTile;
    const int64_t nvalid64 = np - tbase < kTile ? np - tbase : kTile;
    const int nvalid = (int)nvalid64;
    // this tile's count of digit tid, and the exclusive scan over digits
    // (the first kMaxRadix / 64 waves)
    uint32_t c = 0, inc = 0;
    if (tid < kMaxRadix) {
        if ((uint32_t)tid < radix) {
            const int64_t hi = (int64_t)tid * tiles + t;
            const uint32_t g0 = hist[hi];
            const uint32_t g1 = hi + 1 < (int64_t)radix * tiles ? hist[hi + 1] : (uint32_t)np;
            c = g1 - g0;
            gbase[tid] = g0;
        }
        inc = c;
#pragma unroll
        for (int off = 1; off < kWave; off <<= 1) {
            const uint32_t v = __shfl_up(inc, off, kWave);
            if (lane >= off) inc += v;
        }
        if (lane == kWave - 1) wsum[w] = inc;
    }
    for (int d = tid; d < NW * kMaxRadix; d += kSortNT) (&wcnt[0][0])[d] = 0;
    __syncthreads();
    if (tid < kMaxRadix) {
        uint32_t wpre = 0;
        for (int j = 0; j < w; ++j) wpre += wsum[j];
        loff[tid] = wpre + inc - c;
    }

    // rank this wave's items (no block barrier inside the loop)
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (kWave - lane));
    uint32_t kv[R], rk[R];
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int li = w * kWItems + k * kWave + lane;
        const int64_t i = tbase + li;
        kv[k] = li < nvalid ? kin[i] : 0u;
    }
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int li = w * kWItems + k * kWave + lane;
        const bool valid = li < nvalid;
        const uint32_t d = (kv[k] >> shift) & mask;
        const uint64_t peers = match_digit(d, bits, valid);
        const uint32_t r = (uint32_t)__popcll(peers & lt);
        // every lane of a group reads the count before its leader advances it
        const uint32_t base = valid ? wcnt[w][d] : 0u;
        __builtin_amdgcn_wave_barrier();
        if (valid && r == 0) wcnt[w][d] = (uint16_t)(base + (uint32_t)__popcll(peers));
        __builtin_amdgcn_wave_barrier();
        rk[k] = valid ? base + r : 0xffffffffu;
    }
    __syncthreads();
    // per digit: exclusive prefix of the waves' counts, plus the digit offset
    for (uint32_t d = tid; d < radix; d += kSortNT) {
        uint32_t run = loff[d];
#pragma unroll
        for (int j = 0; j < NW; ++j) {
            const uint32_t v = wcnt[j][d];
            wcnt[j][d] = (uint16_t)run;
            run += v;
        }
    }
    __syncthreads();
    // rk becomes the item's tile slot
#pragma unroll
    for (int k = 0; k < R; ++k) {
        if (rk[k] == 0xffffffffu) continue;
        const uint32_t d = (kv[k] >> shift) & mask;
        rk[k] = wcnt[w][d] + rk[k];
        sbuf[rk[k]] = kv[k];
    }
    __syncthreads();
    uint32_t pos[RS];
#pragma unroll
    for (int k = 0; k < RS; ++k) {
        const int j = k * kSortNT + tid;
        pos[k] = 0xffffffffu;
        if (j < nvalid) {
            const uint32_t kj = sbuf[j];
            const uint32_t d = (kj >> shift) & mask;
            pos[k] = gbase[d] + ((uint32_t)j - loff[d]);
            kout[pos[k]] = kj;
        }
    }
    // the indices follow (loaded only now, to keep the ranking's registers
    // few enough for two workgroups per CU)
    uint32_t iv[R];
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int li = w * kWItems + k * kWave + lane;
        const int64_t i = tbase + li;
        iv[k] = li < nvalid ? (iin ? iin[i] : (uint32_t)i) : 0u;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < R; ++k)
        if (rk[k] != 0xffffffffu) sbuf[rk[k]] = iv[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < RS; ++k) {
        const int j = k * kSortNT + tid;
        if (pos[k] != 0xffffffffu) iout[pos[k]] = sbuf[j];
    }
}

// cell_start[c] = first sorted slot with key >= c, c = 0..ncell.
__global__ __launch_bounds__(256) void cell_start_kernel(int64_t np, int64_t ncell,
                                                         const uint32_t* __restrict__ key,
                                                         uint32_t* __restrict__ cs) {
    for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j <= np; j += (int64_t)gridDim.x * 256) {
        int64_t lo = (j == 0) ? -1 : (int64_t)key[j - 1];
        int64_t hi = (j == np) ? ncell : (int64_t)key[j];
        lo = lo < ncell ? lo : ncell;  // keys >= ncell are rejected by the caller;
        hi = hi < ncell ? hi : ncell;  // the clamp keeps every store in bounds

        for (int64_t c = lo + 1; c <= hi; ++c) cs[c] = (uint32_t)j;
    }
}

// The payload.  A particle moves about two cells per step in each direction
// (sigma of v dt / h at 512^3), so the eight particles of a cell before the
// push land in eight different cells and the sources of consecutive sorted
// slots are scattered over a few planes: a gather of one 8-byte value per
// slot and array fetches a whole memory sector for it and finds it evicted
// when a neighbour of the same sector is needed (measured: 78 bytes fetched
// per 8-byte value, 9 ms per 8 GB array at 512^3 x 8 ppc).  So the six
// values of a particle travel together as one 64-byte record (x, y | z, vx |
// vy, vz | padding: one memory sector; 48-byte records straddled two),
// written in input order by the push (or packed here), and the sort
// gathers one record per sorted slot and writes the six arrays in sorted
// order (consecutive threads, consecutive slots).
__global__ __launch_bounds__(256) void pack_rec_kernel(int64_t np, const double* __restrict__ x,
                                                       const double* __restrict__ y,
                                                       const double* __restrict__ z,
                                                       const double* __restrict__ vx,
                                                       const double* __restrict__ vy,
                                                       const double* __restrict__ vz,
                                                       double2* __restrict__ rec) {
    for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < np; p += (int64_t)gridDim.x * 256) {
        rec[4 * p] = make_double2(x[p], y[p]);
        rec[4 * p + 1] = make_double2(z[p], vx[p]);
        rec[4 * p + 2] = make_double2(vy[p], vz[p]);
        rec[4 * p + 3] = make_double2(0.0, 0.0);
    }
}

constexpr int kGatherK = 2;  // sorted slots per thread per trip (loads issued together)
__global__ __launch_bounds__(256) void gather_rec_kernel(int64_t np, const uint32_t* __restrict__ perm,
                                                         const double2* __restrict__ rec,
                                                         double* __restrict__ x, double* __restrict__ y,
                                                         double* __restrict__ z, double* __restrict__ vx,
                                                         double* __restrict__ vy, double* __restrict__ vz) {
    const int64_t stride = (int64_t)gridDim.x * 256 * kGatherK;
    for (int64_t j0 = (int64_t)blockIdx.x * 256 * kGatherK + threadIdx.x; j0 < np; j0 += stride) {
        double2 r[kGatherK][3];
#pragma unroll
        for (int k = 0; k < kGatherK; ++k) {
            const int64_t j = j0 + 256 * k;
            if (j < np) {
                const int64_t q = 4 * (int64_t)perm[j];
                r[k][0] = rec[q];
                r[k][1] = rec[q + 1];
                r[k][2] = rec[q + 2];
            }
        }
#pragma unroll
        for (int k = 0; k < kGatherK; ++k) {
            const int64_t j = j0 + 256 * k;
            if (j >= np) break;
            __builtin_nontemporal_store(r[k][0].x, x + j);
            __builtin_nontemporal_store(r[k][0].y, y + j);
            __builtin_nontemporal_store(r[k][1].x, z + j);
            __builtin_nontemporal_store(r[k][1].y, vx + j);
            __builtin_nontemporal_store(r[k][2].x, vy + j);
            __builtin_nontemporal_store(r[k][2].y, vz + j);
        }
    }
}

__global__ void copy_u32_kernel(int64_t n, const uint32_t* __restrict__ a, uint32_t* __restrict__ b) {
    for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < n; j += (int64_t)gridDim.x * 256)
        b[j] = a[j];
}

hipError_t launch_sort_cells(int64_t np, int n, const uint32_t* key,
                             const double* const src[6], double* const dst[6],
                             uint32_t* cell_start, uint32_t* perm_out, SortScratch* sc,
                             hipStream_t s) {
    const int64_t ncell = (int64_t)n * n * n;
    const int64_t tiles = ntiles(np);
    int bits = 0;
    while (((int64_t)1 << bits) < ncell) ++bits;
    // fewest passes of at most kMaxBits bits, the bits spread evenly
    const int passes = bits == 0 ? 1 : (bits + kMaxBits - 1) / kMaxBits;
    const int dbits = bits == 0 ? 1 : (bits + passes - 1) / passes;
    const uint32_t* kin = key;
    const uint32_t* iin = nullptr;  // identity on the first pass
    int cur = 0;
    if (np > 0) {
        for (int ps = 0; ps < passes; ++ps) {
            const int shift = dbits * ps;
            hipLaunchKernelGGL(hist_kernel, dim3((uint32_t)tiles), dim3(kHistNT), 0, s, np, kin, shift,
                               dbits, sc->hist, tiles);
            hipError_t e = exclusive_scan(sc->hist, tiles * ((int64_t)1 << dbits), sc->sums, s);
            if (e != hipSuccess) return e;
            hipLaunchKernelGGL(scatter_kernel, dim3((uint32_t)tiles), dim3(kSortNT), 0, s, np, kin, iin,
                               sc->key[cur], sc->idx[cur], shift, dbits,
                               (const uint32_t*)sc->hist, tiles);
            kin = sc->key[cur];
            iin = sc->idx[cur];
            cur ^= 1;
        }
    }
    const int nbc = (int)((np + 1 + 255) / 256 < 16384 ? (np + 1 + 255) / 256 : 16384);
    hipLaunchKernelGGL(cell_start_kernel, dim3(nbc), dim3(256), 0, s, np, ncell, kin, cell_start);
    if (np > 0) {
        const int nbp = (int)((np + 255) / 256 < 16384 ? (np + 255) / 256 : 16384);
        if (src)
            hipLaunchKernelGGL(pack_rec_kernel, dim3(nbp), dim3(256), 0, s, np, src[0], src[1], src[2],
                               src[3], src[4], src[5], sc->rec);
        const int64_t groups = (np + kGatherK - 1) / kGatherK;
        const int nbg = (int)((groups + 255) / 256 < 32768 ? (groups + 255) / 256 : 32768);
        hipLaunchKernelGGL(gather_rec_kernel, dim3(nbg), dim3(256), 0, s, np, iin,
                           (const double2*)sc->rec, dst[0], dst[1], dst[2], dst[3], dst[4], dst[5]);
        if (perm_out)
            hipLaunchKernelGGL(copy_u32_kernel, dim3(nbp), dim3(256), 0, s, np, iin, perm_out);
    }
    return hipGetLastError();
}

}  // namespace pic
