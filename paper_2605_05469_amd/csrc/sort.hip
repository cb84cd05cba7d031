// sort.hip -- stable sort of particles by cell key, cell_start and the payload
// permutation.
//
// The cell sort keeps every cell's particles contiguous so the deposit can
// gather them per vertex and the push streams through the field in memory
// order.  Ties keep their input order (stable), which makes the result a pure
// function of the input sequence (the oracle's counting sort gives the same
// permutation).
//
// Algorithm: LSD radix sort on 8-bit digits over (key, index) pairs, one pass
// per digit that the largest key needs.  Each pass:
//   1. tile histograms (4096 keys per 256-thread workgroup, LDS counters),
//   2. exclusive scan of the digit-major histogram table,
//   3. stable scatter: inside a tile, keys are ranked in input order -- within
//      a wave by matching equal digits with 8 ballots and counting lower
//      lanes, across the tile's waves and rounds with LDS running counts.
// Then cell_start from the sorted keys and a gather of the six FP64 arrays.
#include "common.hpp"
#include "particles.hpp"

namespace pic {

constexpr int kSortNT = 256;
constexpr int kIPT = 16;                       // items per thread per tile
constexpr int kTile = kSortNT * kIPT;          // 4096
constexpr int kRadix = 256;
constexpr int kScanNT = 256;
constexpr int kScanIPT = 16;
constexpr int kScanTile = kScanNT * kScanIPT;  // 4096

static int64_t ntiles(int64_t np) { return (np + kTile - 1) / kTile; }

size_t sort_scratch_bytes(int64_t np_max) {
    const int64_t cap = np_max > 0 ? np_max : 1;
    const int64_t t = ntiles(cap);
    const int64_t hist = t * kRadix;
    const int64_t sums = (hist + kScanTile - 1) / kScanTile + 1;
    size_t b = 0;
    b += 4 * (size_t)cap * sizeof(uint32_t);
    b += (size_t)(hist + 64) * sizeof(uint32_t);
    b += (size_t)(sums + 1088) * sizeof(uint32_t);
    return b + 1024;
}

void sort_scratch_carve(void* base, int64_t np_max, SortScratch* s) {
    const int64_t cap = np_max > 0 ? np_max : 1;
    const int64_t t = ntiles(cap);
    const int64_t hist = t * kRadix;
    char* p = (char*)base;
    auto take = [&](size_t bytes) {
        char* r = p;
        p += (bytes + 255) & ~(size_t)255;
        return r;
    };
    s->key[0] = (uint32_t*)take((size_t)cap * 4);
    s->key[1] = (uint32_t*)take((size_t)cap * 4);
    s->idx[0] = (uint32_t*)take((size_t)cap * 4);
    s->idx[1] = (uint32_t*)take((size_t)cap * 4);
    s->hist = (uint32_t*)take((size_t)(hist + 64) * 4);
    s->sums = (uint32_t*)take((size_t)((hist + kScanTile - 1) / kScanTile + 1089) * 4);
    s->cap = cap;
}

// ---------------------------------------------------------------- pass 1 --
__global__ __launch_bounds__(kSortNT) void hist_kernel(int64_t np, const uint32_t* __restrict__ key,
                                                        int shift, uint32_t* __restrict__ hist,
                                                        int64_t tiles) {
    __shared__ uint32_t cnt[kRadix];
    const int tid = threadIdx.x;
    cnt[tid] = 0;
    __syncthreads();
    const int64_t t = blockIdx.x;
    const int64_t base = t * kTile;
#pragma unroll
    for (int k = 0; k < kIPT; ++k) {
        const int64_t i = base + (int64_t)k * kSortNT + tid;
        if (i < np) atomicAdd(&cnt[(key[i] >> shift) & (kRadix - 1)], 1u);
    }
    __syncthreads();
    hist[(int64_t)tid * tiles + t] = cnt[tid];
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
// Stable scatter of one tile.  Each wave ranks its own 1024 consecutive
// items (16 rounds of 64) in input order within their digit with a
// wave-private LDS counter per digit: 8 ballots match equal digits inside a
// round, the lowest lane of each match group reads and advances the
// counter, so no block barrier is needed while ranking.  One barrier later
// the per-digit counts of the four waves give each item its tile-local slot
// (digit offset + earlier waves' count + rank), and the tile is placed in
// LDS in digit order; a final loop walks that copy in order, so
// consecutive threads write consecutive slots of each digit's output run
// (coalesced stores).  The tile's digit counts are differences of
// consecutive entries of the scanned, digit-major histogram table.
constexpr int kWItems = kTile / (kSortNT / kWave);  // items per wave (1024)
__global__ __launch_bounds__(kSortNT) void scatter_kernel(int64_t np,
                                                           const uint32_t* __restrict__ kin,
                                                           const uint32_t* __restrict__ iin,
                                                           uint32_t* __restrict__ kout,
                                                           uint32_t* __restrict__ iout, int shift,
                                                           const uint32_t* __restrict__ hist,
                                                           int64_t tiles) {
    constexpr int NW = kSortNT / kWave;
    constexpr int R = kWItems / kWave;  // rounds per wave (16)
    __shared__ uint32_t gbase[kRadix];  // global first slot of each digit for this tile
    __shared__ uint32_t loff[kRadix];   // tile-local first slot of each digit
    __shared__ uint32_t wcnt[NW][kRadix];
    __shared__ uint32_t wsum[NW];
    __shared__ uint32_t skey[kTile];
    __shared__ uint32_t sidx[kTile];
    const int tid = threadIdx.x, lane = tid & (kWave - 1), w = tid / kWave;
    const int64_t t = blockIdx.x;
    const int64_t tbase = t * kTile;
    const int64_t nvalid64 = np - tbase < kTile ? np - tbase : kTile;
    const int nvalid = (int)nvalid64;
    // this tile's count of digit tid, and the exclusive scan over digits
    const int64_t hi = (int64_t)tid * tiles + t;
    const uint32_t g0 = hist[hi];
    const uint32_t g1 = hi + 1 < (int64_t)kRadix * tiles ? hist[hi + 1] : (uint32_t)np;
    const uint32_t c = g1 - g0;
    gbase[tid] = g0;
    uint32_t inc = c;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const uint32_t v = __shfl_up(inc, off, kWave);
        if (lane >= off) inc += v;
    }
    if (lane == kWave - 1) wsum[w] = inc;
#pragma unroll
    for (int j = 0; j < NW; ++j) wcnt[j][tid] = 0;
    __syncthreads();
    uint32_t wpre = 0;
    for (int j = 0; j < w; ++j) wpre += wsum[j];
    loff[tid] = wpre + inc - c;

    // rank this wave's items (no block barrier inside the loop)
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (kWave - lane));
    uint32_t kv[R], iv[R], rk[R];
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int li = w * kWItems + k * kWave + lane;
        const int64_t i = tbase + li;
        const bool valid = li < nvalid;
        kv[k] = valid ? kin[i] : 0u;
        iv[k] = valid ? (iin ? iin[i] : (uint32_t)i) : 0u;
    }
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int li = w * kWItems + k * kWave + lane;
        const bool valid = li < nvalid;
        const uint32_t d = (kv[k] >> shift) & (kRadix - 1);
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
            const uint64_t bl = __ballot((d >> bit) & 1u);
            peers &= ((d >> bit) & 1u) ? bl : ~bl;
        }
        const uint32_t r = (uint32_t)__popcll(peers & lt);
        // every lane of a group reads the count before its leader advances it
        const uint32_t base = valid ? wcnt[w][d] : 0u;
        __builtin_amdgcn_wave_barrier();
        if (valid && r == 0) wcnt[w][d] = base + (uint32_t)__popcll(peers);
        __builtin_amdgcn_wave_barrier();
        rk[k] = valid ? base + r : 0xffffffffu;
    }
    __syncthreads();
    // place the tile in LDS in digit order: digit offset, earlier waves of
    // the same digit, then the rank inside the wave
#pragma unroll
    for (int k = 0; k < R; ++k) {
        if (rk[k] == 0xffffffffu) continue;
        const uint32_t d = (kv[k] >> shift) & (kRadix - 1);
        uint32_t pre = loff[d];
        for (int j = 0; j < w; ++j) pre += wcnt[j][d];
        skey[pre + rk[k]] = kv[k];
        sidx[pre + rk[k]] = iv[k];
    }
    __syncthreads();
    for (int j = tid; j < nvalid; j += kSortNT) {
        const uint32_t kj = skey[j];
        const uint32_t d = (kj >> shift) & (kRadix - 1);
        const uint32_t pos = gbase[d] + ((uint32_t)j - loff[d]);
        kout[pos] = kj;
        iout[pos] = sidx[j];
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

// One payload array per launch: dst[j] = src[perm[j]].  A particle moves
// about two cells per step (sigma of v dt / h at 512^3), so the sources of a
// run of sorted slots are the particles of the same cells' neighbourhood
// before the push: row segments within about +-4 rows and +-4 planes of the
// previous order.  One XCD's L2 (4 MB) cannot hold that window for the rows
// it works on, but the 256 MB Infinity Cache holds it for a whole plane:
// consecutive groups of kPermGroup 256-slot chunks (512K slots, a quarter of
// a 512^3 plane) go to the eight XCDs in turn, so all XCDs gather from the
// same few planes at a time and the rows they re-read stay in the Infinity
// Cache.  Measured at 512^3 x 8 ppc: 10.0 ms per array against 15.1 ms when
// each XCD walked its own contiguous eighth of the output (and 12.2 ms in
// plain dispatch order).  Stores bypass L2 retention.
constexpr int kPermChunk = 256;
constexpr uint32_t kPermGroup = 2048;
__global__ __launch_bounds__(256) void permute1_kernel(int64_t np, const uint32_t* __restrict__ perm,
                                                       const double* __restrict__ src,
                                                       double* __restrict__ dst) {
    // hardware dispatch deals consecutive block ids to the 8 XCDs in turn:
    // block b runs on XCD b % 8 as that XCD's (b / 8)-th block
    const uint32_t b = blockIdx.x, xcd = b & 7u, k = b >> 3;
    const uint32_t full = (gridDim.x / (8u * kPermGroup)) * (8u * kPermGroup);
    const uint32_t lb = b < full ? ((k / kPermGroup) * 8u + xcd) * kPermGroup + (k % kPermGroup) : b;
    const int64_t j = (int64_t)lb * kPermChunk + threadIdx.x;
    if (j < np) __builtin_nontemporal_store(src[perm[j]], dst + j);
}

__global__ void copy_u32_kernel(int64_t n, const uint32_t* __restrict__ a, uint32_t* __restrict__ b) {
    for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < n; j += (int64_t)gridDim.x * 256)
        b[j] = a[j];
}

hipError_t launch_sort_cells(int64_t np, int64_t ncell, const uint32_t* key,
                             const double* const src[6], double* const dst[6],
                             uint32_t* cell_start, uint32_t* perm_out, SortScratch* sc,
                             hipStream_t s) {
    const int64_t tiles = ntiles(np);
    int bits = 0;
    while (((int64_t)1 << bits) < ncell) ++bits;
    const int passes = bits == 0 ? 1 : (bits + 7) / 8;
    const uint32_t* kin = key;
    const uint32_t* iin = nullptr;  // identity on the first pass
    int cur = 0;
    if (np > 0) {
        for (int ps = 0; ps < passes; ++ps) {
            const int shift = 8 * ps;
            hipLaunchKernelGGL(hist_kernel, dim3((uint32_t)tiles), dim3(kSortNT), 0, s, np, kin, shift,
                               sc->hist, tiles);
            hipError_t e = exclusive_scan(sc->hist, tiles * kRadix, sc->sums, s);
            if (e != hipSuccess) return e;
            hipLaunchKernelGGL(scatter_kernel, dim3((uint32_t)tiles), dim3(kSortNT), 0, s, np, kin, iin,
                               sc->key[cur], sc->idx[cur], shift, (const uint32_t*)sc->hist, tiles);
            kin = sc->key[cur];
            iin = sc->idx[cur];
            cur ^= 1;
        }
    }
    const int nbc = (int)((np + 1 + 255) / 256 < 16384 ? (np + 1 + 255) / 256 : 16384);
    hipLaunchKernelGGL(cell_start_kernel, dim3(nbc), dim3(256), 0, s, np, ncell, kin, cell_start);
    if (np > 0) {
        const int nbp = (int)((np + 255) / 256 < 16384 ? (np + 255) / 256 : 16384);
        const uint32_t nchunk = (uint32_t)((np + kPermChunk - 1) / kPermChunk);
        for (int a = 0; a < 6; ++a)
            hipLaunchKernelGGL(permute1_kernel, dim3(nchunk), dim3(256), 0, s, np, iin, src[a], dst[a]);
        if (perm_out)
            hipLaunchKernelGGL(copy_u32_kernel, dim3(nbp), dim3(256), 0, s, np, iin, perm_out);
    }
    return hipGetLastError();
}

}  // namespace pic
