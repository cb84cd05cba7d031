// common.hpp -- shared device helpers of the HIP path (internal).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pic {

constexpr int kWave = 64;

// ---------------------------------------------------------------------------
// Launch geometry helpers.
// Workgroups are dispatched round-robin over the 8 XCDs of an MI355X; each
// XCD has its own L2.  remap_xcd() turns the hardware block id into a logical
// id such that logical ids [j*nb/8, (j+1)*nb/8) all run on XCD j, so tiles
// that share halo data (consecutive logical ids) share an L2.  Requires
// nb % 8 == 0; otherwise the identity is used.
__device__ __forceinline__ uint32_t remap_xcd(uint32_t bid, uint32_t nb) {
    if ((nb & 7u) != 0u) return bid;
    return (bid & 7u) * (nb >> 3) + (bid >> 3);
}
// The same for any nb: XCD j takes the nb / 8 (+1 for j < nb % 8) logical
// ids that follow those of XCDs 0..j-1.
__device__ __forceinline__ uint32_t remap_xcd_any(uint32_t bid, uint32_t nb) {
    const uint32_t j = bid & 7u, q = nb >> 3, r = nb & 7u;
    return j * q + (j < r ? j : r) + (bid >> 3);
}

// ---------------------------------------------------------------------------
// Deterministic block reductions of doubles (fixed shape: lane tree inside a
// wave, then a fixed-order sum over the waves of the block).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

template <int NT, int K>
__device__ __forceinline__ void block_sum(double (&v)[K], double* lds /* K*NT/64 */) {
    const int lane = threadIdx.x & (kWave - 1);
    const int w = threadIdx.x / kWave;
    constexpr int NW = NT / kWave;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        double s = wave_sum(v[k]);
        if (lane == 0) lds[k * NW + w] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            double s = 0.0;
            for (int i = 0; i < NW; ++i) s += lds[k * NW + i];
            v[k] = s;
        }
    }
}

// Sum of partials[0..n) (stride `stride` between the K components) by one
// block in a fixed order: thread t sums indices t, t+NT, ... sequentially,
// then the block tree.  Result valid in thread 0.
template <int NT, int K>
__device__ __forceinline__ void sum_partials(const double* partials, int n, double (&out)[K],
                                             double* lds) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
        double s = 0.0;
        for (int i = threadIdx.x; i < n; i += NT) s += __builtin_nontemporal_load(partials + (size_t)k * n + i);
        out[k] = s;
    }
    block_sum<NT, K>(out, lds);
}

// Ticket for the "last block finishes the reduction" pattern.  Every block
// calls it after writing its partials; returns true in exactly one block
// (the last to arrive), after an acquire fence, and resets the counter.
__device__ __forceinline__ bool last_block(uint32_t* ticket, uint32_t nblocks, int* lds_flag) {
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        uint32_t t = atomicAdd(ticket, 1u);
        bool last = (t == nblocks - 1);
        if (last) atomicExch(ticket, 0u);
        *lds_flag = last ? 1 : 0;
    }
    __syncthreads();
    bool last = *lds_flag != 0;
    if (last) __threadfence();
    return last;
}

}  // namespace pic
