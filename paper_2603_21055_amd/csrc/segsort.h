// Segment sort of 64-bit instance keys by one wavefront (shared by the sort
// kernel and the wave-tile forward, which sorts its own tile's segment).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace sgad {

// ---------------------------------------------------------------------------
// Per-segment ascending sort of 64-bit keys, one wavefront per segment.
// Segments up to 1024 keys are sorted in registers: K = 1..16 keys per lane,
// key i = lane * K + r in register r, padded with all-ones keys to 64 K.  The
// bitonic network takes every comparator ascending (the first step of each
// merge pairs mirrored positions), so exchanges inside a lane are register
// swaps and exchanges across lanes are one xor shuffle per key half.  Longer
// segments are sorted by the same network in LDS (up to kSortLds keys) or in
// place in global memory with virtual +inf padding.
// ---------------------------------------------------------------------------
constexpr int kSortLds = 4096;

__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t v, int m) {
    const int lo = __shfl_xor((int)(uint32_t)v, m, 64);
    const int hi = __shfl_xor((int)(uint32_t)(v >> 32), m, 64);
    return ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
}

template <int K>
__device__ __forceinline__ void sort_in_lane(uint64_t (&x)[K], int j) {
#pragma unroll
    for (int r = 0; r < K; ++r) {
        const int p = r ^ j;
        if (p > r) {
            const uint64_t a = x[r], b = x[p];
            x[r] = a < b ? a : b;
            x[p] = a < b ? b : a;
        }
    }
}

// Ascending bitonic sort of the 64 K keys a wave holds in registers (key
// i = lane * K + r in register r).
template <int K>
__device__ __forceinline__ void wave_sort_regs(uint64_t (&x)[K], int lane) {
#pragma unroll
    for (int k = 2; k <= 64 * K; k <<= 1) {
        if (k <= K) {
            // mirror step inside the lane: r <-> r ^ (k - 1)
#pragma unroll
            for (int r = 0; r < K; ++r) {
                const int p = r ^ (k - 1);
                if (p > r) {
                    const uint64_t a = x[r], b = x[p];
                    x[r] = a < b ? a : b;
                    x[p] = a < b ? b : a;
                }
            }
        } else {
            // mirror step across lanes: (lane, r) <-> (lane ^ (k / K - 1), K - 1 - r),
            // taken in register pairs (r, K - 1 - r)
            const int lm = k / K - 1;
            const bool lower = (lane & (k / (2 * K))) == 0;
#pragma unroll
            for (int r = 0; r < (K + 1) / 2; ++r) {
                const int q = K - 1 - r;
                const uint64_t ya = shfl_xor_u64(x[q], lm);
                const uint64_t yb = shfl_xor_u64(x[r], lm);
                x[r] = lower ? (x[r] < ya ? x[r] : ya) : (x[r] < ya ? ya : x[r]);
                if (q != r) x[q] = lower ? (x[q] < yb ? x[q] : yb) : (x[q] < yb ? yb : x[q]);
            }
        }
#pragma unroll
        for (int j = k >> 2; j >= 1; j >>= 1) {
            if (j < K) {
                sort_in_lane<K>(x, j);
            } else {
                const int lm = j / K;
                const bool lower = (lane & lm) == 0;
#pragma unroll
                for (int r = 0; r < K; ++r) {
                    const uint64_t y = shfl_xor_u64(x[r], lm);
                    x[r] = lower ? (x[r] < y ? x[r] : y) : (x[r] < y ? y : x[r]);
                }
            }
        }
    }
}

template <int K>
__device__ __forceinline__ void wave_sort_segment(uint64_t* g, int n, int lane) {
    uint64_t x[K];
#pragma unroll
    for (int r = 0; r < K; ++r) {
        const int i = lane * K + r;
        x[r] = i < n ? g[i] : ~0ull;
    }
    wave_sort_regs<K>(x, lane);
#pragma unroll
    for (int r = 0; r < K; ++r) {
        const int i = lane * K + r;
        if (i < n) g[i] = x[r];
    }
}

// Bitonic network in place in global memory with virtual +inf padding, by the
// threads of one workgroup.
__device__ __forceinline__ void sort_global_segment(uint64_t* g, int n) {
    const int tid = threadIdx.x;
    int np2 = 1;
    while (np2 < n) np2 <<= 1;
    // long segment: same network in global memory, virtual +inf padding
    for (int k = 2; k <= np2; k <<= 1) {
        const int h = k >> 1;
        for (int p = tid; p < (np2 >> 1); p += blockDim.x) {
            const int blk = p / h, off = p - blk * h;
            const int a = blk * k + off, b = blk * k + k - 1 - off;
            if (b < n) {
                uint64_t x = g[a], y = g[b];
                if (y < x) {
                    g[a] = y;
                    g[b] = x;
                }
            }
        }
        __syncthreads();
        for (int j = k >> 2; j >= 1; j >>= 1) {
            for (int p = tid; p < (np2 >> 1); p += blockDim.x) {
                const int blk = p / j, off = p - blk * j;
                const int a = blk * 2 * j + off, b = a + j;
                if (b < n) {
                    uint64_t x = g[a], y = g[b];
                    if (y < x) {
                        g[a] = y;
                        g[b] = x;
                    }
                }
            }
            __syncthreads();
        }
    }
}


// Ascending sort of g[0, n) by the calling wavefront (lane = threadIdx.x of
// a 64-thread workgroup).  Segments longer than 1024 keys are left to the
// long-segment pass when `long_pass` is set, else sorted in place in global
// memory.
__device__ __forceinline__ void sort_segment(uint64_t* g, int n, int lane, bool long_pass) {
    if (n <= 1) return;
    if (n <= 64) wave_sort_segment<1>(g, n, lane);
    else if (n <= 128) wave_sort_segment<2>(g, n, lane);
    else if (n <= 256) wave_sort_segment<4>(g, n, lane);
    else if (n <= 512) wave_sort_segment<8>(g, n, lane);
    else if (n <= 1024) wave_sort_segment<16>(g, n, lane);
    else if (!long_pass) sort_global_segment(g, n);
}

}  // namespace sgad
