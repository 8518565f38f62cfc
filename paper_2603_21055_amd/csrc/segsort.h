// Cross-lane exchanges of a wavefront (DPP and the gfx950 row-swap permutes),
// the segment sort of 64-bit instance keys by one wavefront (shared by the
// sort kernel and the wave-tile forward, which sorts its own tile's segment)
// and a bit-matrix transpose across lanes (the wave-tile walks' coverage and
// contribution masks).
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

// The value lane ^ m holds, for the lane masks the network uses, without a
// trip through the LDS unit: DPP quad permutations and row mirrors inside a
// row of 16 lanes, two DPP row shifts for a distance of 4 or 8, and the
// row-swapping permutes for 16 and 32 (xor 2^k - 1 = a mirror inside the row,
// then the rows swapped).  Every lane of the wave takes part.
template <int CTRL>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t v) {
    // every lane is written from a lane of its own row: no old value needed
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, CTRL, 0xF, 0xF, false);
}

// Two DPP moves into one register, each writing only its banks (groups of
// four lanes in a row): lanes whose partner is N lanes up take row_shl:N,
// the others row_shr:N, with no select between the two.
template <int CTRL_A, int BANKS_A, int CTRL_B, int BANKS_B>
__device__ __forceinline__ uint32_t dpp_banks(uint32_t v) {
    const int t = __builtin_amdgcn_mov_dpp((int)v, CTRL_A, 0xF, BANKS_A, false);
    return (uint32_t)__builtin_amdgcn_update_dpp(t, (int)v, CTRL_B, 0xF, BANKS_B, false);
}

__device__ __forceinline__ uint32_t xor_rows16(uint32_t v, int lane) {
    const auto p = __builtin_amdgcn_permlane16_swap(v, v, false, false);
    return (lane & 16) ? p[0] : p[1];
}

__device__ __forceinline__ uint32_t xor_rows32(uint32_t v, int lane) {
    const auto p = __builtin_amdgcn_permlane32_swap(v, v, false, false);
    return (lane & 32) ? p[0] : p[1];
}

template <int M>
__device__ __forceinline__ uint32_t xor_lane_u32(uint32_t v, int lane) {
    if constexpr (M == 1) return dpp_u32<0xB1>(v);          // quad_perm [1, 0, 3, 2]
    else if constexpr (M == 2) return dpp_u32<0x4E>(v);     // quad_perm [2, 3, 0, 1]
    else if constexpr (M == 3) return dpp_u32<0x1B>(v);     // quad_perm [3, 2, 1, 0]
    else if constexpr (M == 4) return dpp_banks<0x104, 0x5, 0x114, 0xA>(v);   // row_shl:4 / row_shr:4
    else if constexpr (M == 7) return dpp_u32<0x141>(v);  // row_half_mirror
    else if constexpr (M == 8) return dpp_banks<0x108, 0x3, 0x118, 0xC>(v);   // row_shl:8 / row_shr:8
    else if constexpr (M == 15) return dpp_u32<0x140>(v);  // row_mirror
    else if constexpr (M == 16) return xor_rows16(v, lane);
    else if constexpr (M == 31) return xor_rows16(dpp_u32<0x140>(v), lane);
    else if constexpr (M == 32) return xor_rows32(v, lane);
    else {
        static_assert(M == 63, "lane mask of the bitonic network");
        return xor_rows32(xor_rows16(dpp_u32<0x140>(v), lane), lane);
    }
}

// One butterfly step of a bit-matrix transpose across lanes: lanes l and
// l ^ S swap the off-diagonal S x S blocks of their words (block rows in the
// lanes, block columns in the bits).
template <int S>
__device__ __forceinline__ uint32_t transpose_step(uint32_t x, uint32_t full, int lane) {
    constexpr uint32_t kM = S == 16 ? 0xFFFF0000u : S == 8 ? 0xFF00FF00u : S == 4 ? 0xF0F0F0F0u
                          : S == 2  ? 0xCCCCCCCCu : 0xAAAAAAAAu;
    const uint32_t m = kM & full;
    const uint32_t y = xor_lane_u32<S>(x, lane);
    return (lane & S) ? ((x & m) | ((y >> S) & ~m)) : ((x & ~m) | ((y << S) & m));
}

// Column lane % SUB of the 64 x SUB bit matrix whose row l is lane l's SUB-bit
// word x, as a 64-bit mask over the lanes: the SUB x SUB blocks of each group
// of SUB lanes are transposed by butterfly exchanges (after which lane j of a
// group holds column j of that group's rows), then the 64 / SUB pieces of a
// column are joined across the groups.  Every lane takes part.
template <int SUB>
__device__ __forceinline__ uint64_t bit_column(uint32_t x, int lane) {
    constexpr uint32_t full = SUB == 32 ? 0xFFFFFFFFu : (1u << SUB) - 1u;
    if constexpr (SUB == 32) x = transpose_step<16>(x, full, lane);
    x = transpose_step<8>(x, full, lane);
    x = transpose_step<4>(x, full, lane);
    x = transpose_step<2>(x, full, lane);
    x = transpose_step<1>(x, full, lane);
    uint32_t pair = x;   // the column's bits of rows 0-31 (lanes 0-31) or 32-63 (lanes 32-63)
    if constexpr (SUB == 16) {
        const uint32_t u = xor_rows16(x, lane);
        pair = (lane & 16) ? (u | (x << 16)) : (x | (u << 16));
    }
    const uint32_t v = xor_rows32(pair, lane);
    return (lane & 32) ? (((uint64_t)pair << 32) | v) : (((uint64_t)v << 32) | pair);
}

// DPP = false: ds_bpermute shuffles instead, which cost no VALU issue slots;
// the better choice inside kernels whose other waves keep the VALU busy
// (the wave-tile forward sorts its tile while other waves walk theirs).
template <int M, bool DPP>
__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t v, int lane) {
    uint32_t lo, hi;
    if constexpr (DPP) {
        lo = xor_lane_u32<M>((uint32_t)v, lane);
        hi = xor_lane_u32<M>((uint32_t)(v >> 32), lane);
    } else {
        lo = (uint32_t)__shfl_xor((int)(uint32_t)v, M, 64);
        hi = (uint32_t)__shfl_xor((int)(uint32_t)(v >> 32), M, 64);
    }
    return ((uint64_t)hi << 32) | lo;
}

// One side of a compare-exchange across lanes: lanes marked `upper` keep the
// larger of their key x and their partner's key y, the others the smaller.
// One comparison and one select (keys are unique but for the all-ones
// padding, so a tie keeps an equal value).
__device__ __forceinline__ uint64_t keep_side(uint64_t x, uint64_t y, bool upper) {
    return ((y < x) != upper) ? y : x;
}

// A compare-exchange of two registers of one lane: a, b = min, max.  The
// swap flag is xored with a false the compiler cannot see through, so that
// both selects use the one comparison instead of becoming a min and a max
// that compare again.
__device__ __forceinline__ void cx_in_lane(uint64_t& a, uint64_t& b) {
    int z;
    asm("s_mov_b32 %0, 0" : "=s"(z));
    const bool sw = (b < a) != (z != 0);
    const uint64_t lo = sw ? b : a, hi = sw ? a : b;
    a = lo;
    b = hi;
}

template <int K>
__device__ __forceinline__ void sort_in_lane(uint64_t (&x)[K], int j) {
#pragma unroll
    for (int r = 0; r < K; ++r) {
        const int p = r ^ j;
        if (p > r) cx_in_lane(x[r], x[p]);
    }
}

// Butterfly steps j, j / 2, ..., 1 of a bitonic merge over the 64 K keys a
// wave holds in registers (key i = lane * K + r in register r).
template <int K, int J, bool DPP>
__device__ __forceinline__ void bitonic_steps(uint64_t (&x)[K], int lane) {
    if constexpr (J < K) {
        sort_in_lane<K>(x, J);
    } else {
        constexpr int lm = J / K;
        const bool upper = (lane & lm) != 0;
#pragma unroll
        for (int r = 0; r < K; ++r) x[r] = keep_side(x[r], shfl_xor_u64<lm, DPP>(x[r], lane), upper);
    }
    if constexpr (J > 1) bitonic_steps<K, J / 2, DPP>(x, lane);
}

// Merge stage of size KS (2 .. 64 K) and the stages after it.
template <int K, int KS, bool DPP>
__device__ __forceinline__ void bitonic_stages(uint64_t (&x)[K], int lane) {
    if constexpr (KS <= K) {
        // mirror step inside the lane: r <-> r ^ (KS - 1)
#pragma unroll
        for (int r = 0; r < K; ++r) {
            const int p = r ^ (KS - 1);
            if (p > r) cx_in_lane(x[r], x[p]);
        }
    } else {
        // mirror step across lanes: (lane, r) <-> (lane ^ (KS / K - 1), K - 1 - r),
        // taken in register pairs (r, K - 1 - r)
        constexpr int lm = KS / K - 1;
        const bool upper = (lane & (KS / (2 * K))) != 0;
#pragma unroll
        for (int r = 0; r < (K + 1) / 2; ++r) {
            const int q = K - 1 - r;
            const uint64_t ya = shfl_xor_u64<lm, DPP>(x[q], lane);
            const uint64_t yb = shfl_xor_u64<lm, DPP>(x[r], lane);
            x[r] = keep_side(x[r], ya, upper);
            if (q != r) x[q] = keep_side(x[q], yb, upper);
        }
    }
    if constexpr (KS >= 4) bitonic_steps<K, KS / 4, DPP>(x, lane);
    if constexpr (2 * KS <= 64 * K) bitonic_stages<K, 2 * KS, DPP>(x, lane);
}

// Ascending bitonic sort of the 64 K keys a wave holds in registers (key
// i = lane * K + r in register r).
template <int K, bool DPP = false>
__device__ __forceinline__ void wave_sort_regs(uint64_t (&x)[K], int lane) {
    bitonic_stages<K, 2, DPP>(x, lane);
}

template <int K, bool DPP>
__device__ __forceinline__ void wave_sort_segment(uint64_t* g, int n, int lane) {
    uint64_t x[K];
#pragma unroll
    for (int r = 0; r < K; ++r) {
        const int i = lane * K + r;
        x[r] = i < n ? g[i] : ~0ull;
    }
    wave_sort_regs<K, DPP>(x, lane);
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
template <bool DPP = false>
__device__ __forceinline__ void sort_segment(uint64_t* g, int n, int lane, bool long_pass) {
    if (n <= 1) return;
    if (n <= 64) wave_sort_segment<1, DPP>(g, n, lane);
    else if (n <= 128) wave_sort_segment<2, DPP>(g, n, lane);
    else if (n <= 256) wave_sort_segment<4, DPP>(g, n, lane);
    else if (n <= 512) wave_sort_segment<8, DPP>(g, n, lane);
    else if (n <= 1024) wave_sort_segment<16, DPP>(g, n, lane);
    else if (!long_pass) sort_global_segment(g, n);
}

}  // namespace sgad
