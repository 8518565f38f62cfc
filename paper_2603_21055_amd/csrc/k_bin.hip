// Preprocess (FP64, fixed operation order), tile counting, scan, scatter and
// the per-tile depth sort of the instance lists.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "segsort.h"
#include "sgad_internal.h"

namespace sgad {

// ---------------------------------------------------------------------------
// Wave-aggregated counter increments.  Each lane names at most one counter
// (t < 0: none); lanes naming the same counter are served by one atomic from
// their lowest lane, and each learns its rank among them.  Neighbouring
// Gaussians overlap the same tiles, so a wave issues a handful of atomics
// instead of one per lane.  The grouping is scalar work (lane reads and
// ballots); all leaders then issue one atomic instruction together, whose
// return stays in flight until agg_slot() reads it, so a caller can issue
// several rounds before it waits on the first.
// ---------------------------------------------------------------------------
struct AggRound {
    uint32_t ret;    // the leader's pre-increment value (leaders only; in flight)
    uint32_t rank;   // the lane's rank among the lanes naming its counter
    int leader;      // the lowest lane naming the lane's counter
};

template <bool NEED_POS>
__device__ __forceinline__ AggRound wave_agg_issue(uint32_t* ctr, int64_t t) {
    const int lane = threadIdx.x & 63;
    const int t_lo = (int)(uint32_t)(uint64_t)t, t_hi = (int)(uint32_t)((uint64_t)t >> 32);
    uint64_t active = __ballot(t >= 0);
    AggRound a{0u, 0u, 0};
    uint32_t cnt = 0;   // nonzero on leader lanes: the size of their group
    while (active) {
        const int leader = (int)__builtin_ctzll(active);
        const int64_t tgt = (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readlane(t_hi, leader) << 32) |
                                      (uint32_t)__builtin_amdgcn_readlane(t_lo, leader));
        const uint64_t peers = __ballot(t == tgt) & active;
        if (lane == leader) cnt = (uint32_t)__popcll(peers);
        if ((peers >> lane) & 1ull) {
            a.leader = leader;
            a.rank = (uint32_t)__popcll(peers & ((1ull << lane) - 1ull));
        }
        active &= ~peers;
    }
    if (cnt != 0u) {
        if (NEED_POS) a.ret = atomicAdd(&ctr[t], cnt);
        else atomicAdd(&ctr[t], cnt);
    }
    return a;
}

// The lane's slot of a round: its leader's pre-increment value plus its rank
// (meaningful for lanes that named a counter).
__device__ __forceinline__ uint32_t agg_slot(const AggRound& a) {
    return (uint32_t)__shfl((int)a.ret, a.leader, 64) + a.rank;
}

// The cells of a tile rectangle [x0, x1) x [y0, y1) in row order, one per
// call of next(): the counter index base + y * ntx + x, or -1 past the end.
struct RectWalk {
    int x, y, x0, x1, y1;
    __device__ __forceinline__ RectWalk(int x0_, int x1_, int y0_, int y1_, bool any)
        : x(x0_), y(any && x0_ < x1_ ? y0_ : y1_), x0(x0_), x1(x1_), y1(y1_) {}
    __device__ __forceinline__ int64_t next(int64_t base, int ntx) {
        if (y >= y1) return -1;
        const int64_t t = base + (int64_t)y * ntx + x;
        if (++x == x1) {
            x = x0;
            ++y;
        }
        return t;
    }
};

// Gaussian of this thread: each wavefront takes an 8x8 patch of one keyframe,
// so its Gaussians overlap few distinct tiles per counting round.  Grid: x =
// four patches per 256-thread block, y = pair.  `live` is false for lanes
// past the keyframe edge; they are given pixel 0 of the pair.  (n_pairs * N
// < 2^31, so 32-bit indices suffice.)
struct PatchPos {
    int pair, u, v, pix;
    int u0, v0;   // the patch's first pixel
    bool live;
};

__device__ __forceinline__ PatchPos patch_pos(const Geometry& G) {
    PatchPos p;
    const int lane = threadIdx.x & 63;
    const int patch = (int)blockIdx.x * 4 + ((int)threadIdx.x >> 6);
    const int pw = (G.Wk + 7) >> 3;
    const int pv = patch / pw;
    const int pu = patch - pv * pw;
    const int u = pu * 8 + (lane & 7), v = pv * 8 + (lane >> 3);
    p.pair = (int)blockIdx.y;
    p.u0 = pu * 8;
    p.v0 = pv * 8;
    p.live = u < G.Wk && v < G.Hk;
    p.u = p.live ? u : 0;
    p.v = p.live ? v : 0;
    p.pix = p.v * G.Wk + p.u;
    return p;
}

__device__ __forceinline__ int wave_max_int(int v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
    return v;
}

// ---------------------------------------------------------------------------
// Preprocess one (pair, Gaussian): back-project at |D + delta|, move into the
// view, project, form the dilated screen covariance, its conic and the tile
// rectangle; count the tiles.  Every FP64 operation is written in the order
// the binning contract fixes and none is fused, so the tile rectangles and
// depth keys are reproducible bit for bit by an independent FP64 evaluation.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_preprocess(Geometry G, RenderBufs B) {
#pragma clang fp contract(off)
    const PatchPos pp = patch_pos(G);
    const bool live = pp.live;   // idle lanes compute pixel 0 and write nothing
    const int pair = pp.pair, pix = pp.pix, u = pp.u, v = pp.v;
    const size_t i = (size_t)pair * G.N + pix;
    const PairConst& pc = B.pairs[pair];
    const KfPtrs kp = B.kfs[pc.kf];
    const float Df = kp.depth[pix];
    const float Of = kp.offset[pix];
    const float Rf = kp.radius[pix];
    bool ok = isfinite(Df) && isfinite(Of) && isfinite(Rf);
    if (!ok && live) {
        atomicOr(&B.status->nonfinite, 1u);
        atomicOr(&B.status->sticky, 2u);
    }

    const double s = (double)Df + (double)Of;
    const double d = fabs(s);
    const double xn = ((double)u - pc.kcx) / pc.kfx;
    const double yn = ((double)v - pc.kcy) / pc.kfy;
    const double X0 = d * xn, X1 = d * yn, X2 = d;
    const double* R = pc.R;
    const double x = ((R[0] * X0 + R[1] * X1) + R[2] * X2) + pc.t[0];
    const double y = ((R[3] * X0 + R[4] * X1) + R[5] * X2) + pc.t[1];
    const double z = ((R[6] * X0 + R[7] * X1) + R[8] * X2) + pc.t[2];
    ok = ok && (z >= kZNear) && live;

    uint32_t rx = 0, ry = 0;
    int x0 = 0, x1 = 0, y0 = 0, y1 = 0;
    float fdx = 0.f, fdy = 0.f, fa = 0.f, fb = 0.f, fc = 0.f;
    if (ok) {
        const double tx = x / z;
        const double ty = y / z;
        const double mx = pc.vfx * tx + pc.vcx;
        const double my = pc.vfy * ty + pc.vcy;
        const double jx = pc.vfx / z;
        const double jy = pc.vfy / z;
        const double k00 = (jx * jx) * (1.0 + tx * tx);
        const double k01 = (jx * jy) * (tx * ty);
        const double k11 = (jy * jy) * (1.0 + ty * ty);
        const double r2 = (double)Rf * (double)Rf;
        const double s00 = r2 * k00 + kLowpass;
        const double s01 = r2 * k01;
        const double s11 = r2 * k11 + kLowpass;
        const double det = s00 * s11 - s01 * s01;
        const double ca = s11 / det;
        const double cb = -s01 / det;
        const double cc = s00 / det;
        const double hd = 0.5 * (s00 - s11);
        const double lam = 0.5 * (s00 + s11) + sqrt(hd * hd + s01 * s01);
        const double rho = ceil(3.0 * sqrt(lam));
        // tile sizes are powers of two: scaling by the reciprocal is the
        // exact quotient
        const double itw = 1.0 / (double)G.TW, ith = 1.0 / (double)G.TH;
        double ax0 = floor((mx - rho) * itw);
        double ax1 = floor((mx + rho) * itw) + 1.0;
        double ay0 = floor((my - rho) * ith);
        double ay1 = floor((my + rho) * ith) + 1.0;
        ax0 = fmax(ax0, 0.0);
        ay0 = fmax(ay0, 0.0);
        ax1 = fmin(ax1, (double)G.ntx);
        ay1 = fmin(ay1, (double)G.nty);
        x0 = (int)fmin(ax0, (double)G.ntx);
        x1 = (int)fmax(ax1, 0.0);
        y0 = (int)fmin(ay0, (double)G.nty);
        y1 = (int)fmax(ay1, 0.0);
        if (x1 < x0) x1 = x0;
        if (y1 < y0) y1 = y0;
        rx = (uint32_t)x0 | ((uint32_t)x1 << 16);
        ry = (uint32_t)y0 | ((uint32_t)y1 << 16);
        fdx = (float)(mx - (double)u);
        fdy = (float)(my - (double)v);
        fa = (float)ca;
        fb = (float)cb;
        fc = (float)cc;
    }
    {
        // count the overlapped tiles, one wave-aggregated round per rectangle cell
        const int n = ok ? (x1 - x0) * (y1 - y0) : 0;
        const int nmax = wave_max_int(n);
        const int64_t base = (int64_t)pc.job * G.ntiles;
        RectWalk rw(x0, x1, y0, y1, ok);
        for (int k = 0; k < nmax; ++k) wave_agg_issue<false>(B.tile_count, rw.next(base, G.ntx));
    }
    const float fz = ok ? (float)z : 0.f;
    float c0 = 0.f, c1 = 0.f, c2 = 0.f;
    if (kp.rgb) {
        c0 = kp.rgb[pix];
        c1 = kp.rgb[(size_t)G.N + pix];
        c2 = kp.rgb[2 * (size_t)G.N + pix];
    } else if (kp.sigma) {
        const float sg = kp.sigma[pix];
        c0 = sg * sg;
    }
    {
        // The wave's 64 records (an 8x8 patch: eight rows of eight 64-byte
        // records, 512 contiguous bytes each) pass through LDS, so that each
        // store instruction writes two whole rows instead of 16 bytes at a
        // 64-byte stride per lane (3.6x less time for these stores on the
        // 8-keyframe window).  Idle lanes stage too and store nothing.
        __shared__ float4 s_rec[4][256];
        float4* sr = s_rec[threadIdx.x >> 6];
        const int lane = threadIdx.x & 63;
        sr[4 * lane + 0] = make_float4((float)u, (float)v, fdx, fdy);
        sr[4 * lane + 1] = make_float4(fa, fb, fc, kp.opacity[pix]);
        sr[4 * lane + 2] = make_float4(c0, c1, c2, fz);
        sr[4 * lane + 3] = make_float4(ok ? (float)x : 0.f, ok ? (float)y : 0.f, Rf, s >= 0.0 ? 1.f : -1.f);
        asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");   // the wave's own LDS writes are visible
        float4* rec0 = B.pre.rec + 4 * ((size_t)pair * G.N + (size_t)pp.v0 * G.Wk + pp.u0);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            // float4 q of the patch = part q % 4 of record (q / 4) % 8 of row q / 32
            const int q = j * 64 + lane, row = q >> 5, col = q & 31;
            if (pp.u0 + (col >> 2) < G.Wk && pp.v0 + row < G.Hk) rec0[(size_t)row * 4 * G.Wk + col] = sr[q];
        }
    }
    if (!live) return;
    if (B.pre.dir) {   // (tracking has no adjoint and leaves it out)
        // offset direction: the view-space centre moves by R (xn, yn, 1) per
        // unit of |D + delta|, and |D + delta| by sign(D + delta) per unit of delta
        const double sg = s >= 0.0 ? 1.0 : -1.0;
        B.pre.dir[i] = make_float4((float)(sg * ((R[0] * xn + R[1] * yn) + R[2])),
                                   (float)(sg * ((R[3] * xn + R[4] * yn) + R[5])),
                                   (float)(sg * ((R[6] * xn + R[7] * yn) + R[8])), 0.f);
    }
    B.pre.z[i] = fz;
    B.pre.rx[i] = rx;
    B.pre.ry[i] = ry;
}

// Zero an array with a kernel (no memset nodes, so the launch is graph-safe).
__global__ void k_zero_u32(uint32_t* p, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = 0u;
}

// Two arrays zeroed by one launch.
__global__ void k_zero2_u32(uint32_t* a, int64_t na, uint32_t* b, int64_t nb) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < na + nb; i += stride) {
        if (i < na) a[i] = 0u;
        else b[i - na] = 0u;
    }
}

__global__ void k_fill_f32(float* p, int64_t n, float v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

// ---------------------------------------------------------------------------
// Exclusive scan of the per-(job, tile) counts (and of their 64-entry chunk
// counts) in one 1024-thread block.  Up to 6144 elements: one pass, thread t
// owning ceil(M / 1024) consecutive elements, all loaded before use.  More:
// rounds of 4096 elements, thread t owning elements 4t..4t+3 of a round (a
// wave's accesses cover one contiguous 1 KB span), the counts of up to
// kScanPre rounds loaded up front.  Also publishes the total, the overflow flag and the
// longest segment, and clears the fill counters and the work-queue counter
// (and, with zero_counts, the counts themselves, so that the next call's
// count pass needs no clearing launch).
// ---------------------------------------------------------------------------
constexpr int kScanIt = 4;
constexpr int kScanPre = 4;
constexpr int kScanRound = 1024 * kScanIt;
constexpr int kScanSmall = 6;   // up to 6144 elements: one pass, <= 6 per thread

__global__ __launch_bounds__(1024) void k_scan(uint32_t* __restrict__ count, uint32_t* start, uint32_t* fill,
                                               uint32_t* cstart, int M, uint32_t capacity, DevStatus* st,
                                               int zero_counts) {
    __shared__ uint32_t s_w[16], s_cw[16], s_max[16];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (M <= 1024 * kScanSmall) {
        // one pass: thread t owns [t * per, t * per + per)
        const int per = (M + 1023) / 1024;
        const int b = tid * per;
        uint32_t c[kScanSmall];
#pragma unroll
        for (int j = 0; j < kScanSmall; ++j) c[j] = (j < per && b + j < M) ? count[b + j] : 0u;
        uint32_t sum = 0, csum = 0, mx = 0;
#pragma unroll
        for (int j = 0; j < kScanSmall; ++j) {
            sum += c[j];
            csum += (c[j] + 63u) >> 6;
            mx = max(mx, c[j]);
        }
        uint32_t inc = sum, cinc = csum;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t o = __shfl_up(inc, off, 64), co = __shfl_up(cinc, off, 64);
            if (lane >= off) {
                inc += o;
                cinc += co;
            }
        }
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) mx = max(mx, (uint32_t)__shfl_xor((int)mx, o, 64));
        if (lane == 63) {
            s_w[wave] = inc;
            s_cw[wave] = cinc;
        }
        if (lane == 0) s_max[wave] = mx;
        __syncthreads();
        const uint32_t a0 = lane < 16 ? s_w[lane] : 0u, ca0 = lane < 16 ? s_cw[lane] : 0u;
        uint32_t a = a0, ca = ca0;
#pragma unroll
        for (int off = 1; off < 16; off <<= 1) {
            const uint32_t o = __shfl_up(a, off, 64), co = __shfl_up(ca, off, 64);
            if (lane >= off) {
                a += o;
                ca += co;
            }
        }
        uint32_t run = (uint32_t)__shfl((int)(a - a0), wave, 64) + inc - sum;
        uint32_t crun = (uint32_t)__shfl((int)(ca - ca0), wave, 64) + cinc - csum;
#pragma unroll
        for (int j = 0; j < kScanSmall; ++j) {
            const int i = b + j;
            if (j < per && i < M) {
                start[i] = run;
                cstart[i] = crun;
                fill[i] = 0u;
                if (zero_counts) count[i] = 0u;   // ready for the next count pass
            }
            run += c[j];
            crun += (c[j] + 63u) >> 6;
        }
        const uint32_t tot = (uint32_t)__shfl((int)a, 15, 64), ctot = (uint32_t)__shfl((int)ca, 15, 64);
        if (tid == 0) {
            start[M] = tot;
            cstart[M] = ctot;
            st->total = tot;
            st->overflow = tot > capacity ? 1u : 0u;
            st->queue = 0u;
            uint32_t m = 0;
            for (int w = 0; w < 16; ++w) m = max(m, s_max[w]);
            st->max_seg = m;
        }
        return;
    }
    const int rounds = (M + kScanRound - 1) / kScanRound;
    uint32_t pre[kScanPre][kScanIt];
#pragma unroll
    for (int r = 0; r < kScanPre; ++r)
#pragma unroll
        for (int j = 0; j < kScanIt; ++j) {
            const int i = r * kScanRound + kScanIt * tid + j;
            pre[r][j] = (r < rounds && i < M) ? count[i] : 0u;
        }
    uint32_t carry = 0, ccarry = 0, mx = 0;
    for (int r = 0; r < rounds; ++r) {
        const int i0 = r * kScanRound + kScanIt * tid;
        uint32_t c[kScanIt];
#pragma unroll
        for (int j = 0; j < kScanIt; ++j) {
            c[j] = 0u;
#pragma unroll
            for (int k = 0; k < kScanPre; ++k)
                if (k == r) c[j] = pre[k][j];
            if (r >= kScanPre && i0 + j < M) c[j] = count[i0 + j];
        }
        uint32_t cc[kScanIt], sum = 0, csum = 0;
#pragma unroll
        for (int j = 0; j < kScanIt; ++j) {
            cc[j] = (c[j] + 63u) >> 6;
            sum += c[j];
            csum += cc[j];
            mx = max(mx, c[j]);
        }
        // inclusive scan of the per-thread sums across the wave
        uint32_t inc = sum, cinc = csum;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t o = __shfl_up(inc, off, 64), co = __shfl_up(cinc, off, 64);
            if (lane >= off) {
                inc += o;
                cinc += co;
            }
        }
        if (lane == 63) {
            s_w[wave] = inc;
            s_cw[wave] = cinc;
        }
        __syncthreads();
        // every wave scans the 16 wave totals itself (lanes 0-15)
        const uint32_t a0 = lane < 16 ? s_w[lane] : 0u, ca0 = lane < 16 ? s_cw[lane] : 0u;
        uint32_t a = a0, ca = ca0;
#pragma unroll
        for (int off = 1; off < 16; off <<= 1) {
            const uint32_t o = __shfl_up(a, off, 64), co = __shfl_up(ca, off, 64);
            if (lane >= off) {
                a += o;
                ca += co;
            }
        }
        const uint32_t tot = (uint32_t)__shfl((int)a, 15, 64), ctot = (uint32_t)__shfl((int)ca, 15, 64);
        const uint32_t wo = (uint32_t)__shfl((int)(a - a0), wave, 64);     // exclusive wave offsets
        const uint32_t cwo = (uint32_t)__shfl((int)(ca - ca0), wave, 64);
        uint32_t run = carry + wo + inc - sum, crun = ccarry + cwo + cinc - csum;
#pragma unroll
        for (int j = 0; j < kScanIt; ++j) {
            const int i = i0 + j;
            if (i < M) {
                start[i] = run;
                cstart[i] = crun;
                fill[i] = 0u;
                if (zero_counts) count[i] = 0u;   // ready for the next count pass
            }
            run += c[j];
            crun += cc[j];
        }
        carry += tot;
        ccarry += ctot;
        __syncthreads();   // s_w is rewritten by the next round
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) mx = max(mx, (uint32_t)__shfl_xor((int)mx, o, 64));
    if (lane == 0) s_max[wave] = mx;
    __syncthreads();
    if (tid == 0) {
        start[M] = carry;
        cstart[M] = ccarry;
        st->total = carry;
        st->overflow = carry > capacity ? 1u : 0u;
        st->queue = 0u;
        uint32_t m = 0;
        for (int w = 0; w < 16; ++w) m = max(m, s_max[w]);
        st->max_seg = m;
    }
}

// ---------------------------------------------------------------------------
// Scatter one key per (Gaussian, overlapped tile) into its tile's segment.
// Key = float bits of z << 32 | gid; the order inside a segment is fixed later
// by the sort, so the atomic slot order does not matter.
// ---------------------------------------------------------------------------
constexpr int kScatterBatch = 4;

__global__ __launch_bounds__(256) void k_scatter(Geometry G, RenderBufs B) {
    const PatchPos pp = patch_pos(G);
    const size_t i = (size_t)pp.pair * G.N + pp.pix;
    int x0 = 0, x1 = 0, y0 = 0, y1 = 0;
    uint64_t key = 0;
    int64_t base = 0;
    if (pp.live) {
        const uint32_t rx = B.pre.rx[i], ry = B.pre.ry[i];
        x0 = rx & 0xffff;
        x1 = rx >> 16;
        y0 = ry & 0xffff;
        y1 = ry >> 16;
        const int pix = pp.pix;
        const PairConst& pc = B.pairs[pp.pair];
        const uint32_t gid = (uint32_t)pc.kf * (uint32_t)G.N + (uint32_t)pix;
        key = ((uint64_t)__float_as_uint(B.pre.z[i]) << 32) | gid;
        base = (int64_t)pc.job * G.ntiles;
    }
    const int n = (x0 < x1 && y0 < y1) ? (x1 - x0) * (y1 - y0) : 0;
    const int nmax = wave_max_int(n);
    bool dropped = false;
    RectWalk rw(x0, x1, y0, y1, pp.live);
    // rounds are issued kScatterBatch at a time: their segment starts and
    // fill atomics all in flight before the first slot is read
    for (int k0 = 0; k0 < nmax; k0 += kScatterBatch) {
        int64_t t[kScatterBatch];
        uint32_t st0[kScatterBatch];
        AggRound ar[kScatterBatch];
#pragma unroll
        for (int j = 0; j < kScatterBatch; ++j) {
            t[j] = k0 + j < nmax ? rw.next(base, G.ntx) : -1;
            st0[j] = t[j] >= 0 ? B.tile_start[t[j]] : 0u;
        }
#pragma unroll
        for (int j = 0; j < kScatterBatch; ++j)
            if (k0 + j < nmax) ar[j] = wave_agg_issue<true>(B.tile_fill, t[j]);
#pragma unroll
        for (int j = 0; j < kScatterBatch; ++j) {
            if (k0 + j >= nmax) break;
            const uint32_t r = agg_slot(ar[j]);
            if (t[j] >= 0) {
                const uint32_t pos = st0[j] + r;
                if (pos < B.capacity) B.keys[pos] = key;
                else dropped = true;
            }
        }
    }
    // an instance that did not fit is the overflow the caller must hear of
    if (__ballot(dropped) != 0ull && (threadIdx.x & 63) == 0) atomicOr(&B.status->sticky, 1u);
}

__device__ inline void cmpswap_lds(uint64_t* s, int a, int b) {
    uint64_t x = s[a], y = s[b];
    if (y < x) {
        s[a] = y;
        s[b] = x;
    }
}

__global__ __launch_bounds__(64) void k_sort(Geometry G, RenderBufs B) {
    const int seg = blockIdx.x;
    if (B.status->overflow) return;
    const uint32_t st = B.tile_start[seg];
    const int n = (int)(B.tile_start[seg + 1] - st);
    uint64_t* g = B.keys + st;
    sort_segment<true>(g, n, threadIdx.x, G.sort_long != 0);
}

// Segments of 1025..4096 keys by a 256-thread workgroup: each of the four
// waves sorts a run of np2 / 4 keys (512 or 1024, padded with all-ones keys
// past n) in registers into LDS, then the runs are merged pairwise in two
// levels.  Each thread merges E consecutive outputs of a pair: it finds how
// many of them come from the first run by a binary search along its output
// diagonal (merge path; keys are unique, so the split is unambiguous),
// merges into registers, and writes them back after the whole workgroup has
// read.
template <int K>
__device__ __forceinline__ void sort_run(const uint64_t* g, int n, uint64_t* s, int wave, int lane) {
    uint64_t x[K];
    const int b = wave * 64 * K + lane * K;
#pragma unroll
    for (int r = 0; r < K; ++r) x[r] = b + r < n ? g[b + r] : ~0ull;
    wave_sort_regs<K, true>(x, lane);
#pragma unroll
    for (int r = 0; r < K; ++r) s[b + r] = x[r];
}

template <int NMAX>
__device__ void sort_merge_segment(uint64_t* g, int n, uint64_t* s) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int np2 = n <= 2048 ? 2048 : 4096;
    if constexpr (NMAX <= 2048) {
        sort_run<8>(g, n, s, wave, lane);   // (n <= NMAX here)
    } else {
        if (np2 == 2048) sort_run<8>(g, n, s, wave, lane);
        else sort_run<16>(g, n, s, wave, lane);
    }
    __syncthreads();
    constexpr int kMaxE = 16;
    const int E = np2 / 256;   // outputs per thread: 8 or 16
    for (int width = np2 / 4; width < np2; width <<= 1) {
        const int o0 = tid * E;
        const int base = (o0 / (2 * width)) * (2 * width);
        const uint64_t* A = s + base;
        const uint64_t* Bv = A + width;
        const int o = o0 - base;
        int lo = o > width ? o - width : 0, hi = o < width ? o : width;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (A[mid] < Bv[o - mid - 1]) lo = mid + 1;
            else hi = mid;
        }
        int i = lo, j = o - lo;
        uint64_t out[kMaxE];
#pragma unroll
        for (int e = 0; e < kMaxE; ++e) {
            if (e < E) {
                const uint64_t a = i < width ? A[i] : ~0ull;
                const uint64_t bb = j < width ? Bv[j] : ~0ull;
                const bool ta = j >= width || (i < width && a < bb);
                out[e] = ta ? a : bb;
                i += ta ? 1 : 0;
                j += ta ? 0 : 1;
            }
        }
        __syncthreads();
#pragma unroll
        for (int e = 0; e < kMaxE; ++e)
            if (e < E) s[o0 + e] = out[e];
        __syncthreads();
    }
    for (int k = tid; k < n; k += blockDim.x) g[k] = s[k];
}

// LDS of NMAX keys: merge sort up to min(NMAX, 4096) keys, the bitonic
// network in LDS up to NMAX, else in place in global memory.
template <int NMAX>
__device__ void sort_long_segment(uint64_t* g, int n, uint64_t* s) {
    const int tid = threadIdx.x;
    if (n <= NMAX && n <= 4096 && blockDim.x == 256) {
        sort_merge_segment<NMAX>(g, n, s);
        return;
    }
    int np2 = 1;
    while (np2 < n) np2 <<= 1;
    if (np2 <= NMAX) {
        for (int k = tid; k < np2; k += blockDim.x) s[k] = k < n ? g[k] : ~0ull;
        __syncthreads();
        for (int k = 2; k <= np2; k <<= 1) {
            const int h = k >> 1;
            for (int p = tid; p < (np2 >> 1); p += blockDim.x) {
                const int blk = p / h, off = p - blk * h;
                cmpswap_lds(s, blk * k + off, blk * k + k - 1 - off);
            }
            __syncthreads();
            for (int j = k >> 2; j >= 1; j >>= 1) {
                for (int p = tid; p < (np2 >> 1); p += blockDim.x) {
                    const int blk = p / j, off = p - blk * j;
                    const int a = blk * 2 * j + off;
                    cmpswap_lds(s, a, a + j);
                }
                __syncthreads();
            }
        }
        for (int k = tid; k < n; k += blockDim.x) g[k] = s[k];
        return;
    }
    sort_global_segment(g, n);
}

// Segments longer than 1024 keys, launched when the previous forward of the
// workload had one (the scan records the longest segment), and always for
// tracking; one workgroup per segment (long segments come in numbers when
// several keyframes overlap a view).  NMAX = 2048 when the previous forward's
// longest segment fit (twice the workgroups per CU), else 4096.
template <int NMAX>
__global__ __launch_bounds__(256) void k_sort_long(Geometry G, RenderBufs B) {
    __shared__ uint64_t s[NMAX];
    if (B.status->overflow) return;
    const int seg = blockIdx.x;
    const uint32_t st = B.tile_start[seg];
    const int n = (int)(B.tile_start[seg + 1] - st);
    if (n <= 1024) return;
    sort_long_segment<NMAX>(B.keys + st, n, s);
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
void launch_zero_u32(uint32_t* p, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    int blocks = (int)std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_zero_u32, dim3(blocks), dim3(256), 0, s, p, n);
}

void launch_zero2_u32(uint32_t* a, int64_t na, uint32_t* b, int64_t nb, hipStream_t s) {
    const int64_t n = na + nb;
    if (n <= 0) return;
    int blocks = (int)std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_zero2_u32, dim3(blocks), dim3(256), 0, s, a, na, b, nb);
}

void launch_fill_f32(float* p, int64_t n, float v, hipStream_t s) {
    if (n <= 0) return;
    int blocks = (int)std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_fill_f32, dim3(blocks), dim3(256), 0, s, p, n, v);
}

static dim3 patch_grid(const Geometry& G) {
    const int patches = ((G.Wk + 7) >> 3) * ((G.Hk + 7) >> 3);
    return dim3((unsigned)((patches + 3) / 4), (unsigned)G.n_pairs);
}

void launch_preprocess(const Geometry& G, const RenderBufs& B, hipStream_t s) {
    hipLaunchKernelGGL(k_preprocess, patch_grid(G), dim3(256), 0, s, G, B);
}

void launch_scan(const Geometry& G, const RenderBufs& B, bool zero_counts, hipStream_t s) {
    const int M = G.n_jobs * G.ntiles;
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, B.tile_count, B.tile_start, B.tile_fill,
                       B.chunk_start, M, B.capacity, B.status, zero_counts ? 1 : 0);
}

void launch_scatter(const Geometry& G, const RenderBufs& B, hipStream_t s) {
    hipLaunchKernelGGL(k_scatter, patch_grid(G), dim3(256), 0, s, G, B);
}

// With G.fuse_sort the forward sorts the segments of up to 1024 keys itself
// (and the longer ones when no long pass runs); only the long pass is
// launched here.
void launch_sort(const Geometry& G, const RenderBufs& B, hipStream_t s) {
    const int M = G.n_jobs * G.ntiles;
    if (!G.fuse_sort) hipLaunchKernelGGL(k_sort, dim3(M), dim3(64), 0, s, G, B);
    if (G.sort_long == 1) hipLaunchKernelGGL(k_sort_long<2048>, dim3(M), dim3(256), 0, s, G, B);
    else if (G.sort_long) hipLaunchKernelGGL(k_sort_long<kSortLds>, dim3(M), dim3(256), 0, s, G, B);
}

}  // namespace sgad
