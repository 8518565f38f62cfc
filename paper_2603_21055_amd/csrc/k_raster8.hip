// Wave-tile compositing: one 8x8 tile per wavefront, one lane per pixel, four
// independent tiles per workgroup (no workgroup barriers).
//
// The tile's sorted instance list is taken in super-chunks of SC entries.
// For each 64-entry chunk every lane stages one entry in LDS and computes the
// pixel rectangle that bounds the entry's 3-sigma ellipse inside the tile;
// sixteen wave ballots turn those rectangles into 8 column masks and 8 row
// masks, and pixel (c, r) takes the chunk's candidates as col[c] & row[r].
// Each lane then walks only its own candidates, in list order (forward) or
// reverse list order (backward), so a pixel evaluates ~47 pairs instead of
// the whole list.  The rectangle is a superset of every pair with q <= 9 as
// evaluated in FP32, so the contributor sets and their order are exactly
// those of the full-list walk.
//
// Backward: the ten per-pair gradient terms are added into per-entry LDS
// accumulators laid out component-major (bank = entry index); after each
// super-chunk one lane per entry applies the chain rule to the keyframe
// parameters and the pose.
#include <hip/hip_runtime.h>

#include "raster_common.h"

namespace sgad {

constexpr int kWaves = 4;

__device__ __forceinline__ uint64_t low_bits(int k) { return k >= 64 ? ~0ull : ((1ull << k) - 1ull); }

// Stage chunk `ch` of a super-chunk and publish its coverage masks.
__device__ __forceinline__ void stage_chunk(const Geometry& G, const RenderBufs& B, int job, uint32_t base, int n,
                                            int ch, int lane, float fx0, float fy0, float4 (*se)[3],
                                            uint64_t* sm) {
    const int e = ch * 64 + lane;
    const bool valid = e < n;
    int x0 = 8, x1 = -1, y0 = 8, y1 = -1;
    if (valid) {
        const float4* rec = entry_record(G, B, job, B.keys[base + e]);
        const float4 eu = rec[0], eg = rec[1], ec = rec[2];
        se[e][0] = eu;
        se[e][1] = eg;
        se[e][2] = ec;
        const float mx = (eu.x - fx0) + eu.z, my = (eu.y - fy0) + eu.w;
        const float det = eg.x * eg.z - eg.y * eg.y;
        const float ex = 3.f * sqrtf(eg.z / det) + 1e-3f;
        const float ey = 3.f * sqrtf(eg.x / det) + 1e-3f;
        x0 = max(0, (int)ceilf(mx - ex));
        x1 = min(7, (int)floorf(mx + ex));
        y0 = max(0, (int)ceilf(my - ey));
        y1 = min(7, (int)floorf(my + ey));
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const uint64_t cm = __ballot(valid && x0 <= k && k <= x1);
        const uint64_t rm = __ballot(valid && y0 <= k && k <= y1);
        if (lane == k) sm[ch * 16 + k] = cm;
        if (lane == 8 + k) sm[ch * 16 + 8 + k] = rm;
    }
}

template <int SC>
__global__ __launch_bounds__(256) void k_fwd8(Geometry G, RenderBufs B, FwdOut O) {
    constexpr int NCH = SC / 64;
    __shared__ float4 s_e[kWaves][SC][3];
    __shared__ uint64_t s_m[kWaves][NCH * 16];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int item = xcd_remap(blockIdx.x, gridDim.x) * kWaves + wave;
    if (item >= G.n_jobs * G.ntiles) return;
    const int job = item / G.ntiles;
    const int tile = item - job * G.ntiles;
    const int tx = tile % G.ntx, ty = tile / G.ntx;
    const int lx = lane & 7, ly = lane >> 3;
    const int px = tx * 8 + lx, py = ty * 8 + ly;
    const bool inside = px < G.Wv && py < G.Hv;
    const bool ovf = B.status->overflow != 0u;
    const uint32_t st = B.tile_start[item];
    const uint32_t en = ovf ? st : B.tile_start[item + 1];
    const float fpx = (float)px, fpy = (float)py;
    const float fx0 = (float)(tx * 8), fy0 = (float)(ty * 8);
    float4 (*se)[3] = s_e[wave];
    uint64_t* sm = s_m[wave];
    float T = 1.f, cr = 0.f, cg = 0.f, cb = 0.f, dd = 0.f;
    int cnt = 0;
    uint32_t last = 0;
    bool done = !inside;
    for (uint32_t sc0 = st; sc0 < en; sc0 += SC) {
        const int n = (int)min((uint32_t)SC, en - sc0);
        const int nch = (n + 63) >> 6;
        for (int ch = 0; ch < nch; ++ch) stage_chunk(G, B, job, sc0, n, ch, lane, fx0, fy0, se, sm);
        lds_fence();
        if (!done) {
            int ch = 0;
            uint64_t m = sm[lx] & sm[8 + ly];
            while (true) {
                while (m == 0ull && ch + 1 < nch) {
                    ++ch;
                    m = sm[ch * 16 + lx] & sm[ch * 16 + 8 + ly];
                }
                if (m == 0ull) break;
                const int e = ch * 64 + __builtin_ctzll(m);
                m &= m - 1ull;
                const float4 eu = se[e][0];
                const float dx = (fpx - eu.x) - eu.z, dy = (fpy - eu.y) - eu.w;
                const float4 eg = se[e][1];
                const float q = pair_q(dx, dy, eg.x, eg.y, eg.z);
                if (!(q <= kQCut)) continue;
                const float alpha = fminf(kAlphaMax, eg.w * gauss_of_q(q));
                if (alpha < kAlphaMin) continue;
                const float test = T * (1.f - alpha);
                if (test < kTMin) {
                    done = true;
                    break;
                }
                const float w = alpha * T;
                const float4 c = se[e][2];
                cr += w * c.x;
                cg += w * c.y;
                cb += w * c.z;
                dd += w * c.w;
                T = test;
                ++cnt;
                last = sc0 - st + (uint32_t)e + 1u;
            }
        }
        lds_fence();
        if (__ballot(!done) == 0ull) break;
    }
    if (!inside) return;
    const size_t pix = (size_t)py * G.Wv + px;
    const size_t P = (size_t)G.P;
    const size_t jp = (size_t)job * P + pix;
    if (ovf) {
        const float nan = __builtin_nanf("");
        cr = cg = cb = dd = nan;
        T = nan;
    }
    O.rgb[((size_t)job * 3 + 0) * P + pix] = cr;
    O.rgb[((size_t)job * 3 + 1) * P + pix] = cg;
    O.rgb[((size_t)job * 3 + 2) * P + pix] = cb;
    O.depth[jp] = dd;
    O.alpha[jp] = 1.f - T;
    if (O.count) O.count[jp] = cnt;
    B.Tfinal[jp] = T;
    B.last[jp] = last;
}

template <int SC>
__global__ __launch_bounds__(256) void k_bwd8(Geometry G, RenderBufs B, BwdArgs A) {
    constexpr int NCH = SC / 64;
    __shared__ float4 s_e[kWaves][SC][3];
    __shared__ uint64_t s_m[kWaves][NCH * 16];
    __shared__ float s_acc[kWaves][10][SC];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int item = xcd_remap(blockIdx.x, gridDim.x) * kWaves + wave;
    if (item >= G.n_jobs * G.ntiles) return;
    const int job = item / G.ntiles;
    const int tile = item - job * G.ntiles;
    const int tx = tile % G.ntx, ty = tile / G.ntx;
    const int lx = lane & 7, ly = lane >> 3;
    const int px = tx * 8 + lx, py = ty * 8 + ly;
    const bool inside = px < G.Wv && py < G.Hv;
    const bool ovf = B.status->overflow != 0u;
    const uint32_t st = B.tile_start[item];
    const size_t P = (size_t)G.P;
    float T = 1.f, gC0 = 0.f, gC1 = 0.f, gC2 = 0.f, gD = 0.f, gA = 0.f;
    int last = 0;
    if (inside && !ovf) {
        const size_t pix = (size_t)py * G.Wv + px;
        const size_t jp = (size_t)job * P + pix;
        T = B.Tfinal[jp];
        last = (int)B.last[jp];
        gC0 = A.g_rgb[((size_t)job * 3 + 0) * P + pix];
        gC1 = A.g_rgb[((size_t)job * 3 + 1) * P + pix];
        gC2 = A.g_rgb[((size_t)job * 3 + 2) * P + pix];
        if (A.g_depth) gD = A.g_depth[jp];
        if (A.g_alpha) gA = A.g_alpha[jp];
    }
    int maxlast = last;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) maxlast = max(maxlast, __shfl_xor(maxlast, o, 64));
    const float Tf = T;
    const float fpx = (float)px, fpy = (float)py;
    const float fx0 = (float)(tx * 8), fy0 = (float)(ty * 8);
    float4 (*se)[3] = s_e[wave];
    uint64_t* sm = s_m[wave];
    float (*acc)[SC] = s_acc[wave];
    float S0 = 0.f, S1 = 0.f, S2 = 0.f, SD = 0.f;
    float pose[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (int sc0 = maxlast > 0 ? ((maxlast - 1) / SC) * SC : -1; sc0 >= 0; sc0 -= SC) {
        const int n = min(SC, maxlast - sc0);
        const int nch = (n + 63) >> 6;
        for (int ch = 0; ch < nch; ++ch) {
            stage_chunk(G, B, job, st + (uint32_t)sc0, n, ch, lane, fx0, fy0, se, sm);
            const int e = ch * 64 + lane;
#pragma unroll
            for (int c = 0; c < 10; ++c) acc[c][e] = 0.f;
        }
        lds_fence();
        const int lim = min(n, last - sc0);   // this pixel's entries are e < lim
        if (lim > 0) {
            int ch = (lim - 1) >> 6;
            uint64_t m = sm[ch * 16 + lx] & sm[ch * 16 + 8 + ly] & low_bits(lim - ch * 64);
            while (true) {
                while (m == 0ull && ch > 0) {
                    --ch;
                    m = sm[ch * 16 + lx] & sm[ch * 16 + 8 + ly];
                }
                if (m == 0ull) break;
                const int bit = 63 - __builtin_clzll(m);
                m &= ~(1ull << bit);
                const int e = ch * 64 + bit;
                const float4 eu = se[e][0];
                const float dx = (fpx - eu.x) - eu.z, dy = (fpy - eu.y) - eu.w;
                const float4 eg = se[e][1];
                const float q = pair_q(dx, dy, eg.x, eg.y, eg.z);
                if (!(q <= kQCut)) continue;
                const float Gv = gauss_of_q(q);
                const float raw = eg.w * Gv;
                const float alpha = fminf(kAlphaMax, raw);
                if (alpha < kAlphaMin) continue;
                const float4 c = se[e][2];
                const float inv = 1.f / (1.f - alpha);
                T = T * inv;
                const float w = alpha * T;
                const float gal = gC0 * (c.x * T - S0 * inv) + gC1 * (c.y * T - S1 * inv) +
                                  gC2 * (c.z * T - S2 * inv) + gD * (c.w * T - SD * inv) + gA * Tf * inv;
                S0 += w * c.x;
                S1 += w * c.y;
                S2 += w * c.z;
                SD += w * c.w;
                atomicAdd(&acc[6][e], gD * w);
                atomicAdd(&acc[7][e], gC0 * w);
                atomicAdd(&acc[8][e], gC1 * w);
                atomicAdd(&acc[9][e], gC2 * w);
                if (raw < kAlphaMax) {
                    const float gq = -0.5f * alpha * gal;
                    const float t1 = eg.x * dx + eg.y * dy;
                    const float t2 = eg.y * dx + eg.z * dy;
                    atomicAdd(&acc[5][e], gal * Gv);
                    atomicAdd(&acc[0][e], -2.f * gq * t1);
                    atomicAdd(&acc[1][e], -2.f * gq * t2);
                    atomicAdd(&acc[2][e], gq * dx * dx);
                    atomicAdd(&acc[3][e], 2.f * gq * dx * dy);
                    atomicAdd(&acc[4][e], gq * dy * dy);
                }
            }
        }
        lds_fence();
        for (int e = lane; e < n; e += 64) {
            float v[10];
            bool any = false;
#pragma unroll
            for (int c = 0; c < 10; ++c) {
                v[c] = acc[c][e];
                any |= v[c] != 0.f;
            }
            if (any) flush_entry(G, B, A, job, B.keys[st + (uint32_t)sc0 + (uint32_t)e], v, pose);
        }
        lds_fence();
    }
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        const float sv = wave_sum(pose[c]);
        if (lane == 0) A.pose_part[(size_t)item * 6 + c] = sv;
    }
}

template <int SC>
static void fwd8_t(const Geometry& G, const RenderBufs& B, const FwdOut& O, hipStream_t s) {
    const int items = G.n_jobs * G.ntiles;
    hipLaunchKernelGGL((k_fwd8<SC>), dim3((items + kWaves - 1) / kWaves), dim3(64 * kWaves), 0, s, G, B, O);
}

template <int SC>
static void bwd8_t(const Geometry& G, const RenderBufs& B, const BwdArgs& A, hipStream_t s) {
    const int items = G.n_jobs * G.ntiles;
    hipLaunchKernelGGL((k_bwd8<SC>), dim3((items + kWaves - 1) / kWaves), dim3(64 * kWaves), 0, s, G, B, A);
}

bool launch_fwd8(const Geometry& G, const RenderBufs& B, const FwdOut& O, int sc, hipStream_t s) {
    if (G.TW != 8 || G.TH != 8) return false;
    if (sc == 256) fwd8_t<256>(G, B, O, s);
    else if (sc == 128) fwd8_t<128>(G, B, O, s);
    else return false;
    return true;
}

bool launch_bwd8(const Geometry& G, const RenderBufs& B, const BwdArgs& A, int sc, hipStream_t s) {
    if (G.TW != 8 || G.TH != 8) return false;
    if (sc == 256) bwd8_t<256>(G, B, A, s);
    else if (sc == 128) bwd8_t<128>(G, B, A, s);
    else return false;
    return true;
}

}  // namespace sgad
