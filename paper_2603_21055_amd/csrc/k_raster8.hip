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
// Backward: see k_bwd8 (a pixel-parallel walk that stores per-pair terms and an
// entry-parallel sum over pixels, with no atomics inside the tile).
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

// Backward of one 8x8 tile per wavefront (one wavefront per workgroup).
//
// The tile's list is taken in 64-entry chunks from the back, each chunk in
// sub-chunks of SUB entries from the back, in two phases per sub-chunk:
//  A (lane = pixel): the reverse walk over the pixel's candidates carries the
//    transmittance and the suffix colour sums and stores, per contributing
//    pair, w = alpha T and gq = dL/dq into a [pixel][entry] LDS matrix;
//  B (lane = entry, 64 / SUB pixel groups): every lane sums its entry's pairs
//    over the pixels of its group that wrote anything in the sub-chunk, and
//    clears what it read.
// The per-entry sums are gq-weighted moments of (dx, dy) and gradient-weighted
// sums of w; the conic enters after the sum.  No LDS location is written by two
// lanes at once, and the in-tile summation order is fixed.
template <int SUB>
__global__ __launch_bounds__(64) void k_bwd8(Geometry G, RenderBufs B, BwdArgs A) {
    constexpr int NS = 64 / SUB;        // sub-chunks per chunk = pixel groups in phase B
    constexpr int LS = 2 * SUB + 4;     // floats per matrix row: 16-byte rows, rows 4 banks apart
    __shared__ float4 s_e[64][3];
    __shared__ uint64_t s_m[16];
    __shared__ float4 s_pc[65];
    __shared__ __align__(16) float s_M[65 * LS];   // row 64 stays zero: the idle pixel of phase B
    const int lane = threadIdx.x;
    const int item = xcd_remap(blockIdx.x, gridDim.x);
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
    s_pc[lane] = make_float4(gC0, gC1, gC2, gD);
    if (lane == 0) s_pc[64] = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
    for (int k = 0; k < LS; k += 4) *(float4*)&s_M[lane * LS + k] = make_float4(0.f, 0.f, 0.f, 0.f);
    if (lane < LS / 4) *(float4*)&s_M[64 * LS + lane * 4] = make_float4(0.f, 0.f, 0.f, 0.f);
    int maxlast = last;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) maxlast = max(maxlast, __shfl_xor(maxlast, o, 64));
    const float Tf = T;
    const float fpx = (float)px, fpy = (float)py;
    const float fx0 = (float)(tx * 8), fy0 = (float)(ty * 8);
    const int sub = lane & (SUB - 1), grp = lane / SUB;
    float S0 = 0.f, S1 = 0.f, S2 = 0.f, SD = 0.f;
    float pose[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (int c0 = maxlast > 0 ? ((maxlast - 1) & ~63) : -1; c0 >= 0; c0 -= 64) {
        const int n = min(64, maxlast - c0);
        stage_chunk(G, B, job, st + (uint32_t)c0, n, 0, lane, fx0, fy0, s_e, s_m);
        lds_fence();
        const uint64_t mine = s_m[lx] & s_m[8 + ly];
        const int lim = min(n, last - c0);   // this pixel's entries are e < lim
        float r[10];
#pragma unroll
        for (int k = 0; k < 10; ++k) r[k] = 0.f;
#pragma unroll
        for (int s = NS - 1; s >= 0; --s) {
            // phase A: reverse walk of this pixel's candidates in the sub-chunk
            const int cut = lim - s * SUB;
            uint64_t m = cut <= 0 ? 0ull : ((mine >> (s * SUB)) & low_bits(min(cut, SUB)));
            bool wrote = false;
            while (m != 0ull) {
                const int bit = 63 - __builtin_clzll(m);
                m &= ~(1ull << bit);
                const int e = s * SUB + bit;
                const float4 eu = s_e[e][0];
                const float dx = (fpx - eu.x) - eu.z, dy = (fpy - eu.y) - eu.w;
                const float4 eg = s_e[e][1];
                const float q = pair_q(dx, dy, eg.x, eg.y, eg.z);
                if (!(q <= kQCut)) continue;
                const float Gv = gauss_of_q(q);
                const float raw = eg.w * Gv;
                const float alpha = fminf(kAlphaMax, raw);
                if (alpha < kAlphaMin) continue;
                const float4 c = s_e[e][2];
                const float inv = 1.f / (1.f - alpha);
                T = T * inv;
                const float w = alpha * T;
                const float gal = gC0 * (c.x * T - S0 * inv) + gC1 * (c.y * T - S1 * inv) +
                                  gC2 * (c.z * T - S2 * inv) + gD * (c.w * T - SD * inv) + gA * Tf * inv;
                S0 += w * c.x;
                S1 += w * c.y;
                S2 += w * c.z;
                SD += w * c.w;
                const float gq = raw < kAlphaMax ? -0.5f * alpha * gal : 0.f;
                *(float2*)&s_M[lane * LS + 2 * bit] = make_float2(w, gq);
                wrote = true;
            }
            const uint64_t pm0 = __ballot(wrote);
            lds_fence();
            // phase B: lane = entry s * SUB + sub, pixel group grp
            const float4 eu = s_e[s * SUB + sub][0];
            float a[10];
#pragma unroll
            for (int k = 0; k < 10; ++k) a[k] = 0.f;
            uint64_t pm = pm0;
            while (pm != 0ull) {
                int p = 64;
#pragma unroll
                for (int g = 0; g < NS; ++g) {
                    const int pg = pm != 0ull ? (int)__builtin_ctzll(pm) : 64;
                    pm &= pm - 1ull;
                    p = g == grp ? pg : p;
                }
                float2* cell = (float2*)&s_M[p * LS + 2 * sub];
                const float2 mv = *cell;
                *cell = make_float2(0.f, 0.f);
                const float4 g = s_pc[p];
                const float dx = ((float)(tx * 8 + (p & 7)) - eu.x) - eu.z;
                const float dy = ((float)(ty * 8 + (p >> 3)) - eu.y) - eu.w;
                a[0] += g.x * mv.x;
                a[1] += g.y * mv.x;
                a[2] += g.z * mv.x;
                a[3] += g.w * mv.x;
                a[4] += mv.y;
                const float u = mv.y * dx, v = mv.y * dy;
                a[5] += u;
                a[6] += v;
                a[7] += u * dx;
                a[8] += u * dy;
                a[9] += v * dy;
            }
#pragma unroll
            for (int o = SUB; o < 64; o <<= 1)
#pragma unroll
                for (int k = 0; k < 10; ++k) a[k] += __shfl_xor(a[k], o, 64);
            if (grp == s)
#pragma unroll
                for (int k = 0; k < 10; ++k) r[k] = a[k];
            lds_fence();
        }
        // lane = chunk entry: chain rule to the keyframe parameters and the pose
        if (lane < n) {
            bool any = false;
#pragma unroll
            for (int k = 0; k < 10; ++k) any |= r[k] != 0.f;
            if (any) {
                const float4 eg = s_e[lane][1];
                float v[10];
                v[0] = -2.f * (eg.x * r[5] + eg.y * r[6]);
                v[1] = -2.f * (eg.y * r[5] + eg.z * r[6]);
                v[2] = r[7];
                v[3] = 2.f * r[8];
                v[4] = r[9];
                v[5] = r[4] != 0.f ? -2.f * r[4] / eg.w : 0.f;
                v[6] = r[3];
                v[7] = r[0];
                v[8] = r[1];
                v[9] = r[2];
                flush_entry(G, B, A, job, B.keys[st + (uint32_t)c0 + (uint32_t)lane], v, pose);
            }
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

template <int SUB>
static void bwd8_t(const Geometry& G, const RenderBufs& B, const BwdArgs& A, hipStream_t s) {
    const int items = G.n_jobs * G.ntiles;
    hipLaunchKernelGGL((k_bwd8<SUB>), dim3(items), dim3(64), 0, s, G, B, A);
}

bool launch_fwd8(const Geometry& G, const RenderBufs& B, const FwdOut& O, int sc, hipStream_t s) {
    if (G.TW != 8 || G.TH != 8) return false;
    if (sc == 256) fwd8_t<256>(G, B, O, s);
    else if (sc == 128) fwd8_t<128>(G, B, O, s);
    else return false;
    return true;
}

bool launch_bwd8(const Geometry& G, const RenderBufs& B, const BwdArgs& A, int sub, hipStream_t s) {
    if (G.TW != 8 || G.TH != 8) return false;
    if (sub == 32) bwd8_t<32>(G, B, A, s);
    else if (sub == 16) bwd8_t<16>(G, B, A, s);
    else return false;
    return true;
}

}  // namespace sgad
