// Tile compositing: front-to-back forward and reverse-order adjoint.
//
// One workgroup per (job, tile); one lane per pixel.  The tile's sorted
// instance list is staged through LDS in batches of one entry per lane.
// The backward walks each pixel's contributors in reverse, recovering the
// transmittance by division (no per-pixel lists are stored), reduces each
// entry's gradient across the wave with cross-lane shuffles and across waves
// with LDS atomics, then applies the chain rule to the keyframe parameters
// and the view pose once per (Gaussian, tile) before a few global atomics.
#include <hip/hip_runtime.h>

#include "raster_common.h"

namespace sgad {

// Stage one instance: source pixel (u, v) and screen displacement of the
// mean, conic, opacity, depth and colour.  A pixel's offset from the mean is
// formed as (p - (u, v)) - displacement: the integer part is exact, so the
// only rounding is the last subtraction and the result does not depend on
// the tile the pixel belongs to.
__device__ __forceinline__ void load_entry(const Geometry& G, const RenderBufs& B, int job, uint64_t key,
                                           float4& eu, float4& eg, float4& ec) {
    const uint32_t gid = (uint32_t)key;
    const int kf = kf_of_gid(G, gid);
    const int pix = (int)(gid - (uint32_t)kf * (uint32_t)G.N);
    const int pair = B.pair_of[job * G.n_kf + kf];
    const float4* rec = B.pre.rec + 4 * ((size_t)pair * G.N + pix);
    eu = rec[0];
    eg = rec[1];
    ec = rec[2];
}

template <int TW, int TH>
__global__ __launch_bounds__(TW* TH) void k_fwd(Geometry G, RenderBufs B, FwdOut O) {
    constexpr int NT = TW * TH;
    __shared__ float4 s_u[NT], s_g[NT], s_c[NT];
    publish_status(B);
    const int item = blockIdx.x;
    const int job = item / G.ntiles;
    const int tile = item - job * G.ntiles;
    const int tx = tile % G.ntx, ty = tile / G.ntx;
    const int x0 = tx * TW, y0 = ty * TH;
    const int tid = threadIdx.x;
    const int lx = tid % TW, ly = tid / TW;
    const int px = x0 + lx, py = y0 + ly;
    const bool inside = px < G.Wv && py < G.Hv;
    const bool ovf = B.status->overflow != 0u;
    const uint32_t st = B.tile_start[item];
    const uint32_t en = ovf ? st : B.tile_start[item + 1];
    const float fpx = (float)px, fpy = (float)py;
    float T = 1.f, cr = 0.f, cg = 0.f, cb = 0.f, dd = 0.f;
    int cnt = 0;
    uint32_t last = 0;
    bool done = !inside;
    for (uint32_t b = st; b < en; b += NT) {
        const int n = (int)min((uint32_t)NT, en - b);
        if (tid < n) load_entry(G, B, job, B.keys[b + tid], s_u[tid], s_g[tid], s_c[tid]);
        __syncthreads();
        if (!done) {
            for (int k = 0; k < n; ++k) {
                const float4 e = s_u[k];
                const float dx = (fpx - e.x) - e.z, dy = (fpy - e.y) - e.w;
                const float4 g = s_g[k];
                const float q = pair_q(dx, dy, g.x, g.y, g.z);
                if (!(q <= kQCut)) continue;
                const float alpha = fminf(kAlphaMax, g.w * gauss_of_q(q));
                if (alpha < kAlphaMin) continue;
                const float test = T * (1.f - alpha);
                if (test < kTMin) {
                    done = true;
                    break;
                }
                const float w = alpha * T;
                const float4 c = s_c[k];
                cr += w * c.x;
                cg += w * c.y;
                cb += w * c.z;
                dd += w * c.w;
                T = test;
                ++cnt;
                last = b - st + (uint32_t)k + 1u;
            }
        }
        if (__syncthreads_count(!done) == 0) break;
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

template <int TW, int TH>
__global__ __launch_bounds__(TW* TH) void k_bwd(Geometry G, RenderBufs B, BwdArgs A) {
    constexpr int NT = TW * TH;
    constexpr int NW = (NT + 63) / 64;
    __shared__ float4 s_u[NT], s_g[NT], s_c[NT];
    __shared__ float s_acc[NT][10];
    __shared__ uint32_t s_max;
    __shared__ float s_pose[NW][6];
    const int item = blockIdx.x;
    const int job = item / G.ntiles;
    const int tile = item - job * G.ntiles;
    const int tx = tile % G.ntx, ty = tile / G.ntx;
    const int x0 = tx * TW, y0 = ty * TH;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int lx = tid % TW, ly = tid / TW;
    const int px = x0 + lx, py = y0 + ly;
    const bool inside = px < G.Wv && py < G.Hv;
    const bool ovf = B.status->overflow != 0u;
    const uint32_t st = B.tile_start[item];
    const size_t P = (size_t)G.P;
    float T = 1.f, gC0 = 0.f, gC1 = 0.f, gC2 = 0.f, gD = 0.f, gA = 0.f;
    uint32_t last = 0;
    if (inside && !ovf) {
        const size_t pix = (size_t)py * G.Wv + px;
        const size_t jp = (size_t)job * P + pix;
        T = B.Tfinal[jp];
        last = B.last[jp];
        gC0 = A.g_rgb[((size_t)job * 3 + 0) * P + pix];
        gC1 = A.g_rgb[((size_t)job * 3 + 1) * P + pix];
        gC2 = A.g_rgb[((size_t)job * 3 + 2) * P + pix];
        if (A.g_depth) gD = A.g_depth[jp];
        if (A.g_alpha) gA = A.g_alpha[jp];
    }
    if (tid == 0) s_max = 0u;
    __syncthreads();
    atomicMax(&s_max, last);
    __syncthreads();
    const int maxlast = (int)s_max;
    const float Tf = T;
    const float fpx = (float)px, fpy = (float)py;
    float S0 = 0.f, S1 = 0.f, S2 = 0.f, SD = 0.f;
    float pose[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (int bend = maxlast; bend > 0; bend -= NT) {
        const int bstart = max(0, bend - NT);
        const int n = bend - bstart;
        if (tid < n) load_entry(G, B, job, B.keys[st + bstart + tid], s_u[tid], s_g[tid], s_c[tid]);
#pragma unroll
        for (int c = 0; c < 10; ++c) s_acc[tid][c] = 0.f;
        __syncthreads();
        for (int k = n - 1; k >= 0; --k) {
            float v[10];
#pragma unroll
            for (int c = 0; c < 10; ++c) v[c] = 0.f;
            bool has = false;
            if (bstart + k < (int)last) {
                const float4 e = s_u[k];
                const float dx = (fpx - e.x) - e.z, dy = (fpy - e.y) - e.w;
                const float4 g = s_g[k];
                const float q = pair_q(dx, dy, g.x, g.y, g.z);
                if (q <= kQCut) {
                    const float Gv = gauss_of_q(q);
                    const float raw = g.w * Gv;
                    const float alpha = fminf(kAlphaMax, raw);
                    if (alpha >= kAlphaMin) {
                        has = true;
                        const float4 c = s_c[k];
                        const float inv = 1.f / (1.f - alpha);
                        T = T * inv;
                        const float w = alpha * T;
                        const float gal = gC0 * (c.x * T - S0 * inv) + gC1 * (c.y * T - S1 * inv) +
                                          gC2 * (c.z * T - S2 * inv) + gD * (c.w * T - SD * inv) +
                                          gA * Tf * inv;
                        S0 += w * c.x;
                        S1 += w * c.y;
                        S2 += w * c.z;
                        SD += w * c.w;
                        v[6] = gD * w;
                        v[7] = gC0 * w;
                        v[8] = gC1 * w;
                        v[9] = gC2 * w;
                        if (raw < kAlphaMax) {
                            const float gq = -0.5f * alpha * gal;
                            v[5] = gal * Gv;
                            const float t1 = g.x * dx + g.y * dy;
                            const float t2 = g.y * dx + g.z * dy;
                            v[0] = -2.f * gq * t1;
                            v[1] = -2.f * gq * t2;
                            v[2] = gq * dx * dx;
                            v[3] = 2.f * gq * dx * dy;
                            v[4] = gq * dy * dy;
                        }
                    }
                }
            }
            if (__any(has)) {
#pragma unroll
                for (int c = 0; c < 10; ++c) {
                    const float sv = wave_sum(v[c]);
                    if (lane == 0 && sv != 0.f) atomicAdd(&s_acc[k][c], sv);
                }
            }
        }
        __syncthreads();
        if (tid < n) {
            float v[10];
            bool any = false;
#pragma unroll
            for (int c = 0; c < 10; ++c) {
                v[c] = s_acc[tid][c];
                any |= v[c] != 0.f;
            }
            if (any) flush_entry(G, B, A, job, B.keys[st + bstart + tid], v, pose);
        }
        __syncthreads();
    }
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        const float sv = wave_sum(pose[c]);
        if (lane == 0) s_pose[wave][c] = sv;
    }
    __syncthreads();
    if (tid < 6) {
        float acc = 0.f;
        for (int w = 0; w < NW; ++w) acc += s_pose[w][tid];
        A.pose_part[(size_t)item * 6 + tid] = acc;
    }
}

// Sum the per-tile pose partials of each job in FP64.
__global__ __launch_bounds__(256) void k_pose_reduce(const float* part, int ntiles, float* d_pose) {
    __shared__ double s[256][6];
    const int job = blockIdx.x;
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int t = threadIdx.x; t < ntiles; t += blockDim.x)
        for (int c = 0; c < 6; ++c) acc[c] += (double)part[((size_t)job * ntiles + t) * 6 + c];
    for (int c = 0; c < 6; ++c) s[threadIdx.x][c] = acc[c];
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int c = 0; c < 6; ++c) s[threadIdx.x][c] += s[threadIdx.x + w][c];
        __syncthreads();
    }
    if (threadIdx.x < 6) d_pose[job * 6 + threadIdx.x] = (float)s[0][threadIdx.x];
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
template <int TW, int TH>
static void fwd_t(const Geometry& G, const RenderBufs& B, const FwdOut& O, hipStream_t s) {
    hipLaunchKernelGGL((k_fwd<TW, TH>), dim3(G.n_jobs * G.ntiles), dim3(TW * TH), 0, s, G, B, O);
}

template <int TW, int TH>
static void bwd_t(const Geometry& G, const RenderBufs& B, const BwdArgs& A, hipStream_t s) {
    hipLaunchKernelGGL((k_bwd<TW, TH>), dim3(G.n_jobs * G.ntiles), dim3(TW * TH), 0, s, G, B, A);
}

bool launch_fwd8(const Geometry& G, const RenderBufs& B, const FwdOut& O, int sch, hipStream_t s);
bool launch_bwd8(const Geometry& G, const RenderBufs& B, const BwdArgs& A, int sc, hipStream_t s);

bool launch_fwd(const Geometry& G, const RenderBufs& B, float* rgb, float* depth, float* alpha, int32_t* count,
                hipStream_t s) {
    FwdOut O{rgb, depth, alpha, count};
    if (G.TW == 8 && G.TH == 8) return launch_fwd8(G, B, O, G.sc_fwd, s);
    else if (G.TW == 16 && G.TH == 8) fwd_t<16, 8>(G, B, O, s);
    else if (G.TW == 16 && G.TH == 16) fwd_t<16, 16>(G, B, O, s);
    else if (G.TW == 32 && G.TH == 8) fwd_t<32, 8>(G, B, O, s);
    else return false;
    return true;
}

bool launch_bwd(const Geometry& G, const RenderBufs& B, const float* g_rgb, const float* g_depth,
                const float* g_alpha, const KfGradPtrs* grads, uint32_t lo, uint32_t hi, float* pose_part,
                float* acc, float* d_pose, hipStream_t s) {
    BwdArgs A{g_rgb, g_depth, g_alpha, grads, lo, hi, pose_part, acc};
    // 8x8: the pose sums and the gradient records are finished by
    // launch_bwd_finish, which the caller launches next
    if (G.TW == 8 && G.TH == 8) return launch_bwd8(G, B, A, G.sc_bwd, s);
    else if (G.TW == 16 && G.TH == 8) bwd_t<16, 8>(G, B, A, s);
    else if (G.TW == 16 && G.TH == 16) bwd_t<16, 16>(G, B, A, s);
    else if (G.TW == 32 && G.TH == 8) bwd_t<32, 8>(G, B, A, s);
    else return false;
    if (d_pose) hipLaunchKernelGGL(k_pose_reduce, dim3(G.n_jobs), dim3(256), 0, s, pose_part, G.ntiles, d_pose);
    return true;
}

}  // namespace sgad
