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

#include "sgad_internal.h"

namespace sgad {

// -0.5 * log2(e): exp(-q/2) = 2^(q * kNegHalfLog2e)
constexpr float kNegHalfLog2e = -0.72134752044448170368f;

// q = a dx^2 + 2 b dx dy + c dy^2 with a fixed, unfused-by-the-compiler
// sequence; forward and backward call the same function so their
// contribution decisions agree bit for bit.
__device__ __forceinline__ float pair_q(float dx, float dy, float a, float b, float c) {
#pragma clang fp contract(off)
    const float t = __builtin_fmaf(b + b, dy, a * dx);
    return __builtin_fmaf(dx, t, (c * dy) * dy);
}

__device__ __forceinline__ float gauss_of_q(float q) {
#pragma clang fp contract(off)
    return __builtin_amdgcn_exp2f(q * kNegHalfLog2e);
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

struct FwdOut {
    float* rgb;      // [n_jobs][3][P]
    float* depth;    // [n_jobs][P]
    float* alpha;    // [n_jobs][P]
    int32_t* count;  // [n_jobs][P] or null
};

struct BwdArgs {
    const float* g_rgb;    // [n_jobs][3][P]
    const float* g_depth;  // [n_jobs][P] or null
    const float* g_alpha;  // [n_jobs][P] or null
    const KfGradPtrs* grads;  // [n_kf]
    uint32_t learn_lo, learn_hi;
    float* pose_part;      // [n_jobs * ntiles][6]
};

// Stage one instance: source pixel (u, v) and screen displacement of the
// mean, conic, opacity, depth and colour.  A pixel's offset from the mean is
// formed as (p - (u, v)) - displacement: the integer part is exact, so the
// only rounding is the last subtraction and the result does not depend on
// the tile the pixel belongs to.
__device__ __forceinline__ void load_entry(const Geometry& G, const RenderBufs& B, int job, uint64_t key,
                                           float4& eu, float4& eg, float4& ec) {
    const uint32_t gid = (uint32_t)key;
    const int kf = (int)(gid / (uint32_t)G.N);
    const int pix = (int)(gid - (uint32_t)kf * (uint32_t)G.N);
    const int pair = B.pair_of[job * G.n_kf + kf];
    const size_t idx = (size_t)pair * G.N + pix;
    const int u = pix % G.Wk, v = pix / G.Wk;
    const KfPtrs kp = B.kfs[kf];
    eu = make_float4((float)u, (float)v, B.pre.dx[idx], B.pre.dy[idx]);
    eg = make_float4(B.pre.ca[idx], B.pre.cb[idx], B.pre.cc[idx], kp.opacity[pix]);
    if (kp.rgb)
        ec = make_float4(kp.rgb[pix], kp.rgb[(size_t)G.N + pix], kp.rgb[2 * (size_t)G.N + pix], B.pre.z[idx]);
    else {
        const float sg = kp.sigma ? kp.sigma[pix] : 0.f;
        ec = make_float4(sg * sg, 0.f, 0.f, B.pre.z[idx]);
    }
}

template <int TW, int TH>
__global__ __launch_bounds__(TW* TH) void k_fwd(Geometry G, RenderBufs B, FwdOut O) {
    constexpr int NT = TW * TH;
    __shared__ float4 s_u[NT], s_g[NT], s_c[NT];
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

// Chain rule of one (Gaussian, tile) gradient to the keyframe parameters and
// the view pose (recomputes the view-space geometry in FP32).
// v = [g_mx, g_my, g_a, g_b, g_c, g_o, g_z, g_r, g_g, g_b]
__device__ __forceinline__ void flush_entry(const Geometry& G, const RenderBufs& B, const BwdArgs& A,
                                            int job, uint64_t key, const float* v, float* pose) {
    const uint32_t gid = (uint32_t)key;
    const int kf = (int)(gid / (uint32_t)G.N);
    const int pix = (int)(gid - (uint32_t)kf * (uint32_t)G.N);
    const int pair = B.pair_of[job * G.n_kf + kf];
    const PairConst& pc = B.pairs[pair];
    const KfPtrs kp = B.kfs[kf];
    const int u = pix % G.Wk, vv = pix / G.Wk;
    const float s = kp.depth[pix] + kp.offset[pix];
    const float d = fabsf(s);
    const float sgn = s >= 0.f ? 1.f : -1.f;
    const float r = kp.radius[pix];
    const float xn = ((float)u - (float)pc.kcx) / (float)pc.kfx;
    const float yn = ((float)vv - (float)pc.kcy) / (float)pc.kfy;
    const float X0 = d * xn, X1 = d * yn, X2 = d;
    const float* R = pc.Rf;
    const float x = R[0] * X0 + R[1] * X1 + R[2] * X2 + pc.tf[0];
    const float y = R[3] * X0 + R[4] * X1 + R[5] * X2 + pc.tf[1];
    const float z = R[6] * X0 + R[7] * X1 + R[8] * X2 + pc.tf[2];
    const float fx = (float)pc.vfx, fy = (float)pc.vfy;
    const float iz = 1.f / z, iz2 = iz * iz, iz3 = iz2 * iz, iz4 = iz2 * iz2, iz5 = iz4 * iz;
    const float tx = x * iz, ty = y * iz, jx = fx * iz, jy = fy * iz;
    const float k00 = jx * jx * (1.f + tx * tx), k01 = jx * jy * (tx * ty), k11 = jy * jy * (1.f + ty * ty);
    const float r2 = r * r;
    const float s00 = r2 * k00 + (float)kLowpass, s01 = r2 * k01, s11 = r2 * k11 + (float)kLowpass;
    const float idet = 1.f / (s00 * s11 - s01 * s01);
    const float q00 = s11 * idet, q01 = -s01 * idet, q11 = s00 * idet;
    const float ga = v[2], hb = 0.5f * v[3], gc = v[4];
    const float m00 = ga * q00 + hb * q01, m01 = ga * q01 + hb * q11;
    const float m10 = hb * q00 + gc * q01, m11 = hb * q01 + gc * q11;
    const float gs00 = -(q00 * m00 + q01 * m10);
    const float gs01 = -2.f * (q00 * m01 + q01 * m11);
    const float gs11 = -(q01 * m01 + q11 * m11);
    const float g_r = 2.f * r * (gs00 * k00 + gs01 * k01 + gs11 * k11);
    float gx = r2 * (gs00 * 2.f * fx * fx * x * iz4 + gs01 * fx * fy * y * iz4);
    float gy = r2 * (gs01 * fx * fy * x * iz4 + gs11 * 2.f * fy * fy * y * iz4);
    float gz = r2 * (gs00 * fx * fx * (-2.f * iz3 - 4.f * x * x * iz5) + gs01 * (-4.f * fx * fy * x * y * iz5) +
                     gs11 * fy * fy * (-2.f * iz3 - 4.f * y * y * iz5));
    gx += v[0] * fx * iz;
    gy += v[1] * fy * iz;
    gz += -v[0] * fx * x * iz2 - v[1] * fy * y * iz2 + v[6];
    pose[0] += gx;
    pose[1] += gy;
    pose[2] += gz;
    pose[3] += y * gz - z * gy;
    pose[4] += z * gx - x * gz;
    pose[5] += x * gy - y * gx;
    const bool learn = kf < 32 ? ((A.learn_lo >> kf) & 1u) : ((A.learn_hi >> (kf - 32)) & 1u);
    if (!learn) return;
    const float gxf = R[0] * gx + R[3] * gy + R[6] * gz;
    const float gyf = R[1] * gx + R[4] * gy + R[7] * gz;
    const float gzf = R[2] * gx + R[5] * gy + R[8] * gz;
    const float g_off = (gxf * xn + gyf * yn + gzf) * sgn;
    const KfGradPtrs gp = A.grads[kf];
    atomicAdd(&gp.d_offset[pix], g_off);
    atomicAdd(&gp.d_radius[pix], g_r);
    atomicAdd(&gp.d_opacity[pix], v[5]);
    atomicAdd(&gp.d_rgb[pix], v[7]);
    atomicAdd(&gp.d_rgb[(size_t)G.N + pix], v[8]);
    atomicAdd(&gp.d_rgb[2 * (size_t)G.N + pix], v[9]);
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

bool launch_fwd(const Geometry& G, const RenderBufs& B, float* rgb, float* depth, float* alpha, int32_t* count,
                hipStream_t s) {
    FwdOut O{rgb, depth, alpha, count};
    if (G.TW == 8 && G.TH == 8) fwd_t<8, 8>(G, B, O, s);
    else if (G.TW == 16 && G.TH == 8) fwd_t<16, 8>(G, B, O, s);
    else if (G.TW == 16 && G.TH == 16) fwd_t<16, 16>(G, B, O, s);
    else if (G.TW == 32 && G.TH == 8) fwd_t<32, 8>(G, B, O, s);
    else return false;
    return true;
}

bool launch_bwd(const Geometry& G, const RenderBufs& B, const float* g_rgb, const float* g_depth,
                const float* g_alpha, const KfGradPtrs* grads, uint32_t lo, uint32_t hi, float* pose_part,
                float* d_pose, hipStream_t s) {
    BwdArgs A{g_rgb, g_depth, g_alpha, grads, lo, hi, pose_part};
    if (G.TW == 8 && G.TH == 8) bwd_t<8, 8>(G, B, A, s);
    else if (G.TW == 16 && G.TH == 8) bwd_t<16, 8>(G, B, A, s);
    else if (G.TW == 16 && G.TH == 16) bwd_t<16, 16>(G, B, A, s);
    else if (G.TW == 32 && G.TH == 8) bwd_t<32, 8>(G, B, A, s);
    else return false;
    if (d_pose) hipLaunchKernelGGL(k_pose_reduce, dim3(G.n_jobs), dim3(256), 0, s, pose_part, G.ntiles, d_pose);
    return true;
}

}  // namespace sgad
