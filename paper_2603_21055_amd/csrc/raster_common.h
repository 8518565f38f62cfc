// Device helpers shared by every compositing kernel.  The forward and
// backward of every variant evaluate a (pixel, Gaussian) pair through these
// functions, so their contribution decisions (q <= 9, alpha >= 1/255, the
// 0.99 clamp) agree bit for bit.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

#include "sgad_internal.h"

namespace sgad {

// First workgroup of a forward: hand the call's status to the host (pinned
// memory, read after the call's completion event) and clear the flags that
// the count and scatter passes raise, so that the next call on this slot
// starts clean.  No kernel of the forward reads those flags.
__device__ __forceinline__ void publish_status(const RenderBufs& B) {
    if (B.status_host == nullptr || blockIdx.x != 0) return;
    constexpr unsigned kWords = sizeof(DevStatus) / 4;
    const unsigned t = threadIdx.x;
    if (t < kWords) {
        uint32_t* st = reinterpret_cast<uint32_t*>(B.status);
        B.status_host[t] = st[t];
        if (t == offsetof(DevStatus, nonfinite) / 4 || t == offsetof(DevStatus, sticky) / 4) st[t] = 0u;
    }
}

// -0.5 * log2(e): exp(-q/2) = 2^(q * kNegHalfLog2e)
constexpr float kNegHalfLog2e = -0.72134752044448170368f;

// q = a dx^2 + 2 b dx dy + c dy^2 in a fixed sequence (no contraction left
// to the compiler).
__device__ __forceinline__ float pair_q(float dx, float dy, float a, float b, float c) {
#pragma clang fp contract(off)
    const float t = __builtin_fmaf(b + b, dy, a * dx);
    return __builtin_fmaf(dx, t, (c * dy) * dy);
}

// The same with the conic's b given doubled (b2 = b + b, an exact product,
// so the result is bit for bit pair_q's); the wave-tile walks stage b2.
__device__ __forceinline__ float pair_q2b(float dx, float dy, float a, float b2, float c) {
#pragma clang fp contract(off)
    const float t = __builtin_fmaf(b2, dy, a * dx);
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
    const float* g_rgb;       // [n_jobs][3][P]
    const float* g_depth;     // [n_jobs][P] or null
    const float* g_alpha;     // [n_jobs][P] or null
    const KfGradPtrs* grads;  // [n_kf]
    uint32_t learn_lo, learn_hi;
    float* pose_part;         // [n_jobs * ntiles][6]
    // 8x8 adjoint: per keyframe Gaussian gid = kf * N + pix, 8 floats at
    // acc[8 gid] (offset, radius, opacity, r, g, b, unused, unused) that the
    // tiles add their shares to, moved into the gradient planes afterwards;
    // null: the shares go straight to the planes
    float* acc;
};

// Keyframe of a Gaussian id gid = kf * N + pix.  (gid + 1/2) / N has its
// fractional part at least 1/(2N) >= 2^-32 away from an integer; gid + 1/2 is
// exact in FP64 and the rounding of 1/N and of the product move the quotient
// (below 64) by less than 2^-45, so truncation gives the integer quotient.
__device__ __forceinline__ int kf_of_gid(const Geometry& G, uint32_t gid) {
    return (int)(((double)gid + 0.5) * G.inv_n);
}

// Record of the instance `key` of job `job`.
__device__ __forceinline__ const float4* entry_record(const Geometry& G, const RenderBufs& B, int job,
                                                      uint64_t key) {
    const uint32_t gid = (uint32_t)key;
    const int kf = kf_of_gid(G, gid);
    const int pix = (int)(gid - (uint32_t)kf * (uint32_t)G.N);
    const int pair = B.pair_of[job * G.n_kf + kf];
    return B.pre.rec + 4 * ((size_t)pair * G.N + pix);
}

// Device-scope float add on global memory, without return.  The pointer is
// taken as a global address so the atomic counts only against the vector
// memory counter (a generic-address atomic also holds the LDS counter, which
// every LDS wait would then wait on).
__device__ __forceinline__ void global_add(float* p, float v) {
    using gfloat = __attribute__((address_space(1))) float;
    __hip_atomic_fetch_add((gfloat*)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Chain rule of one (Gaussian, tile) gradient to the keyframe parameters and
// the view pose.  v = [g_mx, g_my, g_a, g_b, g_c, g_o, g_z, g_c0, g_c1, g_c2];
// (fx, fy) the view's focal lengths, z the view depth, r3 = [x, y, r, sign]
// and d the offset direction of the Gaussian's preprocessed data.  Adds the
// pose term to `pose`; for a learnable keyframe writes the parameter
// gradients (offset, radius, opacity, r, g, b) to out and returns true.
__device__ __forceinline__ bool chain_rule_vals(const BwdArgs& A, float fx, float fy, int kf, float z, float4 r3,
                                                float4 d, const float* v, float* pose, float* out) {
    const float x = r3.x, y = r3.y;
    const float r = r3.z;
    // hardware reciprocals (about 1 ulp), far inside the FP32 rounding of the
    // per-entry sums these gradients are formed from
    const float iz = __builtin_amdgcn_rcpf(z), iz2 = iz * iz, iz3 = iz2 * iz, iz4 = iz2 * iz2, iz5 = iz4 * iz;
    const float tx = x * iz, ty = y * iz, jx = fx * iz, jy = fy * iz;
    const float k00 = jx * jx * (1.f + tx * tx), k01 = jx * jy * (tx * ty), k11 = jy * jy * (1.f + ty * ty);
    const float r2 = r * r;
    const float s00 = r2 * k00 + (float)kLowpass, s01 = r2 * k01, s11 = r2 * k11 + (float)kLowpass;
    const float idet = __builtin_amdgcn_rcpf(s00 * s11 - s01 * s01);
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
    if (!learn) return false;
    out[0] = gx * d.x + gy * d.y + gz * d.z;
    out[1] = g_r;
    out[2] = v[5];
    out[3] = v[7];
    out[4] = v[8];
    out[5] = v[9];
    return true;
}

// The same, adding the parameter gradients to the keyframe's gradient planes.
__device__ __forceinline__ void chain_rule(const Geometry& G, const BwdArgs& A, float fx, float fy, int kf,
                                           int pix, float z, float4 r3, float4 d, const float* v, float* pose) {
    float o[6];
    if (!chain_rule_vals(A, fx, fy, kf, z, r3, d, v, pose, o)) return;
    const KfGradPtrs gp = A.grads[kf];
    global_add(&gp.d_offset[pix], o[0]);
    global_add(&gp.d_radius[pix], o[1]);
    global_add(&gp.d_opacity[pix], o[2]);
    global_add(&gp.d_rgb[pix], o[3]);
    global_add(&gp.d_rgb[(size_t)G.N + pix], o[4]);
    global_add(&gp.d_rgb[2 * (size_t)G.N + pix], o[5]);
}

// The same, reading the record of the instance `key` of job `job`.
__device__ __forceinline__ void flush_entry(const Geometry& G, const RenderBufs& B, const BwdArgs& A, int job,
                                            uint64_t key, const float* v, float* pose) {
    const uint32_t gid = (uint32_t)key;
    const int kf = kf_of_gid(G, gid);
    const int pix = (int)(gid - (uint32_t)kf * (uint32_t)G.N);
    const int pair = B.pair_of[job * G.n_kf + kf];
    const size_t i = (size_t)pair * G.N + pix;
    const float4* rec = B.pre.rec + 4 * i;
    const PairConst& pc = B.pairs[pair];
    chain_rule(G, A, (float)pc.vfx, (float)pc.vfy, kf, pix, rec[2].w, rec[3], B.pre.dir[i], v, pose);
}

// Spread consecutive workgroups over the XCDs in contiguous ranges: the
// hardware hands out workgroup ids round-robin to the 8 XCDs, so a workgroup
// on XCD x with local index k is given the k-th item of XCD x's range and
// neighbouring tiles (which share Gaussians) meet in the same L2.
__device__ __forceinline__ int xcd_remap(int b, int nb) {
    const int q = nb >> 3, r = nb & 7;
    const int x = b & 7, k = b >> 3;
    const int base = x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q;
    return base + k;
}

// Order one wavefront's LDS accesses around this point (workgroups of one
// wavefront: no other wave shares the LDS data): the compiler may not move
// memory accesses across it, and the wave waits for its outstanding LDS
// operations.  Global memory operations are not waited for.
__device__ __forceinline__ void wave_lds_sync() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }

}  // namespace sgad
