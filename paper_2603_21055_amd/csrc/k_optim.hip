// L1 terms of the mapping loss (Eq. 1) with their upstream gradients, and a
// multi-tensor Adam step over the per-pixel Gaussian parameters.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "sgad_internal.h"

namespace sgad {

__device__ __forceinline__ float signf(float x) { return x > 0.f ? 1.f : (x < 0.f ? -1.f : 0.f); }

__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ uint32_t wave_sum_u(uint32_t v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Count the valid target-depth pixels (U = [D > 0]) of every job: each
// block writes its partial count (no atomics, nothing to clear first); block
// 0 of a job also clears the job's loss accumulator.  VEC: four pixels per
// thread as one 16-byte load (P divisible by 4, aligned planes).
template <bool VEC>
__global__ __launch_bounds__(256) void k_count_valid(const float* __restrict__ t_depth, int P,
                                                     uint32_t* __restrict__ part, double* loss) {
    const int job = blockIdx.y;
    const float* td = t_depth + (size_t)job * P;
    const int i0 = blockIdx.x * 1024;
    uint32_t c = 0;
    if (VEC) {
        const int i = i0 + 4 * (int)threadIdx.x;
        if (i < P) {
            const float4 d = *reinterpret_cast<const float4*>(td + i);
            c = (d.x > 0.f ? 1u : 0u) + (d.y > 0.f ? 1u : 0u) + (d.z > 0.f ? 1u : 0u) + (d.w > 0.f ? 1u : 0u);
        }
    } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int i = i0 + j * 256 + (int)threadIdx.x;
            if (i < P) c += td[i] > 0.f ? 1u : 0u;
        }
    }
    c = wave_sum_u(c);
    __shared__ uint32_t s_c[4];
    if ((threadIdx.x & 63) == 0) s_c[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        part[(size_t)job * gridDim.x + blockIdx.x] = s_c[0] + s_c[1] + s_c[2] + s_c[3];
        if (blockIdx.x == 0) loss[job] = 0.0;
    }
}

// One pixel's loss terms and upstream gradients.
__device__ __forceinline__ double l1_pixel(float r0, float r1, float r2, float d, float t0, float t1, float t2,
                                           float td, float inv_rgb, float inv_dep, float& g0, float& g1,
                                           float& g2, float& gd) {
    const float e0 = r0 - t0, e1 = r1 - t1, e2 = r2 - t2;
    const float ed = td > 0.f ? d - td : 0.f;
    g0 = signf(e0) * inv_rgb;
    g1 = signf(e1) * inv_rgb;
    g2 = signf(e2) * inv_rgb;
    gd = signf(ed) * inv_dep;
    return (double)(fabsf(e0) * inv_rgb) + (double)(fabsf(e1) * inv_rgb) + (double)(fabsf(e2) * inv_rgb) +
           (double)(fabsf(ed) * inv_dep);
}

// Loss value and upstream grads:
//   L = w_rgb mean|rgb - t_rgb| + w_depth sum_U |D' - D_t| / |U|
// Same grid as k_count_valid; each block first sums the job's nparts partial
// counts (k_count_valid's per block, or the SSIM maps' per tile).
template <bool VEC>
__global__ __launch_bounds__(256) void k_l1(const float* __restrict__ rgb, const float* __restrict__ dep,
                                            const float* __restrict__ t_rgb, const float* __restrict__ t_dep,
                                            int P, float w_rgb, float w_dep, const uint32_t* __restrict__ part,
                                            int nparts, float* __restrict__ g_rgb, float* __restrict__ g_dep,
                                            double* loss) {
    const int job = blockIdx.y;
    __shared__ uint32_t s_c[4];
    __shared__ double s_a[4];
    const size_t jp = (size_t)job * P, j3 = (size_t)job * 3 * P;
    const int i0 = blockIdx.x * 1024;
    // VEC: the thread's four pixels are loaded first, so that their loads
    // and those of the depth counts are in flight together
    const int iv = i0 + 4 * (int)threadIdx.x;
    const bool vin = VEC && iv < P;
    float4 r[3], t[3], d, td;
    if (vin) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            r[c] = *reinterpret_cast<const float4*>(rgb + j3 + (size_t)c * P + iv);
            t[c] = *reinterpret_cast<const float4*>(t_rgb + j3 + (size_t)c * P + iv);
        }
        d = *reinterpret_cast<const float4*>(dep + jp + iv);
        td = *reinterpret_cast<const float4*>(t_dep + jp + iv);
    }
    {
        // eight count loads in flight per thread before any is waited on
        uint32_t c = 0;
        const uint32_t* pj = part + (size_t)job * nparts;
        for (int k0 = 0; k0 < nparts; k0 += 256 * 8) {
            uint32_t v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int k = k0 + u * 256 + (int)threadIdx.x;
                v[u] = k < nparts ? pj[k] : 0u;
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) c += v[u];
        }
        c = wave_sum_u(c);
        if ((threadIdx.x & 63) == 0) s_c[threadIdx.x >> 6] = c;
        __syncthreads();
    }
    const uint32_t nv = s_c[0] + s_c[1] + s_c[2] + s_c[3];
    const float inv_rgb = w_rgb / (3.f * (float)P);
    const float inv_dep = nv ? w_dep / (float)nv : 0.f;
    double acc = 0.0;
    if (VEC) {
        if (vin) {
            float4 g[3], gd;
            acc += l1_pixel(r[0].x, r[1].x, r[2].x, d.x, t[0].x, t[1].x, t[2].x, td.x, inv_rgb, inv_dep, g[0].x,
                            g[1].x, g[2].x, gd.x);
            acc += l1_pixel(r[0].y, r[1].y, r[2].y, d.y, t[0].y, t[1].y, t[2].y, td.y, inv_rgb, inv_dep, g[0].y,
                            g[1].y, g[2].y, gd.y);
            acc += l1_pixel(r[0].z, r[1].z, r[2].z, d.z, t[0].z, t[1].z, t[2].z, td.z, inv_rgb, inv_dep, g[0].z,
                            g[1].z, g[2].z, gd.z);
            acc += l1_pixel(r[0].w, r[1].w, r[2].w, d.w, t[0].w, t[1].w, t[2].w, td.w, inv_rgb, inv_dep, g[0].w,
                            g[1].w, g[2].w, gd.w);
#pragma unroll
            for (int c = 0; c < 3; ++c) *reinterpret_cast<float4*>(g_rgb + j3 + (size_t)c * P + iv) = g[c];
            *reinterpret_cast<float4*>(g_dep + jp + iv) = gd;
        }
    } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int i = i0 + j * 256 + (int)threadIdx.x;
            if (i < P) {
                float g0, g1, g2, gd;
                acc += l1_pixel(rgb[j3 + i], rgb[j3 + P + i], rgb[j3 + 2 * (size_t)P + i], dep[jp + i],
                                t_rgb[j3 + i], t_rgb[j3 + P + i], t_rgb[j3 + 2 * (size_t)P + i], t_dep[jp + i],
                                inv_rgb, inv_dep, g0, g1, g2, gd);
                g_rgb[j3 + i] = g0;
                g_rgb[j3 + P + i] = g1;
                g_rgb[j3 + 2 * (size_t)P + i] = g2;
                g_dep[jp + i] = gd;
            }
        }
    }
    acc = wave_sum_d(acc);
    if ((threadIdx.x & 63) == 0) s_a[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(&loss[job], s_a[0] + s_a[1] + s_a[2] + s_a[3]);
}

// Multi-tensor Adam: group g owns elements [off[g], off[g+1]) of the flat range.

// Step counter of a replayed Adam: t += 1 and the bias corrections
// 1 - beta^t, so every replay of a captured step takes the next t.
// state = [t (int bits), c1, c2, unused].
__global__ void k_adam_tick(float* state, float b1, float b2) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const int t = __float_as_int(state[0]) + 1;
    state[0] = __int_as_float(t);
    state[1] = (float)(1.0 - pow((double)b1, (double)t));
    state[2] = (float)(1.0 - pow((double)b2, (double)t));
}

// One element: the update takes place in the group's space (identity, log or
// logit), with the gradient carried through the space's derivative.
__device__ __forceinline__ void adam_one(float& p, float& g, float& m, float& v, int sp, float lr, float lo,
                                         float hi, float b1, float b2, float eps, float c1, float c2,
                                         int zero_grad) {
    float th = p, gg = g;
    if (sp == 1) {
        p = fmaxf(p, 1e-12f);
        th = logf(p);
        gg *= p;
    } else if (sp == 2) {
        p = fminf(fmaxf(p, 1e-6f), 1.f - 1e-6f);
        th = logf(p / (1.f - p));
        gg *= p * (1.f - p);
    }
    m = b1 * m + (1.f - b1) * gg;
    v = b2 * v + (1.f - b2) * gg * gg;
    const float mh = m / c1, vh = v / c2;
    th -= lr * mh / (sqrtf(vh) + eps);
    if (sp == 1) p = expf(th);
    else if (sp == 2) p = 1.f / (1.f + expf(-th));
    else p = th;
    p = fminf(fmaxf(p, lo), hi);
    if (zero_grad) g = 0.f;
}

// Each block updates 1024 consecutive elements of one group (blocks
// [boff[g], boff[g+1]) belong to group g), so the group's pointers, space
// and hyper-parameters are uniform over the block; groups whose four arrays
// are 16-byte aligned are read and written as float4.
__global__ __launch_bounds__(256) void k_adam(AdamGroups A, float b1, float b2, float eps, float c1, float c2,
                                              int zero_grad, const float* cdev) {
    if (cdev) {
        c1 = cdev[1];
        c2 = cdev[2];
    }
    int gi = 0;
    while (gi + 1 < A.n && (int)blockIdx.x >= A.boff[gi + 1]) ++gi;
    const int64_t n = A.off[gi + 1] - A.off[gi];
    const int64_t b0 = (int64_t)((int)blockIdx.x - A.boff[gi]) * 1024;
    float* P = A.p[gi];
    float* Gr = A.g[gi];
    float* M = A.m[gi];
    float* V = A.v[gi];
    const int sp = A.space[gi];
    const float lr = A.lr[gi], lo = A.lo[gi], hi = A.hi[gi];
    const int64_t k = b0 + 4 * (int64_t)threadIdx.x;
    if (A.vec[gi] && k + 3 >= n) {
        // ragged end of an aligned group: this thread's last < 4 elements
        for (int64_t i = k; i < n; ++i) {
            float p = P[i], g = Gr[i], m = M[i], v = V[i];
            adam_one(p, g, m, v, sp, lr, lo, hi, b1, b2, eps, c1, c2, zero_grad);
            P[i] = p;
            M[i] = m;
            V[i] = v;
            if (zero_grad) Gr[i] = g;
        }
        return;
    }
    if (A.vec[gi]) {
        float4 p = *reinterpret_cast<const float4*>(P + k);
        float4 g = *reinterpret_cast<const float4*>(Gr + k);
        float4 m = *reinterpret_cast<const float4*>(M + k);
        float4 v = *reinterpret_cast<const float4*>(V + k);
        adam_one(p.x, g.x, m.x, v.x, sp, lr, lo, hi, b1, b2, eps, c1, c2, zero_grad);
        adam_one(p.y, g.y, m.y, v.y, sp, lr, lo, hi, b1, b2, eps, c1, c2, zero_grad);
        adam_one(p.z, g.z, m.z, v.z, sp, lr, lo, hi, b1, b2, eps, c1, c2, zero_grad);
        adam_one(p.w, g.w, m.w, v.w, sp, lr, lo, hi, b1, b2, eps, c1, c2, zero_grad);
        *reinterpret_cast<float4*>(P + k) = p;
        *reinterpret_cast<float4*>(M + k) = m;
        *reinterpret_cast<float4*>(V + k) = v;
        if (zero_grad) *reinterpret_cast<float4*>(Gr + k) = g;
        return;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int64_t i = b0 + j * 256 + threadIdx.x;
        if (i < n) {
            float p = P[i], g = Gr[i], m = M[i], v = V[i];
            adam_one(p, g, m, v, sp, lr, lo, hi, b1, b2, eps, c1, c2, zero_grad);
            P[i] = p;
            M[i] = m;
            V[i] = v;
            if (zero_grad) Gr[i] = g;
        }
    }
}

// `part` holds one u32 per (job, block): n_jobs * l1_blocks(P) entries.
int l1_blocks(int P) { return (P + 1023) / 1024; }

// nparts 0: count the valid target depths into part first; else part
// already holds nparts counts per job and loss is already cleared.
void launch_l1(int n_jobs, int P, const float* rgb, const float* dep, const float* t_rgb, const float* t_dep,
               float w_rgb, float w_dep, uint32_t* part, int nparts, float* g_rgb, float* g_dep, double* loss,
               hipStream_t s) {
    const dim3 grid(l1_blocks(P), n_jobs);
    auto al = [](const void* q) { return ((uintptr_t)q & 15u) == 0; };
    const bool vec = P % 4 == 0 && al(rgb) && al(dep) && al(t_rgb) && al(t_dep) && al(g_rgb) && al(g_dep);
    const int np = nparts > 0 ? nparts : (int)grid.x;
    if (vec) {
        if (nparts <= 0) hipLaunchKernelGGL(k_count_valid<true>, grid, dim3(256), 0, s, t_dep, P, part, loss);
        hipLaunchKernelGGL(k_l1<true>, grid, dim3(256), 0, s, rgb, dep, t_rgb, t_dep, P, w_rgb, w_dep, part, np,
                           g_rgb, g_dep, loss);
    } else {
        if (nparts <= 0) hipLaunchKernelGGL(k_count_valid<false>, grid, dim3(256), 0, s, t_dep, P, part, loss);
        hipLaunchKernelGGL(k_l1<false>, grid, dim3(256), 0, s, rgb, dep, t_rgb, t_dep, P, w_rgb, w_dep, part, np,
                           g_rgb, g_dep, loss);
    }
}

// cdev null: bias corrections c1, c2 as given; else advance the device
// counter cdev and take them from it.  Fills in the block offsets and the
// alignment flags of A.
void launch_adam(AdamGroups& A, float b1, float b2, float eps, float c1, float c2, int zero_grad,
                 float* cdev, hipStream_t s) {
    auto al = [](const void* q) { return ((uintptr_t)q & 15u) == 0; };
    A.boff[0] = 0;
    for (int g = 0; g < A.n; ++g) {
        const int64_t n = A.off[g + 1] - A.off[g];
        A.boff[g + 1] = A.boff[g] + (int)((n + 1023) / 1024);
        A.vec[g] = al(A.p[g]) && al(A.g[g]) && al(A.m[g]) && al(A.v[g]) ? 1 : 0;
    }
    const int blocks = A.boff[A.n];
    if (blocks <= 0) return;
    if (cdev) hipLaunchKernelGGL(k_adam_tick, dim3(1), dim3(64), 0, s, cdev, b1, b2);
    hipLaunchKernelGGL(k_adam, dim3(blocks), dim3(256), 0, s, A, b1, b2, eps, c1, c2, zero_grad,
                       (const float*)cdev);
}

}  // namespace sgad
