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

// Count the valid target-depth pixels (U = [D > 0]) of every job.
__global__ __launch_bounds__(256) void k_count_valid(const float* __restrict__ t_depth, int P, uint32_t* count) {
    const int job = blockIdx.y;
    uint32_t c = 0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < P; i += gridDim.x * blockDim.x)
        c += t_depth[(size_t)job * P + i] > 0.f ? 1u : 0u;
    c = wave_sum_u(c);
    __shared__ uint32_t s_c[4];
    if ((threadIdx.x & 63) == 0) s_c[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t t = s_c[0] + s_c[1] + s_c[2] + s_c[3];
        if (t) atomicAdd(&count[job], t);
    }
}

// Loss value and upstream grads:
//   L = w_rgb mean|rgb - t_rgb| + w_depth sum_U |D' - D_t| / |U|
__global__ __launch_bounds__(256) void k_l1(const float* __restrict__ rgb, const float* __restrict__ dep,
                                            const float* __restrict__ t_rgb, const float* __restrict__ t_dep,
                                            int P, float w_rgb, float w_dep, const uint32_t* count,
                                            float* g_rgb, float* g_dep, double* loss) {
    const int job = blockIdx.y;
    const uint32_t nv = count[job];
    const float inv_rgb = w_rgb / (3.f * (float)P);
    const float inv_dep = nv ? w_dep / (float)nv : 0.f;
    double acc = 0.0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < P; i += gridDim.x * blockDim.x) {
        const size_t jp = (size_t)job * P + i;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const size_t k = ((size_t)job * 3 + c) * P + i;
            const float e = rgb[k] - t_rgb[k];
            acc += (double)(fabsf(e) * inv_rgb);
            g_rgb[k] = signf(e) * inv_rgb;
        }
        const float td = t_dep[jp];
        const float e = td > 0.f ? dep[jp] - td : 0.f;
        acc += (double)(fabsf(e) * inv_dep);
        g_dep[jp] = signf(e) * inv_dep;
    }
    acc = wave_sum_d(acc);
    __shared__ double s_a[4];
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

__global__ __launch_bounds__(256) void k_adam(AdamGroups A, float b1, float b2, float eps, float c1, float c2,
                                              int zero_grad, const float* cdev) {
    if (cdev) {
        c1 = cdev[1];
        c2 = cdev[2];
    }
    const int64_t total = A.off[A.n];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        int gi = 0;
        while (gi + 1 < A.n && i >= A.off[gi + 1]) ++gi;
        const int64_t k = i - A.off[gi];
        const int sp = A.space[gi];
        float p = A.p[gi][k];
        float g = A.g[gi][k];
        float th = p;
        if (sp == 1) {
            p = fmaxf(p, 1e-12f);
            th = logf(p);
            g *= p;
        } else if (sp == 2) {
            p = fminf(fmaxf(p, 1e-6f), 1.f - 1e-6f);
            th = logf(p / (1.f - p));
            g *= p * (1.f - p);
        }
        const float m = b1 * A.m[gi][k] + (1.f - b1) * g;
        const float v = b2 * A.v[gi][k] + (1.f - b2) * g * g;
        A.m[gi][k] = m;
        A.v[gi][k] = v;
        const float mh = m / c1, vh = v / c2;
        th -= A.lr[gi] * mh / (sqrtf(vh) + eps);
        if (sp == 1) p = expf(th);
        else if (sp == 2) p = 1.f / (1.f + expf(-th));
        else p = th;
        p = fminf(fmaxf(p, A.lo[gi]), A.hi[gi]);
        A.p[gi][k] = p;
        if (zero_grad) A.g[gi][k] = 0.f;
    }
}

void launch_l1(int n_jobs, int P, const float* rgb, const float* dep, const float* t_rgb, const float* t_dep,
               float w_rgb, float w_dep, uint32_t* count, float* g_rgb, float* g_dep, double* loss,
               hipStream_t s) {
    const int bx = std::min(128, (P + 255) / 256);
    hipLaunchKernelGGL(k_count_valid, dim3(bx, n_jobs), dim3(256), 0, s, t_dep, P, count);
    hipLaunchKernelGGL(k_l1, dim3(bx, n_jobs), dim3(256), 0, s, rgb, dep, t_rgb, t_dep, P, w_rgb, w_dep, count,
                       g_rgb, g_dep, loss);
}

// cdev null: bias corrections c1, c2 as given; else advance the device
// counter cdev and take them from it.
void launch_adam(const AdamGroups& A, float b1, float b2, float eps, float c1, float c2, int zero_grad,
                 float* cdev, hipStream_t s) {
    const int64_t total = A.off[A.n];
    if (total <= 0) return;
    if (cdev) hipLaunchKernelGGL(k_adam_tick, dim3(1), dim3(64), 0, s, cdev, b1, b2);
    const int blocks = (int)std::min<int64_t>((total + 255) / 256, 8192);
    hipLaunchKernelGGL(k_adam, dim3(blocks), dim3(256), 0, s, A, b1, b2, eps, c1, c2, zero_grad,
                       (const float*)cdev);
}

}  // namespace sgad
