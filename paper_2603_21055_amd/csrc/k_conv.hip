// BF16 3x3 convolutions on MFMA (gfx950 v_mfma_f32_16x16x32_bf16) for the
// offset warm-start net: forward with fused bias + ReLU, input gradient with
// the ReLU mask of the layer input fused, weight and bias gradients.
//
// Activations are NHWC bf16 ([H][W][C], C in {1, 4, 32}); weights are
// [9][Cout][Cin] bf16 (tap-major).  Every product accumulates in FP32.
//
// Implicit GEMM per 16x16 output tile and tap: C[co][pixel] += W[co][ci] *
// X[ci][pixel + tap offset].  Operand layouts of the 16x16x32 MFMA: lane l
// holds A[l % 16][8 (l / 16) .. +8], B[8 (l / 16) .. +8][l % 16] and
// C[4 (l / 16) .. +4][l % 16].
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "sgad_internal.h"

namespace sgad {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));

constexpr int kPS = 40;  // LDS pixel stride (bf16 elements) of the input tile

__device__ __forceinline__ bf16x8 zero8() {
    bf16x8 v;
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = (__bf16)0.f;
    return v;
}

// v clamped into [0, n - 1] (n > 0): a load address that is always in bounds
__device__ __forceinline__ int clampi(int v, int n) { return v < 0 ? 0 : (v >= n ? n - 1 : v); }

// MODE 0: y = relu(conv + bias) as bf16 [H][W][COUT]
// MODE 1: y = conv + bias as f32 [H][W] (COUT == 1)
// MODE 2: y = conv * [mask > 0] as bf16 [H][W][COUT] (input gradient through a ReLU)
//
// Persistent: a workgroup loads the weights once and walks 16x16 output
// tiles; the next tile's 18x18 input patch is loaded into registers while
// the MFMAs of the current tile run.  The patch loads read addresses clamped
// into the image and are zeroed outside it when they are stored to LDS, so
// no load waits at a branch.
template <int CIN, int COUT, int MODE>
__global__ __launch_bounds__(256) void k_conv(int H, int W, const __bf16* __restrict__ x,
                                              const __bf16* __restrict__ w, const float* __restrict__ bias,
                                              const __bf16* __restrict__ mask, void* __restrict__ yout) {
    constexpr int MB = (COUT + 15) / 16;
    constexpr int NCH = CIN == 32 ? 4 : 1;          // 8-channel groups loaded per pixel
    constexpr int L = (324 * NCH + 255) / 256;      // patch loads per thread
    __shared__ __attribute__((aligned(16))) __bf16 s_x[18 * 18 * kPS];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int g = lane >> 4, r16 = lane & 15;
    const int ntx = (W + 15) / 16, ntiles = ntx * ((H + 15) / 16);
    bf16x8 A[9][MB];
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
            const int co = mb * 16 + r16;
            bf16x8 v = zero8();
            if (co < COUT) {
                const __bf16* src = w + ((size_t)t * COUT + co) * CIN;
                if (CIN == 32) {
                    v = *(const bf16x8*)(src + g * 8);
                } else if (g == 0) {
#pragma unroll
                    for (int c = 0; c < CIN; ++c) v[c] = src[c];
                }
            }
            A[t][mb] = v;
        }
    // with fewer than 32 input channels only the first 8-channel group of a
    // pixel is loaded; the other groups stay zero from here on
    if (CIN < 32)
        for (int i = tid; i < 324 * 4; i += 256)
            if ((i & 3) != 0) *(bf16x8*)(s_x + (i >> 2) * kPS + (i & 3) * 8) = zero8();
    bf16x8 xv[L];
    auto load_patch = [&](int tile) {
        const int x0 = (tile % ntx) * 16, y0 = (tile / ntx) * 16;
#pragma unroll
        for (int k = 0; k < L; ++k) {
            const int i = tid + 256 * k, pix = i / NCH, ch = i % NCH;
            const int ty = pix / 18, tx = pix - ty * 18;
            const size_t base = ((size_t)clampi(y0 + ty - 1, H) * W + clampi(x0 + tx - 1, W)) * CIN;
            if (CIN == 32) {
                xv[k] = *(const bf16x8*)(x + base + ch * 8);
            } else if (CIN == 4) {
                const bf16x4 v = *(const bf16x4*)(x + base);
                xv[k] = zero8();
#pragma unroll
                for (int c = 0; c < 4; ++c) xv[k][c] = v[c];
            } else {
                xv[k] = zero8();
#pragma unroll
                for (int c = 0; c < CIN; ++c) xv[k][c] = x[base + c];
            }
        }
    };
    int tile = blockIdx.x;
    if (tile < ntiles) load_patch(tile);
    for (; tile < ntiles; tile += gridDim.x) {
        const int x0 = (tile % ntx) * 16, y0 = (tile / ntx) * 16;
        __syncthreads();   // the previous tile's MFMAs have read s_x
#pragma unroll
        for (int k = 0; k < L; ++k) {
            const int i = tid + 256 * k, pix = i / NCH, ch = i % NCH;
            const int ty = pix / 18, tx = pix - ty * 18;
            const int gy = y0 + ty - 1, gx = x0 + tx - 1;
            const bool in = gy >= 0 && gy < H && gx >= 0 && gx < W;
            if (i < 324 * NCH) *(bf16x8*)(s_x + pix * kPS + ch * 8) = in ? xv[k] : zero8();
        }
        __syncthreads();
        if (tile + (int)gridDim.x < ntiles) load_patch(tile + gridDim.x);
        f32x4 acc[MB][4];
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int nb = 0; nb < 4; ++nb) acc[mb][nb] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            const int ky = t / 3, kx = t - ky * 3;
#pragma unroll
            for (int nb = 0; nb < 4; ++nb) {
                const int ry = wave * 4 + nb + ky, rx = r16 + kx;
                const bf16x8 B = *(const bf16x8*)(s_x + (ry * 18 + rx) * kPS + g * 8);
#pragma unroll
                for (int mb = 0; mb < MB; ++mb)
                    acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[t][mb], B, acc[mb][nb], 0, 0, 0);
            }
        }
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) {
            const int py = y0 + wave * 4 + nb, px = x0 + r16;
            if (py >= H || px >= W) continue;
            const size_t p = (size_t)py * W + px;
            if (MODE == 1) {
                if (g == 0) ((float*)yout)[p] = acc[0][nb][0] + bias[0];
                continue;
            }
#pragma unroll
            for (int mb = 0; mb < MB; ++mb) {
                const int co0 = mb * 16 + 4 * g;
                if (co0 >= COUT) continue;
                bf16x4 o;
                if (MODE == 2) {
                    const bf16x4 mk = *(const bf16x4*)(mask + p * COUT + co0);
#pragma unroll
                    for (int e = 0; e < 4; ++e) o[e] = (__bf16)((float)mk[e] > 0.f ? acc[mb][nb][e] : 0.f);
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e) o[e] = (__bf16)fmaxf(acc[mb][nb][e] + bias[co0 + e], 0.f);
                }
                *(bf16x4*)((__bf16*)yout + p * COUT + co0) = o;
            }
        }
    }
}

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// The 8 bf16 that start kx (0, 1 or 2; uniform across the wave) elements
// after a 16-byte aligned LDS address, from one 16-byte and one 4-byte read
// joined by byte shifts (v_alignbyte) instead of eight 2-byte reads.
__device__ __forceinline__ bf16x8 lds_shifted8(const __bf16* p, int kx) {
    const u32x4 lo = *(const u32x4*)p;
    const uint32_t hi = *(const uint32_t*)(p + 8);
    u32x4 o;
    if (kx == 0) {
        o = lo;
    } else if (kx == 1) {
        o[0] = __builtin_amdgcn_alignbyte(lo[1], lo[0], 2);
        o[1] = __builtin_amdgcn_alignbyte(lo[2], lo[1], 2);
        o[2] = __builtin_amdgcn_alignbyte(lo[3], lo[2], 2);
        o[3] = __builtin_amdgcn_alignbyte(hi, lo[3], 2);
    } else {
        o[0] = lo[1];
        o[1] = lo[2];
        o[2] = lo[3];
        o[3] = hi;
    }
    return __builtin_bit_cast(bf16x8, o);
}

// The channels of one NHWC pixel that one load moves (raw bf16 bits):
// 8 (16 bytes) when C is a multiple of 8, else all C.
template <int C>
struct ChanVec {
    static constexpr int V = C % 8 == 0 ? 8 : C;
    typedef unsigned short T __attribute__((ext_vector_type(V)));
    static __device__ __forceinline__ unsigned short get(const T& v, int j) { return v[j]; }
};
template <>
struct ChanVec<1> {
    static constexpr int V = 1;
    typedef unsigned short T;
    static __device__ __forceinline__ unsigned short get(const T& v, int) { return v; }
};

// Weight and bias gradients: dw[t][co][ci] += sum_p dy[p][co] x[p + off(t)][ci],
// db[co] += sum_p dy[p][co].  Each workgroup walks 16x16 tiles and keeps its
// partial sums in registers (the nine taps split evenly over the four waves),
// then stores them as its row of part ([workgroup][9 * COUT * CIN + COUT],
// every entry written); k_wgrad_reduce sums the rows.  Same-address atomics
// from every workgroup on the chip would serialise.
template <int CIN, int COUT>
__global__ __launch_bounds__(256, 2) void k_wgrad(int H, int W, const __bf16* __restrict__ x,
                                               const __bf16* __restrict__ dy, float* __restrict__ part) {
    constexpr int MB = (COUT + 15) / 16, NB = (CIN + 15) / 16;
    constexpr int DS = 264;  // [co][pixel] row stride
    __shared__ __attribute__((aligned(16))) __bf16 s_dy[32 * DS];
    __shared__ __attribute__((aligned(16))) __bf16 s_x[32 * 18 * 24];
    __shared__ float s_db[8][32];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int g = lane >> 4, r16 = lane & 15;
    const int ntx = (W + 15) / 16, nty = (H + 15) / 16, ntiles = ntx * nty;
    // wave w: taps w and w + 4 whole (A and B reused across the row and column
    // blocks), and (row block, column block) unit w of tap 8 if it exists,
    // so the 9 taps' MB * NB units are spread evenly over the four waves
    f32x4 acc[2][MB][NB];
#pragma unroll
    for (int k3 = 0; k3 < 2; ++k3)
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) acc[k3][mb][nb] = f32x4{0.f, 0.f, 0.f, 0.f};
    f32x4 acc8 = f32x4{0.f, 0.f, 0.f, 0.f};
    const bool has8 = wave < MB * NB;
    const int mb8 = has8 ? wave / NB : 0, nb8 = has8 ? wave % NB : 0;
    float dbp = 0.f;
    const int bco = tid & 31, bgrp = tid >> 5;
    // channel rows past COUT / CIN stay zero (the tile loads never write them)
    for (int i = tid; i < (32 - COUT) * DS; i += 256) s_dy[COUT * DS + i] = (__bf16)0.f;
    for (int i = tid; i < (32 - CIN) * 18 * 24; i += 256) s_x[CIN * 18 * 24 + i] = (__bf16)0.f;
    // tile staging: each thread loads whole pixels' channel vectors (up to 16
    // bytes), every global load of the tile issued before the LDS stores
    typedef typename ChanVec<COUT>::T VecY;
    typedef typename ChanVec<CIN>::T VecX;
    constexpr int VY = ChanVec<COUT>::V, NVY = COUT / VY;
    constexpr int VX = ChanVec<CIN>::V, NVX = CIN / VX;
    const unsigned short* dyr = (const unsigned short*)dy;
    const unsigned short* xr = (const unsigned short*)x;
    unsigned short* s_dyr = (unsigned short*)s_dy;
    unsigned short* s_xr = (unsigned short*)s_x;
    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int x0 = (tile % ntx) * 16, y0 = (tile / ntx) * 16;
        // A channel count that is a multiple of 8 is staged two horizontally
        // adjacent pixels per item, stored as 4-byte pairs into the
        // [channel][pixel] tiles (half the LDS writes of one pixel per item).
        constexpr bool PY = COUT % 8 == 0, PX = CIN % 8 == 0;
        constexpr int NY = PY ? 128 * NVY : 256 * NVY;   // items of the dy tile
        constexpr int NX = PX ? 162 * NVX : 324 * NVX;   // items of the x patch
        constexpr int KY = (NY + 255) / 256, KX = (NX + 255) / 256;
        VecY ry[PY ? 2 * KY : KY];
        VecX rx[PX ? 2 * KX : KX];
#pragma unroll
        for (int k = 0; k < KY; ++k) {
            const int i = tid + 256 * k, q = i / NVY, c = (i - q * NVY) * VY;
            if (PY) {
                const int p0 = 2 * q, gy = y0 + (p0 >> 4), gx = x0 + (p0 & 15);
                ry[2 * k] = VecY(0);
                ry[2 * k + 1] = VecY(0);
                if (i < NY && gy < H) {
                    const unsigned short* src = dyr + ((size_t)gy * W + gx) * COUT + c;
                    if (gx < W) ry[2 * k] = *(const VecY*)src;
                    if (gx + 1 < W) ry[2 * k + 1] = *(const VecY*)(src + COUT);
                }
            } else {
                const int gy = y0 + (q >> 4), gx = x0 + (q & 15);
                ry[k] = VecY(0);
                if (i < NY && gy < H && gx < W) ry[k] = *(const VecY*)(dyr + ((size_t)gy * W + gx) * COUT + c);
            }
        }
#pragma unroll
        for (int k = 0; k < KX; ++k) {
            const int i = tid + 256 * k, q = i / NVX, c = (i - q * NVX) * VX;
            if (PX) {
                const int ty = q / 9, tx0 = (q - ty * 9) * 2;
                const int gy = y0 + ty - 1, gx = x0 + tx0 - 1;
                rx[2 * k] = VecX(0);
                rx[2 * k + 1] = VecX(0);
                if (i < NX && gy >= 0 && gy < H) {
                    const unsigned short* src = xr + ((size_t)gy * W + gx) * CIN + c;
                    if (gx >= 0 && gx < W) rx[2 * k] = *(const VecX*)src;
                    if (gx + 1 >= 0 && gx + 1 < W) rx[2 * k + 1] = *(const VecX*)(src + CIN);
                }
            } else {
                const int ty = q / 18, tx = q - ty * 18;
                const int gy = y0 + ty - 1, gx = x0 + tx - 1;
                rx[k] = VecX(0);
                if (i < NX && gy >= 0 && gy < H && gx >= 0 && gx < W)
                    rx[k] = *(const VecX*)(xr + ((size_t)gy * W + gx) * CIN + c);
            }
        }
        __syncthreads();   // the previous tile's MFMA reads are done
#pragma unroll
        for (int k = 0; k < KY; ++k) {
            const int i = tid + 256 * k, q = i / NVY, c = (i - q * NVY) * VY;
            if (i >= NY) continue;
#pragma unroll
            for (int j = 0; j < VY; ++j) {
                if (PY)
                    *(uint32_t*)(s_dyr + (c + j) * DS + 2 * q) =
                        (uint32_t)ChanVec<COUT>::get(ry[2 * k], j) | ((uint32_t)ChanVec<COUT>::get(ry[2 * k + 1], j) << 16);
                else
                    s_dyr[(c + j) * DS + q] = ChanVec<COUT>::get(ry[k], j);
            }
        }
#pragma unroll
        for (int k = 0; k < KX; ++k) {
            const int i = tid + 256 * k, q = i / NVX, c = (i - q * NVX) * VX;
            if (i >= NX) continue;
            if (PX) {
                const int ty = q / 9, tx0 = (q - ty * 9) * 2;
#pragma unroll
                for (int j = 0; j < VX; ++j)
                    *(uint32_t*)(s_xr + ((c + j) * 18 + ty) * 24 + tx0) =
                        (uint32_t)ChanVec<CIN>::get(rx[2 * k], j) | ((uint32_t)ChanVec<CIN>::get(rx[2 * k + 1], j) << 16);
            } else {
                const int ty = q / 18, tx = q - ty * 18;
#pragma unroll
                for (int j = 0; j < VX; ++j) s_xr[((c + j) * 18 + ty) * 24 + tx] = ChanVec<CIN>::get(rx[k], j);
            }
        }
        __syncthreads();
        if (bco < COUT)
            for (int j = 0; j < 32; ++j) dbp += (float)s_dy[bco * DS + bgrp * 32 + j];
#pragma unroll
        for (int k3 = 0; k3 < 2; ++k3) {
            const int t = wave + 4 * k3;
            const int ky = t / 3, kx = t - ky * 3;
#pragma unroll
            for (int ks = 0; ks < 8; ++ks) {
                const int row = 2 * ks + (g >> 1), col = (g & 1) * 8;
                bf16x8 Am[MB];
#pragma unroll
                for (int mb = 0; mb < MB; ++mb)
                    Am[mb] = *(const bf16x8*)(s_dy + (mb * 16 + r16) * DS + 32 * ks + 8 * g);
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) {
                    const int ci = nb * 16 + r16;
                    const bf16x8 Bv = lds_shifted8(s_x + (ci * 18 + row + ky) * 24 + col, kx);
#pragma unroll
                    for (int mb = 0; mb < MB; ++mb)
                        acc[k3][mb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Am[mb], Bv, acc[k3][mb][nb], 0, 0, 0);
                }
            }
        }
        if (has8) {   // tap 8 = (ky, kx) = (2, 2): this wave's unit
#pragma unroll
            for (int ks = 0; ks < 8; ++ks) {
                const int row = 2 * ks + (g >> 1), col = (g & 1) * 8;
                const bf16x8 Am = *(const bf16x8*)(s_dy + (mb8 * 16 + r16) * DS + 32 * ks + 8 * g);
                const bf16x8 Bv = lds_shifted8(s_x + ((nb8 * 16 + r16) * 18 + row + 2) * 24 + col, 2);
                acc8 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Am, Bv, acc8, 0, 0, 0);
            }
        }
    }
    float* __restrict__ dw = part + (size_t)blockIdx.x * (9 * COUT * CIN + COUT);
    if (has8)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int co = mb8 * 16 + 4 * g + e, ci = nb8 * 16 + r16;
            if (co < COUT && ci < CIN) dw[(8 * COUT + co) * CIN + ci] = acc8[e];
        }
#pragma unroll
    for (int k3 = 0; k3 < 2; ++k3) {
        const int t = wave + 4 * k3;
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int co = mb * 16 + 4 * g + e, ci = nb * 16 + r16;
                    if (co < COUT && ci < CIN) dw[(t * COUT + co) * CIN + ci] = acc[k3][mb][nb][e];
                }
    }
    s_db[bgrp][bco] = dbp;
    __syncthreads();
    if (tid < COUT) {
        float s = 0.f;
        for (int k = 0; k < 8; ++k) s += s_db[k][tid];
        dw[9 * COUT * CIN + tid] = s;
    }
}

constexpr int kWgradBlocks = 512;  // persistent weight-gradient workgroups (two per CU)
constexpr int kWgradSplit = 16;    // row groups of the partial-sum reduction

// Partial-sum rows of the weight gradient for callers that cannot allocate
// (sgad_conv3x3_wgrad_noalloc): one row per persistent workgroup, each row
// wide enough for the largest supported layer (9 * 32 * 32 weights + 32
// biases): 512 x 9248 floats = 18.9 MB, held on every device the library
// runs on until the process ends.  Host code never passes this name to a
// kernel: it stands for a host-side shadow there; conv_scratch_setup gives
// each device's own address.
constexpr size_t kWgradScratchFloats = (size_t)kWgradBlocks * (9 * 32 * 32 + 32);
static __device__ __align__(256) float scratch[kWgradScratchFloats];
constexpr int kScratchDevices = 64;

// Device address of the current device's copy of `scratch`, looked up once
// per device (the caller makes `device` current first).
hipError_t conv_scratch_setup(int device, float** out) {
    static std::mutex mu;
    static float* addr[kScratchDevices] = {};
    *out = nullptr;
    if (device < 0 || device >= kScratchDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[device]) {
        float* p = nullptr;
        const hipError_t e = hipGetSymbolAddress((void**)&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[device] = p;
    }
    *out = addr[device];
    return hipSuccess;
}

size_t conv_scratch_bytes() { return sizeof(float) * kWgradScratchFloats; }

// dw[j] (j < ndw) or db[j - ndw] += sum of column j over the nrow rows of
// part ([nrow][S]); blockIdx.y takes rows y, y + kWgradSplit, ...
__global__ __launch_bounds__(256) void k_wgrad_reduce(int S, int ndw, int nrow, const float* __restrict__ part,
                                                      float* dw, float* db) {
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= S) return;
    float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
    int r = blockIdx.y;
    for (; r + 3 * kWgradSplit < nrow; r += 4 * kWgradSplit) {
        s0 += part[(size_t)r * S + j];
        s1 += part[(size_t)(r + kWgradSplit) * S + j];
        s2 += part[(size_t)(r + 2 * kWgradSplit) * S + j];
        s3 += part[(size_t)(r + 3 * kWgradSplit) * S + j];
    }
    for (; r < nrow; r += kWgradSplit) s0 += part[(size_t)r * S + j];
    const float v = (s0 + s1) + (s2 + s3);
    if (j < ndw) atomicAdd(&dw[j], v);
    else atomicAdd(&db[j - ndw], v);
}

// FP32 master weights [9][cout][cin] -> bf16 copy and the transposed,
// tap-flipped bf16 copy used by the input gradient: wt[t][ci][co] = w[8-t][co][ci].
__global__ void k_conv_weights(int cin, int cout, const float* w, __bf16* wb, __bf16* wt) {
    const int n = 9 * cin * cout;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int t = i / (cin * cout), rem = i - t * cin * cout;
        const int co = rem / cin, ci = rem - co * cin;
        const __bf16 v = (__bf16)w[i];
        wb[i] = v;
        if (wt) wt[((size_t)(8 - t) * cin + ci) * cout + co] = v;
    }
}

// Network input (R, G, B, h): h = (D - mean of D over the in-image 3x3
// neighbourhood) / 2 cm.  Depth in metres would be stored in bf16 with a
// 4-31 mm spacing, as coarse as the sensor noise the offsets undo; the
// high-passed depth resolves it.  The sum runs row by row, left to right.
__global__ void k_net_input(int H, int W, const float* rgb, const float* depth, __bf16* x0) {
    const int P = H * W;
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < P; p += gridDim.x * blockDim.x) {
        const int y = p / W, x = p - y * W;
        float s = 0.f;
        int n = 0;
        for (int yy = max(0, y - 1); yy <= min(H - 1, y + 1); ++yy)
            for (int xx = max(0, x - 1); xx <= min(W - 1, x + 1); ++xx) {
                s += depth[yy * W + xx];
                ++n;
            }
        bf16x4 v;
        v[0] = (__bf16)rgb[p];
        v[1] = (__bf16)rgb[P + p];
        v[2] = (__bf16)rgb[2 * P + p];
        v[3] = (__bf16)((depth[p] - s / (float)n) * (1.f / 0.02f));
        *(bf16x4*)(x0 + (size_t)p * 4) = v;
    }
}

// L1 training loss mean|pred - target| and its gradient (bf16, one channel).
__global__ __launch_bounds__(256) void k_offset_l1(int n, const float* pred, const float* target, __bf16* grad, double* loss) {
    double acc = 0.0;
    const float inv = 1.f / (float)n;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const float e = pred[i] - target[i];
        acc += (double)fabsf(e);
        grad[i] = (__bf16)(e > 0.f ? inv : (e < 0.f ? -inv : 0.f));
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) acc += __shfl_xor(acc, o, 64);
    // one atomic per block: same-address FP64 atomics serialise in L2
    __shared__ double s_acc[4];
    if ((threadIdx.x & 63) == 0) s_acc[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(loss, (s_acc[0] + s_acc[1] + s_acc[2] + s_acc[3]) / (double)n);
}

// ---------------------------------------------------------------------------
// host launchers (return false for an unsupported channel configuration)
// ---------------------------------------------------------------------------
constexpr int kConvBlocks = 512;   // persistent conv workgroups

bool launch_conv_fwd(int H, int W, int cin, int cout, int mode, const void* x, const void* w, const float* bias,
                     const void* mask, void* y, hipStream_t s) {
    const dim3 grid(std::min(((W + 15) / 16) * ((H + 15) / 16), kConvBlocks)), blk(256);
    const __bf16* xb = (const __bf16*)x;
    const __bf16* wb = (const __bf16*)w;
    const __bf16* mb = (const __bf16*)mask;
    if (mode == 0 && cin == 4 && cout == 32)
        hipLaunchKernelGGL((k_conv<4, 32, 0>), grid, blk, 0, s, H, W, xb, wb, bias, mb, y);
    else if (mode == 0 && cin == 32 && cout == 32)
        hipLaunchKernelGGL((k_conv<32, 32, 0>), grid, blk, 0, s, H, W, xb, wb, bias, mb, y);
    else if (mode == 1 && cin == 32 && cout == 1)
        hipLaunchKernelGGL((k_conv<32, 1, 1>), grid, blk, 0, s, H, W, xb, wb, bias, mb, y);
    else if (mode == 2 && cin == 32 && cout == 32)
        hipLaunchKernelGGL((k_conv<32, 32, 2>), grid, blk, 0, s, H, W, xb, wb, bias, mb, y);
    else if (mode == 2 && cin == 1 && cout == 32)
        hipLaunchKernelGGL((k_conv<1, 32, 2>), grid, blk, 0, s, H, W, xb, wb, bias, mb, y);
    else
        return false;
    return true;
}

// Workgroups of the weight gradient (one partial-sum row each): two
// persistent workgroups per CU (measured at 640x480: one leaves each wave's
// tile loads exposed).
static int wgrad_blocks(int H, int W) { return std::min(((W + 15) / 16) * ((H + 15) / 16), kWgradBlocks); }

size_t conv_wgrad_part_bytes(int H, int W, int cin, int cout) {
    return (size_t)wgrad_blocks(H, W) * (size_t)(9 * cout * cin + cout) * sizeof(float);
}

bool launch_conv_wgrad(int H, int W, int cin, int cout, const void* x, const void* dy, float* part, float* dw,
                       float* db, hipStream_t s) {
    const int nrow = wgrad_blocks(H, W);
    const dim3 grid(nrow), blk(256);
    const __bf16* xb = (const __bf16*)x;
    const __bf16* db16 = (const __bf16*)dy;
    if (cin == 4 && cout == 32) hipLaunchKernelGGL((k_wgrad<4, 32>), grid, blk, 0, s, H, W, xb, db16, part);
    else if (cin == 32 && cout == 32) hipLaunchKernelGGL((k_wgrad<32, 32>), grid, blk, 0, s, H, W, xb, db16, part);
    else if (cin == 32 && cout == 1) hipLaunchKernelGGL((k_wgrad<32, 1>), grid, blk, 0, s, H, W, xb, db16, part);
    else return false;
    const int ndw = 9 * cout * cin, S = ndw + cout;
    hipLaunchKernelGGL(k_wgrad_reduce, dim3((S + 255) / 256, std::min(nrow, kWgradSplit)), dim3(256), 0, s, S, ndw,
                       nrow, part, dw, db);
    return true;
}

void launch_conv_weights(int cin, int cout, const float* w, void* wb, void* wt, hipStream_t s) {
    const int n = 9 * cin * cout;
    hipLaunchKernelGGL(k_conv_weights, dim3((n + 255) / 256), dim3(256), 0, s, cin, cout, w, (__bf16*)wb,
                       (__bf16*)wt);
}

void launch_net_input(int H, int W, const float* rgb, const float* depth, void* x0, hipStream_t s) {
    const int P = H * W;
    hipLaunchKernelGGL(k_net_input, dim3(std::min(4096, (P + 255) / 256)), dim3(256), 0, s, H, W, rgb, depth,
                       (__bf16*)x0);
}

void launch_offset_l1(int n, const float* pred, const float* target, void* grad, double* loss, hipStream_t s) {
    hipLaunchKernelGGL(k_offset_l1, dim3(std::min(256, (n + 255) / 256)), dim3(256), 0, s, n, pred, target,
                       (__bf16*)grad, loss);
}

}  // namespace sgad
