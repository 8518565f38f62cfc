// Structural-similarity term of the mapping loss (Eq. 1, weight tau): with x
// the observed colour plane and y the rendered one,
//   L_S = 1 - (1 / (3 P)) sum over channels and pixels of SSIM(x, y),
//   SSIM = (2 mu_x mu_y + C1)(2 s_xy + C2) / ((mu_x^2 + mu_y^2 + C1)(s_xx + s_yy + C2)),
// with the SSIM reference's local statistics: an 11 x 11 Gaussian window of
// standard deviation 1.5 (normalised to sum 1) applied as a 'same'
// correlation with zero padding, C1 = 0.01^2, C2 = 0.03^2 (dynamic range 1).
//
// Two launches per call, both over (16 x 16 tile, plane) with a 26 x 26 patch
// (tile plus a 5-pixel halo) in LDS and the window applied as a row pass then
// a column pass:
//   k_ssim_maps: the filtered moments (x, y, x^2 + y^2, xy), SSIM and the three partials
//     dS/dmu_y, dS/de_yy, dS/de_xy per pixel (written), the SSIM sum;
//   k_ssim_grad: the adjoint of the correlation (the same symmetric window)
//     applied to the three maps, giving
//     dL_S/dy = -(1 / (3 P)) [G*(dS/dmu_y) + 2 y G*(dS/de_yy) + x G*(dS/de_xy)],
//     added to the colour gradient with weight tau.
// The moments and everything formed from them are FP64: s_xx = G*x^2 - mu_x^2
// cancels down to ~C2 = 9e-4 on smooth patches, where FP32 moments of unit-
// range colours would leave errors of ~1e-4 relative.  The maps are stored as
// FP32.
#include <hip/hip_runtime.h>

#include "raster_common.h"

namespace sgad {

constexpr int kSsimR = 5;                    // window radius
constexpr int kSsimT = 16;                   // output tile side, one pixel per thread
constexpr int kSsimE = kSsimT + 2 * kSsimR;  // patch side (tile + halo)
constexpr double kSsimC1 = 0.01 * 0.01;
constexpr double kSsimC2 = 0.03 * 0.03;

// Normalised window taps g[k] = exp(-(k - 5)^2 / (2 * 1.5^2)) / sum_j exp(-(j - 5)^2 / 4.5),
// k = 0..10, written out to 17 digits.
__constant__ double c_ssim_g[2 * kSsimR + 1] = {
    0.0010283800844791101, 0.007598758135239185, 0.036000772128430829, 0.10936068950970002,
    0.21300553771125369,   0.26601172486179436,  0.21300553771125369,  0.10936068950970002,
    0.036000772128430829,  0.007598758135239185, 0.0010283800844791101};

// The block's output tile and colour plane.  The 1-D grid is spread over the
// XCDs in contiguous ranges, so that neighbouring tiles, whose patches
// overlap, share an L2.
struct SsimTile {
    int tx, ty, plane, ntx, nty;
};

__device__ __forceinline__ SsimTile ssim_tile(int H, int W) {
    SsimTile t;
    t.ntx = (W + kSsimT - 1) / kSsimT;
    t.nty = (H + kSsimT - 1) / kSsimT;
    const int b = xcd_remap((int)blockIdx.x, (int)gridDim.x);
    const int per = t.ntx * t.nty;
    t.plane = b / per;
    const int r = b - t.plane * per;
    t.ty = r / t.ntx;
    t.tx = r - t.ty * t.ntx;
    return t;
}

// Patch of NPL planes around tile t, zero outside the image: every thread
// issues all of its loads before its first LDS write, so the block waits for
// one round trip to memory instead of three.
template <int NPL>
__device__ __forceinline__ void ssim_load(int H, int W, const SsimTile& t, const float* const* src,
                                          float (*dst)[kSsimE][kSsimE + 1]) {
    constexpr int N = kSsimE * kSsimE, IT = (N + 255) / 256;
    const int ox = t.tx * kSsimT - kSsimR, oy = t.ty * kSsimT - kSsimR;
    float v[IT][NPL];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const int i = (int)threadIdx.x + it * 256;
        const int r = i / kSsimE, c = i - r * kSsimE;
        const int gx = ox + c, gy = oy + r;
        const bool in = i < N && gx >= 0 && gx < W && gy >= 0 && gy < H;
        const size_t o = in ? (size_t)gy * W + gx : 0;
#pragma unroll
        for (int p = 0; p < NPL; ++p) v[it][p] = in ? src[p][o] : 0.f;
    }
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const int i = (int)threadIdx.x + it * 256;
        if (i >= N) continue;
        const int r = i / kSsimE, c = i - r * kSsimE;
#pragma unroll
        for (int p = 0; p < NPL; ++p) dst[p][r][c] = v[it][p];
    }
}

__device__ __forceinline__ double block_sum_d(double v, double* red) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    return (red[0] + red[1]) + (red[2] + red[3]);
}

// Row pass over the patch: thread t < kRowItems filters row t / kRowThreads
// for the kRowOut outputs starting at kRowOut (t % kRowThreads), each of the
// 10 + kRowOut inputs loaded, converted and (for the maps) squared once for
// the outputs it feeds.  Every output sums its 11 taps in tap order, as a
// one-output loop would.
constexpr int kRowOut = 4;
constexpr int kRowThreads = kSsimT / kRowOut;   // items per patch row
constexpr int kRowItems = kSsimE * kRowThreads;
static_assert(kRowItems <= 256, "one row item per thread of the 256-thread block");

// One block per (plane, tile), plane z = colour channel z % 3 of job z / 3.
// dmap [n_jobs * 3][3][H][W]; part[z][tile] = the tile's SSIM sum (written;
// k_ssim_grad adds them to the loss in a fixed order).  With cnt, the blocks
// of each job's first plane also count the tile's valid target depths
// (D > 0) into cnt[job][tile] for the masked depth term, and the job's first
// tile clears loss[job], which the L1 and SSIM terms then add to.
__global__ __launch_bounds__(256) void k_ssim_maps(int H, int W, const float* __restrict__ rgb,
                                                   const float* __restrict__ t_rgb, float* __restrict__ dmap,
                                                   double* __restrict__ part, const float* __restrict__ t_depth,
                                                   uint32_t* __restrict__ cnt, double* loss) {
    __shared__ float s_in[2][kSsimE][kSsimE + 1];    // observed x, rendered y
    // row-filtered x, y, x^2 + y^2, xy: SSIM needs the two variances only
    // as their sum (18.9 KB of LDS per block, eight blocks per CU)
    __shared__ double s_h[4][kSsimE][kSsimT];
    __shared__ double s_red[4];
    __shared__ uint32_t s_cnt[4];
    const SsimTile st = ssim_tile(H, W);
    const int plane = st.plane;
    const size_t P = (size_t)H * W;
    const bool counts = cnt != nullptr && plane % 3 == 0;
    const int cx = st.tx * kSsimT + (int)(threadIdx.x & (kSsimT - 1));
    const int cy = st.ty * kSsimT + (int)(threadIdx.x >> 4);
    float tdep = 0.f;   // loaded first, counted after the filtering
    if (counts && cx < W && cy < H) tdep = t_depth[(size_t)(plane / 3) * P + (size_t)cy * W + cx];
    const float* src[2] = {t_rgb + (size_t)plane * P, rgb + (size_t)plane * P};
    const double* s_g = c_ssim_g;
    ssim_load<2>(H, W, st, src, s_in);
    __syncthreads();
    if (threadIdx.x < kRowItems) {
        const int r = threadIdx.x / kRowThreads, c0 = (threadIdx.x % kRowThreads) * kRowOut;
        double a[kRowOut] = {}, b[kRowOut] = {}, ss[kRowOut] = {}, xy[kRowOut] = {};
#pragma unroll
        for (int j = 0; j < 2 * kSsimR + kRowOut; ++j) {
            const double x = (double)s_in[0][r][c0 + j], y = (double)s_in[1][r][c0 + j];
            const double s2 = x * x + y * y, xyv = x * y;
#pragma unroll
            for (int o = 0; o < kRowOut; ++o) {
                const int k = j - o;
                if (k < 0 || k > 2 * kSsimR) continue;
                const double g = s_g[k];
                a[o] += g * x;
                b[o] += g * y;
                ss[o] += g * s2;
                xy[o] += g * xyv;
            }
        }
#pragma unroll
        for (int o = 0; o < kRowOut; ++o) {
            s_h[0][r][c0 + o] = a[o];
            s_h[1][r][c0 + o] = b[o];
            s_h[2][r][c0 + o] = ss[o];
            s_h[3][r][c0 + o] = xy[o];
        }
    }
    __syncthreads();
    const int tx = threadIdx.x & (kSsimT - 1), ty = threadIdx.x >> 4;
    double m[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k <= 2 * kSsimR; ++k) {
        const double g = s_g[k];
#pragma unroll
        for (int q = 0; q < 4; ++q) m[q] += g * s_h[q][ty + k][tx];
    }
    const int px = st.tx * kSsimT + tx, py = st.ty * kSsimT + ty;
    double S = 0.0;
    if (px < W && py < H) {
        const double mx = m[0], my = m[1];
        const double sxy = m[3] - mx * my;
        const double A1 = 2.0 * mx * my + kSsimC1, A2 = 2.0 * sxy + kSsimC2;
        const double B1 = mx * mx + my * my + kSsimC1, B2 = (m[2] - (mx * mx + my * my)) + kSsimC2;
        // one division: with q = 1 / (B1 B2), S = A1 A2 q, S / A1 = A2 q,
        // S / A2 = A1 q, S / B1 = S B2 q, S / B2 = S B1 q (B1, B2 > 0; A2 may
        // be 0)
        const double q = 1.0 / (B1 * B2);
        S = A1 * A2 * q;
        const double d_my = 2.0 * q * (mx * (A2 - A1) + my * S * (B1 - B2));
        const double d_eyy = -S * B1 * q;
        const double d_exy = 2.0 * A1 * q;
        const size_t o = (size_t)py * W + px;
        float* dm = dmap + (size_t)plane * 3 * P;
        dm[o] = (float)d_my;
        dm[P + o] = (float)d_eyy;
        dm[2 * P + o] = (float)d_exy;
    }
    if (counts) {
        const uint32_t c = (uint32_t)__popcll(__ballot(tdep > 0.f));
        if ((threadIdx.x & 63) == 0) s_cnt[threadIdx.x >> 6] = c;
    }
    const double sum = block_sum_d(S, s_red);   // (its barrier also publishes s_cnt)
    const int tile = st.ty * st.ntx + st.tx;
    if (threadIdx.x == 0) {
        part[(size_t)plane * st.ntx * st.nty + tile] = sum;
        if (counts) {
            const int job = plane / 3;
            cnt[(size_t)job * st.ntx * st.nty + tile] = (s_cnt[0] + s_cnt[1]) + (s_cnt[2] + s_cnt[3]);
            if (tile == 0) loss[job] = 0.0;
        }
    }
}

// Same grid: g_rgb[plane] += -tau / (3 P) [G*d_my + 2 y G*d_eyy + x G*d_exy].
// The first tile of each job's first plane also adds tau (1 - (sum of the
// job's 3 x tiles partial SSIM sums, in index order) / (3 P)) to loss[job].
__global__ __launch_bounds__(256) void k_ssim_grad(int H, int W, const float* __restrict__ rgb,
                                                   const float* __restrict__ t_rgb, const float* __restrict__ dmap,
                                                   const double* __restrict__ part, double tau,
                                                   float* __restrict__ g_rgb, double* loss) {
    __shared__ float s_in[3][kSsimE][kSsimE + 1];
    __shared__ double s_h[3][kSsimE][kSsimT];
    __shared__ double s_red[4];
    const SsimTile st = ssim_tile(H, W);
    const int plane = st.plane;
    const size_t P = (size_t)H * W;
    if (st.tx == 0 && st.ty == 0 && plane % 3 == 0) {
        const int nt = st.ntx * st.nty * 3;
        const double* pp = part + (size_t)plane * st.ntx * st.nty;
        double acc = 0.0;
        for (int i = threadIdx.x; i < nt; i += 256) acc += pp[i];
        const double sum = block_sum_d(acc, s_red);
        if (threadIdx.x == 0) loss[plane / 3] += tau * (1.0 - sum / (3.0 * (double)P));
    }
    const float* dm = dmap + (size_t)plane * 3 * P;
    const float* src[3] = {dm, dm + P, dm + 2 * P};
    const double* s_g = c_ssim_g;
    ssim_load<3>(H, W, st, src, s_in);
    __syncthreads();
    if (threadIdx.x < kRowItems) {
        const int r = threadIdx.x / kRowThreads, c0 = (threadIdx.x % kRowThreads) * kRowOut;
        double a[kRowOut] = {}, b[kRowOut] = {}, d[kRowOut] = {};
#pragma unroll
        for (int j = 0; j < 2 * kSsimR + kRowOut; ++j) {
            const double u = (double)s_in[0][r][c0 + j], v = (double)s_in[1][r][c0 + j],
                         w = (double)s_in[2][r][c0 + j];
#pragma unroll
            for (int o = 0; o < kRowOut; ++o) {
                const int k = j - o;
                if (k < 0 || k > 2 * kSsimR) continue;
                const double g = s_g[k];
                a[o] += g * u;
                b[o] += g * v;
                d[o] += g * w;
            }
        }
#pragma unroll
        for (int o = 0; o < kRowOut; ++o) {
            s_h[0][r][c0 + o] = a[o];
            s_h[1][r][c0 + o] = b[o];
            s_h[2][r][c0 + o] = d[o];
        }
    }
    __syncthreads();
    const int tx = threadIdx.x & (kSsimT - 1), ty = threadIdx.x >> 4;
    const int px = st.tx * kSsimT + tx, py = st.ty * kSsimT + ty;
    if (px >= W || py >= H) return;
    double f0 = 0.0, f1 = 0.0, f2 = 0.0;
#pragma unroll
    for (int k = 0; k <= 2 * kSsimR; ++k) {
        const double g = s_g[k];
        f0 += g * s_h[0][ty + k][tx];
        f1 += g * s_h[1][ty + k][tx];
        f2 += g * s_h[2][ty + k][tx];
    }
    const size_t o = (size_t)plane * P + (size_t)py * W + px;
    const double x = (double)t_rgb[o], y = (double)rgb[o];
    const double gr = -tau / (3.0 * (double)P) * (f0 + 2.0 * y * f1 + x * f2);
    g_rgb[o] = (float)((double)g_rgb[o] + gr);
}

size_t ssim_tiles(int H, int W) {
    return (size_t)((W + kSsimT - 1) / kSsimT) * (size_t)((H + kSsimT - 1) / kSsimT);
}

// Workspace of one call: the maps, then one FP64 partial sum per (plane, tile).
size_t ssim_map_bytes(int n_jobs, int H, int W) {
    const size_t maps = (size_t)n_jobs * 9 * (size_t)H * W * sizeof(float);
    return ((maps + 255) & ~(size_t)255) + (size_t)n_jobs * 3 * ssim_tiles(H, W) * sizeof(double);
}

static double* ssim_part(int n_jobs, int H, int W, void* ws) {
    const size_t maps = (size_t)n_jobs * 9 * (size_t)H * W * sizeof(float);
    return (double*)((char*)ws + ((maps + 255) & ~(size_t)255));
}

// The two launches of the SSIM term; with cnt (n_jobs * ssim_tiles entries)
// the first also counts the valid target depths and clears the loss, so that
// the L1 launch can run between the two without a counting pass of its own.
void launch_ssim_maps(int n_jobs, int H, int W, const float* rgb, const float* t_rgb, void* ws,
                      const float* t_depth, uint32_t* cnt, double* loss, hipStream_t s) {
    const dim3 grid((unsigned)(ssim_tiles(H, W) * 3 * n_jobs)), blk(256);
    hipLaunchKernelGGL(k_ssim_maps, grid, blk, 0, s, H, W, rgb, t_rgb, (float*)ws, ssim_part(n_jobs, H, W, ws),
                       t_depth, cnt, loss);
}

void launch_ssim_grad(int n_jobs, int H, int W, const float* rgb, const float* t_rgb, float w_ssim, void* ws,
                      float* g_rgb, double* loss, hipStream_t s) {
    const dim3 grid((unsigned)(ssim_tiles(H, W) * 3 * n_jobs)), blk(256);
    hipLaunchKernelGGL(k_ssim_grad, grid, blk, 0, s, H, W, rgb, t_rgb, (const float*)ws,
                       ssim_part(n_jobs, H, W, ws), (double)w_ssim, g_rgb, loss);
}

}  // namespace sgad
