// Per-pixel depth-distribution tracking: forward-mode compositing with six
// pose tangents, fused residual / Jacobian / normal-equation reduction, and an
// on-device FP64 Gauss-Newton solve with the SE(3) update.
//
// Model (abstract; Sec. 3.3 attaches a Gaussian to each back-projected
// point): geometry Gaussians of the previous frame are splatted into the new
// view with sigma^2 as the only colour channel, giving per pixel A, D' and
// S = sum w sigma^2; mu = D'/A, s^2 = S/A.  A pixel is valid iff A >= 0.9 and
// D_obs > 0; r = (D_obs - mu)/s and J = dr/dxi = -(dD' - mu dA)/(A s) with s
// held fixed.  H = sum J^T J, g = sum J^T r, l = sum(-r^2/2 - ln s - ln(2pi)/2).
#include <hip/hip_runtime.h>

#include "raster_common.h"
#include "segsort.h"
#include "sgad_internal.h"

namespace sgad {

constexpr float kNegHalfLog2eT = -0.72134752044448170368f;
constexpr float kAValid = 0.9f;
constexpr int kTrackVals = 29;   // 21 H (upper triangle) + 6 g + loglik + valid count
constexpr int kTraceStride = 40; // per-iteration trace record (doubles)

__device__ __forceinline__ float tq(float dx, float dy, float a, float b, float c) {
#pragma clang fp contract(off)
    const float t = __builtin_fmaf(b + b, dy, a * dx);
    return __builtin_fmaf(dx, t, (c * dy) * dy);
}

__device__ __forceinline__ float twave_sum(float v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Relative pose of the geometry keyframe in the view whose world->camera pose
// is the device FP64 state, same operation order as the host version.
__device__ void make_track_pair(const double* pose, const sgad_pose& kf_pose, const sgad_cam& kc,
                                const sgad_cam& vc, PairConst* out) {
#pragma clang fp contract(off)
    PairConst pc;
    double Rf[9], tf[3];
    for (int i = 0; i < 9; ++i) Rf[i] = (double)kf_pose.R[i];
    for (int i = 0; i < 3; ++i) tf[i] = (double)kf_pose.t[i];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            const double a = pose[i * 3 + 0] * Rf[j * 3 + 0];
            const double b = pose[i * 3 + 1] * Rf[j * 3 + 1];
            const double c = pose[i * 3 + 2] * Rf[j * 3 + 2];
            const double ab = a + b;
            pc.R[i * 3 + j] = ab + c;
        }
    for (int i = 0; i < 3; ++i) {
        const double a = pc.R[i * 3 + 0] * tf[0];
        const double b = pc.R[i * 3 + 1] * tf[1];
        const double c = pc.R[i * 3 + 2] * tf[2];
        const double ab = a + b;
        const double abc = ab + c;
        pc.t[i] = pose[9 + i] - abc;
    }
    for (int i = 0; i < 9; ++i) pc.Rf[i] = (float)pc.R[i];
    for (int i = 0; i < 3; ++i) pc.tf[i] = (float)pc.t[i];
    pc.kfx = kc.fx;
    pc.kfy = kc.fy;
    pc.kcx = kc.cx;
    pc.kcy = kc.cy;
    pc.vfx = vc.fx;
    pc.vfy = vc.fy;
    pc.vcx = vc.cx;
    pc.vcy = vc.cy;
    pc.job = 0;
    pc.kf = 0;
    *out = pc;
}

__global__ void k_track_pair(const double* pose, sgad_pose kf_pose, sgad_cam kc, sgad_cam vc, PairConst* out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    make_track_pair(pose, kf_pose, kc, vc, out);
}

// 96 bytes per entry in LDS; the Jacobian's jx = fx / z and jy = fy / z are
// formed by the walk as fx * (1/z), fy * (1/z), the products the entry would
// have stored.
struct TrackEntry {
    float4 u;   // u, v, dx, dy
    float4 g;   // conic a, b, c, opacity
    float4 c;   // sigma^2, z, x, y
    float4 m;   // 1/z, dmx/dz, dmy/dz, dc/dz
    float4 q0;  // da/dx, da/dy, da/dz, db/dx
    float4 q1;  // db/dy, db/dz, dc/dx, dc/dy
};

__device__ void load_track_entry(const Geometry& G, const RenderBufs& B, uint64_t key, TrackEntry& e) {
    const uint32_t gid = (uint32_t)key;
    const int pix = (int)gid;   // one keyframe
    const PairConst& pc = B.pairs[0];
    const float4* rec = B.pre.rec + 4 * (size_t)pix;
    const float4 r1 = rec[1], r2v = rec[2], r3 = rec[3];
    const float a = r1.x, b = r1.y, c = r1.z;
    e.u = rec[0];
    e.g = r1;
    const float r = r3.z;
    const float x = r3.x, y = r3.y, z = r2v.w;
    const float sg2 = r2v.x;
    const float fx = (float)pc.vfx, fy = (float)pc.vfy;
    const float iz = 1.f / z, iz2 = iz * iz, iz3 = iz2 * iz, iz4 = iz2 * iz2, iz5 = iz4 * iz;
    const float r2 = r * r;
    e.c = make_float4(sg2, z, x, y);
    e.m = make_float4(iz, -fx * x * iz2, -fy * y * iz2, 0.f);
    // dSigma/dX_k (s00, s01, s11), k = x, y, z
    const float p[3] = {r2 * 2.f * fx * fx * x * iz4, 0.f, r2 * fx * fx * (-2.f * iz3 - 4.f * x * x * iz5)};
    const float q[3] = {r2 * fx * fy * y * iz4, r2 * fx * fy * x * iz4, -4.f * r2 * fx * fy * x * y * iz5};
    const float t[3] = {0.f, r2 * 2.f * fy * fy * y * iz4, r2 * fy * fy * (-2.f * iz3 - 4.f * y * y * iz5)};
    float da[3], db[3], dc[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        // d(Q) = -Q dS Q for Q = [[a, b], [b, c]], dS = [[p, q], [q, t]]
        const float ap = a * p[k] + b * q[k], aq = a * q[k] + b * t[k];
        const float bp = b * p[k] + c * q[k], bq = b * q[k] + c * t[k];
        da[k] = -(a * ap + b * aq);
        db[k] = -(a * bp + b * bq);
        dc[k] = -(b * bp + c * bq);
    }
    e.q0 = make_float4(da[0], da[1], da[2], db[0]);
    e.q1 = make_float4(db[1], db[2], dc[0], dc[1]);
    e.m.w = dc[2];
}

template <int TW, int TH>
__global__ __launch_bounds__(TW* TH) void k_track(Geometry G, RenderBufs B, const float* __restrict__ obs,
                                                  float* part) {
    constexpr int NT = TW * TH;
    constexpr int NW = (NT + 63) / 64;
    __shared__ TrackEntry s_e[NT];
    __shared__ float s_red[NW][kTrackVals];
    const int item = blockIdx.x;
    const int tx = item % G.ntx, ty = item / G.ntx;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int px = tx * TW + tid % TW, py = ty * TH + tid / TW;
    const bool inside = px < G.Wv && py < G.Hv;
    const bool ovf = B.status->overflow != 0u;
    const uint32_t st = B.tile_start[item];
    const uint32_t en = ovf ? st : B.tile_start[item + 1];
    const float fpx = (float)px, fpy = (float)py;
    const float vfx = (float)B.pairs[0].vfx, vfy = (float)B.pairs[0].vfy;
    float T = 1.f, Dp = 0.f, Ss = 0.f;
    float dD[6] = {0, 0, 0, 0, 0, 0}, dT[6] = {0, 0, 0, 0, 0, 0};
    bool done = !inside;
    for (uint32_t b0 = st; b0 < en; b0 += NT) {
        const int n = (int)min((uint32_t)NT, en - b0);
        if (tid < n) load_track_entry(G, B, B.keys[b0 + tid], s_e[tid]);
        __syncthreads();
        if (!done) {
            for (int k = 0; k < n; ++k) {
                const float4 eu = s_e[k].u;
                const float dx = (fpx - eu.x) - eu.z, dy = (fpy - eu.y) - eu.w;
                const float4 g = s_e[k].g;
                const float qv = tq(dx, dy, g.x, g.y, g.z);
                if (!(qv <= kQCut)) continue;
                const float Gv = __builtin_amdgcn_exp2f(qv * kNegHalfLog2eT);
                const float raw = g.w * Gv;
                const float alpha = fminf(kAlphaMax, raw);
                if (alpha < kAlphaMin) continue;
                const float om = 1.f - alpha;
                const float test = T * om;
                if (test < kTMin) {
                    done = true;
                    break;
                }
                const float4 ec = s_e[k].c;
                const float w = alpha * T;
                float da[6];
                if (raw < kAlphaMax) {
                    const float4 em = s_e[k].m, q0 = s_e[k].q0, q1 = s_e[k].q1;
                    const float jx = vfx * em.x, jy = vfy * em.x;
                    const float gmx = -2.f * (g.x * dx + g.y * dy);
                    const float gmy = -2.f * (g.y * dx + g.z * dy);
                    const float ga = dx * dx, gb = 2.f * dx * dy, gc = dy * dy;
                    const float vx = gmx * jx + ga * q0.x + gb * q0.w + gc * q1.z;
                    const float vy = gmy * jy + ga * q0.y + gb * q1.x + gc * q1.w;
                    const float vz = gmx * em.y + gmy * em.z + ga * q0.z + gb * q1.y + gc * em.w;
                    const float x = ec.z, y = ec.w, z = ec.y;
                    const float h = -0.5f * alpha;
                    da[0] = h * vx;
                    da[1] = h * vy;
                    da[2] = h * vz;
                    da[3] = h * (y * vz - z * vy);
                    da[4] = h * (z * vx - x * vz);
                    da[5] = h * (x * vy - y * vx);
                } else {
#pragma unroll
                    for (int j = 0; j < 6; ++j) da[j] = 0.f;
                }
                // dz/dxi = (0, 0, 1, y, -x, 0)
                const float dz[6] = {0.f, 0.f, 1.f, ec.w, -ec.z, 0.f};
#pragma unroll
                for (int j = 0; j < 6; ++j) {
                    const float dw = da[j] * T + alpha * dT[j];
                    dD[j] += dw * ec.y + w * dz[j];
                    dT[j] = dT[j] * om - T * da[j];
                }
                Dp += w * ec.y;
                Ss += w * ec.x;
                T = test;
            }
        }
        if (__syncthreads_count(!done) == 0) break;
    }
    // per-pixel residual, Jacobian and contributions
    float vals[kTrackVals];
#pragma unroll
    for (int i = 0; i < kTrackVals; ++i) vals[i] = 0.f;
    if (inside) {
        const float A = 1.f - T;
        const float o = obs[(size_t)py * G.Wv + px];
        if (A >= kAValid && o > 0.f) {
            const float mu = Dp / A;
            const float sd = sqrtf(Ss / A);
            const float r = (o - mu) / sd;
            const float k = -1.f / (A * sd);
            float J[6];
#pragma unroll
            for (int j = 0; j < 6; ++j) J[j] = k * (dD[j] + mu * dT[j]);  // dA = -dT
            int q = 0;
#pragma unroll
            for (int i = 0; i < 6; ++i)
#pragma unroll
                for (int j = i; j < 6; ++j) vals[q++] = J[i] * J[j];
#pragma unroll
            for (int i = 0; i < 6; ++i) vals[21 + i] = J[i] * r;
            vals[27] = -0.5f * r * r - logf(sd) - 0.91893853320467274178f;
            vals[28] = 1.f;
        }
    }
#pragma unroll
    for (int i = 0; i < kTrackVals; ++i) {
        const float sv = twave_sum(vals[i]);
        if (lane == 0) s_red[wave][i] = sv;
    }
    __syncthreads();
    if (tid < kTrackVals) {
        float acc = 0.f;
        for (int w = 0; w < NW; ++w) acc += s_red[w][tid];
        part[(size_t)tid * gridDim.x + item] = acc;   // value-major: [value][item]
    }
}

// One pixel's contribution of one entry (front-to-back order): the same
// operations as the workgroup-tile walk, in the same order.  Returns false
// when the pixel stops before this entry (T would fall below kTMin).
struct TrackPix {
    float T, Dp, Ss, dD[6], dT[6];
};

__device__ __forceinline__ bool track_step(TrackPix& s, const TrackEntry& e, float fpx, float fpy, float vfx,
                                           float vfy) {
    const float4 eu = e.u;
    const float dx = (fpx - eu.x) - eu.z, dy = (fpy - eu.y) - eu.w;
    const float4 g = e.g;
    const float qv = tq(dx, dy, g.x, g.y, g.z);
    if (!(qv <= kQCut)) return true;
    const float Gv = __builtin_amdgcn_exp2f(qv * kNegHalfLog2eT);
    const float raw = g.w * Gv;
    const float alpha = fminf(kAlphaMax, raw);
    if (alpha < kAlphaMin) return true;
    const float om = 1.f - alpha;
    const float test = s.T * om;
    if (test < kTMin) return false;
    const float4 ec = e.c;
    const float w = alpha * s.T;
    float da[6];
    if (raw < kAlphaMax) {
        const float4 em = e.m, q0 = e.q0, q1 = e.q1;
        const float jx = vfx * em.x, jy = vfy * em.x;
        const float gmx = -2.f * (g.x * dx + g.y * dy);
        const float gmy = -2.f * (g.y * dx + g.z * dy);
        const float ga = dx * dx, gb = 2.f * dx * dy, gc = dy * dy;
        const float vx = gmx * jx + ga * q0.x + gb * q0.w + gc * q1.z;
        const float vy = gmy * jy + ga * q0.y + gb * q1.x + gc * q1.w;
        const float vz = gmx * em.y + gmy * em.z + ga * q0.z + gb * q1.y + gc * em.w;
        const float x = ec.z, y = ec.w, z = ec.y;
        const float h = -0.5f * alpha;
        da[0] = h * vx;
        da[1] = h * vy;
        da[2] = h * vz;
        da[3] = h * (y * vz - z * vy);
        da[4] = h * (z * vx - x * vz);
        da[5] = h * (x * vy - y * vx);
    } else {
#pragma unroll
        for (int j = 0; j < 6; ++j) da[j] = 0.f;
    }
    // dz/dxi = (0, 0, 1, y, -x, 0)
    const float dz[6] = {0.f, 0.f, 1.f, ec.w, -ec.z, 0.f};
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        const float dw = da[j] * s.T + alpha * s.dT[j];
        s.dD[j] += dw * ec.y + w * dz[j];
        s.dT[j] = s.dT[j] * om - s.T * da[j];
    }
    s.Dp += w * ec.y;
    s.Ss += w * ec.x;
    s.T = test;
    return true;
}

// Per-pixel residual, Jacobian and the 29 normal-equation terms.
__device__ __forceinline__ void track_terms(const TrackPix& s, float o, float (&vals)[kTrackVals]) {
#pragma unroll
    for (int i = 0; i < kTrackVals; ++i) vals[i] = 0.f;
    const float A = 1.f - s.T;
    if (A >= kAValid && o > 0.f) {
        const float mu = s.Dp / A;
        const float sd = sqrtf(s.Ss / A);
        const float r = (o - mu) / sd;
        const float k = -1.f / (A * sd);
        float J[6];
#pragma unroll
        for (int j = 0; j < 6; ++j) J[j] = k * (s.dD[j] + mu * s.dT[j]);  // dA = -dT
        int q = 0;
#pragma unroll
        for (int i = 0; i < 6; ++i)
#pragma unroll
            for (int j = i; j < 6; ++j) vals[q++] = J[i] * J[j];
#pragma unroll
        for (int i = 0; i < 6; ++i) vals[21 + i] = J[i] * r;
        vals[27] = -0.5f * r * r - logf(sd) - 0.91893853320467274178f;
        vals[28] = 1.f;
    }
}

// 8x8 wave tiles, four per 256-thread workgroup (one partial record per
// workgroup).  Each wave sorts its tile's segment (segments over 1024 keys
// were sorted by the long pass), then per 64-entry chunk publishes the
// derived entries and 16 ballots of their pixel rectangles (3-sigma bounds
// of the q <= 9 ellipse), and each lane walks only its own candidates: the
// entries it skips have q > 9 at its pixel, so every pixel performs the same
// operations in the same order as in the workgroup-tile kernel.
__global__ __launch_bounds__(256) void k_track8(Geometry G, RenderBufs B, const float* __restrict__ obs,
                                                float* part) {
    __shared__ TrackEntry s_e[4][64];
    __shared__ uint64_t s_m[4][16];
    __shared__ float s_red[4][kTrackVals];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int item = blk * 4 + wave;
    const bool tile_ok = item < G.ntiles;
    const int tx = tile_ok ? item % G.ntx : 0, ty = tile_ok ? item / G.ntx : 0;
    const int lx = lane & 7, ly = lane >> 3;
    const int px = tx * 8 + lx, py = ty * 8 + ly;
    const bool inside = tile_ok && px < G.Wv && py < G.Hv;
    const bool ovf = B.status->overflow != 0u;
    const uint32_t st = tile_ok ? B.tile_start[item] : 0u;
    const int len = (ovf || !tile_ok) ? 0 : (int)(B.tile_start[item + 1] - st);
    if (G.fuse_sort) sort_segment(B.keys + st, len, lane, true);
    __syncthreads();   // sorted keys visible to every lane
    const float fpx = (float)px, fpy = (float)py;
    const float fx0 = (float)(tx * 8), fy0 = (float)(ty * 8);
    const float vfx = (float)B.pairs[0].vfx, vfy = (float)B.pairs[0].vfy;
    TrackPix s;
    s.T = 1.f;
    s.Dp = 0.f;
    s.Ss = 0.f;
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        s.dD[j] = 0.f;
        s.dT[j] = 0.f;
    }
    bool done = !inside;
    TrackEntry* se = s_e[wave];
    uint64_t* sm = s_m[wave];
    uint64_t key = lane < len ? B.keys[st + lane] : 0ull;
    for (int c0 = 0; c0 < len; c0 += 64) {
        const int n = min(64, len - c0);
        // tile columns (bits 0-7) and rows (bits 8-15) the entry's 3-sigma
        // rectangle (plus 1e-3 px, which covers the hardware reciprocal and
        // square root) overlaps; sm[k] / sm[8 + k]: the entries covering
        // column / row k, by one transpose across lanes
        uint32_t cover = 0u;
        if (lane < n) {
            TrackEntry e;
            load_track_entry(G, B, key, e);
            se[lane] = e;
            const float mx = (e.u.x - fx0) + e.u.z, my = (e.u.y - fy0) + e.u.w;
            const float idet = __builtin_amdgcn_rcpf(e.g.x * e.g.z - e.g.y * e.g.y);
            const float ex = 3.f * __builtin_amdgcn_sqrtf(e.g.z * idet) + 1e-3f;
            const float ey = 3.f * __builtin_amdgcn_sqrtf(e.g.x * idet) + 1e-3f;
            const int x0 = max(0, (int)ceilf(mx - ex)), x1 = min(7, (int)floorf(mx + ex));
            const int y0 = max(0, (int)ceilf(my - ey)), y1 = min(7, (int)floorf(my + ey));
            if (x0 <= x1 && y0 <= y1)
                cover = ((0xFFu << x0) & (0xFFu >> (7 - x1))) | (((0xFFu << y0) & (0xFFu >> (7 - y1))) << 8);
        }
        const uint64_t col = bit_column<16>(cover, lane);
        if (lane < 16) sm[lane] = col;
        wave_lds_sync();   // (this wave's own LDS region)
        // the next chunk's key while this one is walked
        key = lane < len - c0 - 64 ? B.keys[st + (uint32_t)(c0 + 64 + lane)] : 0ull;
        if (!done) {
            uint64_t m = sm[lx] & sm[8 + ly];
            while (m != 0ull) {
                const int b = (int)__builtin_ctzll(m);
                m &= m - 1ull;
                if (!track_step(s, se[b], fpx, fpy, vfx, vfy)) {
                    done = true;
                    break;
                }
            }
        }
        if (__ballot(!done) == 0ull) break;
        wave_lds_sync();   // walk reads done before the next publish
    }
    float vals[kTrackVals];
    track_terms(s, inside ? obs[(size_t)py * G.Wv + px] : 0.f, vals);
#pragma unroll
    for (int i = 0; i < kTrackVals; ++i) {
        const float sv = twave_sum(vals[i]);
        if (lane == 0) s_red[wave][i] = sv;
    }
    __syncthreads();
    if (threadIdx.x < kTrackVals) {
        const int t = threadIdx.x;
        part[(size_t)t * gridDim.x + blk] = (s_red[0][t] + s_red[1][t]) + (s_red[2][t] + s_red[3][t]);
    }
}

// Partial records k_track / k_track8 write (one per tile, or per four tiles).
int track_parts(const Geometry& G) { return (G.TW == 8 && G.TH == 8) ? (G.ntiles + 3) / 4 : G.ntiles; }

// FP64 sum of the tile partials, damped Cholesky solve, Exp(dxi) * pose.
__device__ bool chol6(const double* A, double* L) {
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j <= i; ++j) {
            double s = A[i * 6 + j];
            for (int k = 0; k < j; ++k) s -= L[i * 6 + k] * L[j * 6 + k];
            if (i == j) {
                if (!(s > 0.0)) return false;
                L[i * 6 + i] = sqrt(s);
            } else {
                L[i * 6 + j] = s / L[j * 6 + j];
            }
        }
    return true;
}

// Also forms the next iteration's relative pose (`next`, when not null).
__global__ __launch_bounds__(512) void k_track_solve(const float* part, int nitems, double* pose, double* trace,
                                                      int it, const DevStatus* st, sgad_pose kf_pose, sgad_cam kc,
                                                      sgad_cam vc, PairConst* next) {
    __shared__ double s_acc[8][kTrackVals];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    double acc[kTrackVals];
#pragma unroll
    for (int i = 0; i < kTrackVals; ++i) acc[i] = 0.0;
    for (int t = tid; t < nitems; t += blockDim.x)
#pragma unroll
        for (int i = 0; i < kTrackVals; ++i) acc[i] += (double)part[(size_t)i * nitems + t];
#pragma unroll
    for (int i = 0; i < kTrackVals; ++i) {
        double v = acc[i];
        for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
        if (lane == 0) s_acc[wave][i] = v;
    }
    __syncthreads();
    if (tid != 0) return;
    double S[kTrackVals];
    for (int i = 0; i < kTrackVals; ++i) {
        double v = 0.0;
        for (int w = 0; w < 8; ++w) v += s_acc[w][i];
        S[i] = v;
    }
    double H[36], g[6];
    int q = 0;
    for (int i = 0; i < 6; ++i)
        for (int j = i; j < 6; ++j) {
            H[i * 6 + j] = S[q];
            H[j * 6 + i] = S[q];
            ++q;
        }
    for (int i = 0; i < 6; ++i) g[i] = S[21 + i];
    double tr = 0.0;
    for (int i = 0; i < 6; ++i) tr += H[i * 6 + i];
    double lam = 0.0, L[36], dxi[6] = {0, 0, 0, 0, 0, 0};
    bool ok = false;
    for (int attempt = 0; attempt < 12 && !st->overflow; ++attempt) {
        double A[36];
        for (int i = 0; i < 36; ++i) A[i] = H[i];
        for (int i = 0; i < 6; ++i) A[i * 6 + i] += lam;
        for (int i = 0; i < 36; ++i) L[i] = 0.0;
        if (chol6(A, L)) {
            ok = true;
            break;
        }
        lam = lam == 0.0 ? 1e-9 * tr : lam * 10.0;
    }
    if (ok) {
        double y[6];
        for (int i = 0; i < 6; ++i) {
            double s = -g[i];
            for (int k = 0; k < i; ++k) s -= L[i * 6 + k] * y[k];
            y[i] = s / L[i * 6 + i];
        }
        for (int i = 5; i >= 0; --i) {
            double s = y[i];
            for (int k = i + 1; k < 6; ++k) s -= L[k * 6 + i] * dxi[k];
            dxi[i] = s / L[i * 6 + i];
        }
    }
    double* rec = trace + (size_t)it * kTraceStride;
    for (int i = 0; i < 21; ++i) rec[i] = S[i];
    for (int i = 0; i < 6; ++i) rec[21 + i] = g[i];
    rec[27] = S[27];
    rec[28] = S[28];
    rec[29] = ok ? lam : -1.0;
    for (int i = 0; i < 6; ++i) rec[30 + i] = dxi[i];
    // Exp(dxi) = [[R, V rho], [0, 1]], R = I + A K + B K^2, V = I + B K + C K^2
    const double* rho = dxi;
    const double* phi = dxi + 3;
    const double th2 = phi[0] * phi[0] + phi[1] * phi[1] + phi[2] * phi[2];
    const double th = sqrt(th2);
    double Ac, Bc, Cc;
    if (th < 1e-4) {
        Ac = 1.0 - th2 / 6.0 + th2 * th2 / 120.0;
        Bc = 0.5 - th2 / 24.0 + th2 * th2 / 720.0;
        Cc = 1.0 / 6.0 - th2 / 120.0 + th2 * th2 / 5040.0;
    } else {
        Ac = sin(th) / th;
        Bc = (1.0 - cos(th)) / th2;
        Cc = (th - sin(th)) / (th2 * th);
    }
    const double K[9] = {0, -phi[2], phi[1], phi[2], 0, -phi[0], -phi[1], phi[0], 0};
    double K2[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) s += K[i * 3 + k] * K[k * 3 + j];
            K2[i * 3 + j] = s;
        }
    double Re[9], V[9];
    for (int i = 0; i < 9; ++i) {
        const double I = (i % 4 == 0) ? 1.0 : 0.0;
        Re[i] = I + Ac * K[i] + Bc * K2[i];
        V[i] = I + Bc * K[i] + Cc * K2[i];
    }
    double te[3];
    for (int i = 0; i < 3; ++i) te[i] = V[i * 3 + 0] * rho[0] + V[i * 3 + 1] * rho[1] + V[i * 3 + 2] * rho[2];
    double Rn[9], tn[3];
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j)
            Rn[i * 3 + j] = Re[i * 3 + 0] * pose[0 * 3 + j] + Re[i * 3 + 1] * pose[1 * 3 + j] +
                            Re[i * 3 + 2] * pose[2 * 3 + j];
        tn[i] = Re[i * 3 + 0] * pose[9] + Re[i * 3 + 1] * pose[10] + Re[i * 3 + 2] * pose[11] + te[i];
    }
    for (int i = 0; i < 9; ++i) pose[i] = Rn[i];
    for (int i = 0; i < 3; ++i) pose[9 + i] = tn[i];
    if (next) make_track_pair(pose, kf_pose, kc, vc, next);
}

void launch_track_pair(const double* pose, const sgad_pose& kf_pose, const sgad_cam& kc, const sgad_cam& vc,
                       PairConst* out, hipStream_t s) {
    hipLaunchKernelGGL(k_track_pair, dim3(1), dim3(64), 0, s, pose, kf_pose, kc, vc, out);
}

bool launch_track(const Geometry& G, const RenderBufs& B, const float* obs, float* part, hipStream_t s) {
    if (G.TW == 16 && G.TH == 16)
        hipLaunchKernelGGL((k_track<16, 16>), dim3(G.ntiles), dim3(256), 0, s, G, B, obs, part);
    else if (G.TW == 8 && G.TH == 8)
        hipLaunchKernelGGL(k_track8, dim3(track_parts(G)), dim3(256), 0, s, G, B, obs, part);
    else if (G.TW == 16 && G.TH == 8)
        hipLaunchKernelGGL((k_track<16, 8>), dim3(G.ntiles), dim3(128), 0, s, G, B, obs, part);
    else if (G.TW == 32 && G.TH == 8)
        hipLaunchKernelGGL((k_track<32, 8>), dim3(G.ntiles), dim3(256), 0, s, G, B, obs, part);
    else
        return false;
    return true;
}

void launch_track_solve(const float* part, int nitems, double* pose, double* trace, int it, const DevStatus* st,
                        const sgad_pose& kf_pose, const sgad_cam& kc, const sgad_cam& vc, PairConst* next,
                        hipStream_t s) {
    hipLaunchKernelGGL(k_track_solve, dim3(1), dim3(512), 0, s, part, nitems, pose, trace, it, st, kf_pose, kc, vc,
                       next);
}

}  // namespace sgad
