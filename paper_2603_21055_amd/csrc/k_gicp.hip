// Tracking a depth frame against a set of geometry Gaussians with
// Generalized ICP (Sec. 3.3, Eq. 2; the supplement's sampling ratio R and
// neighbour count K_c; Tab. 11's point-to-surface correspondences and
// "ellipse" scale normalisation).
//
// A set holds the Gaussians of one frame's stride-R pixel grid, SoA, FP64:
//   [12][n] = x y z | c00 c01 c02 c11 c12 c22 | nx ny nz
// (point in its camera's frame, normalised covariance, normal).  A grid
// pixel without depth has z = 0 there and is never a neighbour or a source.
//
// k_gicp_prepare   one wavefront per grid point: back-projection, its K_c
//                  nearest points of the set (squared distance ((dx^2 +
//                  dy^2) + dz^2), ties by index, a register top-K, searched
//                  in growing windows of grid cells until a distance bound
//                  proves the window exact), their covariance, a cyclic
//                  Jacobi eigen-decomposition, C' = U diag(max(l0/l2, eps),
//                  max(l1/l2, eps), 1) U^T and the normal (smallest).
// k_gicp_linearise_wave one wavefront per source point: X = R a + t, its
//                  K_c nearest target points within D_MAX (the search split
//                  over the lanes), the one with the smallest
//                  (n . e)^2 + eps |e|^2 (first minimum in distance rank);
//                  M = (C_b + R C_a R^T)^-1, J = [-I | [X]x], per-block FP64
//                  partial sums of H = J^T M J (21), g = J^T M e (6),
//                  e^T M e and the count.  The target is a frame's set
//                  (windows of grid cells) or the global set T (shells of
//                  voxels of a hash).
// k_gicp_solve     one block: the partial sums in a fixed order, damped
//                  Cholesky (1e-9 tr H, x10 per retry), dxi = -H^-1 g,
//                  P <- Exp(dxi) P on the device pose, and a trace record.
// Every decision (neighbour sets, correspondences, the distance cut) is
// taken in FP64 with the operation order written here and no contraction,
// so an independent FP64 evaluation in the same order reproduces it.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <algorithm>
#include <climits>
#include <cmath>

#include "sgad_internal.h"

namespace sgad {

constexpr int kGicpMaxK = 32;
constexpr double kGicpEps = 1e-3;
constexpr double kGicpDMax = 0.1;
constexpr int kGicpVals = 29;      // H upper triangle (21), g (6), cost, pair count
constexpr int kGicpTrace = 48;     // trace record: H 21, g 6, cost, n, lambda, dxi 6, R 9, t 3

// Top-K in registers, sorted by (distance, index); every comparison is on
// the pair, so the result does not depend on the order candidates arrive in.
template <int KM>
struct TopK {
    double d[KM];
    int i[KM];
    double worst;
    int worst_i;
};

template <int KM>
__device__ __forceinline__ void topk_init(TopK<KM>& t) {
#pragma unroll
    for (int s = 0; s < KM; ++s) {
        t.d[s] = DBL_MAX;
        t.i[s] = INT_MAX;
    }
    t.worst = DBL_MAX;
    t.worst_i = INT_MAX;
}

template <int KM>
__device__ __forceinline__ void topk_insert(TopK<KM>& t, int k, double d, int j) {
    double cd = d;
    int ci = j;
#pragma unroll
    for (int s = 0; s < KM; ++s) {
        if (s < k) {
            const bool sw = cd < t.d[s] || (cd == t.d[s] && ci < t.i[s]);
            const double td = sw ? t.d[s] : cd;
            const int ti = sw ? t.i[s] : ci;
            t.d[s] = sw ? cd : t.d[s];
            t.i[s] = sw ? ci : t.i[s];
            cd = td;
            ci = ti;
        }
    }
    double w = t.d[0];
    int wi = t.i[0];
#pragma unroll
    for (int s = 0; s < KM; ++s)
        if (s == k - 1) {
            w = t.d[s];
            wi = t.i[s];
        }
    t.worst = w;
    t.worst_i = wi;
}

// Pixel grid a set was sampled on: camera, stride and grid size.
struct GicpGrid {
    double fx, fy, cx, cy;
    int R, gw, gh;
    double m;   // max over the image of |(x, y, 1)|
};

constexpr int kGicpWin = 4;   // half-width (cells) of the first window; doubled until exact

// The k nearest points of `set` (a grid of gw x gh cells) to q: windows of
// growing half-width around the cell q projects to, each new ring of cells
// scanned, until the window provably holds the k nearest.  A point c on the
// ray of a pixel p is at least |q| sin(angle(q, p)) from q, and with r_q, r_p
// the rays (x, y, 1), |q| sin(angle) = q_z |r_q x r_p| / |r_p| >= q_z D / M,
// D the larger of |x_p - x_q| and |y_p - y_q| and M the largest |r_p| over the
// image.  For pixels outside the window, D is at least the normalised
// distance from q's projection to the nearest column or row outside it, so
// once the window's k-th distance is below (q_z D / M)^2 no point outside can
// enter.  A window covering the whole grid is exact by itself; q behind the
// camera scans the whole grid.
//
// With dmax2 finite only points within squared distance dmax2 are candidates
// (the list is the k nearest among them), and the search also ends once no
// point outside the window can be that close.
template <int KM>
__device__ void knn_grid(const double* __restrict__ set, int n, const GicpGrid& g, int k, double qx, double qy,
                         double qz, TopK<KM>& t, double dmax2) {
#pragma clang fp contract(off)
    topk_init(t);
    int cu = 0, cv = 0, w = g.gw + g.gh;      // behind the camera: the whole grid at once
    double u = 0.0, v = 0.0;
    if (qz > 0.0) {
        u = g.fx * (qx / qz) + g.cx;
        v = g.fy * (qy / qz) + g.cy;
        cu = (int)fmin(fmax(rint(u / g.R), 0.0), (double)(g.gw - 1));
        cv = (int)fmin(fmax(rint(v / g.R), 0.0), (double)(g.gh - 1));
        w = kGicpWin;
    }
    int found = 0;
    int lo_u = 1, hi_u = 0, lo_v = 1, hi_v = 0;   // region scanned so far (empty)
    while (true) {
        const int nlo_u = max(0, cu - w), nhi_u = min(g.gw - 1, cu + w);
        const int nlo_v = max(0, cv - w), nhi_v = min(g.gh - 1, cv + w);
        for (int j = nlo_v; j <= nhi_v; ++j)
            for (int i = nlo_u; i <= nhi_u; ++i) {
                if (i >= lo_u && i <= hi_u && j >= lo_v && j <= hi_v) continue;   // scanned before
                const int c = j * g.gw + i;
                const double pz = set[2 * (size_t)n + c];
                if (pz == 0.0) continue;
                const double dx = qx - set[c], dy = qy - set[(size_t)n + c], dz = qz - pz;
                const double d = (dx * dx + dy * dy) + dz * dz;
                if (!(d <= dmax2)) continue;
                ++found;
                if (d < t.worst || (d == t.worst && c < t.worst_i)) topk_insert(t, k, d, c);
            }
        lo_u = nlo_u;
        hi_u = nhi_u;
        lo_v = nlo_v;
        hi_v = nhi_v;
        const bool all = lo_u == 0 && hi_u == g.gw - 1 && lo_v == 0 && hi_v == g.gh - 1;
        if (all) return;
        // normalised distance from q's projection to the nearest column / row outside
        double D = DBL_MAX;
        if (lo_u > 0) D = fmin(D, (u - (double)((lo_u - 1) * g.R)) / g.fx);
        if (hi_u < g.gw - 1) D = fmin(D, ((double)((hi_u + 1) * g.R) - u) / g.fx);
        if (lo_v > 0) D = fmin(D, (v - (double)((lo_v - 1) * g.R)) / g.fy);
        if (hi_v < g.gh - 1) D = fmin(D, ((double)((hi_v + 1) * g.R) - v) / g.fy);
        if (D > 0.0) {
            const double lb = qz * D / g.m;
            const double lb2 = lb * lb * (1.0 - 1e-12);
            if (found >= k && t.worst < lb2) return;
            if (lb2 >= dmax2) return;      // nothing outside is a candidate
        }
        w *= 2;
    }
}

// Cyclic Jacobi eigen-decomposition of a symmetric 3x3 matrix a (row-major,
// overwritten); eigenvalues in w, eigenvectors in the columns of v.
__device__ void jacobi3(double* a, double* w, double* v) {
    for (int i = 0; i < 9; ++i) v[i] = (i % 4 == 0) ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 32; ++sweep) {
        const double off = a[1] * a[1] + a[2] * a[2] + a[5] * a[5];
        const double scale = a[0] * a[0] + a[4] * a[4] + a[8] * a[8];
        if (off <= 1e-30 * scale || off == 0.0) break;
        for (int p = 0; p < 2; ++p)
            for (int q = p + 1; q < 3; ++q) {
                const double apq = a[p * 3 + q];
                if (apq == 0.0) continue;
                const double app = a[p * 3 + p], aqq = a[q * 3 + q];
                const double theta = (aqq - app) / (2.0 * apq);
                const double tt = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                const double c = 1.0 / sqrt(tt * tt + 1.0), s = tt * c;
                for (int r = 0; r < 3; ++r) {       // A <- A J
                    const double arp = a[r * 3 + p], arq = a[r * 3 + q];
                    a[r * 3 + p] = c * arp - s * arq;
                    a[r * 3 + q] = s * arp + c * arq;
                }
                for (int r = 0; r < 3; ++r) {       // A <- J^T A
                    const double apr = a[p * 3 + r], aqr = a[q * 3 + r];
                    a[p * 3 + r] = c * apr - s * aqr;
                    a[q * 3 + r] = s * apr + c * aqr;
                }
                for (int r = 0; r < 3; ++r) {       // V <- V J
                    const double vrp = v[r * 3 + p], vrq = v[r * 3 + q];
                    v[r * 3 + p] = c * vrp - s * vrq;
                    v[r * 3 + q] = s * vrp + c * vrq;
                }
            }
    }
    w[0] = a[0];
    w[1] = a[4];
    w[2] = a[8];
}

// Grid point g = (gy, gx) of a stride-R grid: a = D ((u - cx) / fx, (v - cy) / fy, 1).
__global__ __launch_bounds__(256) void k_gicp_points(const float* __restrict__ depth, int H, int W, int R,
                                                     double fx, double fy, double cx, double cy,
                                                     double* __restrict__ set, int n) {
#pragma clang fp contract(off)
    const int gw = (W + R - 1) / R;
    const int g = (int)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n) return;
    const int gy = g / gw, gx = g - gy * gw;
    const int u = gx * R, v = gy * R;
    const double d = (double)depth[(size_t)v * W + u];
    double x = 0.0, y = 0.0, z = 0.0;
    if (d > 0.0) {
        x = d * (((double)u - cx) / fx);
        y = d * (((double)v - cy) / fy);
        z = d;
    }
    set[g] = x;
    set[(size_t)n + g] = y;
    set[2 * (size_t)n + g] = z;
}

// ---------------------------------------------------------------------------
// Global map T: world Gaussians [12][capacity] (the layout of a set, rows of
// stride `capacity`), at most one per voxel of side `voxel`, found through an
// open-addressing hash of the voxel coordinates (linear probing, `slots` a
// power of two).  keys: packed voxel or kEmpty; vals: the Gaussian's index,
// or, while an insertion runs, -(1 + lowest frame index claiming the voxel).
// ---------------------------------------------------------------------------
constexpr long long kEmpty = -1;
constexpr long long kVoxelBias = 1 << 20;   // voxel coordinates in [-2^20, 2^20) per axis
constexpr int kMapMaxShell = 40;           // voxel >= D_MAX / 32 ends the search by r = 33

__device__ __forceinline__ long long voxel_pack(long long x, long long y, long long z) {
    return ((x + kVoxelBias) << 42) | ((y + kVoxelBias) << 21) | (z + kVoxelBias);
}

__device__ __forceinline__ bool voxel_in_range(long long x, long long y, long long z) {
    return x >= -kVoxelBias && x < kVoxelBias && y >= -kVoxelBias && y < kVoxelBias && z >= -kVoxelBias &&
           z < kVoxelBias;
}

__device__ __forceinline__ int voxel_hash(long long key, int mask) {
    return (int)(((unsigned long long)key * 0x9E3779B97F4A7C15ull) >> 32) & mask;
}

// Slot of `key`, or -1 when absent.
__device__ __forceinline__ int map_find(const long long* keys, int mask, long long key) {
    int s = voxel_hash(key, mask);
    for (int p = 0; p <= mask; ++p) {
        const long long k = keys[s];
        if (k == key) return s;
        if (k == kEmpty) return -1;
        s = (s + 1) & mask;
    }
    return -1;
}

// Wave-wide count of the entries of the lanes' lists below b.
template <int KM>
__device__ __forceinline__ int wave_count_below(const TopK<KM>& t, int k, double b) {
    int c = 0;
#pragma unroll
    for (int q = 0; q < KM; ++q) c += (q < k && t.d[q] < b) ? 1 : 0;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) c += __shfl_xor(c, o, 64);
    return c;
}

struct GridTarget {
    const double* d;
    size_t stride;
    int n;
    GicpGrid g;
    double dmax2;   // candidates within this squared distance (DBL_MAX: all)
    // knn_grid's windows with the cells of each new ring split over the
    // lanes of a wavefront (each lane keeping its own list); the window
    // stops once the lanes together hold k entries below the bound, or the
    // bound passes D_MAX.  Called by every lane with the same query.
    template <int KM>
    __device__ void wave_knn(int k, double qx, double qy, double qz, int lane, TopK<KM>& t) const {
#pragma clang fp contract(off)
        topk_init(t);
        int cu = 0, cv = 0, w = g.gw + g.gh;
        double u = 0.0, v = 0.0;
        if (qz > 0.0) {
            u = g.fx * (qx / qz) + g.cx;
            v = g.fy * (qy / qz) + g.cy;
            cu = (int)fmin(fmax(rint(u / g.R), 0.0), (double)(g.gw - 1));
            cv = (int)fmin(fmax(rint(v / g.R), 0.0), (double)(g.gh - 1));
            w = kGicpWin;
        }
        int lo_u = 1, hi_u = 0, lo_v = 1, hi_v = 0;
        while (true) {
            const int nlo_u = max(0, cu - w), nhi_u = min(g.gw - 1, cu + w);
            const int nlo_v = max(0, cv - w), nhi_v = min(g.gh - 1, cv + w);
            const int wu = nhi_u - nlo_u + 1, nc = wu * (nhi_v - nlo_v + 1);
            for (int p = lane; p < nc; p += 64) {
                const int j = nlo_v + p / wu, i = nlo_u + p % wu;
                if (i >= lo_u && i <= hi_u && j >= lo_v && j <= hi_v) continue;
                const int c = j * g.gw + i;
                const double pz = d[2 * stride + c];
                if (pz == 0.0) continue;
                const double dx = qx - d[c], dy = qy - d[stride + c], dz = qz - pz;
                const double dd = (dx * dx + dy * dy) + dz * dz;
                if (!(dd <= dmax2)) continue;
                if (dd < t.worst || (dd == t.worst && c < t.worst_i)) topk_insert(t, k, dd, c);
            }
            lo_u = nlo_u;
            hi_u = nhi_u;
            lo_v = nlo_v;
            hi_v = nhi_v;
            if (lo_u == 0 && hi_u == g.gw - 1 && lo_v == 0 && hi_v == g.gh - 1) return;
            double D = DBL_MAX;
            if (lo_u > 0) D = fmin(D, (u - (double)((lo_u - 1) * g.R)) / g.fx);
            if (hi_u < g.gw - 1) D = fmin(D, ((double)((hi_u + 1) * g.R) - u) / g.fx);
            if (lo_v > 0) D = fmin(D, (v - (double)((lo_v - 1) * g.R)) / g.fy);
            if (hi_v < g.gh - 1) D = fmin(D, ((double)((hi_v + 1) * g.R) - v) / g.fy);
            if (D > 0.0) {
                const double lb = qz * D / g.m;
                const double lb2 = lb * lb * (1.0 - 1e-12);
                if (wave_count_below(t, k, lb2) >= k) return;
                if (lb2 >= dmax2) return;
            }
            w *= 2;
        }
    }
};

// The k nearest map Gaussians within D_MAX of q: shells of voxels at growing
// Chebyshev distance r from q's voxel.  A Gaussian outside the cube of shells
// scanned so far is at least the distance f from q to the cube's nearest face
// (less 1e-9 m for the rounding of the voxel assignment), so the search can
// end once k candidates are closer than f, or f is beyond D_MAX.  Queries
// outside the map's coordinate range find nothing.
struct MapTarget {
    const double* d;
    size_t stride;
    const long long* keys;
    const int* vals;
    int mask;
    double voxel;

    template <int KM>
    __device__ __forceinline__ void visit(long long x, long long y, long long z, double qx, double qy, double qz,
                                          int k, double dmax2, TopK<KM>& t, int& found) const {
#pragma clang fp contract(off)
        const int sl = map_find(keys, mask, voxel_pack(x, y, z));
        if (sl < 0) return;
        const int c = vals[sl];
        if (c < 0) return;
        const double ex = qx - d[c], ey = qy - d[stride + c], ez = qz - d[2 * stride + c];
        const double dd = (ex * ex + ey * ey) + ez * ez;
        if (!(dd <= dmax2)) return;
        ++found;
        if (dd < t.worst || (dd == t.worst && c < t.worst_i)) topk_insert(t, k, dd, c);
    }

    // The shells with each shell's voxels split over the lanes of a
    // wavefront, each lane keeping its own list; the shells stop once the
    // lanes together hold k entries closer than the scanned cube's faces, or
    // the faces pass D_MAX.  Called by every lane with the same query.
    template <int KM>
    __device__ void wave_knn(int k, double x, double y, double z, int lane, TopK<KM>& t) const {
#pragma clang fp contract(off)
        topk_init(t);
        const double dmax2 = kGicpDMax * kGicpDMax;
        const double lim = (double)(kVoxelBias - kMapMaxShell - 1);
        const double ux = x / voxel, uy = y / voxel, uz = z / voxel;
        if (!(fabs(ux) < lim && fabs(uy) < lim && fabs(uz) < lim)) return;
        const long long cx = (long long)floor(ux), cy = (long long)floor(uy), cz = (long long)floor(uz);
        int found = 0;
        for (int r = 0; r <= kMapMaxShell; ++r) {
            const int side = 2 * r + 1, npos = side * side * side;
            for (int p = lane; p < npos; p += 64) {
                const int dz = p / (side * side) - r, rem = p % (side * side);
                const int dy = rem / side - r, dx = rem % side - r;
                if (max(abs(dx), max(abs(dy), abs(dz))) != r) continue;
                visit(cx + dx, cy + dy, cz + dz, x, y, z, k, dmax2, t, found);
            }
            const double f = fmin(fmin(fmin(x - (double)(cx - r) * voxel, (double)(cx + r + 1) * voxel - x),
                                       fmin(y - (double)(cy - r) * voxel, (double)(cy + r + 1) * voxel - y)),
                                  fmin(z - (double)(cz - r) * voxel, (double)(cz + r + 1) * voxel - z)) -
                             1e-9;
            if (f <= 0.0) continue;
            const double f2 = f * f;
            if (wave_count_below(t, k, f2) >= k) return;
            if (f2 > dmax2) return;
        }
    }
};

// The terms of one pair (source point i of the set src moved to X by the
// pose (Rm, t), target j): H (upper triangle), g, e^T M e and the count, with
// M = (C_b + R C_a R^T)^-1, J = [-I | [X]x], e = b - X.
__device__ __forceinline__ void gicp_pair_terms(const double* __restrict__ src, int ns, int i, const double* Rm,
                                                double X0, double X1, double X2, const double* __restrict__ tgt,
                                                size_t nt, int j, double* acc) {
#pragma clang fp contract(off)
    // C = C_b + R C_a R^T
    const double ca[9] = {src[(size_t)3 * ns + i], src[(size_t)4 * ns + i], src[(size_t)5 * ns + i],
                          src[(size_t)4 * ns + i], src[(size_t)6 * ns + i], src[(size_t)7 * ns + i],
                          src[(size_t)5 * ns + i], src[(size_t)7 * ns + i], src[(size_t)8 * ns + i]};
    double RC[9];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c)
            RC[r * 3 + c] = Rm[r * 3 + 0] * ca[0 * 3 + c] + Rm[r * 3 + 1] * ca[1 * 3 + c] + Rm[r * 3 + 2] * ca[2 * 3 + c];
    double C[9];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c)
            C[r * 3 + c] = RC[r * 3 + 0] * Rm[c * 3 + 0] + RC[r * 3 + 1] * Rm[c * 3 + 1] + RC[r * 3 + 2] * Rm[c * 3 + 2];
    const double cb[6] = {tgt[3 * nt + j], tgt[4 * nt + j], tgt[5 * nt + j],
                          tgt[6 * nt + j], tgt[7 * nt + j], tgt[8 * nt + j]};
    C[0] += cb[0];
    C[1] += cb[1];
    C[2] += cb[2];
    C[3] += cb[1];
    C[4] += cb[3];
    C[5] += cb[4];
    C[6] += cb[2];
    C[7] += cb[4];
    C[8] += cb[5];
    // M = C^-1 by the adjugate (C symmetric positive definite)
    const double m00 = C[4] * C[8] - C[5] * C[7], m01 = C[2] * C[7] - C[1] * C[8], m02 = C[1] * C[5] - C[2] * C[4];
    const double m11 = C[0] * C[8] - C[2] * C[6], m12 = C[2] * C[3] - C[0] * C[5], m22 = C[0] * C[4] - C[1] * C[3];
    const double det = C[0] * m00 + C[1] * (C[5] * C[6] - C[3] * C[8]) + C[2] * (C[3] * C[7] - C[4] * C[6]);
    const double id = 1.0 / det;
    const double M[9] = {m00 * id, m01 * id, m02 * id, m01 * id, m11 * id, m12 * id, m02 * id, m12 * id, m22 * id};
    const double e[3] = {tgt[j] - X0, tgt[nt + j] - X1, tgt[2 * nt + j] - X2};
    // J = [-I | [X]x] (3 x 6)
    const double X[3] = {X0, X1, X2};
    double J[18];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) J[r * 6 + c] = (r == c) ? -1.0 : 0.0;
    J[0 * 6 + 3] = 0.0;   J[0 * 6 + 4] = -X[2]; J[0 * 6 + 5] = X[1];
    J[1 * 6 + 3] = X[2];  J[1 * 6 + 4] = 0.0;   J[1 * 6 + 5] = -X[0];
    J[2 * 6 + 3] = -X[1]; J[2 * 6 + 4] = X[0];  J[2 * 6 + 5] = 0.0;
    double MJ[18], Me[3];
    for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 6; ++c) MJ[r * 6 + c] = M[r * 3 + 0] * J[0 * 6 + c] + M[r * 3 + 1] * J[1 * 6 + c] + M[r * 3 + 2] * J[2 * 6 + c];
        Me[r] = M[r * 3 + 0] * e[0] + M[r * 3 + 1] * e[1] + M[r * 3 + 2] * e[2];
    }
    int q = 0;
    for (int r = 0; r < 6; ++r)
        for (int c = r; c < 6; ++c) acc[q++] = J[0 * 6 + r] * MJ[0 * 6 + c] + J[1 * 6 + r] * MJ[1 * 6 + c] + J[2 * 6 + r] * MJ[2 * 6 + c];
    for (int r = 0; r < 6; ++r) acc[21 + r] = J[0 * 6 + r] * Me[0] + J[1 * 6 + r] * Me[1] + J[2 * 6 + r] * Me[2];
    acc[27] = e[0] * Me[0] + e[1] * Me[1] + e[2] * Me[2];
    acc[28] = 1.0;
}

// Double-precision (value, index) minimum over the wavefront, ties by index.
__device__ __forceinline__ void wave_argmin(double& d, int& idx) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        const double od = __shfl_xor(d, o, 64);
        const int oi = __shfl_xor(idx, o, 64);
        if (od < d || (od == d && oi < idx)) {
            d = od;
            idx = oi;
        }
    }
}

// The k smallest entries of the lanes' sorted lists, in (distance, index)
// order: lane r < k receives the r-th (INT_MAX index past the last).
template <int KM>
__device__ __forceinline__ void wave_take_k(TopK<KM>& t, int k, int lane, double& cd, int& ci) {
    cd = DBL_MAX;
    ci = INT_MAX;
    for (int r = 0; r < k; ++r) {
        double bd = t.d[0];
        int bi = t.i[0];
        wave_argmin(bd, bi);
        if (bi == INT_MAX) break;
        if (lane == r) {
            cd = bd;
            ci = bi;
        }
        if (t.i[0] == bi) {   // the owner drops its head
#pragma unroll
            for (int q = 0; q + 1 < KM; ++q) {
                t.d[q] = t.d[q + 1];
                t.i[q] = t.i[q + 1];
            }
            t.d[KM - 1] = DBL_MAX;
            t.i[KM - 1] = INT_MAX;
        }
    }
}

// Runs after k_gicp_points: reads the coordinate rows, writes rows 3..11.
template <int KM>
__global__ __launch_bounds__(512) void k_gicp_prepare(int k, double* __restrict__ set, int n, GicpGrid grid) {
#pragma clang fp contract(off)
    // one wavefront per grid point: the lanes split the neighbour search,
    // lane 0 forms the covariance from the K_c nearest in order
    __shared__ int s_nb[8][kGicpMaxK];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = (int)blockIdx.x * 8 + wave;
    if (g >= n) return;   // wave-uniform
    const double qx = set[g], qy = set[(size_t)n + g], qz = set[2 * (size_t)n + g];
    if (qz == 0.0) {
        if (lane >= 3 && lane < 12) set[(size_t)lane * n + g] = 0.0;
        return;
    }
    TopK<KM> t;
    {
        GridTarget tg{set, (size_t)n, n, grid, DBL_MAX};
        TopK<KM> tl;
        tg.template wave_knn<KM>(k, qx, qy, qz, lane, tl);
        double cd;
        int ci;
        wave_take_k(tl, k, lane, cd, ci);
        if (lane < k) s_nb[wave][lane] = ci;
    }
    // lane 0 reads what the wave's lanes wrote: wait for the LDS stores
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    if (lane != 0) return;
    topk_init(t);
#pragma unroll
    for (int q = 0; q < KM; ++q)
        if (q < k) t.i[q] = s_nb[wave][q];
    int kk = 0;
    double mx = 0.0, my = 0.0, mz = 0.0;
#pragma unroll
    for (int s = 0; s < KM; ++s)
        if (s < k && t.i[s] != INT_MAX) {
            const int j = t.i[s];
            mx += set[j];
            my += set[(size_t)n + j];
            mz += set[2 * (size_t)n + j];
            ++kk;
        }
    mx /= (double)kk;
    my /= (double)kk;
    mz /= (double)kk;
    double c[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int s = 0; s < KM; ++s)
        if (s < k && t.i[s] != INT_MAX) {
            const int j = t.i[s];
            const double dx = set[j] - mx, dy = set[(size_t)n + j] - my, dz = set[2 * (size_t)n + j] - mz;
            c[0] += dx * dx;
            c[1] += dx * dy;
            c[2] += dx * dz;
            c[4] += dy * dy;
            c[5] += dy * dz;
            c[8] += dz * dz;
        }
    for (int i = 0; i < 9; ++i) c[i] /= (double)kk;
    c[3] = c[1];
    c[6] = c[2];
    c[7] = c[5];
    double w[3], v[9];
    jacobi3(c, w, v);
    // ascending order of the eigenvalues
    int o[3] = {0, 1, 2};
    if (w[o[0]] > w[o[1]]) { const int x = o[0]; o[0] = o[1]; o[1] = x; }
    if (w[o[1]] > w[o[2]]) { const int x = o[1]; o[1] = o[2]; o[2] = x; }
    if (w[o[0]] > w[o[1]]) { const int x = o[0]; o[0] = o[1]; o[1] = x; }
    const double l2 = w[o[2]];
    double sc[3];
    if (l2 > 0.0) {
        sc[0] = fmax(w[o[0]] / l2, kGicpEps);
        sc[1] = fmax(w[o[1]] / l2, kGicpEps);
        sc[2] = 1.0;
    } else {
        sc[0] = kGicpEps;
        sc[1] = kGicpEps;
        sc[2] = 1.0;
    }
    double cn[6] = {0, 0, 0, 0, 0, 0};   // c00 c01 c02 c11 c12 c22
    for (int e = 0; e < 3; ++e) {
        const double ux = v[0 * 3 + o[e]], uy = v[1 * 3 + o[e]], uz = v[2 * 3 + o[e]];
        cn[0] += sc[e] * ux * ux;
        cn[1] += sc[e] * ux * uy;
        cn[2] += sc[e] * ux * uz;
        cn[3] += sc[e] * uy * uy;
        cn[4] += sc[e] * uy * uz;
        cn[5] += sc[e] * uz * uz;
    }
    for (int r = 0; r < 6; ++r) set[(size_t)(3 + r) * n + g] = cn[r];
    set[(size_t)9 * n + g] = v[0 * 3 + o[0]];
    set[(size_t)10 * n + g] = v[1 * 3 + o[0]];
    set[(size_t)11 * n + g] = v[2 * 3 + o[0]];
}

// GICP linearisation with one wavefront per source point (eight per block):
// the target's wave_knn splits the neighbour search over the lanes, each
// keeping its own top-K list; the K nearest are then taken from the lanes'
// sorted lists in (distance, index) order, lane r receiving the r-th; the
// lanes evaluate their candidate's surface distance, and the pair's terms are
// formed by lane 0.  Same results as the one-thread searches of the targets,
// with 64 times as many threads at work.
constexpr int kWavePoints = 8;   // source points (wavefronts) per block of the linearisation

template <int KM, class Target>
__global__ __launch_bounds__(64 * kWavePoints) void k_gicp_linearise_wave(const double* __restrict__ src, int ns,
                                                                          Target tg, int k,
                                                                          const double* __restrict__ pose,
                                                                          double* __restrict__ part,
                                                                          int* __restrict__ corr) {
#pragma clang fp contract(off)
    __shared__ double s_acc[kWavePoints][kGicpVals];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int i = (int)blockIdx.x * kWavePoints + wave;
    double Rm[9], tv[3];
#pragma unroll
    for (int r = 0; r < 9; ++r) Rm[r] = pose[r];
#pragma unroll
    for (int r = 0; r < 3; ++r) tv[r] = pose[9 + r];
    const bool in = i < ns;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    if (in) {
        a0 = src[i];
        a1 = src[(size_t)ns + i];
        a2 = src[2 * (size_t)ns + i];
    }
    const double X0 = ((Rm[0] * a0 + Rm[1] * a1) + Rm[2] * a2) + tv[0];
    const double X1 = ((Rm[3] * a0 + Rm[4] * a1) + Rm[5] * a2) + tv[1];
    const double X2 = ((Rm[6] * a0 + Rm[7] * a1) + Rm[8] * a2) + tv[2];
    // wave-uniform: every lane holds the same point
    const bool active = in && a2 != 0.0;
    int j = -1;
    if (active) {
        TopK<KM> t;
        tg.template wave_knn<KM>(k, X0, X1, X2, lane, t);
        // the K nearest, one per round, into lanes 0 .. K-1
        double cd;
        int ci;
        wave_take_k(t, k, lane, cd, ci);
        // the closest surface element, first minimum in distance order
        const double* tgt = tg.d;
        const size_t nt = tg.stride;
        double ds = DBL_MAX;
        int rank = INT_MAX;
        if (ci != INT_MAX) {
            const int c2 = ci;
            const double e0 = X0 - tgt[c2], e1 = X1 - tgt[nt + c2], e2 = X2 - tgt[2 * nt + c2];
            const double n0 = tgt[9 * nt + c2], n1 = tgt[10 * nt + c2], n2 = tgt[11 * nt + c2];
            const double dn = (n0 * e0 + n1 * e1) + n2 * e2;
            const double ee = (e0 * e0 + e1 * e1) + e2 * e2;
            ds = dn * dn + kGicpEps * ee;
            rank = lane;
        }
        wave_argmin(ds, rank);
        if (rank != INT_MAX) j = __shfl(ci, rank, 64);
    }
    double acc[kGicpVals];
#pragma unroll
    for (int q = 0; q < kGicpVals; ++q) acc[q] = 0.0;
    if (lane == 0) {
        if (corr && in) corr[i] = j;
        if (j >= 0) gicp_pair_terms(src, ns, i, Rm, X0, X1, X2, tg.d, tg.stride, j, acc);
#pragma unroll
        for (int q = 0; q < kGicpVals; ++q) s_acc[wave][q] = acc[q];
    }
    __syncthreads();
    if (threadIdx.x < kGicpVals) {
        const int q = threadIdx.x;
        double v = 0.0;
        for (int w = 0; w < kWavePoints; ++w) v += s_acc[w][q];
        part[(size_t)blockIdx.x * kGicpVals + q] = v;
    }
}

// Sum of the partial records in a fixed order (blocks of 1024 threads):
// value q's blocks b = r (mod 32) summed in block order by thread 32 q + r,
// then the 32 partial sums in r order.
constexpr int kSumStrands = 32;

__device__ __forceinline__ void gicp_sum(const double* part, int nb, double* S) {
    __shared__ double s_p[kGicpVals][kSumStrands];
    const int t = threadIdx.x;
    if (t < kGicpVals * kSumStrands) {
        const int q = t / kSumStrands, r = t % kSumStrands;
        double v = 0.0;
#pragma unroll 4
        for (int b = r; b < nb; b += kSumStrands) v += part[(size_t)b * kGicpVals + q];
        s_p[q][r] = v;
    }
    __syncthreads();
    if (t < kGicpVals) {
        double v = 0.0;
        for (int r = 0; r < kSumStrands; ++r) v += s_p[t][r];
        S[t] = v;
    }
}

__global__ __launch_bounds__(1024) void k_gicp_sum(const double* part, int nb, double* out) {
    __shared__ double S[kGicpVals];
    gicp_sum(part, nb, S);
    __syncthreads();
    if (threadIdx.x < kGicpVals) out[threadIdx.x] = S[threadIdx.x];
}

__device__ bool gicp_chol6(const double* A, double* L) {
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

// One Gauss-Newton step on the device pose; trace record `it` if trace.
__global__ __launch_bounds__(1024) void k_gicp_solve(const double* part, int nb, double* pose, double* trace, int it) {
    __shared__ double S[kGicpVals];
    gicp_sum(part, nb, S);
    __syncthreads();
    if (threadIdx.x != 0) return;
    double Hm[36], g[6];
    int q = 0;
    for (int i = 0; i < 6; ++i)
        for (int j = i; j < 6; ++j) {
            Hm[i * 6 + j] = S[q];
            Hm[j * 6 + i] = S[q];
            ++q;
        }
    for (int i = 0; i < 6; ++i) g[i] = S[21 + i];
    double tr = 0.0;
    for (int i = 0; i < 6; ++i) tr += Hm[i * 6 + i];
    double lam = 0.0, L[36], dxi[6] = {0, 0, 0, 0, 0, 0};
    bool ok = false;
    for (int attempt = 0; attempt < 12; ++attempt) {
        double A[36];
        for (int i = 0; i < 36; ++i) A[i] = Hm[i];
        for (int i = 0; i < 6; ++i) A[i * 6 + i] += lam;
        for (int i = 0; i < 36; ++i) L[i] = 0.0;
        if (gicp_chol6(A, L)) {
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
    // Exp(dxi) = [[Re, V rho], [0, 1]]: Re = I + A K + B K^2, V = I + B K + C K^2
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
    double K2[9], Re[9], V[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            K2[i * 3 + j] = K[i * 3 + 0] * K[0 * 3 + j] + K[i * 3 + 1] * K[1 * 3 + j] + K[i * 3 + 2] * K[2 * 3 + j];
    for (int i = 0; i < 9; ++i) {
        const double I = (i % 4 == 0) ? 1.0 : 0.0;
        Re[i] = I + Ac * K[i] + Bc * K2[i];
        V[i] = I + Bc * K[i] + Cc * K2[i];
    }
    double Rn[9], tn[3];
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j)
            Rn[i * 3 + j] = Re[i * 3 + 0] * pose[0 * 3 + j] + Re[i * 3 + 1] * pose[1 * 3 + j] + Re[i * 3 + 2] * pose[2 * 3 + j];
        tn[i] = Re[i * 3 + 0] * pose[9] + Re[i * 3 + 1] * pose[10] + Re[i * 3 + 2] * pose[11] +
                (V[i * 3 + 0] * rho[0] + V[i * 3 + 1] * rho[1] + V[i * 3 + 2] * rho[2]);
    }
    if (trace) {
        double* rec = trace + (size_t)it * kGicpTrace;
        for (int i = 0; i < 27; ++i) rec[i] = S[i];
        rec[27] = S[27];
        rec[28] = S[28];
        rec[29] = ok ? lam : -1.0;
        for (int i = 0; i < 6; ++i) rec[30 + i] = dxi[i];
        for (int i = 0; i < 9; ++i) rec[36 + i] = pose[i];
        for (int i = 0; i < 3; ++i) rec[45 + i] = pose[9 + i];
    }
    for (int i = 0; i < 9; ++i) pose[i] = Rn[i];
    for (int i = 0; i < 3; ++i) pose[9 + i] = tn[i];
}

int gicp_grid_points(int H, int W, int R) { return ((H + R - 1) / R) * ((W + R - 1) / R); }

static GicpGrid gicp_grid(const sgad_cam& cam, int R) {
    GicpGrid g;
    g.fx = cam.fx;
    g.fy = cam.fy;
    g.cx = cam.cx;
    g.cy = cam.cy;
    g.R = R;
    g.gw = (cam.W + R - 1) / R;
    g.gh = (cam.H + R - 1) / R;
    // the largest |(x, y, 1)| over the image is at a corner
    double m = 0.0;
    for (int cy = 0; cy < 2; ++cy)
        for (int cx = 0; cx < 2; ++cx) {
            const double x = ((double)(cx ? cam.W - 1 : 0) - g.cx) / g.fx;
            const double y = ((double)(cy ? cam.H - 1 : 0) - g.cy) / g.fy;
            m = std::max(m, std::sqrt(1.0 + x * x + y * y));
        }
    g.m = m;
    return g;
}
int gicp_blocks(int n) { return (n + 255) / 256; }
int gicp_vals() { return kGicpVals; }
int gicp_trace_stride() { return kGicpTrace; }
int gicp_max_k() { return kGicpMaxK; }

void launch_gicp_prepare(const float* depth, int H, int W, int R, const sgad_cam& cam, int k, double* set,
                         hipStream_t s) {
    const int n = gicp_grid_points(H, W, R);
    const dim3 grid(gicp_blocks(n)), blk(256);
    hipLaunchKernelGGL(k_gicp_points, grid, blk, 0, s, depth, H, W, R, (double)cam.fx, (double)cam.fy,
                       (double)cam.cx, (double)cam.cy, set, n);
    const dim3 wgrid((n + 7) / 8), wblk(512);
    if (k <= 16) hipLaunchKernelGGL(k_gicp_prepare<16>, wgrid, wblk, 0, s, k, set, n, gicp_grid(cam, R));
    else hipLaunchKernelGGL(k_gicp_prepare<kGicpMaxK>, wgrid, wblk, 0, s, k, set, n, gicp_grid(cam, R));
}

int gicp_wave_blocks(int n) { return (n + kWavePoints - 1) / kWavePoints; }

template <class Target>
static void linearise_wave(const double* src, int ns, const Target& tg, int k, const double* pose, double* part,
                           int* corr, hipStream_t s) {
    const dim3 grid(gicp_wave_blocks(ns)), blk(64 * kWavePoints);
    if (k <= 16)
        hipLaunchKernelGGL((k_gicp_linearise_wave<16, Target>), grid, blk, 0, s, src, ns, tg, k, pose, part, corr);
    else
        hipLaunchKernelGGL((k_gicp_linearise_wave<kGicpMaxK, Target>), grid, blk, 0, s, src, ns, tg, k, pose, part,
                           corr);
}

void launch_gicp_linearise(const double* src, int ns, const double* tgt, int nt, const sgad_cam& tcam, int tR,
                           int k, const double* pose, double* part, int* corr, hipStream_t s) {
    GridTarget tg{tgt, (size_t)nt, nt, gicp_grid(tcam, tR), kGicpDMax * kGicpDMax};
    linearise_wave(src, ns, tg, k, pose, part, corr, s);
}

void launch_gicp_linearise_map(const double* src, int ns, const sgad_gmap& m, int k, const double* pose,
                               double* part, int* corr, hipStream_t s) {
    MapTarget tg{m.data, (size_t)m.capacity, (const long long*)m.keys, m.vals, m.slots - 1, m.voxel};
    linearise_wave(src, ns, tg, k, pose, part, corr, s);
}

// ---------------------------------------------------------------------------
// Map maintenance
// ---------------------------------------------------------------------------
__global__ void k_gmap_reset(long long* keys, int* vals, int slots, int* count) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < slots; i += gridDim.x * blockDim.x) {
        keys[i] = kEmpty;
        vals[i] = INT_MIN;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) *count = 0;
}

// World point of frame Gaussian i under the camera-to-world pose, in the
// fixed order ((r0 a0 + r1 a1) + r2 a2) + t.
__device__ __forceinline__ void world_point(const double* set, int n, int i, const double* P, double* w) {
#pragma clang fp contract(off)
    const double a0 = set[i], a1 = set[(size_t)n + i], a2 = set[2 * (size_t)n + i];
    for (int r = 0; r < 3; ++r) w[r] = ((P[3 * r] * a0 + P[3 * r + 1] * a1) + P[3 * r + 2] * a2) + P[9 + r];
}

__device__ __forceinline__ bool voxel_of(const double* w, double voxel, long long* key) {
    const long long x = (long long)floor(w[0] / voxel), y = (long long)floor(w[1] / voxel),
                    z = (long long)floor(w[2] / voxel);
    if (!voxel_in_range(x, y, z)) return false;
    *key = voxel_pack(x, y, z);
    return true;
}

// Pass 1: every valid frame Gaussian whose voxel is not already in the map
// claims it; among one frame's claims on a voxel the lowest index wins.
__global__ __launch_bounds__(256) void k_gmap_claim(const double* __restrict__ set, int n, const double* pose,
                                                    long long* keys, int* vals, int mask, double voxel) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || set[2 * (size_t)n + i] == 0.0) return;
    double P[12];
    for (int r = 0; r < 12; ++r) P[r] = pose[r];
    double w[3];
    world_point(set, n, i, P, w);
    long long key;
    if (!voxel_of(w, voxel, &key)) return;
    int s = voxel_hash(key, mask);
    for (int p = 0; p <= mask; ++p) {
        long long k = keys[s];
        if (k == kEmpty) {
            const long long prev = (long long)atomicCAS((unsigned long long*)&keys[s], (unsigned long long)kEmpty,
                                                        (unsigned long long)key);
            k = prev == kEmpty ? key : prev;
        }
        if (k == key) {
            if (vals[s] < 0) atomicMax(&vals[s], -(i + 1));   // existing voxels hold an index >= 0
            return;
        }
        s = (s + 1) & mask;
    }
}

// Pass 2 (one block): the winners in index order are appended after the
// map's current count (up to the capacity), moved into the world, and
// their voxels finalised with their map index.
__global__ __launch_bounds__(1024) void k_gmap_commit(const double* __restrict__ set, int n, const double* pose,
                                                      const long long* keys, int* vals, int mask, double voxel,
                                                      double* data, int cap, int* count) {
    __shared__ int s_sum[16];
    __shared__ int s_base;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    double P[12];
    for (int r = 0; r < 12; ++r) P[r] = pose[r];
    const int per = (n + 1023) / 1024, b = tid * per;
    auto winner = [&](int i, int* slot) -> bool {
        if (set[2 * (size_t)n + i] == 0.0) return false;
        double w[3];
        world_point(set, n, i, P, w);
        long long key;
        if (!voxel_of(w, voxel, &key)) return false;
        const int s = map_find(keys, mask, key);
        if (s < 0 || vals[s] != -(i + 1)) return false;
        *slot = s;
        return true;
    };
    int mine = 0;
    for (int i = b; i < min(n, b + per); ++i) {
        int sl;
        mine += winner(i, &sl) ? 1 : 0;
    }
    // exclusive scan of the per-thread counts
    int inc = mine;
    for (int o = 1; o < 64; o <<= 1) {
        const int v = __shfl_up(inc, o, 64);
        if (lane >= o) inc += v;
    }
    if (lane == 63) s_sum[wave] = inc;
    if (tid == 0) s_base = *count;
    __syncthreads();
    int off = 0;
    for (int w = 0; w < wave; ++w) off += s_sum[w];
    int pos = s_base + off + inc - mine;
    for (int i = b; i < min(n, b + per); ++i) {
        int sl;
        if (!winner(i, &sl)) continue;
        if (pos < cap) {
            double w[3];
            world_point(set, n, i, P, w);
            const double ca[9] = {set[(size_t)3 * n + i], set[(size_t)4 * n + i], set[(size_t)5 * n + i],
                                  set[(size_t)4 * n + i], set[(size_t)6 * n + i], set[(size_t)7 * n + i],
                                  set[(size_t)5 * n + i], set[(size_t)7 * n + i], set[(size_t)8 * n + i]};
            double RC[9], C[9];
            for (int r = 0; r < 3; ++r)
                for (int c = 0; c < 3; ++c)
                    RC[r * 3 + c] = P[r * 3] * ca[c] + P[r * 3 + 1] * ca[3 + c] + P[r * 3 + 2] * ca[6 + c];
            for (int r = 0; r < 3; ++r)
                for (int c = 0; c < 3; ++c)
                    C[r * 3 + c] = RC[r * 3] * P[c * 3] + RC[r * 3 + 1] * P[c * 3 + 1] + RC[r * 3 + 2] * P[c * 3 + 2];
            const double nx = set[(size_t)9 * n + i], ny = set[(size_t)10 * n + i], nz = set[(size_t)11 * n + i];
            const size_t st = (size_t)cap;
            data[pos] = w[0];
            data[st + pos] = w[1];
            data[2 * st + pos] = w[2];
            data[3 * st + pos] = C[0];
            data[4 * st + pos] = C[1];
            data[5 * st + pos] = C[2];
            data[6 * st + pos] = C[4];
            data[7 * st + pos] = C[5];
            data[8 * st + pos] = C[8];
            for (int r = 0; r < 3; ++r) data[(9 + r) * st + pos] = P[r * 3] * nx + P[r * 3 + 1] * ny + P[r * 3 + 2] * nz;
            vals[sl] = pos;
        } else {
            vals[sl] = INT_MIN;   // T is full: the voxel stays free for later frames
        }
        ++pos;
    }
    __syncthreads();
    if (tid == 1023) *count = min(cap, pos);
}

void launch_gmap_reset(const sgad_gmap& m, hipStream_t s) {
    hipLaunchKernelGGL(k_gmap_reset, dim3(std::min(1024, (m.slots + 255) / 256)), dim3(256), 0, s,
                       (long long*)m.keys, m.vals, m.slots, m.count);
}

void launch_gmap_insert(const sgad_gmap& m, const double* set, int n, const double* pose, hipStream_t s) {
    hipLaunchKernelGGL(k_gmap_claim, dim3(gicp_blocks(n)), dim3(256), 0, s, set, n, pose, (long long*)m.keys,
                       m.vals, m.slots - 1, m.voxel);
    hipLaunchKernelGGL(k_gmap_commit, dim3(1), dim3(1024), 0, s, set, n, pose, (const long long*)m.keys, m.vals,
                       m.slots - 1, m.voxel, m.data, m.capacity, m.count);
}

// Depth holes (<= 0) filled by D'/A where A >= alpha_min; valid depths kept.
__global__ void k_fill_depth(int P, const float* depth, const float* rdepth, const float* ralpha, float alpha_min,
                             float* out) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < P; i += gridDim.x * blockDim.x) {
        const float d = depth[i];
        float o = d;
        if (!(d > 0.f)) o = ralpha[i] >= alpha_min ? rdepth[i] / ralpha[i] : 0.f;
        out[i] = o;
    }
}

void launch_fill_depth(int P, const float* depth, const float* rdepth, const float* ralpha, float alpha_min,
                       float* out, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_depth, dim3(std::min(4096, (P + 255) / 256)), dim3(256), 0, s, P, depth, rdepth,
                       ralpha, alpha_min, out);
}

void launch_gicp_sum(const double* part, int nb, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_gicp_sum, dim3(1), dim3(1024), 0, s, part, nb, out);
}

void launch_gicp_solve(const double* part, int nb, double* pose, double* trace, int it, hipStream_t s) {
    hipLaunchKernelGGL(k_gicp_solve, dim3(1), dim3(1024), 0, s, part, nb, pose, trace, it);
}

}  // namespace sgad
