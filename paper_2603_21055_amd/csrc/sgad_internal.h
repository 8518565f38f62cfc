// Internal structures shared by the host API and the HIP kernels of libsgad.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/sgad.h"

namespace sgad {

// Splatting constants (see the conventions in sgad.h).
constexpr double kLowpass = 0.3;
constexpr float kAlphaMin = 1.0f / 255.0f;
constexpr float kAlphaMax = 0.99f;
constexpr float kTMin = 1e-4f;
constexpr double kZNear = 0.2;
constexpr float kQCut = 9.0f;
constexpr int kMaxKf = 64;
constexpr int kMaxAdamGroups = 32;
constexpr int kMaxGraphAdam = 8;   // Adam calls one captured graph may hold

// Relative transform and intrinsics of one (job, keyframe) pair.
struct PairConst {
    double R[9];   // R_rel = R_view R_kf^T (FP64, fixed operation order)
    double t[3];   // t_rel = t_view - R_rel t_kf
    double kfx, kfy, kcx, kcy;  // keyframe intrinsics
    double vfx, vfy, vcx, vcy;  // view intrinsics
    float Rf[9], tf[3];         // the same transform rounded to float
    int32_t job, kf;
};

struct KfPtrs {
    const float* depth;
    const float* offset;
    const float* radius;
    const float* opacity;
    const float* rgb;
    const float* sigma;
};

struct KfGradPtrs {
    float* d_rgb;
    float* d_opacity;
    float* d_radius;
    float* d_offset;
};

// Device-side status latched by kernels.
struct DevStatus {
    uint32_t total;      // instances after the count pass (all jobs)
    uint32_t overflow;   // total > capacity
    uint32_t nonfinite;  // a non-finite input was seen
    uint32_t queue;      // work-queue counter of persistent kernels
    uint32_t sticky;     // bit 0: an overflow, bit 1: a non-finite input, since the call began
    uint32_t max_seg;    // longest (job, tile) instance list of the call
};

// Preprocessed per (pair, Gaussian) data.  rec holds one 64-byte record per
// Gaussian (one cache line per gather):
//   [u, v, dx, dy] [a, b, c, o] [c0, c1, c2, z] [x, y, r, sign(D + delta)]
// (dx, dy) = projected mean - (u, v) in view pixels, (a, b, c) the conic,
// o the opacity, c0..c2 the colour (sigma^2 in c0 for tracking), z the view
// depth, (x, y) the view-space centre, r the radius.
struct Preproc {
    float4* rec;   // [n_pairs * N * 4]
    float4* dir;   // [n_pairs * N]: d(view-space centre)/d(offset) = sign(D + delta) R_rel (xn, yn, 1), 0; null: not written
    uint32_t* rx;  // tile x0 | x1 << 16
    uint32_t* ry;  // tile y0 | y1 << 16
    float* z;      // view depth (float), the sort key source
};

struct Geometry {
    int n_kf, n_jobs, n_pairs;
    int Hk, Wk, N;        // keyframe size, N = Hk * Wk
    int Hv, Wv, P;        // view size
    int TW, TH, ntx, nty, ntiles;
    int sc_fwd = 4;    // 64-entry chunks the 8x8 forward publishes at once (1, 2 or 4)
    int sort_long = 2; // long-segment sort pass: 0 none (the register sort takes all), 1 LDS for up to
                       // 2048 keys, 2 up to 4096
    int sc_bwd = 16;   // backward sub-chunk of the 8x8 kernels (16 or 32 entries)
    int fuse_sort = 0; // the 8x8 forward sorts its own segment (no separate sort launch)
    double inv_n = 0.0;   // 1 / N: the keyframe of a Gaussian id without an integer division
};

struct RenderBufs {
    const PairConst* pairs;   // [n_pairs]
    const KfPtrs* kfs;        // [n_kf]
    const int32_t* pair_of;   // [n_jobs * n_kf] -> pair index or -1
    Preproc pre;
    uint32_t* tile_count;     // [n_jobs * ntiles]
    uint32_t* tile_start;     // [n_jobs * ntiles + 1]
    uint32_t* tile_fill;      // [n_jobs * ntiles]
    uint32_t* chunk_start;    // [n_jobs * ntiles + 1]: exclusive scan of ceil(count / 64)
    uint64_t* keys;           // [capacity]
    uint64_t* cmask;          // [chunks][64]: per 64-entry chunk and pixel, the contributing entries
    uint32_t capacity;
    float* Tfinal;            // [n_jobs * P]
    uint32_t* last;           // [n_jobs * P]
    DevStatus* status;
    uint32_t* status_host;    // device address of the call's pinned host copy of *status, or null
};

// Multi-tensor Adam: group g owns elements [off[g], off[g+1]) of the flat range.
struct AdamGroups {
    int n;
    float* p[kMaxAdamGroups];
    float* g[kMaxAdamGroups];
    float* m[kMaxAdamGroups];
    float* v[kMaxAdamGroups];
    int64_t off[kMaxAdamGroups + 1];
    float lr[kMaxAdamGroups];
    float lo[kMaxAdamGroups];
    float hi[kMaxAdamGroups];
    int space[kMaxAdamGroups];
    int boff[kMaxAdamGroups + 1];   // first block of each group (set by the launcher)
    int vec[kMaxAdamGroups];        // all four arrays 16-byte aligned
};

}  // namespace sgad
