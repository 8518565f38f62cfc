// Wave-tile compositing: one 8x8 tile per wavefront (one wavefront per
// workgroup, no barriers), one lane per pixel.
//
// The tile's sorted instance list is taken in chunks of 64 entries.  For each
// chunk every lane publishes one entry in LDS and computes the pixel rectangle
// that bounds the entry's 3-sigma ellipse inside the tile; sixteen wave ballots
// turn those rectangles into 8 column masks and 8 row masks, and pixel (c, r)
// takes the chunk's candidates as col[c] & row[r].  Each lane then walks only
// its own candidates, in list order (forward) or reverse list order
// (backward), so a pixel evaluates ~47 pairs instead of the whole list.  The
// rectangle is a superset of every pair with q <= 9 as evaluated in FP32, so
// the contributor sets and their order are exactly those of the full-list
// walk.
//
// Latency hiding: the records of the next chunk are gathered from HBM into
// registers while the current chunk is walked (keys two chunks ahead, records
// one chunk ahead), and the walks take two candidates per round, whose
// evaluations (LDS reads, q, exp, alpha) are independent of each other.
#include <hip/hip_runtime.h>

#include "raster_common.h"
#include "segsort.h"

namespace sgad {

__device__ __forceinline__ uint64_t low_bits(int k) { return k >= 64 ? ~0ull : ((1ull << k) - 1ull); }

// One lane's share of a chunk, gathered from HBM: its entry's key and record.
struct ChunkRegs {
    uint64_t key;
    float4 r0, r1, r2;
};

// Key of entry `e` of the list starting at `base` (0 when e >= n).
__device__ __forceinline__ uint64_t fetch_key(const RenderBufs& B, uint32_t base, int e, int n) {
    return e < n ? B.keys[base + (uint32_t)e] : 0ull;
}

// Record of `key` (pair looked up in the job's pair table `pof`).
__device__ __forceinline__ void fetch_record(const Geometry& G, const RenderBufs& B, const int* pof, bool valid,
                                             ChunkRegs& c) {
    if (!valid) return;
    const uint32_t gid = (uint32_t)c.key;
    const int kf = kf_of_gid(G, gid);
    const int pix = (int)(gid - (uint32_t)kf * (uint32_t)G.N);
    const size_t i = (size_t)pof[kf] * G.N + pix;
    const float4* rec = B.pre.rec + 4 * i;
    c.r0 = rec[0];
    c.r1 = rec[1];
    c.r2 = rec[2];
}

// Publish a chunk in LDS (records and coverage masks).  sm[k] (k < 8) is the
// set of the chunk's entries whose pixel rectangle covers tile column k,
// sm[8 + k] those covering tile row k: each entry lane forms its 8 column
// bits and 8 row bits, and one transpose across lanes gives lane j the set
// of column j of those 16-bit rows.  The rectangle is the 3-sigma extent
// plus 1e-3 pixels, which covers the ~1 ulp of the hardware reciprocal and
// square root; pixels inside it are tested exactly by the walk.
__device__ __forceinline__ void publish_chunk(const ChunkRegs& c, bool valid, int lane, float fx0, float fy0,
                                              float4 (*se)[3], uint64_t* sm) {
    uint32_t cover = 0u;   // bits 0-7: tile columns, 8-15: tile rows
    if (valid) {
        const float4 eu = c.r0, eg = c.r1;
        se[lane][0] = eu;
        se[lane][1] = make_float4(eg.x, eg.y + eg.y, eg.z, eg.w);   // b staged doubled
        se[lane][2] = c.r2;
        const float mx = (eu.x - fx0) + eu.z, my = (eu.y - fy0) + eu.w;
        const float idet = __builtin_amdgcn_rcpf(eg.x * eg.z - eg.y * eg.y);
        const float ex = 3.f * __builtin_amdgcn_sqrtf(eg.z * idet) + 1e-3f;
        const float ey = 3.f * __builtin_amdgcn_sqrtf(eg.x * idet) + 1e-3f;
        const int x0 = max(0, (int)ceilf(mx - ex)), x1 = min(7, (int)floorf(mx + ex));
        const int y0 = max(0, (int)ceilf(my - ey)), y1 = min(7, (int)floorf(my + ey));
        if (x0 <= x1 && y0 <= y1)
            cover = ((0xFFu << x0) & (0xFFu >> (7 - x1))) | (((0xFFu << y0) & (0xFFu >> (7 - y1))) << 8);
    }
    const uint64_t col = bit_column<16>(cover, lane);
    if (lane < 16) sm[lane] = col;
}

// The backward's gather of one record (separate values rather than a struct,
// so that everything stays in registers).
__device__ __forceinline__ void fetch_bwd(const Geometry& G, const RenderBufs& B, const int* pof, bool valid,
                                          uint64_t key, float4& r0, float4& r1, float4& r2, float4& r3,
                                          float4& d) {
    if (!valid) return;
    const uint32_t gid = (uint32_t)key;
    const int kf = kf_of_gid(G, gid);
    const int pix = (int)(gid - (uint32_t)kf * (uint32_t)G.N);
    const size_t i = (size_t)pof[kf] * G.N + pix;
    const float4* rec = B.pre.rec + 4 * i;
    r0 = rec[0];
    r1 = rec[1];
    r2 = rec[2];
    r3 = rec[3];
    d = B.pre.dir[i];
}

// Tile coordinates of a work item and its pair table in LDS.
struct TileItem {
    int job, tx, ty;
};

__device__ __forceinline__ TileItem tile_item(const Geometry& G, const RenderBufs& B, int item, int lane,
                                              int* pof) {
    TileItem t;
    t.job = item / G.ntiles;
    const int tile = item - t.job * G.ntiles;
    t.tx = tile % G.ntx;
    t.ty = tile / G.ntx;
    pof[lane] = lane < G.n_kf ? B.pair_of[t.job * G.n_kf + lane] : -1;
    return t;
}

// Two front-to-back compositing steps with opacities a0 then a1 (0: a skipped
// candidate, which changes nothing), evaluated without branches so that the
// two candidates' work can overlap.  A step that would take T below kTMin
// ends the pixel's walk: neither it nor the step after it is applied.
// Returns the number of steps applied (0, 1 or 2); T >= kTMin on entry.
__device__ __forceinline__ int composite2(float a0, float4 c0, float a1, float4 c1, float& T, float& cr, float& cg,
                                          float& cb, float& dd) {
    const float t0 = T * (1.f - a0);
    const bool ok0 = t0 >= kTMin;
    const float t1 = t0 * (1.f - a1);
    const bool ok1 = ok0 && t1 >= kTMin;
    const float w0 = ok0 ? a0 * T : 0.f;
    const float w1 = ok1 ? a1 * t0 : 0.f;
    cr += w0 * c0.x;
    cg += w0 * c0.y;
    cb += w0 * c0.z;
    dd += w0 * c0.w;
    cr += w1 * c1.x;
    cg += w1 * c1.y;
    cb += w1 * c1.z;
    dd += w1 * c1.w;
    T = ok1 ? t1 : (ok0 ? t0 : T);
    return ok1 ? 2 : (ok0 ? 1 : 0);
}

__global__ __launch_bounds__(64) void k_fwd8(Geometry G, RenderBufs B, FwdOut O) {
    __shared__ float4 s_e[64][3];
    __shared__ uint64_t s_m[16];
    __shared__ int s_pof[64];
    const int lane = threadIdx.x;
    publish_status(B);
    const int item = xcd_remap(blockIdx.x, gridDim.x);
    if (item >= G.n_jobs * G.ntiles) return;
    const TileItem ti = tile_item(G, B, item, lane, s_pof);
    const int job = ti.job;
    const int lx = lane & 7, ly = lane >> 3;
    const int px = ti.tx * 8 + lx, py = ti.ty * 8 + ly;
    const bool inside = px < G.Wv && py < G.Hv;
    const bool ovf = B.status->overflow != 0u;
    const uint32_t st = B.tile_start[item];
    const int len = ovf ? 0 : (int)(B.tile_start[item + 1] - st);
    const uint32_t cs = B.chunk_start[item];   // this tile's first contributor-mask chunk
    if (G.fuse_sort) {
        // depth order of this tile's segment; the barrier makes the sorted
        // keys visible to every lane before the walk reads them
        sort_segment(B.keys + st, len, lane, G.sort_long != 0);
        __syncthreads();
    }
    const float fpx = (float)px, fpy = (float)py;
    const float fx0 = (float)(ti.tx * 8), fy0 = (float)(ti.ty * 8);
    float T = 1.f, cr = 0.f, cg = 0.f, cb = 0.f, dd = 0.f;
    int cnt = 0;
    uint32_t last = 0;
    bool done = !inside;
    wave_lds_sync();
    ChunkRegs cur{}, nxt{};
    cur.key = fetch_key(B, st, lane, len);
    fetch_record(G, B, s_pof, lane < len, cur);
    nxt.key = fetch_key(B, st + 64u, lane, len - 64);
    for (int c0 = 0; c0 < len; c0 += 64) {
        const int n = min(64, len - c0);
        publish_chunk(cur, lane < n, lane, fx0, fy0, s_e, s_m);
        wave_lds_sync();
        // gather ahead: records of the next chunk, keys of the one after
        fetch_record(G, B, s_pof, lane < len - c0 - 64, nxt);
        const uint64_t key2 = fetch_key(B, st + (uint32_t)(c0 + 128), lane, len - c0 - 128);
        uint64_t cm = 0ull;   // entries of this chunk the pixel takes
        if (!done) {
            uint64_t m = s_m[lx] & s_m[8 + ly];
            // two candidates per round: their q, alpha evaluations are independent
            while (m != 0ull) {
                const int b0 = (int)__builtin_ctzll(m);
                m &= m - 1ull;
                const bool two = m != 0ull;
                const int b1 = two ? (int)__builtin_ctzll(m) : b0;
                if (two) m &= m - 1ull;
                const float4 eu0 = s_e[b0][0], eg0 = s_e[b0][1], ec0 = s_e[b0][2];
                const float4 eu1 = s_e[b1][0], eg1 = s_e[b1][1], ec1 = s_e[b1][2];
                const float dx0 = (fpx - eu0.x) - eu0.z, dy0 = (fpy - eu0.y) - eu0.w;
                const float dx1 = (fpx - eu1.x) - eu1.z, dy1 = (fpy - eu1.y) - eu1.w;
                const float q0 = pair_q2b(dx0, dy0, eg0.x, eg0.y, eg0.z);
                const float q1 = pair_q2b(dx1, dy1, eg1.x, eg1.y, eg1.z);
                const float al0 = fminf(kAlphaMax, eg0.w * gauss_of_q(q0));
                const float al1 = fminf(kAlphaMax, eg1.w * gauss_of_q(q1));
                const bool v0 = q0 <= kQCut && al0 >= kAlphaMin;
                const bool v1 = two && q1 <= kQCut && al1 >= kAlphaMin;
                // a skipped candidate composites with alpha 0, which leaves
                // T and the sums exactly as they are
                const int ap = composite2(v0 ? al0 : 0.f, ec0, v1 ? al1 : 0.f, ec1, T, cr, cg, cb, dd);
                const bool u0 = v0 && ap >= 1, u1 = v1 && ap == 2;
                cm |= (u0 ? 1ull << b0 : 0ull) | (u1 ? 1ull << b1 : 0ull);
                if (ap < 2) {
                    done = true;
                    break;
                }
            }
        }
        // the count and the last entry taken follow from the chunk's mask
        if (cm != 0ull) {
            cnt += __popcll(cm);
            last = (uint32_t)(c0 + 64 - __builtin_clzll(cm));
        }
        B.cmask[((size_t)cs + (size_t)(c0 >> 6)) * 64 + lane] = cm;
        if (__ballot(!done) == 0ull) break;
        cur = nxt;
        nxt.key = key2;
        wave_lds_sync();
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

// Forward over super-chunks of SCH published chunks: each lane walks its
// candidates across all SCH chunks without waiting at chunk boundaries, so a
// wave runs the per-super-chunk maximum over lanes instead of the sum of the
// per-chunk maxima (depth order is spatially correlated: with one
// 256-entry super-chunk a 640x480 tile needs ~25 rounds instead of ~65).
template <int SCH>
__global__ __launch_bounds__(64) void k_fwd8s(Geometry G, RenderBufs B, FwdOut O) {
    constexpr int SPAN = 64 * SCH;
    __shared__ float4 s_e[SPAN][3];
    __shared__ uint64_t s_m[SCH][16];
    __shared__ int s_pof[64];
    const int lane = threadIdx.x;
    publish_status(B);
    const int item = xcd_remap(blockIdx.x, gridDim.x);
    if (item >= G.n_jobs * G.ntiles) return;
    const TileItem ti = tile_item(G, B, item, lane, s_pof);
    const int job = ti.job;
    const int lx = lane & 7, ly = lane >> 3;
    const int px = ti.tx * 8 + lx, py = ti.ty * 8 + ly;
    const bool inside = px < G.Wv && py < G.Hv;
    const bool ovf = B.status->overflow != 0u;
    const uint32_t st = B.tile_start[item];
    const int len = ovf ? 0 : (int)(B.tile_start[item + 1] - st);
    const uint32_t cs = B.chunk_start[item];   // this tile's first contributor-mask chunk
    if (G.fuse_sort) {
        // depth order of this tile's segment; the barrier makes the sorted
        // keys visible to every lane before the walk reads them
        sort_segment(B.keys + st, len, lane, G.sort_long != 0);
        __syncthreads();
    }
    const float fpx = (float)px, fpy = (float)py;
    const float fx0 = (float)(ti.tx * 8), fy0 = (float)(ti.ty * 8);
    float T = 1.f, cr = 0.f, cg = 0.f, cb = 0.f, dd = 0.f;
    int cnt = 0;
    uint32_t last = 0;
    bool done = !inside;
    wave_lds_sync();
    uint64_t keys[SCH];
#pragma unroll
    for (int i = 0; i < SCH; ++i) keys[i] = fetch_key(B, st + (uint32_t)(64 * i), lane, len - 64 * i);
    for (int c0 = 0; c0 < len; c0 += SPAN) {
        const int n = min(SPAN, len - c0);
        const int nch = (n + 63) >> 6;
        ChunkRegs r[SCH];
#pragma unroll
        for (int i = 0; i < SCH; ++i) {
            r[i].key = keys[i];
            fetch_record(G, B, s_pof, lane < n - 64 * i, r[i]);
        }
        // keys of the next super-chunk while this one is walked
#pragma unroll
        for (int i = 0; i < SCH; ++i)
            keys[i] = fetch_key(B, st + (uint32_t)(c0 + SPAN + 64 * i), lane, len - c0 - SPAN - 64 * i);
#pragma unroll
        for (int i = 0; i < SCH; ++i)
            publish_chunk(r[i], lane < n - 64 * i, lane, fx0, fy0, s_e + 64 * i, s_m[i]);
        wave_lds_sync();
        uint64_t cm[SCH];
#pragma unroll
        for (int i = 0; i < SCH; ++i) cm[i] = 0ull;
        if (!done) {
            int ch = 0;
            uint64_t m = s_m[0][lx] & s_m[0][8 + ly];
            while (true) {
                while (m == 0ull && ch + 1 < nch) {
                    ++ch;
                    m = s_m[ch][lx] & s_m[ch][8 + ly];
                }
                if (m == 0ull) break;
                const int e0 = ch * 64 + (int)__builtin_ctzll(m);
                m &= m - 1ull;
                while (m == 0ull && ch + 1 < nch) {
                    ++ch;
                    m = s_m[ch][lx] & s_m[ch][8 + ly];
                }
                const bool two = m != 0ull;
                const int e1 = two ? ch * 64 + (int)__builtin_ctzll(m) : e0;
                if (two) m &= m - 1ull;
                const float4 eu0 = s_e[e0][0], eg0 = s_e[e0][1], ec0 = s_e[e0][2];
                const float4 eu1 = s_e[e1][0], eg1 = s_e[e1][1], ec1 = s_e[e1][2];
                const float dx0 = (fpx - eu0.x) - eu0.z, dy0 = (fpy - eu0.y) - eu0.w;
                const float dx1 = (fpx - eu1.x) - eu1.z, dy1 = (fpy - eu1.y) - eu1.w;
                const float q0 = pair_q2b(dx0, dy0, eg0.x, eg0.y, eg0.z);
                const float q1 = pair_q2b(dx1, dy1, eg1.x, eg1.y, eg1.z);
                const float al0 = fminf(kAlphaMax, eg0.w * gauss_of_q(q0));
                const float al1 = fminf(kAlphaMax, eg1.w * gauss_of_q(q1));
                const bool v0 = q0 <= kQCut && al0 >= kAlphaMin;
                const bool v1 = two && q1 <= kQCut && al1 >= kAlphaMin;
                const int ap = composite2(v0 ? al0 : 0.f, ec0, v1 ? al1 : 0.f, ec1, T, cr, cg, cb, dd);
                const bool u0 = v0 && ap >= 1, u1 = v1 && ap == 2;
#pragma unroll
                for (int i = 0; i < SCH; ++i)
                    cm[i] |= ((u0 && (e0 >> 6) == i) ? 1ull << (e0 & 63) : 0ull) |
                             ((u1 && (e1 >> 6) == i) ? 1ull << (e1 & 63) : 0ull);
                if (ap < 2) {
                    done = true;
                    break;
                }
            }
        }
#pragma unroll
        for (int i = 0; i < SCH; ++i) {
            if (cm[i] != 0ull) {
                cnt += __popcll(cm[i]);
                last = (uint32_t)(c0 + 64 * i + 64 - __builtin_clzll(cm[i]));
            }
            if (i < nch) B.cmask[((size_t)cs + (size_t)(c0 >> 6) + i) * 64 + lane] = cm[i];
        }
        if (__ballot(!done) == 0ull) break;
        wave_lds_sync();
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

// Backward of one 8x8 tile per wavefront.
//
// The tile's list is taken in 64-entry chunks from the back, each chunk in
// sub-chunks of SUB entries from the back, in two phases per sub-chunk:
//  A (lane = pixel): the reverse walk over the pixel's candidates carries the
//    transmittance and the suffix colour sums and stores, per contributing
//    pair, w = alpha T and gq = -2 dL/dq into a [pixel][entry] LDS matrix;
//  B (lane = entry, 64 / SUB lanes per entry): a bit-matrix transpose across
//    lanes turns the per-pixel contribution masks into per-entry pixel sets,
//    and each lane sums its entry's pairs over the contributing pixels of its
//    class.
// The per-entry sums are gq-weighted moments of (dx, dy) and gradient-weighted
// sums of w; the conic and the factor -1/2 of dL/dq enter after the sum (a
// power of two, so the results are those of scaling each term).  No LDS
// location is written by two lanes at once, and the in-tile summation order
// is fixed.  After a chunk, lane e applies the chain rule of entry e from the
// record it gathered.
template <int SUB>
__global__ __launch_bounds__(64) void k_bwd8(Geometry G, RenderBufs B, BwdArgs A) {
    constexpr int NS = 64 / SUB;        // sub-chunks per chunk = pixel groups in phase B
    constexpr int LS = 2 * SUB + 2;     // floats per matrix row: rows 2 banks apart
    __shared__ float4 s_e[64][3];
    __shared__ float4 s_pc[64];
    __shared__ int s_pof[64];
    __shared__ __align__(16) float s_M[64 * LS];   // [pixel][entry] (w, gq); a cell is read only if written
    const int lane = threadIdx.x;
    const int item = xcd_remap(blockIdx.x, gridDim.x);
    if (item >= G.n_jobs * G.ntiles) return;
    const TileItem ti = tile_item(G, B, item, lane, s_pof);
    const int job = ti.job;
    const int lx = lane & 7, ly = lane >> 3;
    const int px = ti.tx * 8 + lx, py = ti.ty * 8 + ly;
    const bool inside = px < G.Wv && py < G.Hv;
    const bool ovf = B.status->overflow != 0u;
    const uint32_t st = B.tile_start[item];
    const size_t P = (size_t)G.P;
    float T = 1.f, gC0 = 0.f, gC1 = 0.f, gC2 = 0.f, gD = 0.f, gA = 0.f;
    int last = 0;
    if (inside && !ovf) {
        const size_t pix = (size_t)py * G.Wv + px;
        const size_t jp = (size_t)job * P + pix;
        T = B.Tfinal[jp];
        last = (int)B.last[jp];
        gC0 = A.g_rgb[((size_t)job * 3 + 0) * P + pix];
        gC1 = A.g_rgb[((size_t)job * 3 + 1) * P + pix];
        gC2 = A.g_rgb[((size_t)job * 3 + 2) * P + pix];
        if (A.g_depth) gD = A.g_depth[jp];
        if (A.g_alpha) gA = A.g_alpha[jp];
    }
    s_pc[lane] = make_float4(gC0, gC1, gC2, gD);
    int maxlast = last;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) maxlast = max(maxlast, __shfl_xor(maxlast, o, 64));
    const float gATf = gA * T;   // alpha-channel term of dL/dalpha: gA T_final / (1 - alpha)
    const float fpx = (float)px, fpy = (float)py;
    const float fx0 = (float)(ti.tx * 8), fy0 = (float)(ti.ty * 8);
    const int sub = lane & (SUB - 1), grp = lane / SUB;
    // g . S - gA T_final, carried as one scalar: g . S is the upstream
    // colour/depth gradient dotted with the suffix sum of w c over the later
    // contributors
    float H = -gATf;
    float pose[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    wave_lds_sync();
    // the view's focal lengths (every pair of a job shares the view)
    float vfx, vfy;
    {
        const uint64_t has = __ballot(lane < G.n_kf && s_pof[lane] >= 0);
        const int f0 = has != 0ull ? (int)__builtin_ctzll(has) : 0;
        const PairConst& pc0 = B.pairs[max(0, s_pof[f0])];
        vfx = (float)pc0.vfx;
        vfy = (float)pc0.vfy;
    }
    // chunks c0 = top, top - 64, ..., 0; every chunk below the top one is full
    const int top = maxlast > 0 ? ((maxlast - 1) & ~63) : -1;
    // current and next chunk: key, record and offset direction of the lane's entry
    uint64_t ck = 0ull, nk = 0ull;
    float4 c0r, c1r, c2r, c3r, cdr, n0r, n1r, n2r, n3r, ndr;
    const uint32_t cs = B.chunk_start[item];   // this tile's first contributor-mask chunk
    uint64_t mine = 0ull, mine_nxt = 0ull;
    if (top >= 0) {
        ck = fetch_key(B, st + (uint32_t)top, lane, maxlast - top);
        fetch_bwd(G, B, s_pof, lane < maxlast - top, ck, c0r, c1r, c2r, c3r, cdr);
        mine = B.cmask[((size_t)cs + (size_t)(top >> 6)) * 64 + lane];
        if (top >= 64) nk = B.keys[st + (uint32_t)(top - 64 + lane)];
    }
    for (int c0 = top; c0 >= 0; c0 -= 64) {
        const int n = min(64, maxlast - c0);
        if (lane < n) {
            s_e[lane][0] = c0r;
            s_e[lane][1] = make_float4(c1r.x, c1r.y + c1r.y, c1r.z, c1r.w);   // b staged doubled
            s_e[lane][2] = c2r;
        }
        wave_lds_sync();
        // gather ahead: records and masks of the next chunk, keys of the one after
        if (c0 >= 64) {
            fetch_bwd(G, B, s_pof, true, nk, n0r, n1r, n2r, n3r, ndr);
            mine_nxt = B.cmask[((size_t)cs + (size_t)((c0 - 64) >> 6)) * 64 + lane];
        }
        const uint64_t key2 = c0 >= 128 ? B.keys[st + (uint32_t)(c0 - 128 + lane)] : 0ull;
        const int lim = min(n, last - c0);   // this pixel's entries are e < lim
        // partial sums of each sub-chunk's entries over this lane's pixel
        // class; summed over the NS classes after the last sub-chunk
        float acc[NS][10];
#pragma unroll
        for (int s = NS - 1; s >= 0; --s) {
            // phase A: reverse walk of this pixel's contributors in the sub-chunk
            // (the forward's decisions), two per round
            const int cut = lim - s * SUB;
            // entries of the sub-chunk this pixel contributed to
            const uint32_t cmask = cut <= 0 ? 0u : (uint32_t)((mine >> (s * SUB)) & low_bits(min(cut, SUB)));
            // dL/dalpha = sum_c g_c (c T - S_c / (1 - alpha)) + gA T_final / (1 - alpha)
            //           = T (g . c) - (g . S - gA T_final) / (1 - alpha)
            // cell `bit` of the pixel's matrix row gets (w, gq); the row's
            // padding cell (bit = SUB) takes the write of an absent second
            // candidate, whose alpha 0 leaves T and H exactly as they are
            auto contribute = [&](float alpha, float raw, float4 c, int bit) {
                const float inv = __builtin_amdgcn_rcpf(1.f - alpha);
                T = T * inv;
                const float w = alpha * T;
                const float gc = gC0 * c.x + gC1 * c.y + gC2 * c.z + gD * c.w;
                const float gal = T * gc - inv * H;
                H += w * gc;
                const float gq = raw < kAlphaMax ? alpha * gal : 0.f;   // -2 dL/dq
                *(float2*)&s_M[lane * LS + 2 * bit] = make_float2(w, gq);
            };
            // walked from its last entry: bit-reversed, the next entry is the
            // lowest set bit
            uint32_t m = __builtin_bitreverse32(cmask);
            while (m != 0u) {
                const int z0 = (int)__builtin_ctz(m);
                m &= m - 1u;
                const bool two = m != 0u;
                const int z1 = two ? (int)__builtin_ctz(m) : z0;
                m &= m - 1u;
                const int b0 = 31 - z0, b1 = 31 - z1;
                const float4* r0 = s_e[s * SUB + b0];
                const float4* r1 = s_e[s * SUB + b1];
                const float4 eu0 = r0[0], eg0 = r0[1], ec0 = r0[2];
                const float4 eu1 = r1[0], eg1 = r1[1], ec1 = r1[2];
                const float dx0 = (fpx - eu0.x) - eu0.z, dy0 = (fpy - eu0.y) - eu0.w;
                const float dx1 = (fpx - eu1.x) - eu1.z, dy1 = (fpy - eu1.y) - eu1.w;
                const float q0 = pair_q2b(dx0, dy0, eg0.x, eg0.y, eg0.z);
                const float q1 = pair_q2b(dx1, dy1, eg1.x, eg1.y, eg1.z);
                const float raw0 = eg0.w * gauss_of_q(q0);
                const float raw1 = eg1.w * gauss_of_q(q1);
                const float al0 = fminf(kAlphaMax, raw0);
                const float al1 = two ? fminf(kAlphaMax, raw1) : 0.f;
                contribute(al0, raw0, ec0, b0);
                contribute(al1, raw1, ec1, two ? b1 : SUB);
            }
            // transpose the contributions: lane (grp, sub) takes the pixel set
            // of entry `sub`
            const uint64_t emask = bit_column<SUB>(cmask, lane);
            wave_lds_sync();   // phase A's matrix cells, for the other lanes
            // phase B: lane = entry s * SUB + sub; the NS lanes of an entry
            // split its contributing pixels by a checkerboard class (NS = 4:
            // (x mod 2, y mod 2); NS = 2: (x + y) mod 2), which balances
            // compact footprints better than columns, and each walks only
            // the cells phase A wrote
            const float4 eu0 = s_e[s * SUB + sub][0];
            const float mxl = (eu0.x - fx0) + eu0.z, myl = (eu0.y - fy0) + eu0.w;
            const uint64_t cls = NS == 4   ? 0x0055005500550055ull << ((grp & 1) + 8 * (grp >> 1))
                                 : NS == 2 ? (grp ? ~0xAA55AA55AA55AA55ull : 0xAA55AA55AA55AA55ull)
                                           : ~0ull;
            float* a = acc[s];
#pragma unroll
            for (int k = 0; k < 10; ++k) a[k] = 0.f;
            uint64_t pm = emask & cls;
            while (pm != 0ull) {
                const int p = (int)__builtin_ctzll(pm);
                pm &= pm - 1ull;
                const float2 mv = *(const float2*)&s_M[p * LS + 2 * sub];
                const float4 gv = s_pc[p];
                const float dx = (float)(p & 7) - mxl;
                const float dy = (float)(p >> 3) - myl;
                a[0] += gv.x * mv.x;
                a[1] += gv.y * mv.x;
                a[2] += gv.z * mv.x;
                a[3] += gv.w * mv.x;
                a[4] += mv.y;
                const float u = mv.y * dx, v = mv.y * dy;
                a[5] += u;
                a[6] += v;
                a[7] += u * dx;
                a[8] += u * dy;
                a[9] += v * dy;
            }
            wave_lds_sync();
        }
        // reduce-scatter over the classes: lane (grp, sub) ends with the sums
        // of entry grp * SUB + sub; each exchange halves what a lane holds
        float r[10];
        if constexpr (NS == 4) {
            const bool hi32 = (lane & 32) != 0, hi16 = (lane & 16) != 0;
            float h[2][10];
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int k = 0; k < 10; ++k) {
                    const float keep = hi32 ? acc[2 + j][k] : acc[j][k];
                    const float send = hi32 ? acc[j][k] : acc[2 + j][k];
                    h[j][k] = keep + __shfl_xor(send, 32, 64);
                }
#pragma unroll
            for (int k = 0; k < 10; ++k) {
                const float keep = hi16 ? h[1][k] : h[0][k];
                const float send = hi16 ? h[0][k] : h[1][k];
                r[k] = keep + __shfl_xor(send, 16, 64);
            }
        } else {
            static_assert(NS == 2, "sub-chunks of 16 or 32 entries");
            const bool hi32 = (lane & 32) != 0;
#pragma unroll
            for (int k = 0; k < 10; ++k) {
                const float keep = hi32 ? acc[1][k] : acc[0][k];
                const float send = hi32 ? acc[0][k] : acc[1][k];
                r[k] = keep + __shfl_xor(send, 32, 64);
            }
        }
        // lane = chunk entry: chain rule to the keyframe parameters and the pose
        int gidx = -1;   // the entry's keyframe Gaussian when it has parameter gradients
        float gv[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        if (lane < n) {
            bool any = false;
#pragma unroll
            for (int k = 0; k < 10; ++k) any |= r[k] != 0.f;
            if (any) {
                const float4 eg = c1r;
                float v[10];
                // r[4..9] hold -2 x the dL/dq-weighted sums
                v[0] = eg.x * r[5] + eg.y * r[6];
                v[1] = eg.y * r[5] + eg.z * r[6];
                v[2] = -0.5f * r[7];
                v[3] = -r[8];
                v[4] = -0.5f * r[9];
                v[5] = r[4] != 0.f ? r[4] * __builtin_amdgcn_rcpf(eg.w) : 0.f;
                v[6] = r[3];
                v[7] = r[0];
                v[8] = r[1];
                v[9] = r[2];
                const uint32_t gid = (uint32_t)ck;
                const int kf = kf_of_gid(G, gid);
                if (chain_rule_vals(A, vfx, vfy, kf, c2r.w, c3r, cdr, v, pose, gv)) gidx = (int)gid;
            }
        }
        // the shares go out eight lanes per entry, one lane per value of the
        // entry's 32-byte accumulator record, so that one atomic instruction
        // covers eight records instead of 64 scattered words; staged in the
        // matrix area, which the next chunk's phase A overwrites
        const uint64_t has = __ballot(gidx >= 0);
        if (has != 0ull) {
            float* st = s_M;
            *(float4*)&st[lane * 8] = make_float4(gv[0], gv[1], gv[2], gv[3]);
            *(float4*)&st[lane * 8 + 4] = make_float4(gv[4], gv[5], __int_as_float(gidx), 0.f);
            wave_lds_sync();
            const int sub8 = lane & 7, grp8 = lane >> 3;
#pragma unroll
            for (int rr = 0; rr < 8; ++rr) {
                if (((has >> (8 * rr)) & 0xffull) == 0ull) continue;
                const int e = rr * 8 + grp8;
                const int id = __float_as_int(st[e * 8 + 6]);
                const float val = st[e * 8 + sub8];
                if (id >= 0 && sub8 < 6) global_add(&A.acc[(size_t)id * 8 + sub8], val);
            }
        }
        ck = nk;
        c0r = n0r;
        c1r = n1r;
        c2r = n2r;
        c3r = n3r;
        cdr = ndr;
        nk = key2;
        mine = mine_nxt;
        wave_lds_sync();
    }
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        const float sv = wave_sum(pose[c]);
        if (lane == 0) A.pose_part[(size_t)item * 6 + c] = sv;
    }
}

bool launch_fwd8(const Geometry& G, const RenderBufs& B, const FwdOut& O, int sch, hipStream_t s) {
    if (G.TW != 8 || G.TH != 8) return false;
    const dim3 grid(G.n_jobs * G.ntiles), block(64);
    if (sch == 1) hipLaunchKernelGGL(k_fwd8, grid, block, 0, s, G, B, O);
    else if (sch == 2) hipLaunchKernelGGL((k_fwd8s<2>), grid, block, 0, s, G, B, O);
    else if (sch == 4) hipLaunchKernelGGL((k_fwd8s<4>), grid, block, 0, s, G, B, O);
    else return false;
    return true;
}

// After the 8x8 adjoint, in one launch: blocks [0, n_pose) sum each job's
// per-tile pose partials in FP64 (a fixed order: 32 strided partial sums per
// component, then those in index order); the other blocks move the
// accumulated parameter gradients of the learnable keyframes into their
// gradient planes (+=) and clear the accumulator records for the next
// adjoint (records that received nothing are left alone).
constexpr int kFinishThreads = 192;   // a multiple of the 6 pose components

__global__ __launch_bounds__(kFinishThreads) void k_bwd_finish(int N, int bpk, const KfGradPtrs* __restrict__ grads,
                                                               uint32_t lo, uint32_t hi, float* __restrict__ acc,
                                                               const float* __restrict__ part, int ntiles,
                                                               float* __restrict__ d_pose, int n_pose) {
    const int tid = threadIdx.x;
    if ((int)blockIdx.x < n_pose) {
        __shared__ double s[kFinishThreads];
        const int job = blockIdx.x;
        const float* pj = part + (size_t)job * ntiles * 6;
        const int n = ntiles * 6;
        double a = 0.0;
        for (int f = tid; f < n; f += kFinishThreads) a += (double)pj[f];
        s[tid] = a;
        __syncthreads();
        if (tid < 6) {
            double t = 0.0;
            for (int g = 0; g < kFinishThreads / 6; ++g) t += s[g * 6 + tid];
            d_pose[job * 6 + tid] = (float)t;
        }
        return;
    }
    const int b = (int)blockIdx.x - n_pose;
    const int kf = b / bpk;
    const int i = (b - kf * bpk) * kFinishThreads + tid;
    const bool learn = kf < 32 ? ((lo >> kf) & 1u) : ((hi >> (kf - 32)) & 1u);
    if (!learn || i >= N) return;
    float4* a = (float4*)acc + ((size_t)kf * N + i) * 2;
    const float4 x = a[0], y = a[1];
    if (x.x != 0.f || x.y != 0.f || x.z != 0.f || x.w != 0.f || y.x != 0.f || y.y != 0.f) {
        const KfGradPtrs gp = grads[kf];
        gp.d_offset[i] += x.x;
        gp.d_radius[i] += x.y;
        gp.d_opacity[i] += x.z;
        gp.d_rgb[i] += x.w;
        gp.d_rgb[(size_t)N + i] += y.x;
        gp.d_rgb[2 * (size_t)N + i] += y.y;
        const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
        a[0] = z4;
        a[1] = z4;
    }
}

void launch_bwd_finish(const Geometry& G, const KfGradPtrs* grads, uint32_t lo, uint32_t hi, float* acc,
                       const float* pose_part, float* d_pose, hipStream_t s) {
    const int bpk = (G.N + kFinishThreads - 1) / kFinishThreads;
    const int n_pose = d_pose ? G.n_jobs : 0;
    hipLaunchKernelGGL(k_bwd_finish, dim3(n_pose + bpk * G.n_kf), dim3(kFinishThreads), 0, s, G.N, bpk, grads,
                       lo, hi, acc, pose_part, G.ntiles, d_pose, n_pose);
}

template <int SUB>
static void bwd8_t(const Geometry& G, const RenderBufs& B, const BwdArgs& A, hipStream_t s) {
    hipLaunchKernelGGL((k_bwd8<SUB>), dim3(G.n_jobs * G.ntiles), dim3(64), 0, s, G, B, A);
}

bool launch_bwd8(const Geometry& G, const RenderBufs& B, const BwdArgs& A, int sub, hipStream_t s) {
    if (G.TW != 8 || G.TH != 8 || !A.acc) return false;
    if (sub == 32) bwd8_t<32>(G, B, A, s);
    else if (sub == 16) bwd8_t<16>(G, B, A, s);
    else return false;
    return true;
}

}  // namespace sgad
