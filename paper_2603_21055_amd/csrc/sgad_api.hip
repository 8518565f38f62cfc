// Host side of the C ABI: context, saved render state, workspace sizing,
// relative-pose tables, launches and asynchronous error latching.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "sgad_internal.h"

namespace sgad {
void launch_zero_u32(uint32_t* p, int64_t n, hipStream_t s);
void launch_fill_f32(float* p, int64_t n, float v, hipStream_t s);
void launch_zero2_u32(uint32_t* a, int64_t na, uint32_t* b, int64_t nb, hipStream_t s);
void launch_preprocess(const Geometry& G, const RenderBufs& B, hipStream_t s);
void launch_scan(const Geometry& G, const RenderBufs& B, bool zero_counts, hipStream_t s);
void launch_scatter(const Geometry& G, const RenderBufs& B, hipStream_t s);
void launch_sort(const Geometry& G, const RenderBufs& B, hipStream_t s);
bool launch_fwd(const Geometry& G, const RenderBufs& B, float* rgb, float* depth, float* alpha, int32_t* count,
                hipStream_t s);
bool launch_bwd(const Geometry& G, const RenderBufs& B, const float* g_rgb, const float* g_depth,
                const float* g_alpha, const KfGradPtrs* grads, uint32_t lo, uint32_t hi, float* pose_part,
                float* acc, float* d_pose, hipStream_t s);
void launch_bwd_finish(const Geometry& G, const KfGradPtrs* grads, uint32_t lo, uint32_t hi, float* acc,
                       const float* pose_part, float* d_pose, hipStream_t s);
void launch_l1(int n_jobs, int P, const float* rgb, const float* dep, const float* t_rgb, const float* t_dep,
               float w_rgb, float w_dep, uint32_t* count, int nparts, float* g_rgb, float* g_dep, double* loss,
               hipStream_t s);
int l1_blocks(int P);
size_t ssim_map_bytes(int n_jobs, int H, int W);
size_t ssim_tiles(int H, int W);
int gicp_grid_points(int H, int W, int R);
int gicp_blocks(int n);
int gicp_vals();
int gicp_max_k();
void launch_gicp_prepare(const float* depth, int H, int W, int R, const sgad_cam& cam, int k, double* set,
                         hipStream_t s);
void launch_gicp_linearise(const double* src, int ns, const double* tgt, int nt, const sgad_cam& tcam, int tR,
                           int k, const double* pose, double* part, int* corr, hipStream_t s);
void launch_gicp_sum(const double* part, int nb, double* out, hipStream_t s);
void launch_gicp_linearise_map(const double* src, int ns, const sgad_gmap& m, int k, const double* pose,
                               double* part, int* corr, hipStream_t s);
int gicp_wave_blocks(int n);
void launch_gmap_reset(const sgad_gmap& m, hipStream_t s);
void launch_gmap_insert(const sgad_gmap& m, const double* set, int n, const double* pose, hipStream_t s);
void launch_fill_depth(int P, const float* depth, const float* rdepth, const float* ralpha, float alpha_min,
                       float* out, hipStream_t s);
void launch_gicp_solve(const double* part, int nb, double* pose, double* trace, int it, hipStream_t s);
void launch_ssim_maps(int n_jobs, int H, int W, const float* rgb, const float* t_rgb, void* ws,
                      const float* t_depth, uint32_t* cnt, double* loss, hipStream_t s);
void launch_ssim_grad(int n_jobs, int H, int W, const float* rgb, const float* t_rgb, float w_ssim, void* ws,
                      float* g_rgb, double* loss, hipStream_t s);
void launch_adam(AdamGroups& A, float b1, float b2, float eps, float c1, float c2, int zero_grad,
                 float* cdev, hipStream_t s);
bool launch_conv_fwd(int H, int W, int cin, int cout, int mode, const void* x, const void* w, const float* bias,
                     const void* mask, void* y, hipStream_t s);
size_t conv_wgrad_part_bytes(int H, int W, int cin, int cout);
hipError_t conv_scratch_setup(int device, float** out);
size_t conv_scratch_bytes();
bool launch_conv_wgrad(int H, int W, int cin, int cout, const void* x, const void* dy, float* part, float* dw, float* db,
                       hipStream_t s);
void launch_conv_weights(int cin, int cout, const float* w, void* wb, void* wt, hipStream_t s);
void launch_net_input(int H, int W, const float* rgb, const float* depth, void* x0, hipStream_t s);
void launch_offset_l1(int n, const float* pred, const float* target, void* grad, double* loss, hipStream_t s);
void launch_track_pair(const double* pose, const sgad_pose& kf_pose, const sgad_cam& kc, const sgad_cam& vc,
                       PairConst* out, hipStream_t s);
bool launch_track(const Geometry& G, const RenderBufs& B, const float* obs, float* part, hipStream_t s);
int track_parts(const Geometry& G);
void launch_track_solve(const float* part, int nitems, double* pose, double* trace, int it, const DevStatus* st,
                        const sgad_pose& kf_pose, const sgad_cam& kc, const sgad_cam& vc, PairConst* next,
                        hipStream_t s);
}  // namespace sgad

using namespace sgad;

namespace {

struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
};

struct PinBuf {
    void* p = nullptr;
    size_t bytes = 0;
};

}  // namespace

struct sgad_saved {
    bool in_use = false;
    const sgad_graph* owner = nullptr;  // captured into this graph: never reused or resized
    Geometry G{};
    hipStream_t stream = nullptr;
    // device buffers (grow-only)
    DevBuf params, pre, tiles, keys, pix, pose_part, status, gradptrs, cmask;
    DevBuf gacc;   // 8x8 adjoint's per-Gaussian gradient accumulator, kept zero between adjoints
    uint32_t capacity = 0;
    uint32_t last_max_seg = 0xffffffffu;  // longest segment seen by the last finished forward
    bool sized = false;
    size_t size_key[5] = {0, 0, 0, 0, 0};  // workload the capacity was sized for
    // pinned staging
    PinBuf up, up_grad;
    // host copies of what the device parameter blocks hold: an unchanged
    // block (every iteration of a mapping loop) is not uploaded again
    std::vector<char> stage, last_up, stage_grad, last_up_grad;
    DevStatus* status_h = nullptr;
    uint32_t* status_dev = nullptr;   // status_h as the forward kernel writes it (null: copied instead)
    int zeroed_M = -1;                // the tile counts [0, M) and the flags are known to be clear
    void* zeroed_tiles = nullptr;     // ... in this allocation of the tile buffer
    hipEvent_t ev_up = nullptr, ev_up_grad = nullptr, ev_status = nullptr;
    bool up_pending = false, up_grad_pending = false, status_pending = false;
    RenderBufs B{};
};

// A captured sequence of library calls and what it holds on to.
struct sgad_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<sgad_saved*> slots;
    DevBuf adam;
    // per timed kernel: its two event-record nodes (events swapped per launch)
    std::vector<std::pair<std::string, std::pair<hipGraphNode_t, hipGraphNode_t>>> timed;
    std::vector<hipEvent_t> events;  // the events the nodes were captured with
};

// Optional per-kernel timing: a pair of hipEvents recorded on the launch
// stream around every library kernel, accumulated per kernel name.
struct KernelTimer {
    bool on = false;
    std::string only;  // time only this kernel name (empty: all)
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pool;
    size_t used = 0;
    std::vector<std::pair<std::string, size_t>> pending;  // name, pool index
    std::vector<std::string> names;
    std::vector<double> ms;
    std::vector<long> count;
};

struct sgad_ctx {
    int device = 0;
    std::string err;
    sgad_status latched = SGAD_OK;
    std::string latched_msg;
    int tile_w = 0, tile_h = 0;  // 0,0: autotuned per workload
    int var_scf = 4, var_scb = 16;  // 8x8 kernel variant when the tile is set by hand
    int last_tw = 8, last_th = 8, last_scf = 4, last_scb = 16;
    // autotuner: configurations measured per workload key, and a forced
    // configuration used while measuring
    struct TuneEntry {
        size_t key[6];
        int tw, th, scf, scb;
        float ms;
    };
    std::vector<TuneEntry> tune;
    bool force = false;
    int ftw = 8, fth = 8, fscf = 4, fscb = 16;
    std::vector<sgad_saved*> slots;
    KernelTimer timer;
    // stream capture of library calls into a graph (sgad_graph_begin/end)
    struct Capture {
        bool on = false;
        hipStream_t cap = nullptr;    // private non-blocking stream the calls are recorded on
        DevBuf adam;                  // Adam step counters of the graph being built
        int n_adam = 0;
        int adam_t0[kMaxGraphAdam] = {};
        std::vector<sgad_saved*> slots;
        std::vector<std::pair<std::string, std::pair<hipEvent_t, hipEvent_t>>> timed;
    } capture;
    DevBuf scratch;  // small per-context scratch (loss counters)
    DevBuf conv_part;  // conv weight-gradient partial sums (one row per workgroup)
    DevBuf ssim_maps;  // SSIM partial-derivative maps of the loss call ([n_jobs * 3][3][H][W] floats)
    DevBuf gicp_part;  // GICP per-block partial sums of the normal equations
    float* conv_scratch = nullptr;  // this device's static partial-sum rows (sgad_conv3x3_wgrad_noalloc)
    struct Track {
        bool sized = false;
        Geometry G{};
        RenderBufs B{};
        DevBuf params, pre, tiles, keys, part, status, trace;
        uint32_t capacity = 0;
        // what a captured graph depends on
        const void* key[8] = {};
        int key_iters = 0, key_tw = 0, key_th = 0;
        sgad_cam kc{}, vc{};
        sgad_pose kpose{};
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        hipStream_t cap = nullptr;
        DevStatus* status_h = nullptr;
        hipEvent_t ev_status = nullptr;
        bool status_pending = false;
    } track;
};

namespace {

// Append an event-record node to the graph being captured on `s` and make it
// the stream's capture dependency (explicit node, so it does not rely on
// external event records in stream capture).
hipError_t capture_event_node(hipStream_t s, hipEvent_t ev) {
    hipStreamCaptureStatus st;
    unsigned long long id = 0;
    hipGraph_t g = nullptr;
    const hipGraphNode_t* deps = nullptr;
    size_t nd = 0;
    hipError_t e = hipStreamGetCaptureInfo_v2(s, &st, &id, &g, &deps, &nd);
    if (e != hipSuccess) return e;
    if (st != hipStreamCaptureStatusActive || !g) return hipErrorIllegalState;
    hipGraphNode_t n = nullptr;
    e = hipGraphAddEventRecordNode(&n, g, deps, nd, ev);
    if (e != hipSuccess) return e;
    return hipStreamUpdateCaptureDependencies(s, &n, 1, hipStreamSetCaptureDependencies);
}

// RAII scope that brackets one launch with timing events when enabled.
struct TimeScope {
    sgad_ctx* c;
    size_t idx = (size_t)-1;
    hipStream_t s;
    bool cap = false;
    hipEvent_t ca = nullptr, cb = nullptr;
    TimeScope(sgad_ctx* ctx, const char* name, hipStream_t stream) : c(ctx), s(stream) {
        KernelTimer& t = c->timer;
        if (!t.on) return;
        if (!t.only.empty() && t.only != name) return;
        if (c->capture.on) {
            // recorded as event nodes of the graph; sgad_graph_launch gives
            // them fresh events on every launch
            if (hipEventCreate(&ca) != hipSuccess) return;
            if (hipEventCreate(&cb) != hipSuccess) {
                (void)hipEventDestroy(ca);
                ca = nullptr;
                return;
            }
            if (capture_event_node(s, ca) != hipSuccess) {
                (void)hipEventDestroy(ca);
                (void)hipEventDestroy(cb);
                return;
            }
            cap = true;
            c->capture.timed.push_back({name, {ca, cb}});
            return;
        }
        if (t.used == t.pool.size()) {
            hipEvent_t a, b;
            if (hipEventCreate(&a) != hipSuccess) return;
            if (hipEventCreate(&b) != hipSuccess) {
                (void)hipEventDestroy(a);
                return;
            }
            t.pool.emplace_back(a, b);
        }
        idx = t.used++;
        (void)hipEventRecord(t.pool[idx].first, s);
        t.pending.emplace_back(name, idx);
    }
    ~TimeScope() {
        if (cap) (void)capture_event_node(s, cb);
        if (idx != (size_t)-1) (void)hipEventRecord(c->timer.pool[idx].second, s);
    }
};

// A fresh timing event pair from the pool, queued for timer_collect.
bool timer_pair(sgad_ctx* c, const std::string& name, hipEvent_t* a, hipEvent_t* b) {
    KernelTimer& t = c->timer;
    if (t.used == t.pool.size()) {
        hipEvent_t x, y;
        if (hipEventCreate(&x) != hipSuccess) return false;
        if (hipEventCreate(&y) != hipSuccess) {
            (void)hipEventDestroy(x);
            return false;
        }
        t.pool.emplace_back(x, y);
    }
    const size_t idx = t.used++;
    *a = t.pool[idx].first;
    *b = t.pool[idx].second;
    t.pending.emplace_back(name, idx);
    return true;
}

void timer_collect(sgad_ctx* c) {
    KernelTimer& t = c->timer;
    for (auto& pr : t.pending) {
        auto& ev = t.pool[pr.second];
        (void)hipEventSynchronize(ev.second);
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, ev.first, ev.second) != hipSuccess) continue;
        size_t k = 0;
        while (k < t.names.size() && t.names[k] != pr.first) ++k;
        if (k == t.names.size()) {
            t.names.push_back(pr.first);
            t.ms.push_back(0.0);
            t.count.push_back(0);
        }
        t.ms[k] += ms;
        t.count[k] += 1;
    }
    t.pending.clear();
    t.used = 0;
}

}  // namespace

namespace {

sgad_status fail(sgad_ctx* c, sgad_status s, const std::string& m) {
    if (c) c->err = m;
    return s;
}

#define HIPCHK(ctx, expr)                                                                     \
    do {                                                                                      \
        hipError_t _e = (expr);                                                               \
        if (_e != hipSuccess)                                                                 \
            return fail(ctx, SGAD_EHIP, std::string(#expr) + ": " + hipGetErrorString(_e));  \
    } while (0)

hipError_t ensure(DevBuf& b, size_t bytes, hipStream_t s) {
    if (bytes == 0) bytes = 256;
    if (b.bytes >= bytes) return hipSuccess;
    if (b.p) {
        hipError_t e = hipStreamSynchronize(s);
        if (e != hipSuccess) return e;
        e = hipFree(b.p);
        if (e != hipSuccess) return e;
    }
    b.p = nullptr;
    b.bytes = 0;
    hipError_t e = hipMalloc(&b.p, bytes);
    if (e != hipSuccess) return e;
    b.bytes = bytes;
    return hipSuccess;
}

// ensure() that refuses to allocate while calls are being captured (a
// captured call must find its workspace sized by an earlier eager call).
hipError_t ensure_c(sgad_ctx* c, DevBuf& b, size_t bytes, hipStream_t s) {
    if (c->capture.on) return b.bytes >= (bytes ? bytes : 256) ? hipSuccess : hipErrorNotSupported;
    return ensure(b, bytes, s);
}

// The stream a call enqueues on: the caller's, or the capture stream.
hipStream_t pick_stream(const sgad_ctx* c, void* stream) {
    return c->capture.on ? c->capture.cap : (hipStream_t)stream;
}

hipError_t ensure_pin(PinBuf& b, size_t bytes) {
    if (b.bytes >= bytes) return hipSuccess;
    if (b.p) {
        hipError_t e = hipHostFree(b.p);
        if (e != hipSuccess) return e;
    }
    b.p = nullptr;
    b.bytes = 0;
    hipError_t e = hipHostMalloc(&b.p, bytes, hipHostMallocDefault);
    if (e != hipSuccess) return e;
    b.bytes = bytes;
    return hipSuccess;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Device buffers of one saved slot (a forward and its adjoint), in bytes;
// the forward allocates exactly these and sgad_workspace_bytes reports them.
struct SlotBytes {
    size_t params, pre, tiles, pix, pose_part, status, keys, cmask, gradptrs, gacc;
    size_t total() const {
        return params + pre + tiles + pix + pose_part + status + keys + cmask + gradptrs + gacc;
    }
};

SlotBytes slot_bytes(int n_kf, int n_pairs, int n_jobs, size_t N, size_t P, size_t M, size_t capacity) {
    SlotBytes b{};
    const size_t o_kfs = align256(sizeof(PairConst) * n_pairs);
    const size_t o_pof = align256(o_kfs + sizeof(KfPtrs) * n_kf);
    b.params = align256(o_pof + sizeof(int32_t) * n_jobs * n_kf);
    b.pre = (size_t)n_pairs * N * 92 + 256;
    b.tiles = (4 * M + 2) * 4 + 256;
    b.pix = (size_t)n_jobs * P * 8;
    b.pose_part = M * 6 * 4;
    b.status = sizeof(DevStatus);
    b.keys = capacity * 8;
    b.cmask = (capacity / 64 + M + 1) * 64 * 8;
    b.gradptrs = align256(sizeof(KfGradPtrs) * n_kf);
    b.gacc = (size_t)n_kf * N * 32;
    return b;
}

// Instance capacity: the first-use guess before any count, and the size
// after an exact count.
size_t first_capacity(size_t NP) { return std::min<size_t>(NP * 3 + 65536, 0xffffffffu); }
size_t counted_capacity(size_t total) { return std::min<size_t>(total + total / 4 + 65536, 0xffffffffu); }

void latch(sgad_ctx* c, sgad_status st, const char* msg) {
    if (c->latched != SGAD_OK) return;
    c->latched = st;
    c->latched_msg = msg;
}

void latch_status(sgad_ctx* c, const DevStatus& st) {
    if (st.nonfinite || (st.sticky & 2u)) latch(c, SGAD_EDATA, "non-finite depth, offset or radius in a keyframe");
    if (st.overflow || (st.sticky & 1u))
        latch(c, SGAD_ERANGE, "instance list overflow (outputs of that call are NaN); capacity grows on the next call");
}

// Read device-side conditions of finished calls without blocking.
void poll(sgad_ctx* c, bool block) {
    if (c->capture.on) return;   // no queries while calls are being recorded
    if (c->track.status_pending) {
        bool done = block ? hipEventSynchronize(c->track.ev_status) == hipSuccess
                          : hipEventQuery(c->track.ev_status) == hipSuccess;
        if (done) {
            c->track.status_pending = false;
            latch_status(c, *c->track.status_h);
            if (c->track.status_h->sticky & 1u) c->track.sized = false;
        }
    }
    for (sgad_saved* s : c->slots) {
        if (!s->status_pending) continue;
        if (block) (void)hipEventSynchronize(s->ev_status);
        else if (hipEventQuery(s->ev_status) != hipSuccess) continue;
        s->status_pending = false;
        const DevStatus st = *s->status_h;
        latch_status(c, st);
        s->last_max_seg = st.max_seg;
        if (st.overflow || (st.sticky & 1u) || st.total > s->capacity - s->capacity / 8)
            s->sized = false;  // re-size on the next forward
    }
}

bool finite_pose(const sgad_pose& p) {
    for (float v : p.R)
        if (!std::isfinite(v)) return false;
    for (float v : p.t)
        if (!std::isfinite(v)) return false;
    return true;
}

bool cam_ok(const sgad_cam& c) {
    return c.H > 0 && c.W > 0 && c.H < 32768 && c.W < 32768 && std::isfinite(c.fx) && std::isfinite(c.fy) &&
           std::isfinite(c.cx) && std::isfinite(c.cy) && c.fx != 0.f && c.fy != 0.f;
}

// T_rel = T_view T_kf^-1 in FP64 with the operation order of the binning contract.
#pragma clang fp contract(off)
void relative_pose(const sgad_pose& v, const sgad_pose& f, PairConst& pc) {
    double Rv[9], Rf[9], tv[3], tf[3];
    for (int i = 0; i < 9; ++i) {
        Rv[i] = (double)v.R[i];
        Rf[i] = (double)f.R[i];
    }
    for (int i = 0; i < 3; ++i) {
        tv[i] = (double)v.t[i];
        tf[i] = (double)f.t[i];
    }
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double a = Rv[i * 3 + 0] * Rf[j * 3 + 0];
            double b = Rv[i * 3 + 1] * Rf[j * 3 + 1];
            double c = Rv[i * 3 + 2] * Rf[j * 3 + 2];
            double ab = a + b;
            pc.R[i * 3 + j] = ab + c;
        }
    for (int i = 0; i < 3; ++i) {
        double a = pc.R[i * 3 + 0] * tf[0];
        double b = pc.R[i * 3 + 1] * tf[1];
        double c = pc.R[i * 3 + 2] * tf[2];
        double ab = a + b;
        double abc = ab + c;
        pc.t[i] = tv[i] - abc;
    }
    for (int i = 0; i < 9; ++i) pc.Rf[i] = (float)pc.R[i];
    for (int i = 0; i < 3; ++i) pc.tf[i] = (float)pc.t[i];
}

sgad_saved* acquire(sgad_ctx* c) {
    for (sgad_saved* s : c->slots)
        if (!s->in_use && !s->owner) {
            s->in_use = true;
            return s;
        }
    sgad_saved* s = new sgad_saved();
    if (hipEventCreateWithFlags(&s->ev_up, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&s->ev_up_grad, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&s->ev_status, hipEventDisableTiming) != hipSuccess) {
        delete s;
        return nullptr;
    }
    if (hipHostMalloc((void**)&s->status_h, sizeof(DevStatus), hipHostMallocCoherent | hipHostMallocMapped) !=
        hipSuccess) {
        (void)hipGetLastError();
        s->status_h = nullptr;
        if (hipHostMalloc((void**)&s->status_h, sizeof(DevStatus), hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            delete s;
            return nullptr;
        }
    }
    std::memset(s->status_h, 0, sizeof(DevStatus));
    // the forward's first workgroup writes the status straight into it
    if (hipHostGetDevicePointer((void**)&s->status_dev, s->status_h, 0) != hipSuccess) {
        s->status_dev = nullptr;
        (void)hipGetLastError();
    }
    s->in_use = true;
    c->slots.push_back(s);
    return s;
}

// While capturing: a free slot already sized for this workload key.
sgad_saved* acquire_sized(sgad_ctx* c, const size_t* key) {
    for (sgad_saved* s : c->slots)
        if (!s->in_use && !s->owner && s->sized && std::memcmp(s->size_key, key, 5 * sizeof(size_t)) == 0) {
            s->in_use = true;
            return s;
        }
    return nullptr;
}

void free_slot(sgad_saved* s) {
    for (DevBuf* b : {&s->params, &s->pre, &s->tiles, &s->keys, &s->pix, &s->pose_part, &s->status, &s->gradptrs,
                      &s->cmask, &s->gacc})
        if (b->p) (void)hipFree(b->p);
    for (PinBuf* b : {&s->up, &s->up_grad})
        if (b->p) (void)hipHostFree(b->p);
    if (s->status_h) (void)hipHostFree(s->status_h);
    if (s->ev_up) (void)hipEventDestroy(s->ev_up);
    if (s->ev_up_grad) (void)hipEventDestroy(s->ev_up_grad);
    if (s->ev_status) (void)hipEventDestroy(s->ev_status);
    delete s;
}

bool valid_tile(int w, int h) {
    return (w == 8 && h == 8) || (w == 16 && h == 8) || (w == 16 && h == 16) || (w == 32 && h == 8);
}

}  // namespace

extern "C" {

sgad_status sgad_create(int device, sgad_ctx** out) {
    if (!out) return SGAD_EINVAL;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return SGAD_EINVAL;
    if (hipSetDevice(device) != hipSuccess) return SGAD_EHIP;
    float* scratch = nullptr;
    if (conv_scratch_setup(device, &scratch) != hipSuccess) return SGAD_EHIP;
    sgad_ctx* c = new sgad_ctx();
    c->device = device;
    c->conv_scratch = scratch;
    *out = c;
    return SGAD_OK;
}

void sgad_destroy(sgad_ctx* c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    if (c->capture.on) {
        hipGraph_t g = nullptr;
        (void)hipStreamEndCapture(c->capture.cap, &g);
        if (g) (void)hipGraphDestroy(g);
        c->capture.on = false;
    }
    if (c->capture.cap) (void)hipStreamDestroy(c->capture.cap);
    if (c->capture.adam.p) (void)hipFree(c->capture.adam.p);
    (void)hipDeviceSynchronize();
    for (sgad_saved* s : c->slots) free_slot(s);
    if (c->scratch.p) (void)hipFree(c->scratch.p);
    if (c->conv_part.p) (void)hipFree(c->conv_part.p);
    if (c->ssim_maps.p) (void)hipFree(c->ssim_maps.p);
    if (c->gicp_part.p) (void)hipFree(c->gicp_part.p);
    {
        auto& T = c->track;
        for (DevBuf* b : {&T.params, &T.pre, &T.tiles, &T.keys, &T.part, &T.status, &T.trace})
            if (b->p) (void)hipFree(b->p);
        if (T.exec) (void)hipGraphExecDestroy(T.exec);
        if (T.graph) (void)hipGraphDestroy(T.graph);
        if (T.cap) (void)hipStreamDestroy(T.cap);
        if (T.status_h) (void)hipHostFree(T.status_h);
        if (T.ev_status) (void)hipEventDestroy(T.ev_status);
    }
    for (auto& pr : c->timer.pool) {
        (void)hipEventDestroy(pr.first);
        (void)hipEventDestroy(pr.second);
    }
    delete c;
}

const char* sgad_last_error(const sgad_ctx* c) { return c ? c->err.c_str() : "null context"; }

sgad_status sgad_sync(sgad_ctx* c) {
    if (!c) return SGAD_EINVAL;
    if (c->capture.on) return fail(c, SGAD_EINVAL, "not allowed while capturing a graph");
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, hipDeviceSynchronize());
    poll(c, true);
    sgad_status s = c->latched;
    if (s != SGAD_OK) c->err = c->latched_msg;
    c->latched = SGAD_OK;
    c->latched_msg.clear();
    return s;
}

sgad_status sgad_set_tile(sgad_ctx* c, int w, int h) {
    if (!c) return SGAD_EINVAL;
    if (!(w == 0 && h == 0) && !valid_tile(w, h)) return fail(c, SGAD_EINVAL, "unsupported tile shape");
    c->tile_w = w;
    c->tile_h = h;
    return SGAD_OK;
}

sgad_status sgad_set_tile_variant(sgad_ctx* c, int fwd_chunks, int bwd_sub) {
    if (!c) return SGAD_EINVAL;
    if (!(fwd_chunks == 1 || fwd_chunks == 2 || fwd_chunks == 4) || !(bwd_sub == 16 || bwd_sub == 32))
        return fail(c, SGAD_EINVAL, "unsupported 8x8 kernel variant");
    c->var_scf = fwd_chunks;
    c->var_scb = bwd_sub;
    return SGAD_OK;
}

sgad_status sgad_get_tile(const sgad_ctx* c, int* w, int* h) {
    if (!c || !w || !h) return SGAD_EINVAL;
    *w = c->last_tw;
    *h = c->last_th;
    return SGAD_OK;
}

sgad_status sgad_get_tile_variant(const sgad_ctx* c, int* fwd_chunks, int* bwd_sub) {
    if (!c || !fwd_chunks || !bwd_sub) return SGAD_EINVAL;
    *fwd_chunks = c->last_scf;
    *bwd_sub = c->last_scb;
    return SGAD_OK;
}

sgad_status sgad_workspace_bytes(sgad_ctx* c, int n_kf, const sgad_keyframe* kf, int n_views,
                                 const sgad_cam* vcam, int n_jobs, const sgad_job* jobs, uint64_t instances,
                                 size_t* bytes) {
    if (!c) return SGAD_EINVAL;
    if (!bytes) return fail(c, SGAD_EINVAL, "bytes is null");
    if (n_kf < 1 || n_kf > kMaxKf || !kf) return fail(c, SGAD_EINVAL, "n_kf must be in [1, 64]");
    if (n_views < 1 || !vcam) return fail(c, SGAD_EINVAL, "need at least one view");
    if (n_jobs < 1 || !jobs) return fail(c, SGAD_EINVAL, "need at least one job");
    for (int f = 0; f < n_kf; ++f)
        if (!cam_ok(kf[f].cam) || kf[f].cam.H != kf[0].cam.H || kf[f].cam.W != kf[0].cam.W)
            return fail(c, SGAD_EINVAL, "keyframes must share a valid H x W");
    for (int v = 0; v < n_views; ++v)
        if (!cam_ok(vcam[v]) || vcam[v].H != vcam[0].H || vcam[v].W != vcam[0].W)
            return fail(c, SGAD_EINVAL, "views must share a valid H x W");
    int n_pairs = 0;
    for (int j = 0; j < n_jobs; ++j) {
        if (jobs[j].view < 0 || jobs[j].view >= n_views) return fail(c, SGAD_EINVAL, "job view out of range");
        const uint64_t m = (uint64_t)jobs[j].kf_mask_lo | ((uint64_t)jobs[j].kf_mask_hi << 32);
        if (n_kf < 64 && (m >> n_kf) != 0) return fail(c, SGAD_EINVAL, "job mask names a missing keyframe");
        n_pairs += __builtin_popcountll(m);
    }
    const size_t N = (size_t)kf[0].cam.H * kf[0].cam.W, P = (size_t)vcam[0].H * vcam[0].W;
    // 8x8 tiles give the most (job, tile) items of all tile shapes
    const size_t M = (size_t)n_jobs * (size_t)((vcam[0].W + 7) / 8) * (size_t)((vcam[0].H + 7) / 8);
    const size_t cap = instances ? counted_capacity((size_t)std::min<uint64_t>(instances, 0xffffffffu))
                                 : first_capacity((size_t)n_pairs * N);
    *bytes = slot_bytes(n_kf, n_pairs, n_jobs, N, P, M, cap).total();
    return SGAD_OK;
}

sgad_status sgad_render_fwd(sgad_ctx* c, int n_kf, const sgad_keyframe* kf, int n_views, const sgad_cam* vcam,
                            const sgad_pose* vpose, int n_jobs, const sgad_job* jobs, float* out_rgb,
                            float* out_depth, float* out_alpha, int32_t* out_count, sgad_saved** saved,
                            void* stream) {
    if (!c) return SGAD_EINVAL;
    if (!saved) return fail(c, SGAD_EINVAL, "saved is null");
    *saved = nullptr;
    if (n_kf < 1 || n_kf > kMaxKf || !kf) return fail(c, SGAD_EINVAL, "n_kf must be in [1, 64]");
    if (n_views < 1 || !vcam || !vpose) return fail(c, SGAD_EINVAL, "need at least one view");
    if (n_jobs < 1 || !jobs) return fail(c, SGAD_EINVAL, "need at least one job");
    if (!out_rgb || !out_depth || !out_alpha) return fail(c, SGAD_EINVAL, "null output");
    const sgad_cam& k0 = kf[0].cam;
    for (int f = 0; f < n_kf; ++f) {
        const sgad_keyframe& k = kf[f];
        if (!cam_ok(k.cam)) return fail(c, SGAD_EINVAL, "bad keyframe camera");
        if (k.cam.H != k0.H || k.cam.W != k0.W) return fail(c, SGAD_EINVAL, "keyframes must share H x W");
        if (!k.depth || !k.offset || !k.radius || !k.opacity || (!k.rgb && !k.sigma))
            return fail(c, SGAD_EINVAL, "null keyframe plane");
        if (!finite_pose(k.T_cw)) return fail(c, SGAD_EINVAL, "non-finite keyframe pose");
    }
    for (int v = 0; v < n_views; ++v) {
        if (!cam_ok(vcam[v])) return fail(c, SGAD_EINVAL, "bad view camera");
        if (vcam[v].H != vcam[0].H || vcam[v].W != vcam[0].W) return fail(c, SGAD_EINVAL, "views must share H x W");
        if (!finite_pose(vpose[v])) return fail(c, SGAD_EINVAL, "non-finite view pose");
    }
    int n_pairs = 0;
    for (int j = 0; j < n_jobs; ++j) {
        if (jobs[j].view < 0 || jobs[j].view >= n_views) return fail(c, SGAD_EINVAL, "job view out of range");
        const uint64_t m = (uint64_t)jobs[j].kf_mask_lo | ((uint64_t)jobs[j].kf_mask_hi << 32);
        if (n_kf < 64 && (m >> n_kf) != 0) return fail(c, SGAD_EINVAL, "job mask names a missing keyframe");
        n_pairs += __builtin_popcountll(m);
    }
    if (n_pairs == 0) return fail(c, SGAD_EINVAL, "jobs render no keyframe");
    const int64_t N = (int64_t)k0.H * k0.W;
    if ((int64_t)n_kf * N >= (1ll << 32) || (int64_t)n_pairs * N >= (1ll << 31) || n_pairs > 65535)
        return fail(c, SGAD_ERANGE, "too many Gaussians for one call");
    hipStream_t s = pick_stream(c, stream);
    HIPCHK(c, hipSetDevice(c->device));
    poll(c, false);
    const bool cap = c->capture.on;

    int TW = c->tile_w, TH = c->tile_h, SCF = c->var_scf, SCB = c->var_scb;
    if (c->force) {
        TW = c->ftw;
        TH = c->fth;
        SCF = c->fscf;
        SCB = c->fscb;
    } else if (TW == 0) {
        const size_t key[6] = {(size_t)vcam[0].H, (size_t)vcam[0].W, (size_t)N, (size_t)n_pairs, (size_t)n_jobs,
                               (size_t)n_kf};
        TW = 8;
        TH = 8;
        for (const auto& e : c->tune)
            if (std::memcmp(e.key, key, sizeof(key)) == 0) {
                TW = e.tw;
                TH = e.th;
                SCF = e.scf;
                SCB = e.scb;
            }
    }
    const size_t NP = (size_t)n_pairs * N;
    const size_t M = (size_t)n_jobs * (size_t)((vcam[0].W + TW - 1) / TW) * (size_t)((vcam[0].H + TH - 1) / TH);
    const size_t size_key[5] = {NP, M, (size_t)TW, (size_t)TH, (size_t)n_jobs};
    sgad_saved* S = cap ? acquire_sized(c, size_key) : acquire(c);
    if (!S && cap) {
        std::string why = "capturing a forward needs an earlier eager call of the same workload (slots:";
        for (sgad_saved* x : c->slots)
            why += std::string(" [") + (x->in_use ? "in use " : "") + (x->owner ? "graph " : "") +
                   (x->sized ? "" : "unsized ") +
                   (std::memcmp(x->size_key, size_key, sizeof(size_key)) ? "other-workload" : "same-workload") + "]";
        return fail(c, SGAD_EINVAL, why + ")");
    }
    if (!S) return fail(c, SGAD_ENOMEM, "cannot allocate a saved slot");
    if (cap) c->capture.slots.push_back(S);
    Geometry& G = S->G;
    G.n_kf = n_kf;
    G.n_jobs = n_jobs;
    G.n_pairs = n_pairs;
    G.Hk = k0.H;
    G.Wk = k0.W;
    G.N = (int)N;
    G.inv_n = 1.0 / (double)N;
    G.Hv = vcam[0].H;
    G.Wv = vcam[0].W;
    G.P = G.Hv * G.Wv;
    G.TW = TW;
    G.TH = TH;
    G.ntx = (G.Wv + TW - 1) / TW;
    G.nty = (G.Hv + TH - 1) / TH;
    G.ntiles = G.ntx * G.nty;
    G.sc_fwd = SCF;
    G.sc_bwd = SCB;
    G.fuse_sort = TW == 8 && TH == 8 ? 1 : 0;
    S->stream = s;
    c->last_tw = TW;
    c->last_th = TH;
    c->last_scf = SCF;
    c->last_scb = SCB;

    // parameter block: pairs | kf pointers | pair_of
    const size_t o_pairs = 0;
    const size_t o_kfs = align256(o_pairs + sizeof(PairConst) * n_pairs);
    const size_t o_pof = align256(o_kfs + sizeof(KfPtrs) * n_kf);
    const size_t up_bytes = align256(o_pof + sizeof(int32_t) * n_jobs * n_kf);
    S->stage.assign(up_bytes, 0);
    char* up = S->stage.data();
    PairConst* pairs = (PairConst*)(up + o_pairs);
    KfPtrs* kps = (KfPtrs*)(up + o_kfs);
    int32_t* pof = (int32_t*)(up + o_pof);
    int p = 0;
    for (int j = 0; j < n_jobs; ++j) {
        const uint64_t m = (uint64_t)jobs[j].kf_mask_lo | ((uint64_t)jobs[j].kf_mask_hi << 32);
        const sgad_cam& vc = vcam[jobs[j].view];
        for (int f = 0; f < n_kf; ++f) {
            pof[j * n_kf + f] = -1;
            if (!((m >> f) & 1ull)) continue;
            PairConst& pc = pairs[p];
            relative_pose(vpose[jobs[j].view], kf[f].T_cw, pc);
            pc.kfx = (double)kf[f].cam.fx;
            pc.kfy = (double)kf[f].cam.fy;
            pc.kcx = (double)kf[f].cam.cx;
            pc.kcy = (double)kf[f].cam.cy;
            pc.vfx = (double)vc.fx;
            pc.vfy = (double)vc.fy;
            pc.vcx = (double)vc.cx;
            pc.vcy = (double)vc.cy;
            pc.job = j;
            pc.kf = f;
            pof[j * n_kf + f] = p;
            ++p;
        }
    }
    for (int f = 0; f < n_kf; ++f)
        kps[f] = KfPtrs{kf[f].depth, kf[f].offset, kf[f].radius, kf[f].opacity, kf[f].rgb, kf[f].sigma};
    if (S->stage != S->last_up || S->params.bytes < up_bytes) {
        if (S->up_pending) {
            // the pinned staging buffer is rewritten: wait for its last upload
            // (while capturing nothing is in flight: capture began after a sync)
            if (!cap) HIPCHK(c, hipEventSynchronize(S->ev_up));
            S->up_pending = false;
        }
        if (cap && S->up.bytes < up_bytes) return fail(c, SGAD_EINVAL, "capture would resize the staging buffer");
        if (ensure_pin(S->up, up_bytes) != hipSuccess) return fail(c, SGAD_ENOMEM, "pinned alloc");
        HIPCHK(c, ensure_c(c, S->params, up_bytes, s));
        std::memcpy(S->up.p, up, up_bytes);
        HIPCHK(c, hipMemcpyAsync(S->params.p, S->up.p, up_bytes, hipMemcpyHostToDevice, s));
        if (!cap) {
            HIPCHK(c, hipEventRecord(S->ev_up, s));
            S->up_pending = true;
        }
        S->last_up = S->stage;
    }

    // workspace
    const size_t PJ = (size_t)n_jobs * G.P;
    const SlotBytes sb = slot_bytes(n_kf, n_pairs, n_jobs, (size_t)N, (size_t)G.P, M, 0);
    HIPCHK(c, ensure_c(c, S->pre, sb.pre, s));
    HIPCHK(c, ensure_c(c, S->tiles, sb.tiles, s));
    HIPCHK(c, ensure_c(c, S->pix, sb.pix, s));
    HIPCHK(c, ensure_c(c, S->pose_part, sb.pose_part, s));
    HIPCHK(c, ensure_c(c, S->status, sb.status, s));
    if (S->gacc.bytes < sb.gacc) {
        HIPCHK(c, ensure_c(c, S->gacc, sb.gacc, s));
        launch_fill_f32((float*)S->gacc.p, (int64_t)(S->gacc.bytes / 4), 0.f, s);
    }
    if (std::memcmp(size_key, S->size_key, sizeof(size_key)) != 0) {
        S->sized = false;
        S->last_max_seg = 0xffffffffu;
        std::memcpy(S->size_key, size_key, sizeof(size_key));
    }
    // the long-segment sort pass only when the last forward of this workload
    // had a segment over 1024 keys (or is unknown); else the register sort
    // falls back to a global-memory network for any segment that grew past it
    G.sort_long = S->last_max_seg <= 1024u ? 0 : (S->last_max_seg <= 2048u ? 1 : 2);
    if (!S->sized && S->capacity == 0) {
        // first use: a generous guess that is corrected after the count pass
        const size_t guess = first_capacity(NP);
        HIPCHK(c, ensure(S->keys, guess * 8, s));
        S->capacity = (uint32_t)guess;
    }

    RenderBufs& B = S->B;
    char* pb = (char*)S->params.p;
    B.pairs = (const PairConst*)(pb + o_pairs);
    B.kfs = (const KfPtrs*)(pb + o_kfs);
    B.pair_of = (const int32_t*)(pb + o_pof);
    char* pp = (char*)S->pre.p;
    B.pre.rec = (float4*)pp;
    B.pre.dir = (float4*)(pp + (size_t)NP * 64);
    B.pre.z = (float*)(pp + (size_t)NP * 80);
    B.pre.rx = (uint32_t*)(pp + (size_t)NP * 84);
    B.pre.ry = (uint32_t*)(pp + (size_t)NP * 88);
    uint32_t* tb = (uint32_t*)S->tiles.p;
    B.tile_count = tb;
    B.tile_fill = tb + M;
    B.tile_start = tb + 2 * M;
    B.chunk_start = tb + 3 * M + 1;
    B.keys = (uint64_t*)S->keys.p;
    B.capacity = S->capacity;
    B.cmask = nullptr;
    B.Tfinal = (float*)S->pix.p;
    B.last = (uint32_t*)((char*)S->pix.p + PJ * 4);
    B.status = (DevStatus*)S->status.p;
    B.status_host = S->status_dev;

    // Each call's scan clears the counts it read and its forward clears the
    // flags, so the clearing launch is needed only when the slot's buffers or
    // tile count changed, or the previous call stopped before its forward.
    if (!S->status_dev || S->zeroed_M != M || S->tiles.p != S->zeroed_tiles) {
        TimeScope ts(c, "zero", s);
        launch_zero2_u32((uint32_t*)B.status, sizeof(DevStatus) / 4, B.tile_count, (int64_t)M, s);
    }
    S->zeroed_M = -1;   // until this call's forward is enqueued
    {
        TimeScope ts(c, "preprocess", s);
        launch_preprocess(G, B, s);
    }
    {
        TimeScope ts(c, "scan", s);
        launch_scan(G, B, S->sized, s);   // the sizing pass keeps the counts for its rescan
    }
    if (!S->sized) {
        // size the instance buffer from the exact count (one host wait)
        HIPCHK(c, hipMemcpyAsync(S->status_h, B.status, sizeof(DevStatus), hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipStreamSynchronize(s));
        const uint32_t total = S->status_h->total;
        if ((size_t)total + (size_t)total / 4 > S->capacity || S->capacity == 0) {
            const size_t cap = counted_capacity(total);
            HIPCHK(c, ensure(S->keys, cap * 8, s));
            S->capacity = (uint32_t)cap;
            B.keys = (uint64_t*)S->keys.p;
            B.capacity = S->capacity;
        }
        launch_scan(G, B, true, s);   // same offsets; overflow against the new capacity; counts cleared
        S->sized = true;
    }
    // contributor masks: one u64 per (64-entry chunk, pixel); at most
    // capacity / 64 + M chunks
    HIPCHK(c, ensure_c(c, S->cmask, slot_bytes(n_kf, n_pairs, n_jobs, (size_t)N, (size_t)G.P, M, S->capacity).cmask, s));
    B.cmask = (uint64_t*)S->cmask.p;
    {
        TimeScope ts(c, "scatter", s);
        launch_scatter(G, B, s);
    }
    {
        TimeScope ts(c, "sort", s);
        launch_sort(G, B, s);
    }
    {
        TimeScope ts(c, "composite_fwd", s);
        if (!launch_fwd(G, B, out_rgb, out_depth, out_alpha, out_count, s))
            return fail(c, SGAD_EINVAL, "unsupported tile shape");
    }
    HIPCHK(c, hipGetLastError());
    S->zeroed_M = M;
    S->zeroed_tiles = S->tiles.p;
    if (!cap) {
        // (a captured forward's status is read back after each graph launch)
        if (!S->status_dev)
            HIPCHK(c, hipMemcpyAsync(S->status_h, B.status, sizeof(DevStatus), hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipEventRecord(S->ev_status, s));
        S->status_pending = true;
    }
    *saved = S;
    return SGAD_OK;
}

sgad_status sgad_render_bwd(sgad_ctx* c, sgad_saved* S, const float* g_rgb, const float* g_depth,
                            const float* g_alpha, const sgad_kf_grads* grads, float* d_pose, uint32_t learn_lo,
                            uint32_t learn_hi, void* stream) {
    if (!c) return SGAD_EINVAL;
    if (!S || !S->in_use) return fail(c, SGAD_EINVAL, "invalid saved handle");
    if (!g_rgb) return fail(c, SGAD_EINVAL, "g_rgb is null");
    const Geometry& G = S->G;
    const uint64_t learn = (uint64_t)learn_lo | ((uint64_t)learn_hi << 32);
    for (int f = 0; f < G.n_kf; ++f) {
        if (!((learn >> f) & 1ull)) continue;
        if (!grads || !grads[f].d_rgb || !grads[f].d_opacity || !grads[f].d_radius || !grads[f].d_offset)
            return fail(c, SGAD_EINVAL, "null gradient output for a learnable keyframe");
    }
    hipStream_t s = pick_stream(c, stream);
    const bool cap = c->capture.on;
    HIPCHK(c, hipSetDevice(c->device));
    poll(c, false);
    const size_t gb = align256(sizeof(KfGradPtrs) * G.n_kf);
    S->stage_grad.assign(gb, 0);
    KfGradPtrs* gp = (KfGradPtrs*)S->stage_grad.data();
    for (int f = 0; f < G.n_kf; ++f) {
        if (grads && ((learn >> f) & 1ull))
            gp[f] = KfGradPtrs{grads[f].d_rgb, grads[f].d_opacity, grads[f].d_radius, grads[f].d_offset};
        else
            gp[f] = KfGradPtrs{nullptr, nullptr, nullptr, nullptr};
    }
    if (S->stage_grad != S->last_up_grad || S->gradptrs.bytes < gb) {
        if (S->up_grad_pending) {
            if (!cap) HIPCHK(c, hipEventSynchronize(S->ev_up_grad));
            S->up_grad_pending = false;
        }
        if (cap && (S->up_grad.bytes < gb || S->gradptrs.bytes < gb))
            return fail(c, SGAD_EINVAL, "capturing a backward needs an earlier eager call of the same workload");
        if (ensure_pin(S->up_grad, gb) != hipSuccess) return fail(c, SGAD_ENOMEM, "pinned alloc");
        HIPCHK(c, ensure_c(c, S->gradptrs, gb, s));
        std::memcpy(S->up_grad.p, gp, gb);
        HIPCHK(c, hipMemcpyAsync(S->gradptrs.p, S->up_grad.p, gb, hipMemcpyHostToDevice, s));
        if (!cap) {
            HIPCHK(c, hipEventRecord(S->ev_up_grad, s));
            S->up_grad_pending = true;
        }
        S->last_up_grad = S->stage_grad;
    }
    {
        TimeScope ts(c, "composite_bwd", s);
        if (!launch_bwd(G, S->B, g_rgb, g_depth, g_alpha, (const KfGradPtrs*)S->gradptrs.p, learn_lo, learn_hi,
                        (float*)S->pose_part.p, (float*)S->gacc.p, d_pose, s))
            return fail(c, SGAD_EINVAL, "unsupported tile shape");
    }
    if (G.TW == 8 && G.TH == 8) {
        TimeScope ts(c, "grad_finish", s);
        launch_bwd_finish(G, (const KfGradPtrs*)S->gradptrs.p, learn_lo, learn_hi, (float*)S->gacc.p,
                          (const float*)S->pose_part.p, d_pose, s);
    }
    HIPCHK(c, hipGetLastError());
    return SGAD_OK;
}

sgad_status sgad_timing_enable(sgad_ctx* c, int enable) {
    if (!c) return SGAD_EINVAL;
    if (c->capture.on) return fail(c, SGAD_EINVAL, "not allowed while capturing a graph");
    HIPCHK(c, hipSetDevice(c->device));
    timer_collect(c);
    c->timer.names.clear();
    c->timer.ms.clear();
    c->timer.count.clear();
    c->timer.on = enable != 0;
    return SGAD_OK;
}

sgad_status sgad_timing_only(sgad_ctx* c, const char* name) {
    if (!c) return SGAD_EINVAL;
    c->timer.only = name ? name : "";
    return SGAD_OK;
}

sgad_status sgad_timing_report(sgad_ctx* c, char* buf, size_t cap) {
    if (!c || !buf || cap == 0) return SGAD_EINVAL;
    if (c->capture.on) return fail(c, SGAD_EINVAL, "not allowed while capturing a graph");
    HIPCHK(c, hipSetDevice(c->device));
    timer_collect(c);
    std::string out;
    char line[256];
    for (size_t k = 0; k < c->timer.names.size(); ++k) {
        snprintf(line, sizeof(line), "%s %ld %.6f\n", c->timer.names[k].c_str(), c->timer.count[k], c->timer.ms[k]);
        out += line;
    }
    if (out.size() + 1 > cap) return fail(c, SGAD_ERANGE, "timing report buffer too small");
    std::memcpy(buf, out.c_str(), out.size() + 1);
    return SGAD_OK;
}

sgad_status sgad_l1_loss(sgad_ctx* c, int n_jobs, int H, int W, const float* rgb, const float* depth,
                         const float* t_rgb, const float* t_depth, float w_rgb, float w_depth, float* g_rgb,
                         float* g_depth, double* loss, void* stream) {
    if (!c) return SGAD_EINVAL;
    if (n_jobs < 1 || H < 1 || W < 1) return fail(c, SGAD_EINVAL, "bad sizes");
    if (!rgb || !depth || !t_rgb || !t_depth || !g_rgb || !g_depth || !loss)
        return fail(c, SGAD_EINVAL, "null pointer");
    hipStream_t s = pick_stream(c, stream);
    HIPCHK(c, hipSetDevice(c->device));
    if ((int64_t)H * W > INT32_MAX / 2) return fail(c, SGAD_ERANGE, "image too large");
    HIPCHK(c, ensure_c(c, c->scratch, (size_t)n_jobs * l1_blocks(H * W) * 4, s));
    uint32_t* cnt = (uint32_t*)c->scratch.p;
    TimeScope ts(c, "l1_loss", s);
    launch_l1(n_jobs, H * W, rgb, depth, t_rgb, t_depth, w_rgb, w_depth, cnt, 0, g_rgb, g_depth, loss, s);
    HIPCHK(c, hipGetLastError());
    return SGAD_OK;
}

sgad_status sgad_eq1_loss(sgad_ctx* c, int n_jobs, int H, int W, const float* rgb, const float* depth,
                          const float* t_rgb, const float* t_depth, float w_rgb, float w_ssim, float w_depth,
                          float* g_rgb, float* g_depth, double* loss, void* stream) {
    if (!c) return SGAD_EINVAL;
    if (n_jobs < 1 || H < 1 || W < 1) return fail(c, SGAD_EINVAL, "bad sizes");
    if (n_jobs > 65535 / 3) return fail(c, SGAD_ERANGE, "at most 21845 jobs");
    if (!rgb || !depth || !t_rgb || !t_depth || !g_rgb || !g_depth || !loss)
        return fail(c, SGAD_EINVAL, "null pointer");
    if (!std::isfinite(w_rgb) || !std::isfinite(w_ssim) || !std::isfinite(w_depth))
        return fail(c, SGAD_EINVAL, "non-finite weight");
    hipStream_t s = pick_stream(c, stream);
    HIPCHK(c, hipSetDevice(c->device));
    if ((int64_t)H * W > INT32_MAX / 2) return fail(c, SGAD_ERANGE, "image too large");
    // valid-depth counts: one per (job, L1 block), or per (job, SSIM tile)
    // when the SSIM maps count them
    const size_t nparts = w_ssim != 0.f ? ssim_tiles(H, W) : (size_t)l1_blocks(H * W);
    HIPCHK(c, ensure_c(c, c->scratch, (size_t)n_jobs * nparts * 4, s));
    if (w_ssim != 0.f) HIPCHK(c, ensure_c(c, c->ssim_maps, ssim_map_bytes(n_jobs, H, W), s));
    uint32_t* cnt = (uint32_t*)c->scratch.p;
    if (w_ssim != 0.f) {
        {
            TimeScope ts(c, "ssim_maps", s);
            launch_ssim_maps(n_jobs, H, W, rgb, t_rgb, c->ssim_maps.p, t_depth, cnt, loss, s);
        }
        {
            TimeScope ts(c, "l1_loss", s);
            launch_l1(n_jobs, H * W, rgb, depth, t_rgb, t_depth, w_rgb, w_depth, cnt, (int)nparts, g_rgb, g_depth,
                      loss, s);
        }
        TimeScope ts(c, "ssim_grad", s);
        launch_ssim_grad(n_jobs, H, W, rgb, t_rgb, w_ssim, c->ssim_maps.p, g_rgb, loss, s);
    } else {
        TimeScope ts(c, "l1_loss", s);
        launch_l1(n_jobs, H * W, rgb, depth, t_rgb, t_depth, w_rgb, w_depth, cnt, 0, g_rgb, g_depth, loss, s);
    }
    HIPCHK(c, hipGetLastError());
    return SGAD_OK;
}

int32_t sgad_gicp_set_size(int H, int W, int ratio) {
    if (H < 1 || W < 1 || ratio < 1) return -1;
    const int64_t n = (int64_t)((H + ratio - 1) / ratio) * ((W + ratio - 1) / ratio);
    return n > (int64_t)INT32_MAX / 12 ? -1 : (int32_t)n;
}

sgad_status sgad_gicp_prepare(sgad_ctx* c, const float* depth, const sgad_cam* cam, int ratio, int k, double* set,
                              void* stream) {
    if (!c) return SGAD_EINVAL;
    if (!depth || !cam || !set) return fail(c, SGAD_EINVAL, "null pointer");
    if (cam->H < 1 || cam->W < 1 || ratio < 1) return fail(c, SGAD_EINVAL, "bad sizes");
    if (!(std::isfinite(cam->fx) && std::isfinite(cam->fy) && cam->fx > 0.f && cam->fy > 0.f &&
          std::isfinite(cam->cx) && std::isfinite(cam->cy)))
        return fail(c, SGAD_EINVAL, "bad intrinsics");
    if (k < 1 || k > gicp_max_k()) return fail(c, SGAD_ERANGE, "K_c must be 1..32");
    if (sgad_gicp_set_size(cam->H, cam->W, ratio) < 1) return fail(c, SGAD_ERANGE, "set too large");
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t s = pick_stream(c, stream);
    TimeScope ts(c, "gicp_prepare", s);
    launch_gicp_prepare(depth, cam->H, cam->W, ratio, *cam, k, set, s);
    HIPCHK(c, hipGetLastError());
    return SGAD_OK;
}

static sgad_status gicp_args(sgad_ctx* c, const double* src, int n_src, const double* tgt, int n_tgt,
                             const sgad_cam* tcam, int tratio, int k, const double* pose) {
    if (!src || !tgt || !pose || !tcam) return fail(c, SGAD_EINVAL, "null pointer");
    if (n_src < 1 || n_tgt < 1) return fail(c, SGAD_EINVAL, "empty set");
    if (n_src > INT32_MAX / 12 || n_tgt > INT32_MAX / 12) return fail(c, SGAD_ERANGE, "set too large");
    if (k < 1 || k > gicp_max_k()) return fail(c, SGAD_ERANGE, "K_c must be 1..32");
    if (tratio < 1 || sgad_gicp_set_size(tcam->H, tcam->W, tratio) != n_tgt)
        return fail(c, SGAD_EINVAL, "target camera and ratio do not give n_tgt grid points");
    if (!(std::isfinite(tcam->fx) && std::isfinite(tcam->fy) && tcam->fx > 0.f && tcam->fy > 0.f &&
          std::isfinite(tcam->cx) && std::isfinite(tcam->cy)))
        return fail(c, SGAD_EINVAL, "bad intrinsics");
    return SGAD_OK;
}

sgad_status sgad_gicp_linearise(sgad_ctx* c, const double* src, int n_src, const double* tgt, int n_tgt,
                                const sgad_cam* tgt_cam, int tgt_ratio, int k, const double* pose, double* out,
                                int32_t* corr, void* stream) {
    if (!c) return SGAD_EINVAL;
    if (const sgad_status st = gicp_args(c, src, n_src, tgt, n_tgt, tgt_cam, tgt_ratio, k, pose)) return st;
    if (!out) return fail(c, SGAD_EINVAL, "null pointer");
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t s = pick_stream(c, stream);
    const int nb = gicp_wave_blocks(n_src);
    HIPCHK(c, ensure_c(c, c->gicp_part, (size_t)nb * gicp_vals() * sizeof(double), s));
    double* part = (double*)c->gicp_part.p;
    TimeScope ts(c, "gicp_linearise", s);
    launch_gicp_linearise(src, n_src, tgt, n_tgt, *tgt_cam, tgt_ratio, k, pose, part, corr, s);
    launch_gicp_sum(part, nb, out, s);
    HIPCHK(c, hipGetLastError());
    return SGAD_OK;
}

sgad_status sgad_gicp_track(sgad_ctx* c, const double* src, int n_src, const double* tgt, int n_tgt,
                            const sgad_cam* tgt_cam, int tgt_ratio, int k, double* pose, int iters, double* trace,
                            void* stream) {
    if (!c) return SGAD_EINVAL;
    if (const sgad_status st = gicp_args(c, src, n_src, tgt, n_tgt, tgt_cam, tgt_ratio, k, pose)) return st;
    if (iters < 1) return fail(c, SGAD_EINVAL, "iters must be >= 1");
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t s = pick_stream(c, stream);
    const int nb = gicp_wave_blocks(n_src);
    HIPCHK(c, ensure_c(c, c->gicp_part, (size_t)nb * gicp_vals() * sizeof(double), s));
    double* part = (double*)c->gicp_part.p;
    TimeScope ts(c, "gicp_iteration", s);
    for (int it = 0; it < iters; ++it) {
        launch_gicp_linearise(src, n_src, tgt, n_tgt, *tgt_cam, tgt_ratio, k, pose, part, nullptr, s);
        launch_gicp_solve(part, nb, pose, trace, it, s);
    }
    HIPCHK(c, hipGetLastError());
    return SGAD_OK;
}

static sgad_status gmap_args(sgad_ctx* c, const sgad_gmap* m) {
    if (!m || !m->data || !m->keys || !m->vals || !m->count) return fail(c, SGAD_EINVAL, "null pointer");
    if (m->capacity < 1 || m->capacity > INT32_MAX / 12) return fail(c, SGAD_ERANGE, "capacity out of range");
    if (m->slots < 2 || (m->slots & (m->slots - 1)) != 0 || m->slots / 2 < m->capacity)
        return fail(c, SGAD_EINVAL, "slots must be a power of two >= 2 * capacity");
    if (!(std::isfinite(m->voxel) && m->voxel >= 0.1 / 32)) return fail(c, SGAD_ERANGE, "voxel below D_MAX / 32");
    return SGAD_OK;
}

sgad_status sgad_gmap_reset(sgad_ctx* c, const sgad_gmap* m, void* stream) {
    if (!c) return SGAD_EINVAL;
    if (const sgad_status st = gmap_args(c, m)) return st;
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t s = pick_stream(c, stream);
    launch_gmap_reset(*m, s);
    HIPCHK(c, hipGetLastError());
    return SGAD_OK;
}

sgad_status sgad_gmap_insert(sgad_ctx* c, const sgad_gmap* m, const double* set, int n, const double* pose,
                             void* stream) {
    if (!c) return SGAD_EINVAL;
    if (const sgad_status st = gmap_args(c, m)) return st;
    if (!set || !pose) return fail(c, SGAD_EINVAL, "null pointer");
    if (n < 1) return fail(c, SGAD_EINVAL, "empty set");
    if (n > INT32_MAX / 12) return fail(c, SGAD_ERANGE, "set too large");
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t s = pick_stream(c, stream);
    TimeScope ts(c, "gmap_insert", s);
    launch_gmap_insert(*m, set, n, pose, s);
    HIPCHK(c, hipGetLastError());
    return SGAD_OK;
}

static sgad_status gicp_map_args(sgad_ctx* c, const double* src, int n_src, const sgad_gmap* m, int k,
                                 const double* pose) {
    if (const sgad_status st = gmap_args(c, m)) return st;
    if (!src || !pose) return fail(c, SGAD_EINVAL, "null pointer");
    if (n_src < 1) return fail(c, SGAD_EINVAL, "empty set");
    if (n_src > INT32_MAX / 12) return fail(c, SGAD_ERANGE, "set too large");
    if (k < 1 || k > gicp_max_k()) return fail(c, SGAD_ERANGE, "K_c must be 1..32");
    return SGAD_OK;
}

sgad_status sgad_gicp_linearise_map(sgad_ctx* c, const double* src, int n_src, const sgad_gmap* m, int k,
                                    const double* pose, double* out, int32_t* corr, void* stream) {
    if (!c) return SGAD_EINVAL;
    if (const sgad_status st = gicp_map_args(c, src, n_src, m, k, pose)) return st;
    if (!out) return fail(c, SGAD_EINVAL, "null pointer");
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t s = pick_stream(c, stream);
    const int nb = gicp_wave_blocks(n_src);
    HIPCHK(c, ensure_c(c, c->gicp_part, (size_t)nb * gicp_vals() * sizeof(double), s));
    double* part = (double*)c->gicp_part.p;
    TimeScope ts(c, "gicp_linearise_map", s);
    launch_gicp_linearise_map(src, n_src, *m, k, pose, part, corr, s);
    launch_gicp_sum(part, nb, out, s);
    HIPCHK(c, hipGetLastError());
    return SGAD_OK;
}

sgad_status sgad_gicp_track_map(sgad_ctx* c, const double* src, int n_src, const sgad_gmap* m, int k, double* pose,
                                int iters, double* trace, void* stream) {
    if (!c) return SGAD_EINVAL;
    if (const sgad_status st = gicp_map_args(c, src, n_src, m, k, pose)) return st;
    if (iters < 1) return fail(c, SGAD_EINVAL, "iters must be >= 1");
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t s = pick_stream(c, stream);
    const int nb = gicp_wave_blocks(n_src);
    HIPCHK(c, ensure_c(c, c->gicp_part, (size_t)nb * gicp_vals() * sizeof(double), s));
    double* part = (double*)c->gicp_part.p;
    TimeScope ts(c, "gicp_map_iteration", s);
    for (int it = 0; it < iters; ++it) {
        launch_gicp_linearise_map(src, n_src, *m, k, pose, part, nullptr, s);
        launch_gicp_solve(part, nb, pose, trace, it, s);
    }
    HIPCHK(c, hipGetLastError());
    return SGAD_OK;
}

sgad_status sgad_fill_depth(sgad_ctx* c, int P, const float* depth, const float* rdepth, const float* ralpha,
                            float alpha_min, float* out, void* stream) {
    if (!c) return SGAD_EINVAL;
    if (!depth || !rdepth || !ralpha || !out) return fail(c, SGAD_EINVAL, "null pointer");
    if (P < 1) return fail(c, SGAD_EINVAL, "bad sizes");
    if (!(alpha_min > 0.f && alpha_min <= 1.f)) return fail(c, SGAD_EINVAL, "alpha_min must be in (0, 1]");
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t s = pick_stream(c, stream);
    launch_fill_depth(P, depth, rdepth, ralpha, alpha_min, out, s);
    HIPCHK(c, hipGetLastError());
    return SGAD_OK;
}

sgad_status sgad_adam_step(sgad_ctx* c, int n_groups, const sgad_adam_group* groups, int step, float beta1,
                           float beta2, float eps, int zero_grad, void* stream) {
    if (!c) return SGAD_EINVAL;
    if (n_groups < 1 || n_groups > kMaxAdamGroups || !groups) return fail(c, SGAD_ERANGE, "1..32 groups");
    if (step < 1) return fail(c, SGAD_EINVAL, "step counts from 1");
    AdamGroups A{};
    A.n = n_groups;
    A.off[0] = 0;
    for (int g = 0; g < n_groups; ++g) {
        const sgad_adam_group& G = groups[g];
        if (G.n < 0 || (G.n > 0 && (!G.param || !G.grad || !G.m || !G.v)))
            return fail(c, SGAD_EINVAL, "bad adam group");
        A.p[g] = G.param;
        A.g[g] = G.grad;
        A.m[g] = G.m;
        A.v[g] = G.v;
        A.lr[g] = G.lr;
        A.lo[g] = G.lo;
        A.hi[g] = G.hi;
        if (G.space < 0 || G.space > 2) return fail(c, SGAD_EINVAL, "unknown adam space");
        A.space[g] = G.space;
        A.off[g + 1] = A.off[g] + G.n;
    }
    if (A.off[n_groups] > ((int64_t)1 << 40)) return fail(c, SGAD_ERANGE, "more than 2^40 Adam elements");
    hipStream_t s = pick_stream(c, stream);
    HIPCHK(c, hipSetDevice(c->device));
    const float c1 = (float)(1.0 - std::pow((double)beta1, step));
    const float c2 = (float)(1.0 - std::pow((double)beta2, step));
    float* cdev = nullptr;
    if (c->capture.on) {
        // a replayed step must advance t: the graph keeps a device counter
        // that starts at step - 1 and is incremented by each launch
        auto& C = c->capture;
        if (C.n_adam == kMaxGraphAdam) return fail(c, SGAD_ERANGE, "too many Adam calls in one captured graph");
        C.adam_t0[C.n_adam] = step - 1;
        cdev = (float*)C.adam.p + 4 * C.n_adam;
        ++C.n_adam;
    }
    TimeScope ts(c, "adam", s);
    launch_adam(A, beta1, beta2, eps, c1, c2, zero_grad, cdev, s);
    HIPCHK(c, hipGetLastError());
    return SGAD_OK;
}

sgad_status sgad_graph_begin(sgad_ctx* c, void* stream) {
    if (!c) return SGAD_EINVAL;
    auto& C = c->capture;
    if (C.on) return fail(c, SGAD_EINVAL, "a capture is already open");
    HIPCHK(c, hipSetDevice(c->device));
    // nothing of this context may be in flight while its staging buffers are
    // rewritten by the captured calls
    HIPCHK(c, hipStreamSynchronize((hipStream_t)stream));
    HIPCHK(c, hipDeviceSynchronize());
    poll(c, true);
    if (!C.cap) HIPCHK(c, hipStreamCreateWithFlags(&C.cap, hipStreamNonBlocking));
    HIPCHK(c, ensure(C.adam, sizeof(float) * 4 * kMaxGraphAdam, C.cap));
    C.n_adam = 0;
    C.slots.clear();
    C.timed.clear();
    HIPCHK(c, hipStreamBeginCapture(C.cap, hipStreamCaptureModeThreadLocal));
    C.on = true;
    return SGAD_OK;
}

sgad_status sgad_graph_end(sgad_ctx* c, sgad_graph** out) {
    if (!c) return SGAD_EINVAL;
    auto& C = c->capture;
    if (!C.on) return fail(c, SGAD_EINVAL, "no capture is open");
    C.on = false;
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(C.cap, &graph);
    auto drop_timed = [&]() {
        for (auto& t : C.timed) {
            (void)hipEventDestroy(t.second.first);
            (void)hipEventDestroy(t.second.second);
        }
        C.timed.clear();
    };
    if (e != hipSuccess || !graph || !out) {
        if (graph) (void)hipGraphDestroy(graph);
        drop_timed();
        if (!out) return fail(c, SGAD_EINVAL, "out is null");
        return fail(c, SGAD_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    }
    sgad_graph* g = new sgad_graph();
    g->graph = graph;
    // map the timing events to their event-record nodes
    if (!C.timed.empty()) {
        size_t n = 0;
        std::vector<hipGraphNode_t> nodes;
        if (hipGraphGetNodes(graph, nullptr, &n) == hipSuccess && n > 0) {
            nodes.resize(n);
            if (hipGraphGetNodes(graph, nodes.data(), &n) != hipSuccess) nodes.clear();
        }
        for (auto& t : C.timed) {
            hipGraphNode_t na = nullptr, nb = nullptr;
            for (hipGraphNode_t nd : nodes) {
                hipGraphNodeType ty;
                hipEvent_t ev = nullptr;
                if (hipGraphNodeGetType(nd, &ty) != hipSuccess || ty != hipGraphNodeTypeEventRecord) continue;
                if (hipGraphEventRecordNodeGetEvent(nd, &ev) != hipSuccess) continue;
                if (ev == t.second.first) na = nd;
                if (ev == t.second.second) nb = nd;
            }
            if (na && nb) g->timed.push_back({t.first, {na, nb}});
        }
    }
    hipError_t ie = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
    if (ie != hipSuccess) {
        (void)hipGraphDestroy(graph);
        drop_timed();
        delete g;
        return fail(c, SGAD_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(ie));
    }
    // the nodes keep referring to these events until they are swapped
    for (auto& t : C.timed) {
        g->events.push_back(t.second.first);
        g->events.push_back(t.second.second);
    }
    C.timed.clear();
    // the graph owns the Adam counters and the slots it was captured with
    g->adam = C.adam;
    C.adam = DevBuf{};
    if (C.n_adam > 0) {
        float init[4 * kMaxGraphAdam] = {};
        for (int k = 0; k < C.n_adam; ++k) {
            int t0 = C.adam_t0[k];
            std::memcpy(&init[4 * k], &t0, sizeof(int));
        }
        HIPCHK(c, hipMemcpy(g->adam.p, init, sizeof(init), hipMemcpyHostToDevice));
    }
    for (sgad_saved* S : C.slots) {
        S->owner = g;
        g->slots.push_back(S);
    }
    C.slots.clear();
    *out = g;
    return SGAD_OK;
}

sgad_status sgad_graph_launch(sgad_ctx* c, sgad_graph* g, void* stream) {
    if (!c || !g) return SGAD_EINVAL;
    if (c->capture.on) return fail(c, SGAD_EINVAL, "not allowed while capturing a graph");
    hipStream_t s = (hipStream_t)stream;
    HIPCHK(c, hipSetDevice(c->device));
    poll(c, false);
    if (c->timer.on)
        for (auto& t : g->timed) {
            hipEvent_t a, b;
            if (!timer_pair(c, t.first, &a, &b)) break;
            HIPCHK(c, hipGraphExecEventRecordNodeSetEvent(g->exec, t.second.first, a));
            HIPCHK(c, hipGraphExecEventRecordNodeSetEvent(g->exec, t.second.second, b));
        }
    HIPCHK(c, hipGraphLaunch(g->exec, s));
    for (sgad_saved* S : g->slots) {
        // read back what the replayed forwards found, as an eager forward does
        if (S->status_pending) continue;
        if (!S->status_dev)
            HIPCHK(c, hipMemcpyAsync(S->status_h, S->B.status, sizeof(DevStatus), hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipEventRecord(S->ev_status, s));
        S->status_pending = true;
    }
    return SGAD_OK;
}

sgad_status sgad_graph_destroy(sgad_ctx* c, sgad_graph* g) {
    if (!c || !g) return SGAD_EINVAL;
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, hipDeviceSynchronize());
    poll(c, true);
    for (sgad_saved* S : g->slots) S->owner = nullptr;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    for (hipEvent_t e : g->events) (void)hipEventDestroy(e);
    if (g->adam.p) (void)hipFree(g->adam.p);
    delete g;
    return SGAD_OK;
}

sgad_status sgad_saved_release(sgad_ctx* c, sgad_saved* S) {
    if (!c || !S) return SGAD_EINVAL;
    for (sgad_saved* x : c->slots)
        if (x == S) {
            S->in_use = false;
            return SGAD_OK;
        }
    return fail(c, SGAD_EINVAL, "handle does not belong to this context");
}

sgad_status sgad_saved_instances(sgad_ctx* c, const sgad_saved* S, int job, uint32_t* tile_ranges,
                                 uint64_t* keys, size_t cap, size_t* n_keys, int* n_tiles) {
    if (!c || !S || !S->in_use || !n_keys || !n_tiles) return SGAD_EINVAL;
    if (c->capture.on) return fail(c, SGAD_EINVAL, "not allowed while capturing a graph");
    const Geometry& G = S->G;
    if (job < 0 || job >= G.n_jobs) return fail(c, SGAD_EINVAL, "job out of range");
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, hipStreamSynchronize(S->stream));
    DevStatus st;
    HIPCHK(c, hipMemcpy(&st, S->B.status, sizeof(st), hipMemcpyDeviceToHost));
    if (st.overflow) return fail(c, SGAD_ERANGE, "instance list overflowed");
    std::vector<uint32_t> start(G.ntiles + 1);
    HIPCHK(c, hipMemcpy(start.data(), S->B.tile_start + (size_t)job * G.ntiles, (G.ntiles + 1) * 4,
                        hipMemcpyDeviceToHost));
    const size_t n = start[G.ntiles] - start[0];
    *n_keys = n;
    *n_tiles = G.ntiles;
    if (tile_ranges)
        for (int t = 0; t < G.ntiles; ++t) {
            tile_ranges[2 * t] = start[t] - start[0];
            tile_ranges[2 * t + 1] = start[t + 1] - start[0];
        }
    if (keys) {
        if (cap < n) return fail(c, SGAD_ERANGE, "key buffer too small");
        HIPCHK(c, hipMemcpy(keys, S->B.keys + start[0], n * 8, hipMemcpyDeviceToHost));
    }
    return SGAD_OK;
}

sgad_status sgad_track_gn(sgad_ctx* c, const sgad_keyframe* geo, const sgad_cam* vcam, const float* obs_depth,
                          double* pose, int iters, double* trace, uint32_t flags, void* stream) {
    if (!c) return SGAD_EINVAL;
    if (c->capture.on) return fail(c, SGAD_EINVAL, "not allowed while capturing a graph");
    if (!geo || !vcam || !obs_depth || !pose) return fail(c, SGAD_EINVAL, "null argument");
    if (iters < 1 || iters > 1000) return fail(c, SGAD_ERANGE, "iters must be in [1, 1000]");
    if (!cam_ok(geo->cam) || !cam_ok(*vcam)) return fail(c, SGAD_EINVAL, "bad camera");
    if (!geo->depth || !geo->offset || !geo->radius || !geo->opacity || !geo->sigma)
        return fail(c, SGAD_EINVAL, "geometry keyframe needs depth, offset, radius, opacity and sigma");
    if (!finite_pose(geo->T_cw)) return fail(c, SGAD_EINVAL, "non-finite keyframe pose");
    hipStream_t s = (hipStream_t)stream;
    HIPCHK(c, hipSetDevice(c->device));
    poll(c, false);
    auto& T = c->track;
    int TW = c->tile_w ? c->tile_w : 8, TH = c->tile_h ? c->tile_h : 8;
    Geometry& G = T.G;
    const int64_t N = (int64_t)geo->cam.H * geo->cam.W;
    const bool same_shape = T.sized && G.Hk == geo->cam.H && G.Wk == geo->cam.W && G.Hv == vcam->H &&
                            G.Wv == vcam->W && G.TW == TW && G.TH == TH;
    G.n_kf = 1;
    G.n_jobs = 1;
    G.n_pairs = 1;
    G.Hk = geo->cam.H;
    G.Wk = geo->cam.W;
    G.N = (int)N;
    G.inv_n = 1.0 / (double)N;
    G.Hv = vcam->H;
    G.Wv = vcam->W;
    G.P = G.Hv * G.Wv;
    G.TW = TW;
    G.TH = TH;
    G.ntx = (G.Wv + TW - 1) / TW;
    G.nty = (G.Hv + TH - 1) / TH;
    G.ntiles = G.ntx * G.nty;
    G.fuse_sort = TW == 8 && TH == 8 ? 1 : 0;   // the wave-tile kernel sorts its own segments
    const size_t M = (size_t)G.ntiles;
    if (!T.status_h) {
        HIPCHK(c, hipHostMalloc((void**)&T.status_h, sizeof(DevStatus), hipHostMallocDefault));
        HIPCHK(c, hipEventCreateWithFlags(&T.ev_status, hipEventDisableTiming));
        HIPCHK(c, hipStreamCreateWithFlags(&T.cap, hipStreamNonBlocking));
    }
    if (T.status_pending) {
        HIPCHK(c, hipEventSynchronize(T.ev_status));
        T.status_pending = false;
        latch_status(c, *T.status_h);
    }
    HIPCHK(c, ensure(T.params, 1024, s));
    HIPCHK(c, ensure(T.pre, (size_t)N * 92 + 256, s));
    HIPCHK(c, ensure(T.tiles, (4 * M + 2) * 4 + 256, s));
    HIPCHK(c, ensure(T.part, M * 32 * 4, s));
    HIPCHK(c, ensure(T.status, sizeof(DevStatus), s));
    HIPCHK(c, ensure(T.trace, (size_t)iters * 40 * 8, s));
    double* tr = trace ? trace : (double*)T.trace.p;
    RenderBufs& B = T.B;
    char* pb = (char*)T.params.p;
    B.pairs = (const PairConst*)pb;
    B.kfs = (const KfPtrs*)(pb + 512);
    B.pair_of = (const int32_t*)(pb + 768);
    char* pp = (char*)T.pre.p;
    B.pre.rec = (float4*)pp;
    B.pre.dir = nullptr;   // no adjoint: the offset directions are not needed
    B.pre.z = (float*)(pp + (size_t)N * 80);
    B.pre.rx = (uint32_t*)(pp + (size_t)N * 84);
    B.pre.ry = (uint32_t*)(pp + (size_t)N * 88);
    uint32_t* tb = (uint32_t*)T.tiles.p;
    B.tile_count = tb;
    B.tile_fill = tb + M;
    B.tile_start = tb + 2 * M;
    B.chunk_start = tb + 3 * M + 1;
    B.cmask = nullptr;
    B.status = (DevStatus*)T.status.p;
    B.Tfinal = nullptr;
    B.last = nullptr;
    // constant tables: keyframe pointers and the single pair index
    {
        KfPtrs kp{geo->depth, geo->offset, geo->radius, geo->opacity, nullptr, geo->sigma};
        int32_t zero = 0;
        HIPCHK(c, hipMemcpyAsync((char*)T.params.p + 512, &kp, sizeof(kp), hipMemcpyHostToDevice, s));
        HIPCHK(c, hipMemcpyAsync((char*)T.params.p + 768, &zero, 4, hipMemcpyHostToDevice, s));
    }
    PairConst* pair_dev = (PairConst*)T.params.p;
    if (!same_shape || !T.sized) {
        // sizing pass at the starting pose (one host wait)
        B.keys = nullptr;
        B.capacity = 0;
        launch_track_pair(pose, geo->T_cw, geo->cam, *vcam, pair_dev, s);
        launch_zero_u32((uint32_t*)B.status, sizeof(DevStatus) / 4, s);
        launch_zero_u32(B.tile_count, (int64_t)M, s);
        launch_preprocess(G, B, s);
        launch_scan(G, B, false, s);
        HIPCHK(c, hipMemcpyAsync(T.status_h, B.status, sizeof(DevStatus), hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipStreamSynchronize(s));
        const size_t cap = std::min<size_t>((size_t)T.status_h->total * 3 / 2 + 65536, 0xffffffffu);
        if (cap > T.capacity) {
            HIPCHK(c, ensure(T.keys, cap * 8, s));
            T.capacity = (uint32_t)cap;
        }
        T.sized = true;
    }
    B.keys = (uint64_t*)T.keys.p;
    B.capacity = T.capacity;
    const void* key[8] = {geo->depth, geo->offset, geo->radius, geo->opacity, geo->sigma, obs_depth, pose, tr};
    // Each iteration's scan clears the counts it read and rewrites total,
    // overflow and queue; a non-finite flag, once raised, stays for the call.
    auto enqueue = [&](hipStream_t q) -> bool {
        launch_zero2_u32((uint32_t*)B.status, sizeof(DevStatus) / 4, B.tile_count, (int64_t)M, q);
        launch_track_pair(pose, geo->T_cw, geo->cam, *vcam, pair_dev, q);
        for (int it = 0; it < iters; ++it) {
            launch_preprocess(G, B, q);
            launch_scan(G, B, true, q);
            launch_scatter(G, B, q);
            launch_sort(G, B, q);
            if (!launch_track(G, B, obs_depth, (float*)T.part.p, q)) return false;
            // the solve also forms the next iteration's relative pose
            launch_track_solve((const float*)T.part.p, track_parts(G), pose, tr, it, B.status, geo->T_cw,
                               geo->cam, *vcam, it + 1 < iters ? pair_dev : nullptr, q);
        }
        return true;
    };
    if (flags & 1u) {
        bool reuse = T.exec && T.key_iters == iters && T.key_tw == TW && T.key_th == TH &&
                     std::memcmp(T.key, key, sizeof(key)) == 0 && std::memcmp(&T.kc, &geo->cam, sizeof(sgad_cam)) == 0 &&
                     std::memcmp(&T.vc, vcam, sizeof(sgad_cam)) == 0 &&
                     std::memcmp(&T.kpose, &geo->T_cw, sizeof(sgad_pose)) == 0 && T.B.capacity == B.capacity;
        if (!reuse) {
            if (T.exec) (void)hipGraphExecDestroy(T.exec);
            if (T.graph) (void)hipGraphDestroy(T.graph);
            T.exec = nullptr;
            T.graph = nullptr;
            // the capture stream must see the tables written above
            HIPCHK(c, hipStreamSynchronize(s));
            HIPCHK(c, hipStreamBeginCapture(T.cap, hipStreamCaptureModeThreadLocal));
            const bool ok = enqueue(T.cap);
            hipGraph_t g = nullptr;
            HIPCHK(c, hipStreamEndCapture(T.cap, &g));
            if (!ok) {
                (void)hipGraphDestroy(g);
                return fail(c, SGAD_EINVAL, "unsupported tile shape");
            }
            T.graph = g;
            HIPCHK(c, hipGraphInstantiate(&T.exec, g, nullptr, nullptr, 0));
            std::memcpy(T.key, key, sizeof(key));
            T.key_iters = iters;
            T.key_tw = TW;
            T.key_th = TH;
            T.kc = geo->cam;
            T.vc = *vcam;
            T.kpose = geo->T_cw;
        }
        TimeScope ts(c, "track_graph", s);
        HIPCHK(c, hipGraphLaunch(T.exec, s));
    } else {
        TimeScope ts(c, "track_loop", s);
        if (!enqueue(s)) return fail(c, SGAD_EINVAL, "unsupported tile shape");
    }
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipMemcpyAsync(T.status_h, B.status, sizeof(DevStatus), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipEventRecord(T.ev_status, s));
    T.status_pending = true;
    return SGAD_OK;
}

sgad_status sgad_autotune(sgad_ctx* c, int n_kf, const sgad_keyframe* kf, int n_views, const sgad_cam* vcam,
                          const sgad_pose* vpose, int n_jobs, const sgad_job* jobs, int reps, int* best_tw,
                          int* best_th, float* best_ms, void* stream) {
    if (!c) return SGAD_EINVAL;
    if (c->capture.on) return fail(c, SGAD_EINVAL, "not allowed while capturing a graph");
    if (reps < 1 || reps > 1000) return fail(c, SGAD_ERANGE, "reps must be in [1, 1000]");
    if (n_kf < 1 || n_kf > kMaxKf || !kf || n_views < 1 || !vcam || n_jobs < 1 || !jobs)
        return fail(c, SGAD_EINVAL, "bad workload");
    hipStream_t s = (hipStream_t)stream;
    HIPCHK(c, hipSetDevice(c->device));
    const int64_t N = (int64_t)kf[0].cam.H * kf[0].cam.W;
    const int64_t P = (int64_t)vcam[0].H * vcam[0].W;
    int n_pairs = 0;
    for (int j = 0; j < n_jobs; ++j)
        n_pairs += __builtin_popcountll((uint64_t)jobs[j].kf_mask_lo | ((uint64_t)jobs[j].kf_mask_hi << 32));
    // scratch: outputs, upstream grads (a constant), keyframe grads, pose
    DevBuf buf;
    const size_t fo = (size_t)n_jobs * P * 5, fu = (size_t)n_jobs * P * 5, fg = (size_t)n_kf * N * 6;
    HIPCHK(c, ensure(buf, (fo + fu + fg + (size_t)n_jobs * 6) * 4, s));
    float* base = (float*)buf.p;
    float *o_rgb = base, *o_dep = o_rgb + n_jobs * P * 3, *o_alp = o_dep + n_jobs * P;
    float *u_rgb = base + fo, *u_dep = u_rgb + n_jobs * P * 3, *u_alp = u_dep + n_jobs * P;
    float* kg = base + fo + fu;
    float* dpose = kg + fg;
    launch_fill_f32(u_rgb, (int64_t)fu, 1e-6f, s);
    std::vector<sgad_kf_grads> grads(n_kf);
    for (int f = 0; f < n_kf; ++f) {
        float* g = kg + (size_t)f * N * 6;
        grads[f] = sgad_kf_grads{g, g + 3 * N, g + 4 * N, g + 5 * N};
    }
    struct Cand {
        int tw, th, scf, scb;
    };
    const Cand cands[] = {{16, 16, 0, 0}, {16, 8, 0, 0}, {32, 8, 0, 0}, {8, 8, 4, 16}, {8, 8, 1, 16},
                          {8, 8, 2, 16},  {8, 8, 4, 32}, {8, 8, 1, 32}, {8, 8, 2, 32}};
    hipEvent_t e0, e1;
    HIPCHK(c, hipEventCreate(&e0));
    HIPCHK(c, hipEventCreate(&e1));
    float best = 1e30f;
    Cand bc = cands[3];
    sgad_status rs = SGAD_OK;
    for (const Cand& cd : cands) {
        c->force = true;
        c->ftw = cd.tw;
        c->fth = cd.th;
        c->fscf = cd.scf ? cd.scf : 4;
        c->fscb = cd.scb ? cd.scb : 16;
        float ms_tot = 0.f;
        for (int r = 0; r <= reps && rs == SGAD_OK; ++r) {  // r == 0 is a warm-up
            sgad_saved* sv = nullptr;
            if (r == 1) (void)hipEventRecord(e0, s);
            rs = sgad_render_fwd(c, n_kf, kf, n_views, vcam, vpose, n_jobs, jobs, o_rgb, o_dep, o_alp, nullptr,
                                 &sv, stream);
            if (rs != SGAD_OK) break;
            rs = sgad_render_bwd(c, sv, u_rgb, u_dep, u_alp, grads.data(), dpose, 0xffffffffu, 0xffffffffu, stream);
            (void)sgad_saved_release(c, sv);
        }
        if (rs != SGAD_OK) break;
        (void)hipEventRecord(e1, s);
        (void)hipEventSynchronize(e1);
        (void)hipEventElapsedTime(&ms_tot, e0, e1);
        const float ms = ms_tot / reps;
        if (ms < best) {
            best = ms;
            bc = cd;
        }
    }
    c->force = false;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(s);
    if (buf.p) (void)hipFree(buf.p);
    if (rs != SGAD_OK) return rs;
    {
        sgad_ctx::TuneEntry te{};
        const size_t key[6] = {(size_t)vcam[0].H, (size_t)vcam[0].W, (size_t)N, (size_t)n_pairs, (size_t)n_jobs,
                               (size_t)n_kf};
        std::memcpy(te.key, key, sizeof(key));
        te.tw = bc.tw;
        te.th = bc.th;
        te.scf = bc.scf ? bc.scf : 4;
        te.scb = bc.scb ? bc.scb : 16;
        te.ms = best;
        bool found = false;
        for (auto& e : c->tune)
            if (std::memcmp(e.key, key, sizeof(key)) == 0) {
                e = te;
                found = true;
            }
        if (!found) c->tune.push_back(te);
    }
    if (best_tw) *best_tw = bc.tw;
    if (best_th) *best_th = bc.th;
    if (best_ms) *best_ms = best;
    return SGAD_OK;
}

// ---------------------------------------------------------------- conv net
static bool conv_dims_ok(int H, int W) { return H > 0 && W > 0 && H < 65536 && W < 65536; }
// the conv kernels move a pixel's channels (and a weight row) in 16-byte loads
static bool conv_aligned(const void* p) { return ((uintptr_t)p & 15) == 0; }

sgad_status sgad_conv_weights(sgad_ctx* c, int cin, int cout, const float* w, uint16_t* w_bf16, uint16_t* wt_bf16,
                              void* stream) {
    if (!c) return SGAD_EINVAL;
    if (cin < 1 || cout < 1 || cin > 32 || cout > 32 || !w || !w_bf16) return fail(c, SGAD_EINVAL, "bad weights");
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t s = pick_stream(c, stream);
    TimeScope ts(c, "conv_weights", s);
    launch_conv_weights(cin, cout, w, w_bf16, wt_bf16, s);
    HIPCHK(c, hipGetLastError());
    return SGAD_OK;
}

sgad_status sgad_conv3x3_fwd(sgad_ctx* c, int H, int W, int cin, int cout, int mode, const uint16_t* x,
                             const uint16_t* w_bf16, const float* bias, void* y, void* stream) {
    if (!c) return SGAD_EINVAL;
    if (!conv_dims_ok(H, W) || !x || !w_bf16 || !bias || !y) return fail(c, SGAD_EINVAL, "bad conv arguments");
    if (mode != SGAD_CONV_RELU_BF16 && mode != SGAD_CONV_LINEAR_F32) return fail(c, SGAD_EINVAL, "bad conv mode");
    if (!conv_aligned(x) || !conv_aligned(w_bf16) || !conv_aligned(y))
        return fail(c, SGAD_EINVAL, "conv pointers must be 16-byte aligned");
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t s = pick_stream(c, stream);
    TimeScope ts(c, "conv_fwd", s);
    if (!launch_conv_fwd(H, W, cin, cout, mode, x, w_bf16, bias, nullptr, y, s))
        return fail(c, SGAD_EINVAL, "unsupported (cin, cout, mode)");
    HIPCHK(c, hipGetLastError());
    return SGAD_OK;
}

sgad_status sgad_conv3x3_dgrad(sgad_ctx* c, int H, int W, int cin, int cout, const uint16_t* dy,
                               const uint16_t* wt_bf16, const uint16_t* mask, uint16_t* dx, void* stream) {
    if (!c) return SGAD_EINVAL;
    if (!conv_dims_ok(H, W) || !dy || !wt_bf16 || !mask || !dx) return fail(c, SGAD_EINVAL, "bad dgrad arguments");
    if (!conv_aligned(dy) || !conv_aligned(wt_bf16) || !conv_aligned(mask) || !conv_aligned(dx))
        return fail(c, SGAD_EINVAL, "conv pointers must be 16-byte aligned");
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t s = pick_stream(c, stream);
    TimeScope ts(c, "conv_dgrad", s);
    // the input gradient is a convolution from cout to cin channels
    if (!launch_conv_fwd(H, W, cout, cin, 2, dy, wt_bf16, nullptr, mask, dx, s))
        return fail(c, SGAD_EINVAL, "unsupported (cin, cout)");
    HIPCHK(c, hipGetLastError());
    return SGAD_OK;
}

sgad_status sgad_conv3x3_wgrad(sgad_ctx* c, int H, int W, int cin, int cout, const uint16_t* x, const uint16_t* dy,
                               float* dw, float* db, void* stream) {
    if (!c) return SGAD_EINVAL;
    if (!conv_dims_ok(H, W) || !x || !dy || !dw || !db) return fail(c, SGAD_EINVAL, "bad wgrad arguments");
    if (!conv_aligned(x) || !conv_aligned(dy)) return fail(c, SGAD_EINVAL, "conv pointers must be 16-byte aligned");
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t s = pick_stream(c, stream);
    TimeScope ts(c, "conv_wgrad", s);
    if (!((cin == 4 && cout == 32) || (cin == 32 && cout == 32) || (cin == 32 && cout == 1)))
        return fail(c, SGAD_EINVAL, "unsupported (cin, cout)");
    HIPCHK(c, ensure_c(c, c->conv_part, conv_wgrad_part_bytes(H, W, cin, cout), s));
    launch_conv_wgrad(H, W, cin, cout, x, dy, (float*)c->conv_part.p, dw, db, s);
    HIPCHK(c, hipGetLastError());
    return SGAD_OK;
}

sgad_status sgad_conv3x3_wgrad_noalloc(sgad_ctx* c, int H, int W, int cin, int cout, const uint16_t* x,
                                       const uint16_t* dy, float* dw, float* db, void* stream) {
    if (!c) return SGAD_EINVAL;
    if (!conv_dims_ok(H, W) || !x || !dy || !dw || !db) return fail(c, SGAD_EINVAL, "bad wgrad arguments");
    if (!conv_aligned(x) || !conv_aligned(dy)) return fail(c, SGAD_EINVAL, "conv pointers must be 16-byte aligned");
    if (!((cin == 4 && cout == 32) || (cin == 32 && cout == 32) || (cin == 32 && cout == 1)))
        return fail(c, SGAD_EINVAL, "unsupported (cin, cout)");
    const size_t need = conv_wgrad_part_bytes(H, W, cin, cout);
    if (need > conv_scratch_bytes()) {
        char msg[160];
        std::snprintf(msg, sizeof msg, "wgrad needs %zu bytes of partial sums, the static scratch holds %zu", need,
                      conv_scratch_bytes());
        return fail(c, SGAD_ERANGE, msg);
    }
    if (!c->conv_scratch) return fail(c, SGAD_EHIP, "static scratch address not set up");
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t s = pick_stream(c, stream);
    launch_conv_wgrad(H, W, cin, cout, x, dy, c->conv_scratch, dw, db, s);
    HIPCHK(c, hipGetLastError());
    return SGAD_OK;
}

sgad_status sgad_net_input(sgad_ctx* c, int H, int W, const float* rgb, const float* depth, uint16_t* x0,
                           void* stream) {
    if (!c) return SGAD_EINVAL;
    if (!conv_dims_ok(H, W) || !rgb || !depth || !x0) return fail(c, SGAD_EINVAL, "bad input arguments");
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t s = pick_stream(c, stream);
    launch_net_input(H, W, rgb, depth, x0, s);
    HIPCHK(c, hipGetLastError());
    return SGAD_OK;
}

sgad_status sgad_offset_l1(sgad_ctx* c, int n, const float* pred, const float* target, uint16_t* grad,
                           double* loss, void* stream) {
    if (!c) return SGAD_EINVAL;
    if (n < 1 || !pred || !target || !grad || !loss) return fail(c, SGAD_EINVAL, "bad loss arguments");
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t s = pick_stream(c, stream);
    launch_zero_u32((uint32_t*)loss, 2, s);
    launch_offset_l1(n, pred, target, grad, loss, s);
    HIPCHK(c, hipGetLastError());
    return SGAD_OK;
}

}  // extern "C"
