"""ctypes binding of libsgad.so (the C ABI in include/sgad.h).

Argument marshalling only: every step of the splat path runs in the HIP
library.  Device memory and streams come from PyTorch; tensors must be
contiguous float32 (int32 for counts) on the context's device.  If the
library is missing this module raises at load time: there is no CPU path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsgad.so")

OK, EINVAL, ERANGE, EHIP, ENOMEM, EDATA = range(6)
STATUS_NAMES = {0: "SGAD_OK", 1: "SGAD_EINVAL", 2: "SGAD_ERANGE", 3: "SGAD_EHIP", 4: "SGAD_ENOMEM",
                5: "SGAD_EDATA"}


class SgadError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class Cam(C.Structure):
    _fields_ = [("H", C.c_int32), ("W", C.c_int32), ("fx", C.c_float), ("fy", C.c_float),
                ("cx", C.c_float), ("cy", C.c_float)]


class Pose(C.Structure):
    _fields_ = [("R", C.c_float * 9), ("t", C.c_float * 3)]


class Keyframe(C.Structure):
    _fields_ = [("cam", Cam), ("T_cw", Pose), ("depth", C.c_void_p), ("offset", C.c_void_p),
                ("radius", C.c_void_p), ("opacity", C.c_void_p), ("rgb", C.c_void_p),
                ("sigma", C.c_void_p)]


class Job(C.Structure):
    _fields_ = [("view", C.c_int32), ("kf_mask_lo", C.c_uint32), ("kf_mask_hi", C.c_uint32)]


class AdamGroup(C.Structure):
    _fields_ = [("param", C.c_void_p), ("grad", C.c_void_p), ("m", C.c_void_p), ("v", C.c_void_p),
                ("n", C.c_int64), ("lr", C.c_float), ("lo", C.c_float), ("hi", C.c_float),
                ("space", C.c_int32)]


SPACE_LINEAR, SPACE_LOG, SPACE_LOGIT = 0, 1, 2


class KfGrads(C.Structure):
    _fields_ = [("d_rgb", C.c_void_p), ("d_opacity", C.c_void_p), ("d_radius", C.c_void_p),
                ("d_offset", C.c_void_p)]


class GMapC(C.Structure):
    _fields_ = [("data", C.c_void_p), ("keys", C.c_void_p), ("vals", C.c_void_p), ("count", C.c_void_p),
                ("capacity", C.c_int32), ("slots", C.c_int32), ("voxel", C.c_double)]


_P = C.c_void_p
_SIGS = {
    "sgad_create": (C.c_int, [C.c_int, C.POINTER(_P)]),
    "sgad_destroy": (None, [_P]),
    "sgad_last_error": (C.c_char_p, [_P]),
    "sgad_sync": (C.c_int, [_P]),
    "sgad_set_tile": (C.c_int, [_P, C.c_int, C.c_int]),
    "sgad_get_tile": (C.c_int, [_P, C.POINTER(C.c_int), C.POINTER(C.c_int)]),
    "sgad_get_tile_variant": (C.c_int, [_P, C.POINTER(C.c_int), C.POINTER(C.c_int)]),
    "sgad_set_tile_variant": (C.c_int, [_P, C.c_int, C.c_int]),
    "sgad_render_fwd": (C.c_int, [_P, C.c_int, C.POINTER(Keyframe), C.c_int, C.POINTER(Cam),
                                  C.POINTER(Pose), C.c_int, C.POINTER(Job), _P, _P, _P, _P,
                                  C.POINTER(_P), _P]),
    "sgad_render_bwd": (C.c_int, [_P, _P, _P, _P, _P, C.POINTER(KfGrads), _P, C.c_uint32, C.c_uint32, _P]),
    "sgad_workspace_bytes": (C.c_int, [_P, C.c_int, C.POINTER(Keyframe), C.c_int, C.POINTER(Cam), C.c_int,
                                       C.POINTER(Job), C.c_uint64, C.POINTER(C.c_size_t)]),
    "sgad_saved_release": (C.c_int, [_P, _P]),
    "sgad_track_gn": (C.c_int, [_P, C.POINTER(Keyframe), C.POINTER(Cam), _P, _P, C.c_int, _P, C.c_uint32,
                                _P]),
    "sgad_timing_enable": (C.c_int, [_P, C.c_int]),
    "sgad_timing_only": (C.c_int, [_P, C.c_char_p]),
    "sgad_l1_loss": (C.c_int, [_P, C.c_int, C.c_int, C.c_int, _P, _P, _P, _P, C.c_float, C.c_float, _P, _P,
                               _P, _P]),
    "sgad_eq1_loss": (C.c_int, [_P, C.c_int, C.c_int, C.c_int, _P, _P, _P, _P, C.c_float, C.c_float, C.c_float,
                                _P, _P, _P, _P]),
    "sgad_gicp_set_size": (C.c_int32, [C.c_int, C.c_int, C.c_int]),
    "sgad_gicp_prepare": (C.c_int, [_P, _P, C.c_void_p, C.c_int, C.c_int, _P, _P]),
    "sgad_gicp_linearise": (C.c_int, [_P, _P, C.c_int, _P, C.c_int, C.c_void_p, C.c_int, C.c_int, _P, _P, _P,
                                      _P]),
    "sgad_gicp_track": (C.c_int, [_P, _P, C.c_int, _P, C.c_int, C.c_void_p, C.c_int, C.c_int, _P, C.c_int, _P,
                                  _P]),
    "sgad_gmap_reset": (C.c_int, [_P, C.POINTER(GMapC), _P]),
    "sgad_gmap_insert": (C.c_int, [_P, C.POINTER(GMapC), _P, C.c_int, _P, _P]),
    "sgad_gicp_linearise_map": (C.c_int, [_P, _P, C.c_int, C.POINTER(GMapC), C.c_int, _P, _P, _P, _P]),
    "sgad_gicp_track_map": (C.c_int, [_P, _P, C.c_int, C.POINTER(GMapC), C.c_int, _P, C.c_int, _P, _P]),
    "sgad_fill_depth": (C.c_int, [_P, C.c_int, _P, _P, _P, C.c_float, _P, _P]),
    "sgad_adam_step": (C.c_int, [_P, C.c_int, C.c_void_p, C.c_int, C.c_float, C.c_float, C.c_float,
                                 C.c_int, _P]),
    "sgad_timing_report": (C.c_int, [_P, C.c_char_p, C.c_size_t]),
    "sgad_conv_weights": (C.c_int, [_P, C.c_int, C.c_int, _P, _P, _P, _P]),
    "sgad_conv3x3_fwd": (C.c_int, [_P, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, _P, _P, _P, _P, _P]),
    "sgad_conv3x3_dgrad": (C.c_int, [_P, C.c_int, C.c_int, C.c_int, C.c_int, _P, _P, _P, _P, _P]),
    "sgad_conv3x3_wgrad": (C.c_int, [_P, C.c_int, C.c_int, C.c_int, C.c_int, _P, _P, _P, _P, _P]),
    "sgad_conv3x3_wgrad_noalloc": (C.c_int, [_P, C.c_int, C.c_int, C.c_int, C.c_int, _P, _P, _P, _P, _P]),
    "sgad_net_input": (C.c_int, [_P, C.c_int, C.c_int, _P, _P, _P, _P]),
    "sgad_offset_l1": (C.c_int, [_P, C.c_int, _P, _P, _P, _P, _P]),
    "sgad_autotune": (C.c_int, [_P, C.c_int, C.POINTER(Keyframe), C.c_int, C.POINTER(Cam), C.POINTER(Pose),
                                C.c_int, C.POINTER(Job), C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int),
                                C.POINTER(C.c_float), _P]),
    "sgad_saved_instances": (C.c_int, [_P, _P, C.c_int, _P, _P, C.c_size_t, C.POINTER(C.c_size_t),
                                       C.POINTER(C.c_int)]),
    "sgad_graph_begin": (C.c_int, [_P, _P]),
    "sgad_graph_end": (C.c_int, [_P, C.POINTER(_P)]),
    "sgad_graph_launch": (C.c_int, [_P, _P, _P]),
    "sgad_graph_destroy": (C.c_int, [_P, _P]),
}

_lib = None


def load(path: str = LIB_PATH):
    """Load libsgad.so and declare the signatures (raises if it is absent)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} not built: run `python -m paper_2603_21055_amd.build`")
    lib = C.CDLL(path)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def declared_symbols(header=None):
    """Names of the functions declared in include/sgad.h."""
    import re
    header = header or os.path.join(os.path.dirname(HERE), "include", "sgad.h")
    txt = open(header).read()
    return sorted(set(re.findall(r"^\s*(?:[\w\*]+\s+)+\**(sgad_\w+)\s*\(", txt, re.M)))


# ----------------------------------------------------------------------------
# marshalling helpers
# ----------------------------------------------------------------------------
def _ptr(t):
    if t is None:
        return None
    return C.c_void_p(t.data_ptr())


class GlobalMap:
    """Device storage of the global set T: data float64 [12, capacity], the
    voxel hash (keys int64, vals int32, 2 x capacity rounded up to a power of
    two) and the count."""

    def __init__(self, device, capacity, voxel=0.02):
        import torch
        capacity = int(capacity)
        slots = 1 << max(1, (2 * capacity - 1).bit_length())
        self.data = torch.zeros((12, capacity), dtype=torch.float64, device=device)
        self.keys = torch.empty(slots, dtype=torch.int64, device=device)
        self.vals = torch.empty(slots, dtype=torch.int32, device=device)
        self.count_t = torch.zeros(1, dtype=torch.int32, device=device)
        self.c = GMapC(self.data.data_ptr(), self.keys.data_ptr(), self.vals.data_ptr(), self.count_t.data_ptr(),
                       capacity, slots, float(voxel))

    def count(self):
        return int(self.count_t.item())

    def view(self):
        """The Gaussians in use, float64 [12, count]."""
        return self.data[:, :self.count()]


def _cam(cam) -> Cam:
    return Cam(int(cam["H"]), int(cam["W"]), float(cam["fx"]), float(cam["fy"]), float(cam["cx"]),
               float(cam["cy"]))


def _pose(R, t) -> Pose:
    p = Pose()
    Rf = np.asarray(R, np.float32).reshape(9)
    tf = np.asarray(t, np.float32).reshape(3)
    for i in range(9):
        p.R[i] = float(Rf[i])
    for i in range(3):
        p.t[i] = float(tf[i])
    return p


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _check_tensor(t, name, dev, dtype=None):
    import torch
    dtype = dtype or torch.float32
    if t is None:
        return
    if not t.is_cuda or t.device != dev:
        raise ValueError(f"{name} must be on {dev}")
    if t.dtype != dtype or not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous {dtype}")


class Context:
    """An sgad_ctx on one device.  Keyframes are dicts with ``cam`` (dict),
    ``R``, ``t`` (numpy, world->camera) and device tensors ``depth``,
    ``offset``, ``radius``, ``opacity``, ``rgb`` (or ``sigma``)."""

    def __init__(self, device: int = 0):
        import torch
        self.lib = load()
        self.device = torch.device("cuda", device)
        h = C.c_void_p()
        self._check(self.lib.sgad_create(device, C.byref(h)), ctx=False)
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            for g in list(getattr(self, "_graphs", [])):
                self.lib.sgad_graph_destroy(self.h, g)
            self.lib.sgad_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st, ctx=True):
        if st != OK:
            msg = self.lib.sgad_last_error(self.h).decode() if ctx else "sgad_create failed"
            raise SgadError(st, msg)

    def sync(self):
        """Wait for the context's work and raise a latched device condition."""
        self._check(self.lib.sgad_sync(self.h))

    def set_tile(self, w: int, h: int):
        self._check(self.lib.sgad_set_tile(self.h, w, h))

    def get_tile(self):
        w, h = C.c_int(), C.c_int()
        self._check(self.lib.sgad_get_tile(self.h, C.byref(w), C.byref(h)))
        return w.value, h.value

    def set_tile_variant(self, fwd_chunks: int, bwd_sub: int):
        """8x8 kernel variant used when the tile is set to (8, 8) by hand."""
        self._check(self.lib.sgad_set_tile_variant(self.h, int(fwd_chunks), int(bwd_sub)))

    def get_tile_variant(self):
        """(forward chunks per super-chunk, adjoint sub-chunk) of the last 8x8 forward."""
        f, b = C.c_int(), C.c_int()
        self._check(self.lib.sgad_get_tile_variant(self.h, C.byref(f), C.byref(b)))
        return f.value, b.value

    def timing(self, enable: bool):
        """Enable/disable per-kernel event timing (resets the accumulators)."""
        self._check(self.lib.sgad_timing_enable(self.h, 1 if enable else 0))

    def timing_only(self, name=None):
        """Time only the kernel `name` (None: every kernel)."""
        self._check(self.lib.sgad_timing_only(self.h, name.encode() if name else None))

    def timing_report(self) -> dict:
        """{kernel name: (launches, total ms)} since timing was enabled."""
        buf = C.create_string_buffer(1 << 16)
        self._check(self.lib.sgad_timing_report(self.h, buf, len(buf)))
        out = {}
        for line in buf.value.decode().splitlines():
            name, n, ms = line.split()
            out[name] = (int(n), float(ms))
        return out

    # -------------------------------------------------------------- render
    def _kf_array(self, kfs):
        arr = (Keyframe * len(kfs))()
        for i, kf in enumerate(kfs):
            for k in ("depth", "offset", "radius", "opacity", "rgb", "sigma"):
                _check_tensor(kf.get(k), f"kf[{i}].{k}", self.device)
            arr[i] = Keyframe(_cam(kf["cam"]), _pose(kf["R"], kf["t"]), _ptr(kf["depth"]),
                              _ptr(kf["offset"]), _ptr(kf["radius"]), _ptr(kf["opacity"]),
                              _ptr(kf.get("rgb")), _ptr(kf.get("sigma")))
        return arr

    @staticmethod
    def _views_jobs(views, jobs):
        cams = (Cam * len(views))(*[_cam(v["cam"]) for v in views])
        poses = (Pose * len(views))(*[_pose(v["R"], v["t"]) for v in views])
        ja = (Job * len(jobs))()
        for i, (v, ids) in enumerate(jobs):
            m = 0
            for f in ids:
                m |= 1 << int(f)
            ja[i] = Job(int(v), m & 0xFFFFFFFF, (m >> 32) & 0xFFFFFFFF)
        return cams, poses, ja

    def autotune(self, kfs, views, jobs, reps=5, stream=None):
        """Time every tile configuration on this workload; returns
        ((tile_w, tile_h), ms per forward + adjoint) of the fastest."""
        kfa = self._kf_array(kfs)
        cams, poses, ja = self._views_jobs(views, jobs)
        tw, th, ms = C.c_int(), C.c_int(), C.c_float()
        st = self.lib.sgad_autotune(self.h, len(kfs), kfa, len(views), cams, poses, len(jobs), ja, int(reps),
                                    C.byref(tw), C.byref(th), C.byref(ms), _stream(stream))
        self._check(st)
        return (tw.value, th.value), ms.value

    def render_fwd(self, kfs, views, jobs, out_rgb, out_depth, out_alpha, out_count=None, stream=None):
        """Enqueue the forward; returns the saved handle (a c_void_p)."""
        kfa = self._kf_array(kfs)
        cams, poses, ja = self._views_jobs(views, jobs)
        for name, t in (("out_rgb", out_rgb), ("out_depth", out_depth), ("out_alpha", out_alpha)):
            _check_tensor(t, name, self.device)
        import torch
        _check_tensor(out_count, "out_count", self.device, torch.int32)
        saved = C.c_void_p()
        st = self.lib.sgad_render_fwd(self.h, len(kfs), kfa, len(views), cams, poses, len(jobs), ja,
                                      _ptr(out_rgb), _ptr(out_depth), _ptr(out_alpha), _ptr(out_count),
                                      C.byref(saved), _stream(stream))
        self._check(st)
        return saved

    def workspace_bytes(self, kfs, views, jobs, instances=0):
        """Device bytes a forward + adjoint of this workload holds (instance
        list sized for `instances` keys; 0: the first call's size)."""
        kfa = self._kf_array(kfs)
        cams, _, ja = self._views_jobs(views, jobs)
        out = C.c_size_t()
        self._check(self.lib.sgad_workspace_bytes(self.h, len(kfs), kfa, len(views), cams, len(jobs), ja,
                                                  int(instances), C.byref(out)))
        return out.value

    def render_bwd(self, saved, g_rgb, g_depth, g_alpha, grads, d_pose, learnable, stream=None):
        """grads: list (len n_kf) of dicts with d_rgb/d_opacity/d_radius/d_offset
        tensors or None; learnable: iterable of keyframe indices."""
        for name, t in (("g_rgb", g_rgb), ("g_depth", g_depth), ("g_alpha", g_alpha), ("d_pose", d_pose)):
            _check_tensor(t, name, self.device)
        ga = (KfGrads * len(grads))()
        for i, g in enumerate(grads):
            if g is None:
                ga[i] = KfGrads(None, None, None, None)
            else:
                for k in ("d_rgb", "d_opacity", "d_radius", "d_offset"):
                    _check_tensor(g[k], f"grads[{i}].{k}", self.device)
                ga[i] = KfGrads(_ptr(g["d_rgb"]), _ptr(g["d_opacity"]), _ptr(g["d_radius"]),
                                _ptr(g["d_offset"]))
        m = 0
        for f in learnable:
            m |= 1 << int(f)
        st = self.lib.sgad_render_bwd(self.h, saved, _ptr(g_rgb), _ptr(g_depth), _ptr(g_alpha), ga,
                                      _ptr(d_pose), m & 0xFFFFFFFF, (m >> 32) & 0xFFFFFFFF,
                                      _stream(stream))
        self._check(st)

    def l1_loss(self, rgb, depth, t_rgb, t_depth, g_rgb, g_depth, loss, w_rgb=0.8, w_depth=1.0,
                stream=None):
        """L1 terms of Eq. 1: writes g_rgb, g_depth and loss [n_jobs] (float64)."""
        import torch
        for name, t in (("rgb", rgb), ("depth", depth), ("t_rgb", t_rgb), ("t_depth", t_depth),
                        ("g_rgb", g_rgb), ("g_depth", g_depth)):
            _check_tensor(t, name, self.device)
        _check_tensor(loss, "loss", self.device, torch.float64)
        nj, Hh, W = depth.shape
        st = self.lib.sgad_l1_loss(self.h, nj, Hh, W, _ptr(rgb), _ptr(depth), _ptr(t_rgb), _ptr(t_depth),
                                   float(w_rgb), float(w_depth), _ptr(g_rgb), _ptr(g_depth), _ptr(loss),
                                   _stream(stream))
        self._check(st)

    def eq1_loss(self, rgb, depth, t_rgb, t_depth, g_rgb, g_depth, loss, w_rgb=0.8, w_ssim=0.2, w_depth=1.0,
                 stream=None):
        """All of Eq. 1 (L1 colour, SSIM, masked L1 depth): writes g_rgb, g_depth
        and loss [n_jobs] (float64)."""
        import torch
        for name, t in (("rgb", rgb), ("depth", depth), ("t_rgb", t_rgb), ("t_depth", t_depth),
                        ("g_rgb", g_rgb), ("g_depth", g_depth)):
            _check_tensor(t, name, self.device)
        _check_tensor(loss, "loss", self.device, torch.float64)
        nj, Hh, W = depth.shape
        st = self.lib.sgad_eq1_loss(self.h, nj, Hh, W, _ptr(rgb), _ptr(depth), _ptr(t_rgb), _ptr(t_depth),
                                    float(w_rgb), float(w_ssim), float(w_depth), _ptr(g_rgb), _ptr(g_depth),
                                    _ptr(loss), _stream(stream))
        self._check(st)

    def adam_step(self, groups, step, beta1=0.9, beta2=0.999, eps=1e-8, zero_grad=True, stream=None):
        """groups: list of (param, grad, m, v, lr, lo, hi[, space]) device tensors
        / floats; space is SPACE_LINEAR (default), SPACE_LOG or SPACE_LOGIT."""
        arr = (AdamGroup * len(groups))()
        for i, grp in enumerate(groups):
            p, g, m, v, lr, lo, hi = grp[:7]
            space = grp[7] if len(grp) > 7 else SPACE_LINEAR
            for name, t in (("param", p), ("grad", g), ("m", m), ("v", v)):
                _check_tensor(t, name, self.device)
            arr[i] = AdamGroup(_ptr(p), _ptr(g), _ptr(m), _ptr(v), p.numel(), float(lr), float(lo), float(hi),
                               int(space))
        st = self.lib.sgad_adam_step(self.h, len(groups), C.cast(arr, C.c_void_p), int(step), float(beta1),
                                     float(beta2), float(eps), 1 if zero_grad else 0, _stream(stream))
        self._check(st)

    def track_gn(self, geo, vcam, obs_depth, pose, iters=30, trace=None, graph=True, stream=None):
        """Gauss-Newton tracking.  pose: device float64 [12] (R row-major, t),
        updated in place; trace: device float64 [iters, 40] or None."""
        import torch
        kfa = self._kf_array([geo])
        cam = _cam(vcam)
        _check_tensor(obs_depth, "obs_depth", self.device)
        _check_tensor(pose, "pose", self.device, torch.float64)
        _check_tensor(trace, "trace", self.device, torch.float64)
        st = self.lib.sgad_track_gn(self.h, kfa, C.byref(cam), _ptr(obs_depth), _ptr(pose), int(iters),
                                    _ptr(trace), 1 if graph else 0, _stream(stream))
        self._check(st)

    # ------------------------------------------------------------------ GICP
    def gicp_set_size(self, H, W, ratio):
        """Points n of a frame's stride-ratio grid (a set is float64 [12, n])."""
        return int(self.lib.sgad_gicp_set_size(int(H), int(W), int(ratio)))

    def gicp_prepare(self, depth, cam, ratio, k, set_, stream=None):
        """Build the GICP set [12, n] (float64, written) of a depth map [H, W]."""
        import torch
        _check_tensor(depth, "depth", self.device)
        _check_tensor(set_, "set", self.device, torch.float64)
        c = _cam(cam)
        self._check(self.lib.sgad_gicp_prepare(self.h, _ptr(depth), C.byref(c), int(ratio), int(k), _ptr(set_),
                                               _stream(stream)))

    def gicp_linearise(self, src, tgt, tgt_cam, ratio, k, pose, out, corr=None, stream=None):
        """One linearisation of Eq. 2 at the device pose (float64 [12]): out
        float64 [29] (H upper triangle, g, cost, pair count); corr int32
        [n_src] or None; tgt_cam / ratio: the target set's camera and stride."""
        import torch
        for name, t in (("src", src), ("tgt", tgt), ("pose", pose), ("out", out)):
            _check_tensor(t, name, self.device, torch.float64)
        _check_tensor(corr, "corr", self.device, torch.int32)
        c = _cam(tgt_cam)
        self._check(self.lib.sgad_gicp_linearise(self.h, _ptr(src), src.shape[1], _ptr(tgt), tgt.shape[1],
                                                 C.byref(c), int(ratio), int(k), _ptr(pose), _ptr(out), _ptr(corr),
                                                 _stream(stream)))

    def gicp_track(self, src, tgt, tgt_cam, ratio, k, pose, iters, trace=None, stream=None):
        """`iters` Gauss-Newton steps on the device pose (float64 [12], in
        place); trace float64 [iters, 48] or None."""
        import torch
        for name, t in (("src", src), ("tgt", tgt), ("pose", pose)):
            _check_tensor(t, name, self.device, torch.float64)
        _check_tensor(trace, "trace", self.device, torch.float64)
        c = _cam(tgt_cam)
        self._check(self.lib.sgad_gicp_track(self.h, _ptr(src), src.shape[1], _ptr(tgt), tgt.shape[1], C.byref(c),
                                             int(ratio), int(k), _ptr(pose), int(iters), _ptr(trace),
                                             _stream(stream)))

    # ------------------------------------------------------- global set T
    def gmap_new(self, capacity, voxel=0.02):
        """An empty global set T of `capacity` Gaussians on this device."""
        m = GlobalMap(self.device, capacity, voxel)
        self.gmap_reset(m)
        return m

    def gmap_reset(self, m, stream=None):
        self._check(self.lib.sgad_gmap_reset(self.h, C.byref(m.c), _stream(stream)))

    def gmap_insert(self, m, set_, pose, stream=None):
        """Add a tracked frame's set [12, n] under its camera-to-world pose
        (device float64 [12])."""
        import torch
        _check_tensor(set_, "set", self.device, torch.float64)
        _check_tensor(pose, "pose", self.device, torch.float64)
        self._check(self.lib.sgad_gmap_insert(self.h, C.byref(m.c), _ptr(set_), set_.shape[1], _ptr(pose),
                                              _stream(stream)))

    def gicp_linearise_map(self, src, m, k, pose, out, corr=None, stream=None):
        """gicp_linearise against T (camera-to-world pose; corr indexes T)."""
        import torch
        for name, t in (("src", src), ("pose", pose), ("out", out)):
            _check_tensor(t, name, self.device, torch.float64)
        _check_tensor(corr, "corr", self.device, torch.int32)
        self._check(self.lib.sgad_gicp_linearise_map(self.h, _ptr(src), src.shape[1], C.byref(m.c), int(k),
                                                     _ptr(pose), _ptr(out), _ptr(corr), _stream(stream)))

    def gicp_track_map(self, src, m, k, pose, iters, trace=None, stream=None):
        """gicp_track against T."""
        import torch
        for name, t in (("src", src), ("pose", pose)):
            _check_tensor(t, name, self.device, torch.float64)
        _check_tensor(trace, "trace", self.device, torch.float64)
        self._check(self.lib.sgad_gicp_track_map(self.h, _ptr(src), src.shape[1], C.byref(m.c), int(k),
                                                 _ptr(pose), int(iters), _ptr(trace), _stream(stream)))

    def fill_depth(self, depth, rdepth, ralpha, out, alpha_min=0.5, stream=None):
        """Depth holes filled by rendered depth / alpha where alpha >= alpha_min."""
        for name, t in (("depth", depth), ("rdepth", rdepth), ("ralpha", ralpha), ("out", out)):
            _check_tensor(t, name, self.device)
        n = depth.numel()
        if not (rdepth.numel() == ralpha.numel() == out.numel() == n):
            raise ValueError("fill_depth: sizes differ")
        self._check(self.lib.sgad_fill_depth(self.h, n, _ptr(depth), _ptr(rdepth), _ptr(ralpha),
                                             float(alpha_min), _ptr(out), _stream(stream)))

    # -------------------------------------------------------------- conv net
    def conv_weights(self, cin, cout, w, w_bf16, wt_bf16=None, stream=None):
        import torch
        _check_tensor(w, "w", self.device)
        _check_tensor(w_bf16, "w_bf16", self.device, torch.bfloat16)
        _check_tensor(wt_bf16, "wt_bf16", self.device, torch.bfloat16)
        self._check(self.lib.sgad_conv_weights(self.h, cin, cout, _ptr(w), _ptr(w_bf16), _ptr(wt_bf16),
                                               _stream(stream)))

    def conv_fwd(self, H, W, cin, cout, mode, x, w_bf16, bias, y, stream=None):
        self._check(self.lib.sgad_conv3x3_fwd(self.h, H, W, cin, cout, mode, _ptr(x), _ptr(w_bf16), _ptr(bias),
                                              _ptr(y), _stream(stream)))

    def conv_dgrad(self, H, W, cin, cout, dy, wt_bf16, mask, dx, stream=None):
        self._check(self.lib.sgad_conv3x3_dgrad(self.h, H, W, cin, cout, _ptr(dy), _ptr(wt_bf16), _ptr(mask),
                                                _ptr(dx), _stream(stream)))

    def conv_wgrad(self, H, W, cin, cout, x, dy, dw, db, stream=None):
        self._check(self.lib.sgad_conv3x3_wgrad(self.h, H, W, cin, cout, _ptr(x), _ptr(dy), _ptr(dw), _ptr(db),
                                                _stream(stream)))

    def conv_wgrad_noalloc(self, H, W, cin, cout, x, dy, dw, db, stream=None):
        self._check(self.lib.sgad_conv3x3_wgrad_noalloc(self.h, H, W, cin, cout, _ptr(x), _ptr(dy), _ptr(dw),
                                                        _ptr(db), _stream(stream)))

    def net_input(self, H, W, rgb, depth, x0, stream=None):
        self._check(self.lib.sgad_net_input(self.h, H, W, _ptr(rgb), _ptr(depth), _ptr(x0), _stream(stream)))

    def offset_l1(self, pred, target, grad, loss, stream=None):
        self._check(self.lib.sgad_offset_l1(self.h, pred.numel(), _ptr(pred), _ptr(target), _ptr(grad),
                                            _ptr(loss), _stream(stream)))

    def release(self, saved):
        self._check(self.lib.sgad_saved_release(self.h, saved))

    # graph capture of library calls (see sgad_graph_begin in include/sgad.h)
    def graph_begin(self, stream=None):
        self._check(self.lib.sgad_graph_begin(self.h, _stream(stream)))

    def graph_end(self):
        g = C.c_void_p()
        self._check(self.lib.sgad_graph_end(self.h, C.byref(g)))
        self.__dict__.setdefault("_graphs", []).append(g)
        return g

    def graph_launch(self, graph, stream=None):
        self._check(self.lib.sgad_graph_launch(self.h, graph, _stream(stream)))

    def graph_destroy(self, graph):
        gs = self.__dict__.get("_graphs", [])
        for i, g in enumerate(gs):
            if g.value == graph.value:
                del gs[i]
                break
        self._check(self.lib.sgad_graph_destroy(self.h, graph))

    def instances(self, saved, job):
        """Sorted instance list of one job: (tile_ranges [n_tiles, 2], keys)."""
        n = C.c_size_t()
        nt = C.c_int()
        self._check(self.lib.sgad_saved_instances(self.h, saved, job, None, None, 0, C.byref(n),
                                                  C.byref(nt)))
        ranges = np.zeros((nt.value, 2), np.uint32)
        keys = np.zeros(max(n.value, 1), np.uint64)
        self._check(self.lib.sgad_saved_instances(self.h, saved, job, ranges.ctypes.data_as(C.c_void_p),
                                                  keys.ctypes.data_as(C.c_void_p), keys.size,
                                                  C.byref(n), C.byref(nt)))
        return ranges, keys[:n.value]


# ----------------------------------------------------------------------------
# convenience: numpy scene -> device tensors
# ----------------------------------------------------------------------------
def to_device(kf: dict, device) -> dict:
    """Copy a numpy keyframe dict (as made by ``synth``) to device tensors."""
    import torch
    out = dict(cam=dict(kf["cam"]), R=np.asarray(kf["R"], np.float32), t=np.asarray(kf["t"], np.float32))
    for k in ("depth", "offset", "radius", "opacity", "rgb", "sigma"):
        if kf.get(k) is not None:
            out[k] = torch.from_numpy(np.ascontiguousarray(kf[k], np.float32)).to(device)
    return out
