"""ctypes binding of librt.so (the C ABI declared in include/rt.h).

Argument marshalling only: every step of the trace runs in the HIP kernels of
librt.so.  There is no fallback: if the library is missing, importing this
module raises.  PyTorch supplies device memory and the stream.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librt.so")

if not os.path.exists(LIB_PATH):
    raise ImportError("paper_2005_05386_amd: %s is not built; run `python -c 'import __graft_entry__ as g; "
                      "g.build()'` (hipcc for gfx950)" % LIB_PATH)

_lib = C.CDLL(LIB_PATH)

RT_OK, RT_EINVAL, RT_ENOMEM, RT_EDEVICE, RT_EUNSUPPORTED, RT_ESTATE = 0, -1, -2, -3, -4, -5
EUCLID, GRAPH_GAUSS, PULLBACK_TWIST, PULLBACK_ZTWIST, PULLBACK_DEFORM, GRAPH_ANISO, GRAPH_QUADRIC = 0, 1, 2, 3, 4, 5, 6
RK4, RK45, EULER = 0, 1, 2
FLAG_TIMING, FLAG_COUNT_WORK, FLAG_SURROGATE, FLAG_BATCH_SEGMENTS = 1, 2, 4, 8

EXPORTS = ["rt_abi_version", "rt_create", "rt_destroy", "rt_last_error", "rt_set_metric", "rt_set_scene",
           "rt_trace", "rt_sync", "rt_get_stats", "rt_tape_bytes", "rt_trace_fwd_ckpt", "rt_loss_l2",
           "rt_trace_bwd", "rt_mlp_work_bytes", "rt_mlp_fwd", "rt_mlp_fwd_grouped", "rt_mlp_bwd", "rt_mse_grad", "rt_adamw_step",
           "rt_surrogate_gen", "rt_surrogate_train_bytes", "rt_surrogate_train", "rt_surrogate_calibrate",
           "rt_surrogate_load", "rt_illuminate", "rt_trace_noalloc"]
NOALLOC_SCRATCH_BYTES = 64 << 20   # RT_NOALLOC_SCRATCH_BYTES
MLP_PARAMS = 134918


class RtError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("rt status %d: %s" % (status, msg))
        self.status = status


class rt_bump(C.Structure):
    _fields_ = [("a", C.c_float), ("cx", C.c_float), ("cy", C.c_float), ("cz", C.c_float), ("sigma", C.c_float)]


class rt_metric(C.Structure):
    _fields_ = [("kind", C.c_int), ("n_sets", C.c_int), ("n_bumps", C.c_int), ("bumps", C.c_void_p),
                ("twist_amp", C.c_float), ("twist_theta0", C.c_float), ("cull_sigmas", C.c_float),
                ("n_deforms", C.c_int), ("deforms", C.c_void_p),
                ("n_abumps", C.c_int), ("abumps", C.c_void_p), ("quadric", C.c_float * 3)]


class rt_scene(C.Structure):
    _fields_ = [("n_spheres", C.c_int), ("spheres", C.c_void_p), ("n_planes", C.c_int), ("planes", C.c_void_p),
                ("n_tori", C.c_int), ("tori", C.c_void_p)]


class rt_camera(C.Structure):
    _fields_ = [("eye", C.c_float * 3), ("forward", C.c_float * 3), ("up", C.c_float * 3),
                ("vfov_deg", C.c_float), ("width", C.c_int), ("height", C.c_int)]


class rt_step_rule(C.Structure):
    _fields_ = [("kind", C.c_int), ("h", C.c_float), ("rtol", C.c_float), ("atol", C.c_float),
                ("h_min", C.c_float), ("h_max", C.c_float), ("t_max", C.c_float), ("cull_every", C.c_int),
                ("pass_steps", C.c_int), ("bisect_iters", C.c_int), ("flags", C.c_int)]


class rt_outputs(C.Structure):
    _fields_ = [("hit", C.c_void_p), ("t", C.c_void_p), ("id", C.c_void_p), ("dir", C.c_void_p),
                ("steps", C.c_void_p)]


class rt_light(C.Structure):
    _fields_ = [("pos", C.c_float * 3), ("h", C.c_float), ("tol", C.c_float), ("max_iters", C.c_int),
                ("max_steps", C.c_int)]


class rt_shading(C.Structure):
    _fields_ = [("shade", C.c_void_p), ("status", C.c_void_p), ("dir", C.c_void_p), ("len", C.c_void_p)]


class rt_stats(C.Structure):
    _fields_ = [("rays", C.c_uint64), ("ray_steps", C.c_uint64), ("attempts", C.c_uint64),
                ("wave_iters", C.c_uint64), ("lane_iters", C.c_uint64), ("bump_list_sum", C.c_uint64),
                ("obj_list_sum", C.c_uint64), ("refined", C.c_uint64), ("acc_evals", C.c_uint64),
                ("bump_evals", C.c_uint64), ("obj_tests", C.c_uint64), ("passes", C.c_int), ("pass_ms", C.c_float),
                ("refine_ms", C.c_float), ("compact_ms", C.c_float), ("total_ms", C.c_float),
                ("crossings", C.c_uint64), ("accepted", C.c_uint64), ("surr_ms", C.c_float),
                ("eligible", C.c_int), ("adj_steps", C.c_uint64), ("adj_bump_terms", C.c_uint64),
                ("adj_recomputed", C.c_uint64),
                ("batch_windows", C.c_uint64), ("batch_replays", C.c_uint64),
                ("refine_evals", C.c_uint64), ("refine_bump_terms", C.c_uint64), ("refine_steps", C.c_uint64)]


_P = C.c_void_p
_lib.rt_abi_version.restype = C.c_int
_lib.rt_create.argtypes = [C.c_int, C.POINTER(_P)]
_lib.rt_create.restype = C.c_int
_lib.rt_destroy.argtypes = [_P]
_lib.rt_destroy.restype = None
_lib.rt_last_error.argtypes = [_P]
_lib.rt_last_error.restype = C.c_char_p
_lib.rt_set_metric.argtypes = [_P, C.POINTER(rt_metric)]
_lib.rt_set_metric.restype = C.c_int
_lib.rt_set_scene.argtypes = [_P, C.POINTER(rt_scene)]
_lib.rt_set_scene.restype = C.c_int
_lib.rt_trace.argtypes = [_P, C.POINTER(rt_camera), C.POINTER(rt_step_rule), C.c_int, C.POINTER(rt_outputs), _P]
_lib.rt_trace.restype = C.c_int
_lib.rt_trace_noalloc.argtypes = [_P, C.POINTER(rt_camera), C.POINTER(rt_step_rule), C.c_int, C.POINTER(rt_outputs), _P]
_lib.rt_trace_noalloc.restype = C.c_int
_lib.rt_illuminate.argtypes = [_P, C.POINTER(rt_camera), C.POINTER(rt_outputs), C.POINTER(rt_light),
                               C.POINTER(rt_shading), _P]
_lib.rt_illuminate.restype = C.c_int
_lib.rt_sync.argtypes = [_P, _P]
_lib.rt_sync.restype = C.c_int
_lib.rt_get_stats.argtypes = [_P, C.POINTER(rt_stats)]
_lib.rt_get_stats.restype = C.c_int
_lib.rt_tape_bytes.argtypes = [C.POINTER(rt_camera), C.c_int, C.c_int, C.c_int]
_lib.rt_tape_bytes.restype = C.c_size_t
_lib.rt_trace_fwd_ckpt.argtypes = [_P, C.POINTER(rt_camera), C.POINTER(rt_step_rule), C.c_int, C.c_int,
                                   C.POINTER(rt_outputs), _P, C.c_size_t, _P]
_lib.rt_trace_fwd_ckpt.restype = C.c_int
_lib.rt_loss_l2.argtypes = [_P, C.POINTER(rt_camera), _P, _P, _P, _P, _P, _P, _P, _P]
_lib.rt_loss_l2.restype = C.c_int
_lib.rt_trace_bwd.argtypes = [_P, _P, _P, _P, _P]
_lib.rt_trace_bwd.restype = C.c_int
_lib.rt_mlp_work_bytes.argtypes = [C.c_int, C.c_int]
_lib.rt_mlp_work_bytes.restype = C.c_size_t
_lib.rt_mlp_fwd.argtypes = [_P, C.c_int, C.c_int, _P, _P, _P, _P, _P, C.c_size_t, _P]
_lib.rt_mlp_fwd.restype = C.c_int
_lib.rt_mlp_bwd.argtypes = [_P, C.c_int, C.c_int, _P, _P, _P, _P, _P, C.c_size_t, _P]
_lib.rt_mlp_bwd.restype = C.c_int
_lib.rt_adamw_step.argtypes = [_P, _P, _P, _P, _P, _P, C.c_size_t, C.c_float, C.c_float, C.c_float, C.c_float,
                               C.c_float, C.c_int, _P]
_lib.rt_adamw_step.restype = C.c_int
_lib.rt_mse_grad.argtypes = [_P, _P, _P, _P, C.c_size_t, C.c_int, _P, _P]
_lib.rt_mse_grad.restype = C.c_int
_lib.rt_surrogate_gen.argtypes = [_P, C.c_int, _P, _P, C.c_int, C.c_float, C.c_int, C.c_uint64, _P, _P, _P, _P]
_lib.rt_surrogate_gen.restype = C.c_int
_lib.rt_mlp_fwd_grouped.argtypes = [_P, C.c_int, _P, _P, _P, _P, _P, _P]
_lib.rt_mlp_fwd_grouped.restype = C.c_int
_lib.rt_surrogate_train_bytes.argtypes = [C.c_int, C.c_int]
_lib.rt_surrogate_train_bytes.restype = C.c_size_t
_lib.rt_surrogate_train.argtypes = [_P, C.c_int, _P, _P, C.c_int, C.c_int, C.c_float, C.c_int, C.c_uint64, C.c_float,
                                    C.c_float, C.c_int, C.c_float, C.c_float, C.c_float, C.c_float, _P, _P, _P, _P,
                                    _P, C.c_size_t, _P, C.c_int, _P]
_lib.rt_surrogate_train.restype = C.c_int
_lib.rt_surrogate_calibrate.argtypes = [_P, C.c_int, C.c_int, _P, _P, _P, _P, C.c_int, _P, _P]
_lib.rt_surrogate_calibrate.restype = C.c_int
_lib.rt_surrogate_load.argtypes = [_P, C.c_int, _P, _P, _P, _P, C.c_int, _P, C.c_int, _P, C.c_int, C.c_float]
_lib.rt_surrogate_load.restype = C.c_int


def lib():
    return _lib


def abi_version():
    return _lib.rt_abi_version()


def camera_struct(cam):
    f3 = lambda v: (C.c_float * 3)(*[float(x) for x in v])
    return rt_camera(f3(cam["eye"]), f3(cam["forward"]), f3(cam["up"]), float(cam["vfov_deg"]),
                     int(cam["width"]), int(cam["height"]))


def rule_struct(r):
    return rt_step_rule(int(r["kind"]), float(r["h"]), float(r.get("rtol", 1e-6)), float(r.get("atol", 1e-6)),
                        float(r.get("h_min", 1e-6)), float(r.get("h_max", r["h"])), float(r["t_max"]),
                        int(r.get("cull_every", 16)), int(r.get("pass_steps", 256)), int(r.get("bisect_iters", 24)),
                        int(r.get("flags", 0)))


class Tracer:
    """One rt_ctx on a HIP device (device=-1: host-only, validation only)."""

    def __init__(self, device=0):
        h = _P()
        st = _lib.rt_create(int(device), C.byref(h))
        if st != RT_OK:
            raise RtError(st, _lib.rt_last_error(None).decode())
        self._h = h
        self.device = device
        self.n_sets = 1
        self._keep = []

    def close(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.rt_destroy(self._h)
        self._h = None

    def __del__(self):
        self.close()

    def _check(self, st):
        if st != RT_OK:
            raise RtError(st, _lib.rt_last_error(self._h).decode())

    def set_metric(self, metric):
        b = np.ascontiguousarray(np.asarray(metric.get("bumps", np.zeros((1, 0, 5))), np.float32))
        if b.ndim == 2:
            b = b[None]
        n_sets, n_bumps = b.shape[0], b.shape[1]
        # deformation rows: a, c (3), spreads (3), v (3) and the optional
        # rotation w (3) of the field V(p) = v + w x (p - c), zero if absent
        d = metric.get("deforms")
        d = np.zeros((1, 0, 13), np.float32) if d is None else np.asarray(d, np.float32)
        d = d[None] if d.ndim == 2 else d
        if d.shape[-1] == 10:
            d = np.concatenate([d, np.zeros(d.shape[:-1] + (3,), np.float32)], axis=-1)
        if d.shape[-1] != 13:
            raise ValueError("deformation rows must have 10 or 13 values")
        d = np.ascontiguousarray(d)
        ab = metric.get("abumps")
        ab = np.zeros((1, 0, 7), np.float32) if ab is None else np.asarray(ab, np.float32)
        ab = np.ascontiguousarray(ab[None] if ab.ndim == 2 else ab)
        if int(metric["kind"]) == PULLBACK_DEFORM:
            n_sets = d.shape[0]
        if int(metric["kind"]) == GRAPH_ANISO:
            n_sets = ab.shape[0]
        if int(metric["kind"]) == GRAPH_QUADRIC:
            n_sets = 1
        q = [float(x) for x in metric.get("quadric", (0.0, 0.0, 0.0))]
        m = rt_metric(int(metric["kind"]), int(n_sets), int(n_bumps), b.ctypes.data if b.size else None,
                      float(metric.get("twist_amp", 0.4)), float(metric.get("twist_theta0", 1.2)),
                      float(metric.get("cull_sigmas", 6.0)), int(d.shape[1]), d.ctypes.data if d.size else None,
                      int(ab.shape[1]), ab.ctypes.data if ab.size else None, (C.c_float * 3)(*q))
        self._check(_lib.rt_set_metric(self._h, C.byref(m)))
        self.n_sets = n_sets

    def set_scene(self, scene):
        sp = np.ascontiguousarray(np.asarray(scene["spheres"], np.float32).reshape(-1, 4))
        pl = np.ascontiguousarray(np.asarray(scene["planes"], np.float32).reshape(-1, 4))
        to = np.ascontiguousarray(np.asarray(scene["tori"], np.float32).reshape(-1, 8))
        s = rt_scene(sp.shape[0], sp.ctypes.data if sp.size else None, pl.shape[0],
                     pl.ctypes.data if pl.size else None, to.shape[0], to.ctypes.data if to.size else None)
        self._check(_lib.rt_set_scene(self._h, C.byref(s)))

    def alloc_outputs(self, camera, with_steps=True):
        import torch
        n = self.n_sets * camera["height"] * camera["width"]
        dev = torch.device("cuda", self.device)
        return dict(hit=torch.empty((n, 3), dtype=torch.float32, device=dev),
                    t=torch.empty(n, dtype=torch.float32, device=dev),
                    id=torch.empty(n, dtype=torch.int32, device=dev),
                    dir=torch.empty((n, 3), dtype=torch.float32, device=dev),
                    steps=torch.empty(n, dtype=torch.int32, device=dev) if with_steps else None)

    def trace_into(self, camera, rule, max_steps, out, stream=None, noalloc=False):
        """Enqueue a trace writing into the tensors of `out` (see
        alloc_outputs); asynchronous on `stream` (torch stream or None for
        torch's current stream).  noalloc: call rt_trace_noalloc, whose
        workspace is the library's static per-GPU array (no device
        allocation inside the call)."""
        import torch
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        n = self.n_sets * camera["height"] * camera["width"]
        for k, shape, dt in (("hit", (n, 3), torch.float32), ("t", (n,), torch.float32),
                             ("id", (n,), torch.int32), ("dir", (n, 3), torch.float32)):
            tns = out[k]
            if tuple(tns.shape) != shape or tns.dtype != dt or not tns.is_cuda or not tns.is_contiguous():
                raise ValueError("output %s must be a contiguous %s cuda tensor of shape %s" % (k, dt, shape))
        steps = out.get("steps")
        if steps is not None and (tuple(steps.shape) != (n,) or steps.dtype != torch.int32):
            raise ValueError("output steps must be an int32 tensor of shape (%d,)" % n)
        o = rt_outputs(out["hit"].data_ptr(), out["t"].data_ptr(), out["id"].data_ptr(), out["dir"].data_ptr(),
                       steps.data_ptr() if steps is not None else None)
        cam = camera_struct(camera)
        r = rule_struct(rule)
        fn = _lib.rt_trace_noalloc if noalloc else _lib.rt_trace
        self._check(fn(self._h, C.byref(cam), C.byref(r), int(max_steps), C.byref(o), C.c_void_p(stream.cuda_stream)))
        return out

    def trace(self, camera, rule, max_steps=None, with_steps=True):
        if max_steps is None:
            max_steps = rule["max_steps"]
        out = self.alloc_outputs(camera, with_steps)
        return self.trace_into(camera, rule, max_steps, out)

    def illuminate(self, camera, traced, light, stream=None):
        """Direct Riemannian illumination of a traced frame by a point light
        (rt_illuminate).  light: dict(pos, h=0.01, tol=1e-4, max_iters=16,
        max_steps=4000).  Returns dict of cuda tensors shade, status, dir,
        len."""
        import torch
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        n = self.n_sets * camera["height"] * camera["width"]
        for k, shape, dt in (("hit", (n, 3), torch.float32), ("id", (n,), torch.int32)):
            tns = traced[k]
            if tuple(tns.shape) != shape or tns.dtype != dt or not tns.is_cuda or not tns.is_contiguous():
                raise ValueError("traced %s must be a contiguous %s cuda tensor of shape %s" % (k, dt, shape))
        dev = traced["hit"].device
        out = dict(shade=torch.empty(n, dtype=torch.float32, device=dev),
                   status=torch.empty(n, dtype=torch.int32, device=dev),
                   dir=torch.empty((n, 3), dtype=torch.float32, device=dev),
                   len=torch.empty(n, dtype=torch.float32, device=dev))
        o = rt_outputs(traced["hit"].data_ptr(), None, traced["id"].data_ptr(), None, None)
        L = rt_light((C.c_float * 3)(*[float(v) for v in light["pos"]]), float(light.get("h", 0.01)),
                     float(light.get("tol", 1e-4)), int(light.get("max_iters", 16)), int(light.get("max_steps", 4000)))
        sh = rt_shading(out["shade"].data_ptr(), out["status"].data_ptr(), out["dir"].data_ptr(), out["len"].data_ptr())
        self._check(_lib.rt_illuminate(self._h, C.byref(camera_struct(camera)), C.byref(o), C.byref(L), C.byref(sh),
                                       C.c_void_p(stream.cuda_stream)))
        return out

    def illuminate_raw(self, camera, hit_ptr, id_ptr, light, shade_ptr, status_ptr, stream_handle=0):
        """rt_illuminate with raw device pointers (validation tests)."""
        o = rt_outputs(hit_ptr or None, None, id_ptr or None, None, None)
        L = rt_light((C.c_float * 3)(*[float(v) for v in light["pos"]]), float(light.get("h", 0.01)),
                     float(light.get("tol", 1e-4)), int(light.get("max_iters", 16)), int(light.get("max_steps", 4000)))
        sh = rt_shading(shade_ptr or None, status_ptr or None, None, None)
        self._check(_lib.rt_illuminate(self._h, C.byref(camera_struct(camera)), C.byref(o), C.byref(L), C.byref(sh),
                                       C.c_void_p(stream_handle)))

    def trace_raw(self, camera, rule, max_steps, out_ptrs, stream_handle, noalloc=False):
        """Enqueue with raw device pointers (hit, t, id, dir, steps-or-0)."""
        o = rt_outputs(*[p if p else None for p in out_ptrs])
        fn = _lib.rt_trace_noalloc if noalloc else _lib.rt_trace
        self._check(fn(self._h, C.byref(camera_struct(camera)), C.byref(rule_struct(rule)), int(max_steps), C.byref(o),
                       C.c_void_p(stream_handle)))

    # ---- differentiation (graph metric, RK4)
    def tape_bytes(self, camera, max_steps, ckpt_every):
        return int(_lib.rt_tape_bytes(C.byref(camera_struct(camera)), int(self.n_sets), int(max_steps),
                                      int(ckpt_every)))

    def trace_fwd_ckpt(self, camera, rule, max_steps, ckpt_every, out=None, tape=None):
        """Trace with the adjoint tape; returns (outputs, tape tensor)."""
        import torch
        stream = torch.cuda.current_stream(self.device)
        if out is None:
            out = self.alloc_outputs(camera)
        nbytes = self.tape_bytes(camera, max_steps, ckpt_every)
        if tape is None or tape.numel() * tape.element_size() < nbytes:
            tape = torch.empty(nbytes // 4 + 1, dtype=torch.float32, device=torch.device("cuda", self.device))
        steps = out.get("steps")
        o = rt_outputs(out["hit"].data_ptr(), out["t"].data_ptr(), out["id"].data_ptr(), out["dir"].data_ptr(),
                       steps.data_ptr() if steps is not None else None)
        self._check(_lib.rt_trace_fwd_ckpt(self._h, C.byref(camera_struct(camera)), C.byref(rule_struct(rule)),
                                           int(max_steps), int(ckpt_every), C.byref(o), C.c_void_p(tape.data_ptr()),
                                           C.c_size_t(tape.numel() * tape.element_size()),
                                           C.c_void_p(stream.cuda_stream)))
        return out, tape

    def loss_l2(self, camera, hit, ids, target_hit, target_id, mask=None, want_grad=True):
        """Masked L2 loss per set (device) and its gradient on the hit map."""
        import torch
        stream = torch.cuda.current_stream(self.device)
        dev = hit.device
        loss = torch.empty(self.n_sets, dtype=torch.float32, device=dev)
        grad = torch.empty_like(hit) if want_grad else None
        m = None
        if mask is not None:
            m = mask.to(device=dev, dtype=torch.uint8).contiguous()
        self._check(_lib.rt_loss_l2(self._h, C.byref(camera_struct(camera)), C.c_void_p(hit.data_ptr()),
                                    C.c_void_p(ids.data_ptr()), C.c_void_p(target_hit.data_ptr()),
                                    C.c_void_p(target_id.data_ptr()), C.c_void_p(m.data_ptr() if m is not None else 0),
                                    C.c_void_p(loss.data_ptr()), C.c_void_p(grad.data_ptr() if grad is not None else 0),
                                    C.c_void_p(stream.cuda_stream)))
        return loss, grad

    def trace_bwd(self, tape, grad_hit, n_bumps):
        import torch
        stream = torch.cuda.current_stream(self.device)
        g = torch.empty((self.n_sets, n_bumps, 5), dtype=torch.float32, device=grad_hit.device)
        gh = grad_hit.contiguous()
        self._check(_lib.rt_trace_bwd(self._h, C.c_void_p(tape.data_ptr()), C.c_void_p(gh.data_ptr()),
                                      C.c_void_p(g.data_ptr()), C.c_void_p(stream.cuda_stream)))
        return g

    # ---- surrogate MLP (BF16 matrix cores)
    def mlp_work(self, n_nets, batch):
        import torch
        nb = int(_lib.rt_mlp_work_bytes(int(n_nets), int(batch)))
        return torch.empty(nb // 4 + 64, dtype=torch.float32, device=torch.device("cuda", self.device))

    def mlp_fwd(self, w_bf16, params, x, work):
        """x [n_nets, batch, 6] float32 cuda -> y [n_nets, batch, 6]."""
        import torch
        n, b = x.shape[0], x.shape[1]
        y = torch.empty((n, b, 6), dtype=torch.float32, device=x.device)
        st = torch.cuda.current_stream(self.device)
        self._check(_lib.rt_mlp_fwd(self._h, n, b, C.c_void_p(w_bf16.data_ptr()), C.c_void_p(params.data_ptr()),
                                    C.c_void_p(x.contiguous().data_ptr()), C.c_void_p(y.data_ptr()),
                                    C.c_void_p(work.data_ptr()), C.c_size_t(work.numel() * 4),
                                    C.c_void_p(st.cuda_stream)))
        return y

    def mlp_fwd_grouped(self, w_bf16, params, x, rows):
        """x [sum(rows), 6] float32 cuda, rows per network -> y [sum(rows), 6]."""
        import torch
        r = np.ascontiguousarray(rows, np.int32)
        x = x.contiguous()
        y = torch.empty_like(x)
        st = torch.cuda.current_stream(self.device)
        self._check(_lib.rt_mlp_fwd_grouped(self._h, int(len(r)), r.ctypes.data, C.c_void_p(w_bf16.data_ptr()),
                                            C.c_void_p(params.data_ptr()), C.c_void_p(x.data_ptr()),
                                            C.c_void_p(y.data_ptr()), C.c_void_p(st.cuda_stream)))
        return y

    def mlp_bwd(self, w_bf16, params, dy, work):
        """Parameter gradient [n_nets, MLP_PARAMS] of sum(dy * y) for the last
        mlp_fwd on `work` (same weights)."""
        import torch
        n, b = dy.shape[0], dy.shape[1]
        g = torch.empty((n, MLP_PARAMS), dtype=torch.float32, device=dy.device)
        st = torch.cuda.current_stream(self.device)
        self._check(_lib.rt_mlp_bwd(self._h, n, b, C.c_void_p(w_bf16.data_ptr()), C.c_void_p(params.data_ptr()),
                                    C.c_void_p(dy.contiguous().data_ptr()), C.c_void_p(g.data_ptr()),
                                    C.c_void_p(work.data_ptr()), C.c_size_t(work.numel() * 4),
                                    C.c_void_p(st.cuda_stream)))
        return g

    def mse_grad(self, y, t, batch):
        """dy = 2 (y - t) / batch; returns (dy, 64 partial sums of squares)."""
        import torch
        dy = torch.empty_like(y)
        part = torch.empty(64, dtype=torch.float32, device=y.device)
        st = torch.cuda.current_stream(self.device)
        self._check(_lib.rt_mse_grad(self._h, C.c_void_p(y.data_ptr()), C.c_void_p(t.contiguous().data_ptr()),
                                     C.c_void_p(dy.data_ptr()), C.c_size_t(y.numel()), int(batch),
                                     C.c_void_p(part.data_ptr()), C.c_void_p(st.cuda_stream)))
        return dy, part

    def adamw(self, params, w_bf16, m, v, grad, lr, step, b1=0.9, b2=0.999, eps=1e-8, wd=0.0):
        import torch
        st = torch.cuda.current_stream(self.device)
        self._check(_lib.rt_adamw_step(self._h, C.c_void_p(params.data_ptr()), C.c_void_p(w_bf16.data_ptr()),
                                       C.c_void_p(m.data_ptr()), C.c_void_p(v.data_ptr()),
                                       C.c_void_p(grad.data_ptr()), C.c_size_t(params.numel()), float(lr),
                                       float(b1), float(b2), float(eps), float(wd), int(step),
                                       C.c_void_p(st.cuda_stream)))

    def surrogate_gen(self, kappa, scale, n_per, h, grid=False, seed=0, mode=None):
        """Crossing data for each shape kappa (mode 0: sin^2 th uniform,
        1: cos-theta grid, 2: sin th uniform, 4 / 6: 0 / 2 with stratified
        draws; grid=True selects mode 1):
        returns x, y [n,n_per,6], aux [n,n_per,4]."""
        import torch
        k = np.ascontiguousarray(kappa, np.float32)
        sc = np.ascontiguousarray(scale, np.float32)
        n = len(k)
        dev = torch.device("cuda", self.device)
        x = torch.empty((n, n_per, 6), dtype=torch.float32, device=dev)
        y = torch.empty((n, n_per, 6), dtype=torch.float32, device=dev)
        aux = torch.empty((n, n_per, 4), dtype=torch.float32, device=dev)
        st = torch.cuda.current_stream(self.device)
        self._check(_lib.rt_surrogate_gen(self._h, n, k.ctypes.data, sc.ctypes.data, int(n_per), float(h),
                                          int(mode if mode is not None else (1 if grid else 0)), int(seed),
                                          C.c_void_p(x.data_ptr()),
                                          C.c_void_p(y.data_ptr()), C.c_void_p(aux.data_ptr()),
                                          C.c_void_p(st.cuda_stream)))
        return x, y, aux

    def surrogate_train(self, kappa, scale, params, w_bf16, m, v, batch, n_steps, h=0.01, mode=0, seed=0,
                        lr=2e-3, lr_min=1e-5, warmup=200, b1=0.9, b2=0.999, eps=1e-8, wd=0.0, log_every=500):
        """Enqueue n_steps training steps of the networks (all in the
        library); returns the loss log [n_steps // log_every, 64] partial
        sums (a device tensor, valid after the stream's work)."""
        import torch
        k = np.ascontiguousarray(kappa, np.float32)
        sc = np.ascontiguousarray(scale, np.float32)
        n = len(k)
        dev = torch.device("cuda", self.device)
        nbytes = int(_lib.rt_surrogate_train_bytes(n, int(batch)))
        work = torch.empty(nbytes // 4 + 64, dtype=torch.float32, device=dev)
        n_log = int(n_steps) // int(log_every)
        log = torch.zeros((max(n_log, 1), 64), dtype=torch.float32, device=dev)
        st = torch.cuda.current_stream(self.device)
        self._check(_lib.rt_surrogate_train(self._h, n, k.ctypes.data, sc.ctypes.data, int(batch), int(n_steps),
                                            float(h), int(mode), int(seed), float(lr), float(lr_min), int(warmup),
                                            float(b1), float(b2), float(eps), float(wd),
                                            C.c_void_p(params.data_ptr()), C.c_void_p(w_bf16.data_ptr()),
                                            C.c_void_p(m.data_ptr()), C.c_void_p(v.data_ptr()),
                                            C.c_void_p(work.data_ptr()), C.c_size_t(work.numel() * 4),
                                            C.c_void_p(log.data_ptr()) if n_log else None, int(log_every),
                                            C.c_void_p(st.cuda_stream)))
        return log[:n_log], work

    def surrogate_calibrate(self, x, pred, target, scale, n_bins):
        """Per-bin decoded error maxima [n, n_bins, 2] of pred against target."""
        import torch
        n, n_per = x.shape[0], x.shape[1]
        sc = np.ascontiguousarray(scale, np.float32)
        err = torch.empty((n, n_bins, 2), dtype=torch.float32, device=x.device)
        st = torch.cuda.current_stream(self.device)
        self._check(_lib.rt_surrogate_calibrate(self._h, int(n), int(n_per), C.c_void_p(x.data_ptr()),
                                                C.c_void_p(pred.data_ptr()), C.c_void_p(target.data_ptr()),
                                                sc.ctypes.data, int(n_bins), C.c_void_p(err.data_ptr()),
                                                C.c_void_p(st.cuda_stream)))
        return err

    def surrogate_load(self, w_bf16, params, scale, arc, err, net_of_bump, tol=1e-3):
        """Copy trained networks and their tables into the tracer."""
        import torch
        self.sync()
        n = int(params.shape[0])
        sc = np.ascontiguousarray(scale, np.float32)
        nob = np.ascontiguousarray(net_of_bump, np.int32)
        arc = arc.contiguous()
        err = err.contiguous()
        self._check(_lib.rt_surrogate_load(self._h, n, C.c_void_p(w_bf16.data_ptr()), C.c_void_p(params.data_ptr()),
                                           sc.ctypes.data, C.c_void_p(arc.data_ptr()), int(arc.shape[1]),
                                           C.c_void_p(err.data_ptr()), int(err.shape[1]), nob.ctypes.data,
                                           int(len(nob)), float(tol)))

    def surrogate_unload(self):
        self._check(_lib.rt_surrogate_load(self._h, 0, None, None, None, None, 2, None, 1, None, 0, 1.0))

    def sync(self, stream=None):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self._check(_lib.rt_sync(self._h, C.c_void_p(stream.cuda_stream)))

    def stats(self):
        s = rt_stats()
        self._check(_lib.rt_get_stats(self._h, C.byref(s)))
        return {k: getattr(s, k) for k, _ in rt_stats._fields_}


def to_numpy(out):
    return {k: (v.cpu().numpy() if v is not None else None) for k, v in out.items()}


def make_trace_function():
    """torch.autograd.Function: hit map of a graph-metric RK4 trace as a
    differentiable function of the bump parameters.

        hit, ids = TraceFn.apply(params, tracer, metric, camera, rule, ckpt_every)

    params [n_sets, n_bumps, 5] (a, cx, cy, cz, sigma); hit [n_sets*H*W, 3].
    The forward uploads params to the context (host copy), traces with the
    adjoint tape; the backward runs the HIP adjoint on the incoming
    gradient of hit (pixels that miss receive none)."""
    import torch

    class TraceFn(torch.autograd.Function):
        @staticmethod
        def forward(ctx, params, tracer, metric, camera, rule, ckpt_every):
            m = dict(metric, bumps=params.detach().float().cpu().numpy())
            tracer.set_metric(m)
            out, tape = tracer.trace_fwd_ckpt(camera, rule, rule["max_steps"], ckpt_every)
            ctx.tracer, ctx.tape, ctx.nb, ctx.pdev = tracer, tape, params.shape[1], params.device
            ctx.mark_non_differentiable(out["id"])
            return out["hit"], out["id"]

        @staticmethod
        def backward(ctx, grad_hit, grad_id):
            g = ctx.tracer.trace_bwd(ctx.tape, grad_hit.float(), ctx.nb)
            return g.to(ctx.pdev), None, None, None, None, None

    return TraceFn
