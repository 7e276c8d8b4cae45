"""Python binding of libsurfsplat (the C ABI in include/surfsplat.h).

Argument marshalling only: every step of the rendering path runs in the HIP
library.  PyTorch provides device memory and the stream.  If the library is
not built (or the device is not a GPU) the calls raise; there is no fallback.
"""
from __future__ import annotations

import ctypes
import dataclasses
import math
import os
from typing import List, Optional, Sequence

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsurfsplat.so")

(SS_OK, SS_ERR_INVALID_ARG, SS_ERR_HIP, SS_ERR_CAPACITY, SS_ERR_STATE, SS_ERR_UNSUPPORTED, SS_ERR_NOMEM,
 SS_ERR_STATIC_LIMIT) = range(8)
SHADE = {"albedo": 0, "splitsum": 1, "normal": 2}
LAUNCH = {"batched": 0, "per_view": 1}

EXPORTED = ["ss_default_options", "ss_create", "ss_destroy", "ss_set_options", "ss_brdf_lut",
            "ss_set_brdf_lut", "ss_reserve", "ss_render", "ss_render_backward", "ss_poll",
            "ss_render_static", "ss_debug_binning", "ss_debug_env_levels", "ss_profile_enable", "ss_profile_read",
            "ss_status_str"]
STATIC_SCRATCH_BYTES = 32 << 20  # SS_STATIC_SCRATCH_BYTES
STAGES = ["envmap", "preprocess", "binning", "raster_forward", "raster_backward",
          "preprocess_backward", "envmap_backward"]


class SurfsplatError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        super().__init__(f"{where}: {status_str(status)} (status {status})")


class ss_options(ctypes.Structure):
    _fields_ = [("r_cut", ctypes.c_float), ("k_max", ctypes.c_int32), ("gamma", ctypes.c_float),
                ("sigma_f", ctypes.c_float), ("shade", ctypes.c_int32), ("tile_w", ctypes.c_int32),
                ("tile_h", ctypes.c_int32), ("lds_batch", ctypes.c_int32), ("launch", ctypes.c_int32),
                ("persistent", ctypes.c_int32), ("depth_stats", ctypes.c_int32), ("mip", ctypes.c_int32),
                ("env_lds", ctypes.c_int32), ("t_min", ctypes.c_float), ("deterministic", ctypes.c_int32),
                ("validate", ctypes.c_int32), ("counters", ctypes.c_int32), ("tonemap", ctypes.c_int32),
                ("seg_len", ctypes.c_int32), ("bwd_walk", ctypes.c_int32)]


class ss_camera(ctypes.Structure):
    _fields_ = [("scene", ctypes.c_int32), ("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("fx", ctypes.c_float), ("fy", ctypes.c_float), ("cx", ctypes.c_float),
                ("cy", ctypes.c_float), ("R", ctypes.c_float * 9), ("t", ctypes.c_float * 3),
                ("znear", ctypes.c_float), ("background", ctypes.c_float * 3)]


_fp = ctypes.POINTER(ctypes.c_float)


class ss_batch(ctypes.Structure):
    _fields_ = [("n_scenes", ctypes.c_int32), ("surfel_offset", ctypes.POINTER(ctypes.c_int64)),
                ("position", ctypes.c_void_p), ("normal", ctypes.c_void_p), ("tangent", ctypes.c_void_p),
                ("scale", ctypes.c_void_p), ("albedo", ctypes.c_void_p), ("roughness", ctypes.c_void_p),
                ("metallic", ctypes.c_void_p), ("envmap", ctypes.POINTER(ctypes.c_void_p)),
                ("env_hw", ctypes.POINTER(ctypes.c_int32)), ("n_views", ctypes.c_int32),
                ("cameras", ctypes.POINTER(ss_camera))]


class ss_outputs(ctypes.Structure):
    _fields_ = [("image", ctypes.c_void_p), ("alpha", ctypes.c_void_p), ("n_layers", ctypes.c_void_p),
                ("cons", ctypes.c_void_p), ("depth", ctypes.c_void_p),
                ("generation", ctypes.POINTER(ctypes.c_int64))]


class ss_grad_in(ctypes.Structure):
    _fields_ = [("d_image", ctypes.c_void_p), ("d_alpha", ctypes.c_void_p), ("d_cons", ctypes.c_void_p),
                ("d_depth", ctypes.c_void_p), ("generation", ctypes.c_int64)]


class ss_grads(ctypes.Structure):
    _fields_ = [("d_position", ctypes.c_void_p), ("d_normal", ctypes.c_void_p),
                ("d_tangent", ctypes.c_void_p), ("d_scale", ctypes.c_void_p),
                ("d_albedo", ctypes.c_void_p), ("d_roughness", ctypes.c_void_p),
                ("d_metallic", ctypes.c_void_p), ("d_envmap", ctypes.POINTER(ctypes.c_void_p)),
                ("screen_grad", ctypes.c_void_p), ("visible_views", ctypes.c_void_p)]


class ss_diag(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("n_records", ctypes.c_int64), ("n_pairs", ctypes.c_int64),
                ("pair_capacity", ctypes.c_int64), ("workspace_bytes", ctypes.c_int64),
                ("generation", ctypes.c_int64), ("n_nonfinite", ctypes.c_int64),
                ("n_evaluated", ctypes.c_int64), ("n_fragments", ctypes.c_int64), ("n_layers", ctypes.c_int64),
                ("sum_layer_weight", ctypes.c_double), ("static_status", ctypes.c_int32),
                ("static_pairs", ctypes.c_int64), ("static_pair_capacity", ctypes.c_int64)]


_LIB = None


def load_library(path: str = LIB_PATH):
    """Load libsurfsplat.so; raises if it has not been built."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(path):
        raise RuntimeError(f"libsurfsplat is not built ({path} missing); run __graft_entry__.build() "
                           "or python paper_2605_05876_amd/build.py")
    L = ctypes.CDLL(path)
    vp = ctypes.c_void_p
    L.ss_default_options.argtypes = [ctypes.POINTER(ss_options)]
    L.ss_create.argtypes = [ctypes.POINTER(ss_options), ctypes.POINTER(vp)]
    L.ss_destroy.argtypes = [vp]
    L.ss_set_options.argtypes = [vp, ctypes.POINTER(ss_options)]
    L.ss_brdf_lut.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, vp]
    L.ss_set_brdf_lut.argtypes = [vp, vp, ctypes.c_int32, ctypes.c_int32, vp]
    L.ss_reserve.argtypes = [vp, ctypes.POINTER(ss_batch), vp, ctypes.POINTER(ctypes.c_size_t)]
    L.ss_render.argtypes = [vp, ctypes.POINTER(ss_batch), ctypes.POINTER(ss_outputs), vp]
    L.ss_render_backward.argtypes = [vp, ctypes.POINTER(ss_batch), ctypes.POINTER(ss_grad_in),
                                     ctypes.POINTER(ss_grads), vp]
    L.ss_poll.argtypes = [vp, ctypes.POINTER(ss_diag)]
    L.ss_render_static.argtypes = [vp, ctypes.POINTER(ss_batch), ctypes.POINTER(ss_outputs), vp]
    L.ss_debug_binning.argtypes = [vp, vp, vp, vp, vp, vp, ctypes.POINTER(ctypes.c_int64),
                                   ctypes.POINTER(ctypes.c_int64), vp]
    L.ss_debug_env_levels.argtypes = [vp, ctypes.c_int32, vp, ctypes.c_int64, vp]
    L.ss_profile_enable.argtypes = [vp, ctypes.c_int32]
    L.ss_profile_read.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
    L.ss_status_str.argtypes = [ctypes.c_int]
    L.ss_status_str.restype = ctypes.c_char_p
    for name in EXPORTED:
        getattr(L, name).restype = ctypes.c_char_p if name == "ss_status_str" else ctypes.c_int
    _LIB = L
    return L


def status_str(s: int) -> str:
    try:
        return load_library().ss_status_str(int(s)).decode()
    except Exception:
        return f"status {s}"


def _check(s, where):
    if s != SS_OK:
        raise SurfsplatError(s, where)


@dataclasses.dataclass
class Options:
    """Mirror of ss_options (defaults: the paper's settings, App. A.1)."""
    r_cut: float = 3.0
    k_max: int = 16
    gamma: float = 2.0 * math.pi
    sigma_f: float = 0.1
    shade: str = "albedo"
    tile_w: int = 16
    tile_h: int = 16
    lds_batch: int = 128        # 0: picked by the library at each reserve
    launch: str = "batched"
    persistent: bool = True
    depth_stats: bool = False   # allow forwards to output the eq:cons_loss term
    mip: str = "centre"         # "centre" (Sec. 3.3.2) | "pixel" (per-pixel Jacobian, Sec. 3.3.1)
    env_lds: int = -1           # split-sum backward: environment gradient floats kept in LDS (-1: all that fit)
    t_min: float = 0.0          # transmittance early-out (0: off)
    deterministic: bool = False  # bitwise reproducible gradients
    validate: bool = False      # count non-finite inputs (ss_poll: n_nonfinite)
    counters: bool = False      # count the raster forward's work (ss_poll)
    tonemap: str = "linear"     # "linear" | "srgb_log" (log-space + sRGB transfer, eq:photo_loss)
    seg_len: int = 0            # split tile lists longer than this (0: 2048, -1: never)
    bwd_walk: str = "auto"      # raster backward walk: "auto" | "rows" | "records"

    def to_c(self) -> ss_options:
        return ss_options(self.r_cut, self.k_max, self.gamma, self.sigma_f, SHADE[self.shade],
                          self.tile_w, self.tile_h, self.lds_batch, LAUNCH[self.launch],
                          1 if self.persistent else 0, 1 if self.depth_stats else 0,
                          {"centre": 0, "pixel": 1}[self.mip], int(self.env_lds), float(self.t_min),
                          1 if self.deterministic else 0, 1 if self.validate else 0,
                          1 if self.counters else 0, {"linear": 0, "srgb_log": 1}[self.tonemap],
                          int(self.seg_len), {"auto": 0, "rows": 1, "records": 2}[self.bwd_walk])


def camera_to_c(cam) -> ss_camera:
    c = ss_camera()
    c.scene = int(getattr(cam, "scene", 0))
    c.width, c.height = int(cam.width), int(cam.height)
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    R = [float(x) for x in list(getattr(cam.R, "ravel", lambda: cam.R)())]
    for i in range(9):
        c.R[i] = R[i]
    for i in range(3):
        c.t[i] = float(cam.t[i])
        c.background[i] = float(cam.background[i])
    c.znear = float(cam.znear)
    return c


def _stream_ptr(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


PARAMS = ["position", "normal", "tangent", "scale", "albedo", "roughness", "metallic"]


class Batch:
    """Device-side batch: parameters [C][N] (float32, contiguous, cuda),
    per-scene surfel offsets, environment maps and cameras."""

    def __init__(self, params: dict, surfel_offset: Sequence[int], cameras: Sequence,
                 envmaps: Optional[List[torch.Tensor]] = None):
        self.params = {k: params[k] for k in PARAMS}
        for k, v in self.params.items():
            if not (v.is_cuda and v.dtype == torch.float32 and v.is_contiguous()):
                raise ValueError(f"{k} must be a contiguous float32 CUDA tensor")
        self.offsets = (ctypes.c_int64 * len(surfel_offset))(*[int(x) for x in surfel_offset])
        self.n_scenes = len(surfel_offset) - 1
        self.cameras = list(cameras)
        self.cams_c = (ss_camera * len(self.cameras))(*[camera_to_c(c) for c in self.cameras])
        self.envmaps = envmaps
        if envmaps is not None:
            self.env_ptrs = (ctypes.c_void_p * self.n_scenes)(*[e.data_ptr() for e in envmaps])
            hw = []
            for e in envmaps:
                hw += [int(e.shape[0]), int(e.shape[1])]
            self.env_hw = (ctypes.c_int32 * len(hw))(*hw)
        self.c = ss_batch()
        self.c.n_scenes = self.n_scenes
        self.c.surfel_offset = self.offsets
        for k in PARAMS:
            setattr(self.c, k, self.params[k].data_ptr())
        if envmaps is not None:
            self.c.envmap = self.env_ptrs
            self.c.env_hw = self.env_hw
        self.c.n_views = len(self.cameras)
        self.c.cameras = self.cams_c
        self.n_pixels = sum(int(c.width) * int(c.height) for c in self.cameras)
        self.n = int(surfel_offset[-1])

    def view_slices(self):
        out, o = [], 0
        for c in self.cameras:
            n = int(c.width) * int(c.height)
            out.append((o, o + n, int(c.height), int(c.width)))
            o += n
        return out


class Renderer:
    """One libsurfsplat context (one stream at a time).

    check_capacity: after each forward outside graph capture, poll the device
    status (this synchronises the stream); when the surfels have moved so far
    that the reserved pair capacity was exceeded, reserve again and render
    again, so no truncated image is ever returned.  Under capture (or with
    check_capacity off) an overflow leaves NaN images and gradients and a
    status for ss_poll."""

    def __init__(self, options: Optional[Options] = None, lut: Optional[torch.Tensor] = None,
                 lut_size=(64, 64), lut_samples: int = 1024, check_capacity: bool = True):
        self.L = load_library()
        self.options = options or Options()
        self.check_capacity = check_capacity
        self.last_generation = 0
        self.ctx = ctypes.c_void_p()
        _check(self.L.ss_create(ctypes.byref(self.options.to_c()), ctypes.byref(self.ctx)), "ss_create")
        self.lut = None
        if self.options.shade == "splitsum":
            self.set_brdf_lut(lut if lut is not None else make_brdf_lut(*lut_size, lut_samples))

    def set_options(self, options: Options):
        self.options = options
        _check(self.L.ss_set_options(self.ctx, ctypes.byref(options.to_c())), "ss_set_options")
        if options.shade == "splitsum" and self.lut is None:
            self.set_brdf_lut(make_brdf_lut())

    def set_brdf_lut(self, lut: torch.Tensor):
        lut = lut.contiguous()
        n_r, n_nv = int(lut.shape[0]), int(lut.shape[1])
        _check(self.L.ss_set_brdf_lut(self.ctx, _ptr(lut), n_nv, n_r, _stream_ptr()), "ss_set_brdf_lut")
        self.lut = lut

    def close(self):
        if self.ctx:
            self.L.ss_destroy(self.ctx)
            self.ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def reserve(self, batch: Batch) -> int:
        ws = ctypes.c_size_t()
        _check(self.L.ss_reserve(self.ctx, ctypes.byref(batch.c), _stream_ptr(), ctypes.byref(ws)), "ss_reserve")
        return int(ws.value)

    def forward(self, batch: Batch, want_layers: bool = False, out=None, want_cons: bool = False,
                want_depth: bool = False):
        """Image [sum HW][3], alpha [sum HW] and layer counts (uint8, if
        want_layers).  With want_cons / want_depth (options.depth_stats needed) a
        fourth result, a dict with the per-pixel depth-consolidation term of
        eq:cons_loss ("cons") and the composited depth ("depth")."""
        dev = batch.params["position"].device
        aux = {}
        if out is None:
            image = torch.empty((batch.n_pixels, 3), device=dev, dtype=torch.float32)
            alpha = torch.empty((batch.n_pixels,), device=dev, dtype=torch.float32)
            nl = torch.empty((batch.n_pixels,), device=dev, dtype=torch.uint8) if want_layers else None
            for k, want in (("cons", want_cons), ("depth", want_depth)):
                if want:
                    aux[k] = torch.empty((batch.n_pixels,), device=dev, dtype=torch.float32)
        elif len(out) == 4:
            image, alpha, nl, aux = out
        else:
            image, alpha, nl = out
        gen = ctypes.c_int64(0)
        o = ss_outputs(image.data_ptr(), alpha.data_ptr(), None if nl is None else nl.data_ptr(),
                       _ptr(aux.get("cons")), _ptr(aux.get("depth")), ctypes.pointer(gen))
        _check(self.L.ss_render(self.ctx, ctypes.byref(batch.c), ctypes.byref(o), _stream_ptr()), "ss_render")
        if self.check_capacity and not torch.cuda.is_current_stream_capturing():
            d = self.poll()
            if d["device_status"] == SS_ERR_CAPACITY:
                self.reserve(batch)
                _check(self.L.ss_render(self.ctx, ctypes.byref(batch.c), ctypes.byref(o), _stream_ptr()),
                       "ss_render")
                d = self.poll()
            _check(d["device_status"], "ss_render (device)")
        self.last_generation = int(gen.value)
        return (image, alpha, nl, aux) if aux else (image, alpha, nl)

    def render_static(self, batch: Batch, out=None, want_layers: bool = False):
        """Forward through ss_render_static (no device allocation in the library:
        the workspace is its fixed per-GPU array).  Returns image, alpha and the
        layer counts (if want_layers); `out` may pass (image, alpha, n_layers)."""
        dev = batch.params["position"].device
        if out is None:
            image = torch.empty((batch.n_pixels, 3), device=dev, dtype=torch.float32)
            alpha = torch.empty((batch.n_pixels,), device=dev, dtype=torch.float32)
            nl = torch.empty((batch.n_pixels,), device=dev, dtype=torch.uint8) if want_layers else None
        else:
            image, alpha, nl = out
        o = ss_outputs(image.data_ptr(), alpha.data_ptr(), None if nl is None else nl.data_ptr(), None, None,
                       None)
        _check(self.L.ss_render_static(self.ctx, ctypes.byref(batch.c), ctypes.byref(o), _stream_ptr()),
               "ss_render_static")
        return image, alpha, nl

    def backward(self, batch: Batch, d_image: torch.Tensor, d_alpha: Optional[torch.Tensor] = None,
                 grads: Optional[dict] = None, want_envmap: bool = True, want_screen_grad: bool = False,
                 d_cons: Optional[torch.Tensor] = None, d_depth: Optional[torch.Tensor] = None,
                 generation: int = 0):
        """Parameter gradients of the last forward.  With want_screen_grad (or
        "screen_grad" / "visible_views" tensors in `grads`) also the
        densification statistic of Sec. 3.6.1: float32 [N] sum over views and
        pixels of |(dL_p/dT1z, dL_p/dT2z)| T4z and int32 [N] visible-view count.
        generation: the number the forward reported (0: the last forward); a
        stale one raises SurfsplatError (SS_ERR_STATE)."""
        dev = batch.params["position"].device
        if grads is None:
            grads = {k: torch.empty_like(batch.params[k]) for k in PARAMS}
            if batch.envmaps is not None and want_envmap:
                grads["envmap"] = [torch.empty_like(e) for e in batch.envmaps]
            if want_screen_grad:
                n = batch.params["position"].shape[1]
                grads["screen_grad"] = torch.empty(n, device=dev, dtype=torch.float32)
                grads["visible_views"] = torch.empty(n, device=dev, dtype=torch.int32)
        d_image = d_image.contiguous()
        d_alpha = None if d_alpha is None else d_alpha.contiguous()
        d_cons = None if d_cons is None else d_cons.contiguous()
        d_depth = None if d_depth is None else d_depth.contiguous()
        gi = ss_grad_in(d_image.data_ptr(), None if d_alpha is None else d_alpha.data_ptr(),
                        None if d_cons is None else d_cons.data_ptr(),
                        None if d_depth is None else d_depth.data_ptr(), int(generation))
        g = ss_grads()
        for k in PARAMS:
            setattr(g, "d_" + k, None if grads.get(k) is None else grads[k].data_ptr())
        for k in ("screen_grad", "visible_views"):
            setattr(g, k, None if grads.get(k) is None else grads[k].data_ptr())
        env_keep = None
        if grads.get("envmap") is not None:
            env_keep = (ctypes.c_void_p * len(grads["envmap"]))(*[e.data_ptr() for e in grads["envmap"]])
            g.d_envmap = env_keep
        _check(self.L.ss_render_backward(self.ctx, ctypes.byref(batch.c), ctypes.byref(gi), ctypes.byref(g),
                                         _stream_ptr()), "ss_render_backward")
        return grads

    def poll(self) -> dict:
        d = ss_diag()
        s = self.L.ss_poll(self.ctx, ctypes.byref(d))
        return dict(status=int(s), device_status=d.status, n_records=d.n_records, n_pairs=d.n_pairs,
                    pair_capacity=d.pair_capacity, workspace_bytes=d.workspace_bytes, generation=d.generation,
                    n_nonfinite=d.n_nonfinite, n_evaluated=d.n_evaluated, n_fragments=d.n_fragments,
                    n_layers=d.n_layers, sum_layer_weight=d.sum_layer_weight, static_status=d.static_status,
                    static_pairs=d.static_pairs, static_pair_capacity=d.static_pair_capacity)

    def profile(self, enable: bool = True):
        _check(self.L.ss_profile_enable(self.ctx, 1 if enable else 0), "ss_profile_enable")

    def profile_read(self) -> dict:
        """{stage: (total ms, launches)} since the previous read (synchronises)."""
        ms = (ctypes.c_double * len(STAGES))()
        cnt = (ctypes.c_int64 * len(STAGES))()
        _check(self.L.ss_profile_read(self.ctx, ms, cnt), "ss_profile_read")
        return {k: (ms[i], cnt[i]) for i, k in enumerate(STAGES)}

    def debug_binning(self, batch: Batch):
        """Binning of the last forward (test access): record keys and pixel
        rectangles, the sorted pair list and the per-tile ranges."""
        dev = batch.params["position"].device
        R = sum(int(batch.offsets[c.scene + 1] - batch.offsets[c.scene]) for c in batch.cameras)
        zb = torch.empty(R, dtype=torch.int32, device=dev)
        rect = torch.empty((R, 4), dtype=torch.int32, device=dev)
        np_ = ctypes.c_int64()
        nt = ctypes.c_int64()
        _check(self.L.ss_debug_binning(self.ctx, None, None, None, None, None, ctypes.byref(np_),
                                       ctypes.byref(nt), _stream_ptr()), "ss_debug_binning")
        keys = torch.empty(max(np_.value, 1), dtype=torch.int64, device=dev)
        vals = torch.empty(max(np_.value, 1), dtype=torch.int32, device=dev)
        ranges = torch.empty((max(nt.value, 1), 2), dtype=torch.int32, device=dev)
        _check(self.L.ss_debug_binning(self.ctx, _ptr(zb), _ptr(rect), _ptr(keys), _ptr(vals), _ptr(ranges),
                                       ctypes.byref(np_), ctypes.byref(nt), _stream_ptr()), "ss_debug_binning")
        n = np_.value
        return dict(rec_zbits=zb, rec_rect=rect, keys=keys[:n], vals=vals[:n], ranges=ranges[:nt.value])

    def debug_env_levels(self, batch: Batch, scene: int = 0):
        """Environment levels 1..6 of a scene as the last forward computed them
        (test access), flattened level by level, each [row][column][rgb]."""
        He, We = (int(x) for x in batch.envmaps[scene].shape[:2])
        n = 3 * sum(max(He >> l, 4) * max(We >> l, 8) for l in range(1, 6)) + 3 * 32 * 64
        out = torch.empty(n, dtype=torch.float32, device=batch.params["position"].device)
        _check(self.L.ss_debug_env_levels(self.ctx, scene, _ptr(out), n, _stream_ptr()), "ss_debug_env_levels")
        return out


def make_brdf_lut(n_nv: int = 64, n_r: int = 64, samples: int = 1024, device="cuda") -> torch.Tensor:
    """Split-sum BRDF table [n_r][n_nv][2] computed on the GPU (ss_brdf_lut)."""
    L = load_library()
    lut = torch.empty((n_r, n_nv, 2), dtype=torch.float32, device=device)
    _check(L.ss_brdf_lut(_ptr(lut), n_nv, n_r, samples, _stream_ptr()), "ss_brdf_lut")
    return lut


class SurfelRenderFunction(torch.autograd.Function):
    """image, alpha = render(surfel parameters, environment maps) with the
    hand-written adjoint of libsurfsplat as backward."""

    @staticmethod
    def forward(ctx, renderer: Renderer, offsets, cameras, position, normal, tangent, scale, albedo,
                roughness, metallic, *envmaps):
        params = dict(position=position.contiguous(), normal=normal.contiguous(),
                      tangent=tangent.contiguous(), scale=scale.contiguous(),
                      albedo=albedo.contiguous(), roughness=roughness.contiguous(),
                      metallic=metallic.contiguous())
        envs = [e.contiguous() for e in envmaps] if envmaps else None
        batch = Batch(params, offsets, cameras, envs)
        image, alpha, _ = renderer.forward(batch)
        ctx.renderer = renderer
        ctx.batch = batch
        ctx.n_env = len(envmaps)
        # the backward must find this forward's state (a second render through the
        # same renderer before backward replaces it: the library then refuses)
        ctx.generation = renderer.last_generation
        return image, alpha

    @staticmethod
    def backward(ctx, d_image, d_alpha):
        batch = ctx.batch
        if d_image is None:
            d_image = torch.zeros((batch.n_pixels, 3), device=batch.params["position"].device)
        g = ctx.renderer.backward(batch, d_image, d_alpha, want_envmap=ctx.n_env > 0, generation=ctx.generation)
        env = g.get("envmap") or []
        return (None, None, None, g["position"], g["normal"], g["tangent"], g["scale"], g["albedo"],
                g["roughness"], g["metallic"], *env)


def render(renderer: Renderer, params: dict, offsets, cameras, envmaps=None):
    """Differentiable render: returns (image [sum HW][3], alpha [sum HW])."""
    envs = list(envmaps) if envmaps else []
    return SurfelRenderFunction.apply(renderer, list(offsets), list(cameras),
                                      *[params[k] for k in PARAMS], *envs)
