"""FP64 CPU oracle of the differentiable EWA surfel rasterizer (test infrastructure).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It shares no code with the GPU renderer: the two meet
only in the seeded inputs of `scenegen`.

Functions follow the paper section by section (see oracle.cpp):
  * `envmap`            -- irradiance and GGX-prefiltered maps (eq:ibl, Sec. 3.4.2)
  * `envmap_adjoint`    -- transpose of that linear map
  * `brdf_lut`          -- split-sum (beta1, beta2) table (eq:ibl)
  * `bin_f32`           -- FP32 cull / depth key / tile rectangle (Sec. 3.2.1, App. A.1)
  * `records`           -- FP64 per-surfel quantities, FP64 cull rule and FP32 binning
  * `sorted_pairs`      -- reference tile lists sorted by (tile, z_start, record)
  * `render`            -- brute-force forward per pixel (Sec. 3.1-3.5, Alg. 1)
  * `render_jvp`        -- exact directional derivative (dual numbers)
  * `render_grad`       -- adjoint (reverse-mode tape)
Parity unpinned by the paper: the BRDF table, the environment-map conventions
and sigma_f, which are readings of silent points (see the tests for the
internal-consistency checks that pin them).
"""
from __future__ import annotations

import ctypes
import dataclasses
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

PARAM_NAMES = ["position", "normal", "tangent", "scale", "albedo", "roughness", "metallic"]
PARAM_ROWS = [3, 3, 3, 2, 3, 1, 1]


def lib():
    global _LIB
    if _LIB is None:
        # ORACLE_LIBRARY: another build of oracle.cpp (the sanitizer test's)
        path = os.environ.get("ORACLE_LIBRARY") or os.path.join(_HERE, "liboracle.so")
        if not os.path.exists(path):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        fpp = ctypes.POINTER(ctypes.c_void_p)
        L.orc_envmap_size.restype = ctypes.c_int
        L.orc_envmap_size.argtypes = [ctypes.c_int, ctypes.c_int]
        L.orc_envmap.argtypes = [dp, ctypes.c_int, ctypes.c_int, dp]
        L.orc_envmap_adjoint.argtypes = [dp, ctypes.c_int, ctypes.c_int, dp]
        L.orc_brdf_lut.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, dp]
        L.orc_set_threads.argtypes = [ctypes.c_int]
        L.orc_bin_f32.argtypes = [fpp, ctypes.c_int, dp, dp, ip, ctypes.POINTER(ctypes.c_uint32), ip, ip]
        L.orc_render.argtypes = [fpp, ctypes.c_int, dp, dp, dp, ctypes.c_int, ctypes.c_int, dp,
                                 ctypes.c_int, ctypes.c_int, ctypes.c_int, ip, dp, dp, ip, dp, dp, ip, dp, dp, ip, dp,
                                 ip]
        L.orc_records.argtypes = [fpp, ctypes.c_int, dp, dp, dp]
        L.orc_render_jvp.argtypes = [fpp, ctypes.c_int, fpp, dp, dp, dp, dp, ctypes.c_int, ctypes.c_int,
                                     dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ip, dp, dp, dp, dp, dp]
        L.orc_render_grad.argtypes = [fpp, ctypes.c_int, dp, dp, dp, ctypes.c_int, ctypes.c_int, dp,
                                      ctypes.c_int, ctypes.c_int, ctypes.c_int, ip, dp, dp, fpp, dp, dp, dp]
        L.orc_screen_grad.argtypes = [fpp, ctypes.c_int, dp, dp, dp, ctypes.c_int, ctypes.c_int, dp,
                                      ctypes.c_int, ctypes.c_int, ctypes.c_int, ip, dp, dp, dp, dp, ip, dp]
        L.orc_pixel_fragments.restype = ctypes.c_int
        L.orc_pixel_fragments.argtypes = [fpp, ctypes.c_int, dp, dp, dp, ctypes.c_int, ctypes.c_int, dp,
                                          ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                          ctypes.c_int, ip, dp, dp, dp, ip]
        _LIB = L
    return _LIB


@dataclasses.dataclass
class Options:
    r_cut: float = 3.0             # App. A.1
    gamma: float = 2.0 * math.pi   # eq:alpha, Sec. 3.5.1
    sigma_f: float = 0.1           # pixel prefilter variance (not given by the paper)
    k_max: int = 16                # App. A.1
    shade: str = "albedo"          # "albedo" | "splitsum" | "normal"
    tile_w: int = 16
    tile_h: int = 16
    mip: str = "centre"            # "centre" (Sec. 3.3.2) | "pixel" (per-pixel Jacobian, Sec. 3.3.1)
    t_min: float = 0.0             # transmittance early-out (0: off; the paper has none)
    tonemap: str = "linear"        # "linear" | "srgb_log" (log-space + sRGB transfer, eq:photo_loss)

    def pack(self):
        f = lambda x: float(np.float32(x))
        return np.array([f(self.r_cut), f(self.gamma), f(self.sigma_f), self.k_max,
                         {"albedo": 0, "splitsum": 1, "normal": 2}[self.shade], self.tile_w, self.tile_h,
                         {"centre": 0, "pixel": 1}[self.mip], f(self.t_min),
                         {"linear": 0, "srgb_log": 1}[self.tonemap]], np.float64)



def set_threads(n: int = 0) -> int:
    """OpenMP threads of the oracle's loops (n > 0 sets it); returns the count."""
    return int(lib().orc_set_threads(int(n)))

def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _iptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def pack_camera(cam) -> np.ndarray:
    f = lambda x: float(np.float32(x))
    out = np.zeros(22, np.float64)
    out[0], out[1] = cam.width, cam.height
    out[2:6] = [f(cam.fx), f(cam.fy), f(cam.cx), f(cam.cy)]
    out[6:15] = np.asarray(cam.R, np.float32).astype(np.float64).ravel()
    out[15:18] = np.asarray(cam.t, np.float32).astype(np.float64)
    out[18] = f(cam.znear)
    out[19:22] = [f(b) for b in cam.background]
    return out


class _Params:
    """Keeps the 7 float32 parameter arrays alive and exposes a void** to them."""

    def __init__(self, scene):
        self.arrs = [np.ascontiguousarray(getattr(scene, k), np.float32) for k in PARAM_NAMES]
        self.n = int(self.arrs[0].shape[1])
        self.ptrs = (ctypes.c_void_p * 7)(*[a.ctypes.data for a in self.arrs])

    @property
    def pp(self):
        return ctypes.cast(self.ptrs, ctypes.POINTER(ctypes.c_void_p))


def map_size(He, We) -> int:
    return int(lib().orc_envmap_size(He, We))


def map_layout(He, We):
    """[(H, W, offset)] for level 0 (= E), specular levels 1..5 and the irradiance map."""
    hs = [He] + [max(He >> l, 4) for l in range(1, 6)] + [32]
    ws = [We] + [max(We >> l, 8) for l in range(1, 6)] + [64]
    out, off = [], 0
    for h, w in zip(hs, ws):
        out.append((h, w, off))
        off += h * w * 3
    return out


def envmap(E: np.ndarray) -> np.ndarray:
    E = np.ascontiguousarray(E, np.float64)
    He, We = E.shape[:2]
    out = np.zeros(map_size(He, We), np.float64)
    lib().orc_envmap(_dptr(E), He, We, _dptr(out))
    return out


def envmap_adjoint(dmaps: np.ndarray, He: int, We: int) -> np.ndarray:
    dmaps = np.ascontiguousarray(dmaps, np.float64)
    dE = np.zeros((He, We, 3), np.float64)
    lib().orc_envmap_adjoint(_dptr(dmaps), He, We, _dptr(dE))
    return dE


def brdf_lut(n_nv: int = 64, n_r: int = 64, samples: int = 1024) -> np.ndarray:
    out = np.zeros((n_r, n_nv, 2), np.float64)
    lib().orc_brdf_lut(n_nv, n_r, samples, _dptr(out))
    return out


def bin_f32(scene, cam, opt: Options):
    P = _Params(scene)
    n = P.n
    keep = np.zeros(n, np.int32)
    zbits = np.zeros(n, np.uint32)
    rect = np.zeros((n, 4), np.int32)
    c = pack_camera(cam)
    o = opt.pack()
    lib().orc_bin_f32(P.pp, n, _dptr(c), _dptr(o), _iptr(keep),
                      zbits.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), _iptr(rect), None)
    return keep, zbits, rect


def pixel_rects(scene, cam, opt: Options):
    """Inclusive pixel rectangles (il, ih, jl, jh) of the FP32 binning, [n][4]."""
    P = _Params(scene)
    n = P.n
    keep = np.zeros(n, np.int32)
    zbits = np.zeros(n, np.uint32)
    rect = np.zeros((n, 4), np.int32)
    prect = np.zeros((n, 4), np.int32)
    c, o = pack_camera(cam), opt.pack()
    lib().orc_bin_f32(P.pp, n, _dptr(c), _dptr(o), _iptr(keep),
                      zbits.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), _iptr(rect), _iptr(prect))
    return prect


def sorted_pairs(keep, zbits, rect, tiles_x, tile_base=0, rec_base=0):
    """Reference tile lists: (key = tile << 32 | z_start bits, value = record), sorted."""
    idx = np.nonzero(keep)[0]
    tiles, recs, zs = [], [], []
    for i in idx:
        tx0, ty0, tx1, ty1 = rect[i]
        ty, tx = np.meshgrid(np.arange(ty0, ty1 + 1), np.arange(tx0, tx1 + 1), indexing="ij")
        t = (ty * tiles_x + tx).ravel() + tile_base
        tiles.append(t)
        recs.append(np.full(t.size, i + rec_base))
        zs.append(np.full(t.size, zbits[i]))
    if not tiles:
        return np.zeros(0, np.uint64), np.zeros(0, np.uint32)
    tiles = np.concatenate(tiles).astype(np.uint64)
    recs = np.concatenate(recs).astype(np.uint32)
    zs = np.concatenate(zs).astype(np.uint64)
    keys = (tiles << np.uint64(32)) | zs
    order = np.lexsort((recs, keys))
    return keys[order], recs[order]


def _maps_lut(maps, lut, He, We, opt):
    if opt.shade == "splitsum":
        # the C side indexes the map set by (He, We) and the table by its shape
        if maps is None or lut is None or He <= 0 or We <= 0:
            raise ValueError("split-sum shading needs maps, lut and env_hw")
        if np.size(maps) != lib().orc_envmap_size(int(He), int(We)):
            raise ValueError("maps do not match env_hw")
    if maps is None:
        maps = np.zeros(1, np.float64)
        He, We = 0, 0
    if lut is None:
        lut = np.zeros((2, 2, 2), np.float64)
    maps = np.ascontiguousarray(maps, np.float64)
    lut = np.ascontiguousarray(lut, np.float64)
    return maps, lut, He, We


def render(scene, cam, opt: Options, pix, maps=None, lut=None, env_hw=(0, 0)):
    """Forward at the listed pixels pix [K][2] (integer x, y); `cons` is the
    per-pixel depth-consolidation term of eq:cons_loss; `viol` the covering
    fragments (FP64 decisions) that the FP32 binning misses (culled surfel, or
    pixel outside its rectangle); `pp_drop`, `pp_drop_w` the count and weight sum
    of the fragments the per-pixel MIP filter would accept outside that
    rectangle (mip = "pixel" only); `n_frag` the fragments accumulated into
    the composited layers."""
    P = _Params(scene)
    pix = np.ascontiguousarray(pix, np.int32).reshape(-1, 2)
    k = pix.shape[0]
    maps, lut, He, We = _maps_lut(maps, lut, *env_hw, opt)
    img = np.zeros((k, 3), np.float64)
    alpha = np.zeros(k, np.float64)
    nl = np.zeros(k, np.int32)
    cm = np.zeros(k, np.float64)
    gm = np.zeros(k, np.float64)
    viol = np.zeros(k, np.int32)
    cons = np.zeros(k, np.float64)
    depth = np.zeros(k, np.float64)
    drop = np.zeros(k, np.int32)
    drop_w = np.zeros(k, np.float64)
    nfrag = np.zeros(k, np.int32)
    c, o = pack_camera(cam), opt.pack()
    lib().orc_render(P.pp, P.n, _dptr(c), _dptr(o), _dptr(maps), He, We, _dptr(lut),
                     lut.shape[1], lut.shape[0], k, _iptr(pix), _dptr(img), _dptr(alpha),
                     _iptr(nl), _dptr(cm), _dptr(gm), _iptr(viol), _dptr(cons), _dptr(depth), _iptr(drop),
                     _dptr(drop_w), _iptr(nfrag))
    return dict(image=img, alpha=alpha, n_layers=nl, cut_margin=cm, gap_margin=gm, viol=viol, cons=cons,
                depth=depth, pp_drop=drop, pp_drop_w=drop_w, n_frag=nfrag)


def records(scene, cam, opt: Options) -> dict:
    """Per-surfel FP64 quantities of one view: T rows, depth interval, the MIP
    filter (Sigma_mip^{-1}, Sigma_mip, n_f), the FP64 cull (keep64, margin =
    (minimum depth over the acceptance ellipse - znear) / c'_z) and the FP32
    binning (keep32, inclusive pixel rectangle il, ih, jl, jh, and stage32: 0-2
    culled (centre not beyond znear, degenerate projection, ellipse not entirely
    beyond znear), 3 empty rectangle, 4 kept)."""
    P = _Params(scene)
    out = np.zeros((P.n, 26), np.float64)
    c, o = pack_camera(cam), opt.pack()
    lib().orc_records(P.pp, P.n, _dptr(c), _dptr(o), _dptr(out))
    return dict(T1=out[:, 0:3], T2=out[:, 3:6], T4=out[:, 6:9], zs=out[:, 9], ze=out[:, 10],
                sinv=out[:, 11:14], sig=out[:, 14:17], nf=out[:, 17], keep64=out[:, 18] > 0,
                margin=out[:, 19], keep32=out[:, 20] > 0, rect=out[:, 21:25].astype(np.int64),
                stage32=out[:, 25].astype(np.int64))


def render_jvp(scene, cam, opt: Options, pix, direction: dict, maps=None, dmaps=None,
               lut=None, env_hw=(0, 0)):
    """Exact directional derivative of image, alpha and cons along `direction`
    (dict of parameter-name -> float64 array of the parameter's shape)."""
    P = _Params(scene)
    pix = np.ascontiguousarray(pix, np.int32).reshape(-1, 2)
    k = pix.shape[0]
    maps, lut, He, We = _maps_lut(maps, lut, *env_hw, opt)
    keep = []
    vp = (ctypes.c_void_p * 7)()
    for j, name in enumerate(PARAM_NAMES):
        if name in direction and direction[name] is not None:
            a = np.ascontiguousarray(direction[name], np.float64)
            keep.append(a)
            vp[j] = a.ctypes.data
        else:
            vp[j] = None
    dm = None if dmaps is None else np.ascontiguousarray(dmaps, np.float64)
    img = np.zeros((k, 3), np.float64)
    img_dot = np.zeros((k, 3), np.float64)
    a_dot = np.zeros(k, np.float64)
    c_dot = np.zeros(k, np.float64)
    z_dot = np.zeros(k, np.float64)
    c, o = pack_camera(cam), opt.pack()
    lib().orc_render_jvp(P.pp, P.n, ctypes.cast(vp, ctypes.POINTER(ctypes.c_void_p)), _dptr(c), _dptr(o),
                         _dptr(maps), _dptr(dm) if dm is not None else None, He, We, _dptr(lut),
                         lut.shape[1], lut.shape[0], k, _iptr(pix), _dptr(img), _dptr(img_dot), _dptr(a_dot),
                         _dptr(c_dot), _dptr(z_dot))
    return dict(image=img, image_dot=img_dot, alpha_dot=a_dot, cons_dot=c_dot, depth_dot=z_dot)


def render_grad(scene, cam, opt: Options, pix, dimage, dalpha=None, maps=None, lut=None,
                env_hw=(0, 0), dcons=None, ddepth=None):
    """Adjoint at the listed pixels (loss weights dimage [K][3], dalpha [K],
    dcons [K] on the depth-consolidation term and ddepth [K] on the composited
    depth): returns dict of parameter
    gradients (float64, parameter shapes) and `maps` (gradient w.r.t. the flat
    map set)."""
    P = _Params(scene)
    n = P.n
    pix = np.ascontiguousarray(pix, np.int32).reshape(-1, 2)
    k = pix.shape[0]
    maps, lut, He, We = _maps_lut(maps, lut, *env_hw, opt)
    dimage = np.ascontiguousarray(dimage, np.float64).reshape(k, 3)
    da = None if dalpha is None else np.ascontiguousarray(dalpha, np.float64).reshape(k)
    grads = [np.zeros((r, n) if r > 1 else (n,), np.float64) for r in PARAM_ROWS]
    gp = (ctypes.c_void_p * 7)(*[g.ctypes.data for g in grads])
    dmaps = np.zeros(maps.size, np.float64)
    dc = None if dcons is None else np.ascontiguousarray(dcons, np.float64).reshape(k)
    dz = None if ddepth is None else np.ascontiguousarray(ddepth, np.float64).reshape(k)
    c, o = pack_camera(cam), opt.pack()
    lib().orc_render_grad(P.pp, n, _dptr(c), _dptr(o), _dptr(maps), He, We, _dptr(lut),
                          lut.shape[1], lut.shape[0], k, _iptr(pix), _dptr(dimage),
                          _dptr(da) if da is not None else None,
                          ctypes.cast(gp, ctypes.POINTER(ctypes.c_void_p)), _dptr(dmaps),
                          _dptr(dc) if dc is not None else None, _dptr(dz) if dz is not None else None)
    out = dict(zip(PARAM_NAMES, grads))
    out["maps"] = dmaps
    return out


def screen_grad(scene, cam, opt: Options, pix, dimage, dalpha=None, maps=None, lut=None,
                env_hw=(0, 0), dcons=None):
    """Densification statistic (Sec. 3.6.1, eq:ss_grad) at the listed pixels:
    per surfel, `abs` = sum over pixels of |(dL_p/dT1z, dL_p/dT2z)| T4z, `vec` =
    the plain sum of those vectors ([2, n]), `visible` = culled-in with a
    non-empty tile rectangle in this view."""
    P = _Params(scene)
    n = P.n
    pix = np.ascontiguousarray(pix, np.int32).reshape(-1, 2)
    k = pix.shape[0]
    maps, lut, He, We = _maps_lut(maps, lut, *env_hw, opt)
    dimage = np.ascontiguousarray(dimage, np.float64).reshape(k, 3)
    da = None if dalpha is None else np.ascontiguousarray(dalpha, np.float64).reshape(k)
    a = np.zeros(n, np.float64)
    vec = np.zeros((2, n), np.float64)
    vis = np.zeros(n, np.int32)
    dc = None if dcons is None else np.ascontiguousarray(dcons, np.float64).reshape(k)
    c, o = pack_camera(cam), opt.pack()
    lib().orc_screen_grad(P.pp, n, _dptr(c), _dptr(o), _dptr(maps), He, We, _dptr(lut),
                          lut.shape[1], lut.shape[0], k, _iptr(pix), _dptr(dimage),
                          _dptr(da) if da is not None else None, _dptr(a), _dptr(vec), _iptr(vis),
                          None if dc is None else _dptr(dc))
    return dict(abs=a, vec=vec, visible=vis.astype(bool))


def pixel_fragments(scene, cam, opt: Options, px: int, py: int, maps=None, lut=None,
                    env_hw=(0, 0), cap: int = 4096):
    """Covering fragments of one pixel in visiting order: record index, z_start,
    z_end, weight, layer (-1 = discarded by the layer cap)."""
    P = _Params(scene)
    maps, lut, He, We = _maps_lut(maps, lut, *env_hw, opt)
    idx = np.zeros(cap, np.int32)
    zs, ze, w = (np.zeros(cap, np.float64) for _ in range(3))
    lay = np.zeros(cap, np.int32)
    c, o = pack_camera(cam), opt.pack()
    k = lib().orc_pixel_fragments(P.pp, P.n, _dptr(c), _dptr(o), _dptr(maps), He, We, _dptr(lut),
                                  lut.shape[1], lut.shape[0], px, py, cap, _iptr(idx), _dptr(zs),
                                  _dptr(ze), _dptr(w), _iptr(lay))
    k = min(k, cap)
    return dict(idx=idx[:k], zs=zs[:k], ze=ze[:k], w=w[:k], layer=lay[:k])


def all_pixels(cam) -> np.ndarray:
    ys, xs = np.meshgrid(np.arange(cam.height), np.arange(cam.width), indexing="ij")
    return np.stack([xs.ravel(), ys.ravel()], axis=1).astype(np.int32)
