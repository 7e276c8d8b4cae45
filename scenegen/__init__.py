"""Seeded synthetic surfel scenes, environment maps and cameras.

This module is the only code shared by the GPU renderer's tests/bench and the
CPU oracle.  It draws inputs; it holds none of the rendering method's
arithmetic (no projection, no kernel, no grouping, no shading).

The paper measures on a point-sampled Stanford Bunny and on Stanford-ORB
captures (Sec. 4, Sec. 4.3); neither is available here, so every scene below is
a seeded synthetic stand-in with the surfel counts, resolutions, scale
distributions and material distributions of the paper's workloads.

Layout of a scene (all float32, structure-of-arrays, N surfels):
    position [3][N], normal [3][N], tangent [3][N], scale [2][N],
    albedo [3][N], roughness [N], metallic [N], envmap [H_e][W_e][3] or None.
Cameras are pinhole, world->camera rotation R (row-major, OpenCV axes: x right,
y down, z forward), translation t, focal lengths and principal point in pixels.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

__all__ = [
    "Scene", "Camera", "Workload", "look_at_camera", "fibonacci_directions",
    "sphere_scene", "torus_scene", "superquadric_scene", "clustered_sphere_scene",
    "lognormal_envmap", "make_config", "CONFIG_NAMES", "plane_scene", "near_plane_workload",
    "tie_planes_workload", "two_spheres_workload", "occluded_planes_workload", "thin_shell_workload",
    "concat_scenes",
]


@dataclasses.dataclass
class Scene:
    position: np.ndarray
    normal: np.ndarray
    tangent: np.ndarray
    scale: np.ndarray
    albedo: np.ndarray
    roughness: np.ndarray
    metallic: np.ndarray
    envmap: Optional[np.ndarray] = None

    @property
    def n(self) -> int:
        return int(self.position.shape[1])

    def params(self):
        return dict(position=self.position, normal=self.normal, tangent=self.tangent,
                    scale=self.scale, albedo=self.albedo, roughness=self.roughness,
                    metallic=self.metallic)

    def subset(self, idx) -> "Scene":
        idx = np.asarray(idx)
        return Scene(self.position[:, idx].copy(), self.normal[:, idx].copy(),
                     self.tangent[:, idx].copy(), self.scale[:, idx].copy(),
                     self.albedo[:, idx].copy(), self.roughness[idx].copy(),
                     self.metallic[idx].copy(), self.envmap)


@dataclasses.dataclass
class Camera:
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    R: np.ndarray            # [3][3] world -> camera, row-major
    t: np.ndarray            # [3]
    znear: float = 0.01
    background: tuple = (0.0, 0.0, 0.0)
    scene: int = 0


@dataclasses.dataclass
class Workload:
    name: str
    scenes: List[Scene]
    cameras: List[Camera]
    shade: str                 # "albedo" or "splitsum"

    @property
    def pixel_views(self) -> int:
        return sum(c.width * c.height for c in self.cameras)

    @property
    def n_surfels(self) -> int:
        return sum(s.n for s in self.scenes)


def _rngs(seed: int, k: int):
    return [np.random.default_rng(s) for s in np.random.SeedSequence(seed).spawn(k)]


def _f32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float32))


def look_at_camera(eye, width, height, fov_y_deg=45.0, target=(0.0, 0.0, 0.0),
                   up=(0.0, 0.0, 1.0), scene=0, znear=0.01, background=(0.0, 0.0, 0.0)) -> Camera:
    """Pinhole camera looking at `target`; vertical field of view `fov_y_deg`."""
    eye = np.asarray(eye, np.float64)
    fwd = np.asarray(target, np.float64) - eye
    fwd /= np.linalg.norm(fwd)
    upv = np.asarray(up, np.float64)
    if abs(float(fwd @ upv)) > 0.99:
        upv = np.array([0.0, 1.0, 0.0])
    right = np.cross(fwd, upv)
    right /= np.linalg.norm(right)
    down = np.cross(fwd, right)
    R = np.stack([right, down, fwd])
    t = -R @ eye
    f = (height / 2.0) / math.tan(math.radians(fov_y_deg) / 2.0)
    return Camera(width, height, float(f), float(f), width / 2.0, height / 2.0,
                  _f32(R), _f32(t), znear, tuple(background), scene)


def fibonacci_directions(n: int) -> np.ndarray:
    i = np.arange(n, dtype=np.float64)
    z = 1.0 - (2.0 * i + 1.0) / n
    r = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    phi = i * math.pi * (3.0 - math.sqrt(5.0))
    return np.stack([r * np.cos(phi), r * np.sin(phi), z], axis=1)


def _tangent_from_normal(nrm: np.ndarray) -> np.ndarray:
    """e_x, or e_y where the normal is nearly parallel to e_x ([3][N])."""
    t = np.zeros_like(nrm)
    near = np.abs(nrm[0]) > 0.9
    t[0, ~near] = 1.0
    t[1, near] = 1.0
    return t


def _inplane_tangent(nrm: np.ndarray, angle: np.ndarray) -> np.ndarray:
    """A unit tangent at `angle` in the plane orthogonal to `nrm` ([3][N])."""
    a = _tangent_from_normal(nrm)
    a = a - (a * nrm).sum(0) * nrm
    a /= np.linalg.norm(a, axis=0)
    b = np.cross(nrm.T, a.T).T
    return np.cos(angle) * a + np.sin(angle) * b


def _svbrdf(rng, n):
    albedo = rng.uniform(0.0, 1.0, size=(3, n))
    rough = rng.uniform(0.05, 1.0, size=n)
    metal = (rng.uniform(0.0, 1.0, size=n) < 0.3).astype(np.float64)
    return albedo, rough, metal


def lognormal_envmap(seed: int, h: int, w: int, sigma: float = 1.5) -> np.ndarray:
    rng = _rngs(seed + 7919, 1)[0]
    return _f32(np.exp(rng.normal(0.0, sigma, size=(h, w, 3))))


def sphere_scene(seed: int, n: int, scale: float = 0.02, svbrdf: bool = False) -> Scene:
    """Uniform points on the unit sphere, radial normals, isotropic scale."""
    r_pos, r_alb, r_mat = _rngs(seed, 3)
    p = r_pos.normal(size=(3, n))
    p /= np.linalg.norm(p, axis=0)
    nrm = p.copy()
    tan = _tangent_from_normal(nrm)
    scl = np.full((2, n), scale)
    if svbrdf:
        alb, rough, metal = _svbrdf(r_mat, n)
    else:
        alb = r_alb.uniform(0.0, 1.0, size=(3, n))
        rough = np.full(n, 0.5)
        metal = np.zeros(n)
    return Scene(_f32(p), _f32(nrm), _f32(tan), _f32(scl), _f32(alb), _f32(rough), _f32(metal))


def _displacement(rng):
    a = int(rng.integers(3, 9))
    b = int(rng.integers(2, 6))
    p1, p2 = rng.uniform(0.0, 2.0 * math.pi, size=2)
    return a, b, p1, p2


def _param_normals(fn, u, v, eps=1e-5):
    """Unit normals of a parametric surface fn(u, v) -> [3][N] by central differences."""
    du = (fn(u + eps, v) - fn(u - eps, v)) / (2 * eps)
    dv = (fn(u, v + eps) - fn(u, v - eps)) / (2 * eps)
    nrm = np.cross(du.T, dv.T).T
    return nrm / np.linalg.norm(nrm, axis=0)


def torus_scene(seed: int, n: int = 200_000, R: float = 1.0, r: float = 0.35,
                amp: float = 0.02, scale_mu=math.log(0.008), scale_sigma=0.3) -> Scene:
    """Area-uniform surfels on a displaced torus (axis z), anisotropic scales, SVBRDF."""
    r_pos, r_disp, r_ang, r_scl, r_mat = _rngs(seed, 5)
    a, b, p1, p2 = _displacement(r_disp)
    th = np.empty(0)
    ph = np.empty(0)
    while th.size < n:      # rejection on the area element (R + r cos phi)/(R + r)
        m = 2 * (n - th.size) + 1024
        t_ = r_pos.uniform(0.0, 2 * math.pi, m)
        f_ = r_pos.uniform(0.0, 2 * math.pi, m)
        keep = r_pos.uniform(0.0, 1.0, m) < (R + r * np.cos(f_)) / (R + r)
        th = np.concatenate([th, t_[keep]])
        ph = np.concatenate([ph, f_[keep]])
    th, ph = th[:n], ph[:n]

    def surf(t_, f_):
        rr = r + amp * np.sin(a * t_ + p1) * np.sin(b * f_ + p2)
        return np.stack([(R + rr * np.cos(f_)) * np.cos(t_),
                         (R + rr * np.cos(f_)) * np.sin(t_),
                         rr * np.sin(f_)])
    pos = surf(th, ph)
    nrm = _param_normals(surf, th, ph)
    # orient outward (away from the tube centre line)
    ctr = np.stack([R * np.cos(th), R * np.sin(th), np.zeros_like(th)])
    flip = ((pos - ctr) * nrm).sum(0) < 0
    nrm[:, flip] *= -1
    tan = _inplane_tangent(nrm, r_ang.uniform(0.0, math.pi, n))
    scl = np.exp(r_scl.normal(scale_mu, scale_sigma, size=(2, n)))
    alb, rough, metal = _svbrdf(r_mat, n)
    return Scene(_f32(pos), _f32(nrm), _f32(tan), _f32(scl), _f32(alb), _f32(rough), _f32(metal))


def _spow(x, e):
    return np.sign(x) * np.abs(x) ** e


class _Superquadric:
    def __init__(self, rng):
        self.ax = rng.uniform(0.25, 0.6, size=3)
        self.e1, self.e2 = rng.uniform(0.3, 1.8, size=2)
        self.c = rng.uniform(-0.5, 0.5, size=3)
        q = rng.normal(size=4)
        q /= np.linalg.norm(q)
        w, x, y, z = q
        self.Rm = np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
                            [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
                            [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])

    def local(self, eta, om):
        a1, a2, a3 = self.ax
        ce, se = np.cos(eta), np.sin(eta)
        return np.stack([a1 * _spow(ce, self.e1) * _spow(np.cos(om), self.e2),
                         a2 * _spow(ce, self.e1) * _spow(np.sin(om), self.e2),
                         a3 * _spow(se, self.e1)])

    def world(self, eta, om):
        return self.Rm @ self.local(eta, om) + self.c[:, None]

    def implicit(self, pw):
        pl = self.Rm.T @ (pw - self.c[:, None])
        x, y, z = np.abs(pl[0]) / self.ax[0], np.abs(pl[1]) / self.ax[1], np.abs(pl[2]) / self.ax[2]
        return (x ** (2 / self.e2) + y ** (2 / self.e2)) ** (self.e2 / self.e1) + z ** (2 / self.e1)

    def grad(self, pw):
        """Gradient of the implicit function in world space ([3][N])."""
        pl = self.Rm.T @ (pw - self.c[:, None])
        a1, a2, a3 = self.ax
        e1, e2 = self.e1, self.e2
        x, y, z = pl[0] / a1, pl[1] / a2, pl[2] / a3
        ax_, ay_, az_ = np.maximum(np.abs(x), 1e-12), np.maximum(np.abs(y), 1e-12), np.maximum(np.abs(z), 1e-12)
        s = ax_ ** (2 / e2) + ay_ ** (2 / e2)
        g = (e2 / e1) * s ** (e2 / e1 - 1)
        gx = g * (2 / e2) * ax_ ** (2 / e2 - 1) * np.sign(x) / a1
        gy = g * (2 / e2) * ay_ ** (2 / e2 - 1) * np.sign(y) / a2
        gz = (2 / e1) * az_ ** (2 / e1 - 1) * np.sign(z) / a3
        return self.Rm @ np.stack([gx, gy, gz])

    def area_density(self, eta, om, eps=1e-5):
        du = (self.local(eta + eps, om) - self.local(eta - eps, om)) / (2 * eps)
        dv = (self.local(eta, om + eps) - self.local(eta, om - eps)) / (2 * eps)
        return np.linalg.norm(np.cross(du.T, dv.T), axis=1)


def superquadric_scene(seed: int, n: int = 1_000_000, k: int = 5,
                       scale_mu=math.log(0.004), scale_sigma=0.5) -> Scene:
    """Union of k seeded superquadrics, area-uniform, interior points removed."""
    r_shape, r_pos, r_ang, r_scl, r_mat, r_mix = _rngs(seed, 6)
    sq = [_Superquadric(r_shape) for _ in range(k)]
    # surface-area estimate and density bound per superquadric on a parameter grid
    eg = np.linspace(-math.pi / 2 + 1e-3, math.pi / 2 - 1e-3, 256)
    og = np.linspace(-math.pi, math.pi, 512)
    E, O = np.meshgrid(eg, og, indexing="ij")
    dens_max, area = [], []
    for s in sq:
        d = s.area_density(E.ravel(), O.ravel())
        dens_max.append(float(np.percentile(d, 99.9)))
        area.append(float(d.mean() * math.pi * 2 * math.pi))
    area = np.asarray(area)
    pts, nrms = [], []
    got = 0
    while got < n:
        need = n - got
        for i, s in enumerate(sq):
            m = int(need * area[i] / area.sum() * 1.6) + 256
            eta = r_pos.uniform(-math.pi / 2, math.pi / 2, m)
            om = r_pos.uniform(-math.pi, math.pi, m)
            d = s.area_density(eta, om)
            keep = r_pos.uniform(0.0, dens_max[i], m) < d
            p = s.world(eta[keep], om[keep])
            inside = np.zeros(p.shape[1], bool)
            for j, o in enumerate(sq):
                if j != i:
                    inside |= o.implicit(p) < 1.0
            p = p[:, ~inside]
            g = s.grad(p)
            g /= np.linalg.norm(g, axis=0)
            pts.append(p)
            nrms.append(g)
            got += p.shape[1]
    pos = np.concatenate(pts, axis=1)
    nrm = np.concatenate(nrms, axis=1)
    sel = r_mix.permutation(pos.shape[1])[:n]
    pos, nrm = pos[:, sel], nrm[:, sel]
    tan = _inplane_tangent(nrm, r_ang.uniform(0.0, math.pi, n))
    scl = np.exp(r_scl.normal(scale_mu, scale_sigma, size=(2, n)))
    alb, rough, metal = _svbrdf(r_mat, n)
    return Scene(_f32(pos), _f32(nrm), _f32(tan), _f32(scl), _f32(alb), _f32(rough), _f32(metal))


def clustered_sphere_scene(seed: int, n: int = 3_000_000, clusters: int = 10, frac: float = 0.7,
                           std: float = 0.05, amp: float = 0.02,
                           scale_mu=math.log(0.002), scale_sigma=0.8) -> Scene:
    """Displaced unit sphere; `frac` of the surfels in tangent-Gaussian clusters."""
    r_c, r_pos, r_disp, r_ang, r_scl, r_mat = _rngs(seed, 6)
    a, b, p1, p2 = _displacement(r_disp)
    nc = int(round(n * frac))
    cen = r_c.normal(size=(3, clusters))
    cen /= np.linalg.norm(cen, axis=0)
    lab = r_pos.integers(0, clusters, nc)
    c = cen[:, lab]
    off = r_pos.normal(0.0, std, size=(3, nc))
    off -= (off * c).sum(0) * c                    # tangent-plane Gaussian
    d1 = c + off
    d1 /= np.linalg.norm(d1, axis=0)               # reproject to the sphere
    d2 = r_pos.normal(size=(3, n - nc))
    d2 /= np.linalg.norm(d2, axis=0)
    dirs = np.concatenate([d1, d2], axis=1)
    th = np.arccos(np.clip(dirs[2], -1, 1))
    ph = np.arctan2(dirs[1], dirs[0])

    def surf(t_, f_):
        rr = 1.0 + amp * np.sin(a * t_ + p1) * np.sin(b * f_ + p2)
        return rr * np.stack([np.sin(t_) * np.cos(f_), np.sin(t_) * np.sin(f_), np.cos(t_)])
    th = np.clip(th, 1e-4, math.pi - 1e-4)
    pos = surf(th, ph)
    nrm = _param_normals(surf, th, ph)
    flip = (nrm * pos).sum(0) < 0
    nrm[:, flip] *= -1
    tan = _inplane_tangent(nrm, r_ang.uniform(0.0, math.pi, n))
    scl = np.exp(r_scl.normal(scale_mu, scale_sigma, size=(2, n)))
    alb, rough, metal = _svbrdf(r_mat, n)
    return Scene(_f32(pos), _f32(nrm), _f32(tan), _f32(scl), _f32(alb), _f32(rough), _f32(metal))


def plane_scene(n_side: int, spacing: float, scale: float, z: float = 0.0, extent=None,
                color=None, seed: int = 0, jitter: float = 0.0) -> Scene:
    """A square lattice of fronto-parallel (normal +z) isotropic surfels in the plane z."""
    rng = _rngs(seed, 2)
    g = (np.arange(n_side) - (n_side - 1) / 2.0) * spacing
    X, Y = np.meshgrid(g, g, indexing="ij")
    n = X.size
    pos = np.stack([X.ravel(), Y.ravel(), np.full(n, z)])
    if jitter:
        pos[2] += rng[0].uniform(-jitter, jitter, n)
    nrm = np.zeros((3, n))
    nrm[2] = 1.0
    tan = np.zeros((3, n))
    tan[0] = 1.0
    scl = np.full((2, n), scale)
    if color is None:
        alb = rng[1].uniform(0, 1, size=(3, n))
    else:
        alb = np.tile(np.asarray(color, np.float64)[:, None], (1, n))
    return Scene(_f32(pos), _f32(nrm), _f32(tan), _f32(scl), _f32(alb),
                 _f32(np.full(n, 0.5)), _f32(np.zeros(n)))


def checkerboard_workload(n_side: int = 2000, extent: float = 10.0, square: float = 0.2,
                          width: int = 800, height: int = 600, eye=(0.0, -10.6, 0.45),
                          target=(0.0, 0.0, 0.0)) -> "Workload":
    """Anti-aliasing test scene: a ground plane z = 0 sampled on an n_side^2 lattice
    over [-extent, extent]^2 (4M surfels by default), isotropic scale = spacing,
    black/white checkerboard albedo of the given square size, seen from a low
    camera so that the plane recedes to the horizon (minification from ~0.1 to
    many surfels per pixel within one frame)."""
    spacing = 2.0 * extent / n_side
    sc = plane_scene(n_side, spacing, spacing, color=(0.0, 0.0, 0.0))
    x, y = sc.position[0].astype(np.float64), sc.position[1].astype(np.float64)
    white = (np.floor(x / square) + np.floor(y / square)).astype(np.int64) % 2 == 0
    sc.albedo = _f32(np.tile(white.astype(np.float64), (3, 1)))
    cam = look_at_camera(eye, width, height, target=target)
    return Workload("checkerboard", [sc], [cam], "albedo")


def concat_scenes(*scenes: Scene) -> Scene:
    """One scene holding the surfels of several (in order); the envmap of the first."""
    cat = lambda k: _f32(np.concatenate([np.asarray(getattr(s, k)) for s in scenes], axis=-1))
    return Scene(cat("position"), cat("normal"), cat("tangent"), cat("scale"), cat("albedo"),
                 cat("roughness"), cat("metallic"), scenes[0].envmap)


def _axis_camera(width, height, f, znear=0.01, background=(0.0, 0.0, 0.0), eye=(0.0, 0.0, 0.0)):
    """Pinhole camera at `eye` looking down +z (R = I)."""
    R = np.eye(3)
    return Camera(width, height, float(f), float(f), width / 2.0, height / 2.0, _f32(R),
                  _f32(-np.asarray(eye, np.float64)), znear, tuple(background), 0)


def near_plane_workload(seed: int = 61, n: int = 3000, width: int = 96, height: int = 80,
                        f: float = 80.0, znear: float = 0.25) -> Workload:
    """Surfels close to the camera: centres at depths U[0.6 znear, 6 znear] and
    lateral positions up to 1.3x the half field of view, random orientations and
    lognormal(ln 0.04, 0.5) scales, so that many straddle the near plane, lie
    partly behind the camera or cross the image border.  SVBRDF and a 16 x 32
    environment; camera at the origin looking down +z with the given znear."""
    r_pos, r_nrm, r_ang, r_scl, r_mat, r_env = _rngs(seed, 6)
    z = r_pos.uniform(0.6 * znear, 6.0 * znear, n)
    hx, hy = 1.3 * (width / 2.0) / f, 1.3 * (height / 2.0) / f
    x = r_pos.uniform(-hx, hx, n) * z
    y = r_pos.uniform(-hy, hy, n) * z
    nrm = r_nrm.normal(size=(3, n))
    nrm /= np.linalg.norm(nrm, axis=0)
    tan = _inplane_tangent(nrm, r_ang.uniform(0, math.pi, n))
    scl = np.exp(r_scl.normal(math.log(0.04), 0.5, size=(2, n)))
    alb, rough, metal = _svbrdf(r_mat, n)
    sc = Scene(_f32(np.stack([x, y, z])), _f32(nrm), _f32(tan), _f32(scl), _f32(alb), _f32(rough), _f32(metal))
    sc.envmap = lognormal_envmap(seed, 16, 32)
    cam = _axis_camera(width, height, f, znear=znear, background=(0.1, 0.2, 0.3))
    return Workload("near_plane", [sc], [cam], "splitsum")


def tie_planes_workload(width: int = 80, height: int = 64, f: float = 90.0, spacing: float = 0.03,
                        scale: float = 0.03, z: float = 2.0, gap: float = 0.5) -> Workload:
    """Adversarial ties of the depth sort: camera at the origin looking down +z at
    fronto-parallel surfels (normal -z, tangent +x), whose depth intervals have
    zero extent, so every surfel of a plane has exactly the same z_start.  Two
    interleaved lattices (red, and blue offset by half a spacing) share the plane
    z; a green lattice at z + gap lies behind them."""
    def lat(off, zz, col, half):
        g = (np.arange(-half, half + 1)) * spacing + off
        X, Y = np.meshgrid(g, g, indexing="ij")
        k = X.size
        pos = np.stack([X.ravel() * zz / z, Y.ravel() * zz / z, np.full(k, zz)])
        nrm = np.tile(np.array([[0.0], [0.0], [-1.0]]), (1, k))
        tan = np.tile(np.array([[1.0], [0.0], [0.0]]), (1, k))
        alb = np.tile(np.asarray(col, np.float64)[:, None], (1, k))
        return Scene(_f32(pos), _f32(nrm), _f32(tan), _f32(np.full((2, k), scale * zz / z)), _f32(alb),
                     _f32(np.full(k, 0.5)), _f32(np.zeros(k)))
    half = int(0.55 * width / f * z / spacing) + 1
    sc = concat_scenes(lat(0.0, z, (1.0, 0.1, 0.1), half), lat(0.5 * spacing, z, (0.1, 0.1, 1.0), half),
                       lat(0.25 * spacing, z + gap, (0.1, 1.0, 0.1), half))
    return Workload("tie_planes", [sc], [_axis_camera(width, height, f)], "albedo")


def _sphere_points(rng_pos, rng_ang, centre, radius, n):
    p = rng_pos.normal(size=(3, n))
    p /= np.linalg.norm(p, axis=0)
    tan = _inplane_tangent(p, rng_ang.uniform(0, math.pi, n))
    return np.asarray(centre, np.float64)[:, None] + radius * p, p, tan


def two_spheres_workload(seed: int = 71, n_each: int = 20_000, width: int = 800, height: int = 600,
                         scale: float = None, shade: str = "albedo") -> Workload:
    """The inter-object edge scene of Sec. 4.4.3: two overlapping point-sampled
    unit spheres, the rear one offset to the right, so that the front
    silhouette, the rear silhouette and the overlap where the front sphere
    occludes the rear one are all in view.  Radial normals; isotropic scale
    about the mean surfel spacing (default 1.2 sqrt(4 pi / n_each)); a warm
    front sphere and a cool rear one (uniform per-surfel albedo jitter).
    Camera 45 deg vertical FOV, looking at the pair from distance 4.5."""
    r = _rngs(seed, 6)
    s = 1.2 * math.sqrt(4 * math.pi / n_each) if scale is None else scale
    pa, na, ta = _sphere_points(r[0], r[1], (-0.35, 0.0, 0.0), 0.6, n_each)
    pb, nb, tb = _sphere_points(r[2], r[3], (0.45, 0.5, 0.1), 0.6, n_each)
    ca = np.clip(np.array([[0.9], [0.5], [0.2]]) + r[4].uniform(-0.1, 0.1, (3, n_each)), 0, 1)
    cb = np.clip(np.array([[0.2], [0.4], [0.9]]) + r[5].uniform(-0.1, 0.1, (3, n_each)), 0, 1)
    mk = lambda p, nn, t, c: Scene(_f32(p), _f32(nn), _f32(t), _f32(np.full((2, n_each), s)), _f32(c),
                                   _f32(np.full(n_each, 0.4)), _f32(np.zeros(n_each)))
    sc = concat_scenes(mk(pa, na, ta, ca), mk(pb, nb, tb, cb))
    if shade == "splitsum":
        sc.envmap = lognormal_envmap(seed, 16, 32)
    cam = look_at_camera((0.0, -4.5, 0.3), width, height, target=(0.05, 0.25, 0.05))
    return Workload("two_spheres", [sc], [cam], shade)


def occluded_planes_workload(width: int = 72, height: int = 60, f: float = 80.0, seed: int = 81) -> Workload:
    """A dense, opaque front plane (spacing s/3, accumulated weight far above the
    opacity saturation) over a sparser second plane, both slightly tilted and
    jittered, random albedo; the back plane is wider, so it is visible around the
    front one."""
    r = _rngs(seed, 4)
    th = math.radians(10.0)

    def plane(z, spacing, s, extent, rng):
        g = np.arange(-extent, extent + 1e-9, spacing)
        X, Y = np.meshgrid(g, g, indexing="ij")
        k = X.size
        X = X.ravel() + rng.uniform(-0.2, 0.2, k) * spacing
        Y = Y.ravel() + rng.uniform(-0.2, 0.2, k) * spacing
        pos = np.stack([X, Y * math.cos(th), z + Y * math.sin(th)])
        nrm = np.tile(np.array([[0.0], [math.sin(th)], [-math.cos(th)]]), (1, k))
        tan = np.tile(np.array([[1.0], [0.0], [0.0]]), (1, k))
        return Scene(_f32(pos), _f32(nrm), _f32(tan), _f32(np.full((2, k), s)),
                     _f32(rng.uniform(0, 1, (3, k))), _f32(np.full(k, 0.5)), _f32(np.zeros(k)))
    front = plane(2.0, 0.01, 0.03, 0.5, r[0])
    back = plane(2.6, 0.04, 0.04, 1.2, r[1])
    cam = _axis_camera(width, height, f, background=(0.3, 0.3, 0.3))
    return Workload("occluded_planes", [concat_scenes(front, back)], [cam], "albedo")


def thin_shell_workload(width: int = 72, height: int = 60, f: float = 80.0, seed: int = 91,
                        sep: float = 0.02) -> Workload:
    """Two near-parallel tilted layers separated by `sep` along the view axis, less
    than their surfels' depth extent (the thin-shell limitation of Sec. 5: the
    interval merge fuses them into one layer), plus a third layer well behind;
    lattice spacing about the surfel scale, random albedo."""
    r = _rngs(seed, 3)
    th = math.radians(35.0)

    def layer(z, rng, off):
        g = np.arange(-0.6, 0.6 + 1e-9, 0.025) + off
        X, Y = np.meshgrid(g, g, indexing="ij")
        k = X.size
        pos = np.stack([X.ravel(), Y.ravel() * math.cos(th), z + Y.ravel() * math.sin(th)])
        nrm = np.tile(np.array([[0.0], [math.sin(th)], [-math.cos(th)]]), (1, k))
        tan = np.tile(np.array([[1.0], [0.0], [0.0]]), (1, k))
        return Scene(_f32(pos), _f32(nrm), _f32(tan), _f32(np.full((2, k), 0.025)),
                     _f32(rng.uniform(0, 1, (3, k))), _f32(np.full(k, 0.5)), _f32(np.zeros(k)))
    sc = concat_scenes(layer(2.0, r[0], 0.0), layer(2.0 + sep, r[1], 0.0123), layer(2.5, r[2], 0.007))
    return Workload("thin_shell", [sc], [_axis_camera(width, height, f)], "albedo")


CONFIG_NAMES = ["C1", "C2", "C3", "C4", "C5"]


def make_config(name: str, n_scale: float = 1.0, res_scale: float = 1.0, views=None) -> Workload:
    """The five synthetic workloads.

    C1: 4,096 surfels on the unit sphere, isotropic scale 0.02, albedo only,
        one 128x128 view from distance 3 (45 deg vertical FOV).
    C2: 200k surfels on a displaced torus, anisotropic lognormal scales, SVBRDF,
        64x128 lognormal(0, 1.5) environment, one 512x512 view.
    C3: 1M surfels on a union of 5 superquadrics, 128x256 environment,
        8 views of 800x800 on a sphere of radius 3.
    C4: 3M surfels, density-clustered displaced sphere, one 1920x1080 view.
    C5: four scenes (50k, 300k, 1M, 2M) with 16 views from 256^2 to 1024^2.
    `n_scale`/`res_scale` shrink a workload for tests; 1.0 is the full size.
    """
    def N(x):
        return max(64, int(round(x * n_scale)))

    def P(x):
        return max(16, int(round(x * res_scale)))
    if name == "C1":
        sc = sphere_scene(1, N(4096), 0.02)
        cams = [look_at_camera((0.0, -3.0, 0.0), P(128), P(128))]
        return Workload(name, [sc], cams, "albedo")
    if name == "C2":
        sc = torus_scene(2, N(200_000))
        sc.envmap = lognormal_envmap(2, 64, 128)
        el = math.radians(30.0)
        eye = (0.0, -3.0 * math.cos(el), 3.0 * math.sin(el))
        cams = [look_at_camera(eye, P(512), P(512))]
        return Workload(name, [sc], cams, "splitsum")
    if name == "C3":
        sc = superquadric_scene(3, N(1_000_000))
        sc.envmap = lognormal_envmap(3, 128, 256)
        nv = 8 if views is None else views
        cams = [look_at_camera(3.0 * d, P(800), P(800)) for d in fibonacci_directions(nv)]
        return Workload(name, [sc], cams, "splitsum")
    if name == "C4":
        sc = clustered_sphere_scene(4, N(3_000_000))
        sc.envmap = lognormal_envmap(4, 128, 256)
        el = math.radians(30.0)
        eye = (0.0, -3.0 * math.cos(el), 3.0 * math.sin(el))
        cams = [look_at_camera(eye, P(1920), P(1080))]
        return Workload(name, [sc], cams, "splitsum")
    if name == "C5":
        s0 = sphere_scene(51, N(50_000), 0.02, svbrdf=True)
        s1 = torus_scene(52, N(300_000))
        s2 = superquadric_scene(53, N(1_000_000))
        s3 = superquadric_scene(54, N(2_000_000))
        scenes = [s0, s1, s2, s3]
        for i, s in enumerate(scenes):
            s.envmap = lognormal_envmap(55 + i, 128, 256)
        res = [256, 512, 768, 1024]
        dirs = fibonacci_directions(16)
        cams = []
        for v in range(16):
            si = v // 4
            r = P(res[v % 4])
            cams.append(look_at_camera(3.0 * dirs[v], r, r, scene=si))
        return Workload(name, scenes, cams, "splitsum")
    raise ValueError(f"unknown workload {name!r}")
