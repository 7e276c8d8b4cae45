"""Split tile lists: lists longer than options.seg_len are walked as segments
in parallel and merged per pixel in list order (the z_max each segment enters
with comes from the segments before it).  At seg_len = 256 the small scenes
below split most tiles into several segments, with layer boundaries, the
16-layer cap and the transmittance early-out falling inside and across
segments.  Checked: oracle parity (image protocol, gradient protocol), the same
decisions as the unsplit walk (layer counts, accumulated fragments, layers),
images and gradients equal to the unsplit ones to FP32 summation order, and a
bitwise reproducible deterministic backward."""
import dataclasses

import numpy as np
import pytest

import scenegen as g
from conftest import axis_camera, make_scene
from parity_util import GRAD_REL_L2, assert_image_parity, rel_l2
from test_gpu_parity import O, _backward_case, _forward_case, all_pix, gpu_run, small_multiview, ss  # noqa: F401

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def stacked_planes():
    """20 tilted sparse planes one behind the other (more than K_max layers)."""
    cam = axis_camera(40, 40, 100.0)
    pos, nrm, tan, scl, alb = [], [], [], [], []
    rng = np.random.default_rng(0)
    th = np.radians(8.0)
    for k in range(20):
        gx, gy = np.meshgrid(np.arange(-4, 5) * 0.0317 + 0.0043 * k, np.arange(-4, 5) * 0.0317 - 0.0029 * k)
        n = gx.size
        pos.append(np.stack([gx.ravel(), gy.ravel() * np.cos(th), 2.0 + 0.05 * k + gy.ravel() * np.sin(th)], 1))
        nrm.append(np.tile([0, -np.sin(th), np.cos(th)], (n, 1)))
        tan.append(np.tile([1.0, 0, 0], (n, 1)))
        scl.append(np.full((n, 2), 0.02))
        alb.append(rng.uniform(0, 1, (n, 3)))
    return [make_scene(*[np.concatenate(x) for x in (pos, nrm, tan, scl, alb)])], [cam], "albedo"


def deep_stack():
    """90 planes of 3 x 3 wide surfels 0.03 apart in depth, each shifted
    sideways by up to 5 px about the corner the four 16 x 16 tiles share: a
    256-entry segment holds about 30 of them, so many pixels reach the 16-layer
    cap inside their first segment, others in a later one or never."""
    cam = axis_camera(32, 32, 100.0)
    pos, nrm, tan, scl, alb = [], [], [], [], []
    rng = np.random.default_rng(1)
    for k in range(90):
        th = np.radians(rng.uniform(-3.0, 3.0))
        ox, oy = rng.uniform(-0.1, 0.1, 2)
        gx, gy = np.meshgrid(np.arange(-1, 2) * 0.06 + ox, np.arange(-1, 2) * 0.06 + oy)
        n = gx.size
        pos.append(np.stack([gx.ravel(), gy.ravel() * np.cos(th), 2.0 + 0.03 * k + gy.ravel() * np.sin(th)], 1))
        nrm.append(np.tile([0, -np.sin(th), np.cos(th)], (n, 1)))
        tan.append(np.tile([1.0, 0, 0], (n, 1)))
        scl.append(np.full((n, 2), 0.05))
        alb.append(rng.uniform(0, 1, (n, 3)))
    return [make_scene(*[np.concatenate(x) for x in (pos, nrm, tan, scl, alb)])], [cam], "albedo"


def _case(name):
    if name == "stacked":
        return stacked_planes()
    if name == "deep":
        return deep_stack()
    if name == "tie_planes":
        w = g.tie_planes_workload()
        c = w.cameras[0]
        return w.scenes, [dataclasses.replace(c, cx=c.cx + 0.3183, cy=c.cy + 0.2718)], w.shade
    if name == "multiview":
        scenes, cams = small_multiview()
        return scenes, cams, "splitsum"
    w = g.two_spheres_workload(n_each=8000, width=200, height=150)
    return w.scenes, w.cameras, w.shade


def _lengths(ss, scenes, cams, opts):
    r = ss.Renderer(opts)
    b = ss.batch_from_scenes(scenes, cams)
    r.forward(b)
    rg = r.debug_binning(b)["ranges"].cpu().numpy().view(np.uint32).astype(np.int64).reshape(-1, 2)
    return rg[:, 1] - rg[:, 0]


@pytest.mark.parametrize("walk", ["rows", "records"])
@pytest.mark.parametrize("name", ["stacked", "deep", "tie_planes", "multiview", "two_spheres"])
def test_split_parity(O, ss, name, walk):
    scenes, cams, shade = _case(name)
    kw = dict(tile_w=16, tile_h=16, seg_len=256, bwd_walk=walk)
    L = _lengths(ss, scenes, cams, ss.Options(shade=shade, tile_w=16, tile_h=16, seg_len=256))
    kw["exact_ties"] = name == "tie_planes"
    assert (L > 256).sum() >= 2, L.max()      # several tiles are split
    rep = _forward_case(O, ss, scenes, cams, shade, lambda c, v: all_pix(c), **kw)
    print(name, "longest list", int(L.max()))
    assert_image_parity(rep)
    errs = _backward_case(O, ss, scenes, cams, shade, lambda c, v: all_pix(c), **kw)
    assert max(errs.values()) <= GRAD_REL_L2, errs


@pytest.mark.parametrize("name,t_min,k_max", [("stacked", 0.0, 16), ("stacked", 0.02, 16), ("deep", 0.0, 16),
                                              ("deep", 0.0, 5), ("deep", 1e-3, 16), ("tie_planes", 0.0, 16),
                                              ("multiview", 0.0, 16), ("two_spheres", 0.0, 16)])
def test_split_matches_unsplit(ss, name, t_min, k_max):
    """The same per-pixel decisions as the unsplit walk: identical layer counts
    and work counters (fragments, layers); images and gradients equal up to the
    FP32 summation order of layers that span a segment boundary."""
    scenes, cams, shade = _case(name)
    n_pix = sum(c.width * c.height for c in cams)
    rng = np.random.default_rng(3)
    G = rng.normal(size=(n_pix, 3))
    Ga = rng.normal(size=n_pix)
    out = []
    for seg in (256, -1):
        opts = ss.Options(shade=shade, tile_w=16, tile_h=16, seg_len=seg, counters=True, t_min=t_min, k_max=k_max)
        r, b, img, a, nl, gr = gpu_run(ss, scenes, cams, opts, G, Ga)
        out.append((img, a, nl, gr, r.poll()))
    (i0, a0, n0, g0, d0), (i1, a1, n1, g1, d1) = out
    assert np.array_equal(n0, n1)
    assert d0["n_fragments"] == d1["n_fragments"] and d0["n_layers"] == d1["n_layers"], (d0, d1)
    assert abs(d0["sum_layer_weight"] - d1["sum_layer_weight"]) <= 1e-5 * d1["sum_layer_weight"]
    np.testing.assert_allclose(i0, i1, rtol=1e-5, atol=1e-7)
    np.testing.assert_allclose(a0, a1, rtol=1e-5, atol=1e-7)
    pos = np.linalg.norm(g1["position"])
    for k in ("position", "normal", "scale", "albedo"):
        if np.linalg.norm(g1[k]) < 1e-6 * pos:
            continue
        assert rel_l2(g0[k], g1[k]) <= 1e-5, k


@pytest.mark.parametrize("walk", ["rows", "records"])
def test_split_deterministic_bitwise(ss, walk):
    scenes, cams, shade = _case("multiview")
    opts = ss.Options(shade=shade, tile_w=16, tile_h=16, seg_len=256, deterministic=True, bwd_walk=walk)
    b = ss.batch_from_scenes(scenes, cams)
    gen = torch.Generator("cuda").manual_seed(5)
    G = torch.randn((b.n_pixels, 3), device="cuda", generator=gen)
    runs = []
    for r in (ss.Renderer(opts), ss.Renderer(opts)):
        img, a, _ = r.forward(b)
        gr = r.backward(b, G)
        torch.cuda.synchronize()
        runs.append((img.clone(), {k: gr[k].clone() for k in ss.PARAMS}))
    assert torch.equal(runs[0][0], runs[1][0])
    for k in ss.PARAMS:
        assert torch.equal(runs[0][1][k], runs[1][1][k]), k
