"""The allocation-free forward (ss_render_static, for callers that cannot
allocate device memory) against ss_render, through the C ABI.

Forward images are deterministic (every pixel sums its fragments in list
order) and the allocation-free path never splits long tile lists, so against
ss_render with unsplit lists the two entry points must agree bit for bit.  Two calls in a row,
the second with a smaller batch (and another shading mode), check that the
shared fixed workspace is cleared and re-laid out per call."""
import ctypes
import math

import numpy as np
import pytest

import scenegen as g

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ss():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_2605_05876_amd as m
    m.load_library()
    return m


def _splitsum_case():
    sc = g.torus_scene(22, 20_000, scale_mu=math.log(0.02), scale_sigma=0.3)
    sc.envmap = g.lognormal_envmap(22, 16, 32)
    el = math.radians(30.0)
    cams = [g.look_at_camera((0.0, -3.0 * math.cos(el), 3.0 * math.sin(el)), 96, 96),
            g.look_at_camera((3.0, 0.0, 0.4), 80, 64)]
    return [sc], cams, "splitsum"


def _albedo_case():
    w = g.make_config("C1", n_scale=0.5, res_scale=0.5)   # 2048 surfels, 64 x 64
    return w.scenes, w.cameras, "albedo"


def _compare(ss, scenes, cams, shade):
    opts = ss.Options(shade=shade, tile_w=16, tile_h=8, seg_len=-1)
    b = ss.batch_from_scenes(scenes, cams)
    ref = ss.Renderer(opts)
    img0, a0, nl0 = ref.forward(b, want_layers=True)
    d0 = ref.poll()
    assert d0["status"] == 0, d0
    r = ss.Renderer(opts)
    # poison the outputs so that a pixel the static path does not write shows
    img = torch.full_like(img0, float("nan"))
    a = torch.full_like(a0, float("nan"))
    nl = torch.full_like(nl0, 255)
    r.render_static(b, out=(img, a, nl))
    d = r.poll()
    torch.cuda.synchronize()
    assert d["status"] == 0 and d["static_status"] == 0, d
    assert d["static_pairs"] == d0["n_pairs"], (d, d0)
    assert d["static_pair_capacity"] >= d["static_pairs"]
    assert torch.equal(img, img0), float((img - img0).abs().max())
    assert torch.equal(a, a0)
    assert torch.equal(nl, nl0)
    assert d0["n_pairs"] > 0 and float(a0.max()) > 0.1
    return d


def test_static_render_matches_render_twice(ss):
    d1 = _compare(ss, *_splitsum_case())
    d2 = _compare(ss, *_albedo_case())          # smaller batch, other shading mode
    assert d2["static_pairs"] < d1["static_pairs"]


def test_static_render_rejects_oversized_batch(ss):
    w = g.make_config("C1", n_scale=0.5, res_scale=0.5)
    cam = g.look_at_camera(np.array([0.0, -3.0, 0.0]), 4096, 4096)   # 16.8 M pixels > the array
    b = ss.batch_from_scenes(w.scenes, [cam])
    r = ss.Renderer(ss.Options())
    img = torch.empty((b.n_pixels, 3), device="cuda")
    a = torch.empty((b.n_pixels,), device="cuda")
    L = ss.load_library()
    o = ss.surfsplat.ss_outputs(img.data_ptr(), a.data_ptr(), None, None, None, None)
    s = L.ss_render_static(r.ctx, ctypes.byref(b.c), ctypes.byref(o),
                           ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert s == ss.SS_ERR_STATIC_LIMIT
    per_view = ss.Renderer(ss.Options(launch="per_view"))
    s = L.ss_render_static(per_view.ctx, ctypes.byref(b.c), ctypes.byref(o),
                           ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert s == ss.SS_ERR_UNSUPPORTED
