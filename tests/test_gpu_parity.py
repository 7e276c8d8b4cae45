"""GPU parity: the HIP renderer (through the C ABI) against the CPU oracle.

Binning is compared bit for bit; images and gradients with the protocol of
parity_util (FP32 against FP64, decision-margin pixels excluded).
"""
import math

import numpy as np
import pytest

import scenegen as g
from parity_util import (GRAD_REL_L2, assert_image_parity, compare_images, decision_ok,
                         oracle_forward, oracle_maps, oracle_options, per_surfel_report, pixel_index, rel_l2)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def O():
    import oracle
    oracle.lib()
    return oracle


@pytest.fixture(scope="module")
def ss():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_2605_05876_amd as m
    m.load_library()
    return m


def all_pix(cam):
    ys, xs = np.meshgrid(np.arange(cam.height), np.arange(cam.width), indexing="ij")
    return np.stack([xs.ravel(), ys.ravel()], 1).astype(np.int32)


def sample_pix(cam, k, seed, frac=0.6):
    """k seeded pixels, uniform over the central `frac` of the view."""
    rng = np.random.default_rng(seed)
    w0, h0 = int(cam.width * (1 - frac) / 2), int(cam.height * (1 - frac) / 2)
    xs = rng.integers(w0, cam.width - w0, k)
    ys = rng.integers(h0, cam.height - h0, k)
    p = np.unique(np.stack([xs, ys], 1), axis=0)
    return p.astype(np.int32)


def gpu_run(ss, scenes, cams, opts, G=None, Ga=None):
    r = ss.Renderer(opts)
    b = ss.batch_from_scenes(scenes, cams)
    img, a, nl = r.forward(b, want_layers=True)
    d = r.poll()
    assert d["status"] == 0, d
    grads = None
    if G is not None:
        gt = torch.from_numpy(np.ascontiguousarray(G, np.float32)).cuda()
        ga = None if Ga is None else torch.from_numpy(np.ascontiguousarray(Ga, np.float32)).cuda()
        grads = r.backward(b, gt, ga)
        grads = {k: ([e.cpu().numpy() for e in v] if isinstance(v, list) else v.cpu().numpy())
                 for k, v in grads.items()}
    torch.cuda.synchronize()
    return r, b, img.cpu().numpy(), a.cpu().numpy(), nl.cpu().numpy(), grads


def small_c2():
    sc = g.torus_scene(22, 20_000, scale_mu=math.log(0.02), scale_sigma=0.3)
    sc.envmap = g.lognormal_envmap(22, 16, 32)
    el = math.radians(30.0)
    cam = g.look_at_camera((0.0, -3.0 * math.cos(el), 3.0 * math.sin(el)), 96, 96)
    return [sc], [cam]


def small_multiview():
    sc = g.superquadric_scene(33, 30_000, scale_mu=math.log(0.012), scale_sigma=0.5)
    sc.envmap = g.lognormal_envmap(33, 16, 32)
    cams = [g.look_at_camera(3.0 * d, 72, 56) for d in g.fibonacci_directions(3)]
    return [sc], cams


# ---------------------------------------------------------------- binning
# Tile counts cover every pair-sort pass count: C1 16x16 and MV (one radix pass),
# C1 8x8 (two), one 16x16 tile (none), BIG 8x8 with 69696 tiles (17 bits: a 9-bit
# and an 8-bit pass), HUGE 8x8 with 135424 tiles (18 bits: three passes); MV per
# view sorts each view on its own.
@pytest.mark.parametrize("case,tile,launch", [("C1", (16, 16), "batched"), ("C1", (8, 8), "batched"),
                                              ("C2s", (16, 16), "batched"), ("MV", (16, 8), "batched"),
                                              ("MV", (32, 16), "batched"), ("MV", (16, 8), "per_view"),
                                              ("ONE_TILE", (16, 16), "batched"), ("BIG", (8, 8), "batched"),
                                              ("HUGE", (8, 8), "batched")])
def test_binning_bit_exact(O, ss, case, tile, launch):
    if case == "C1":
        w = g.make_config("C1")
        scenes, cams, shade = w.scenes, w.cameras, "albedo"
    elif case == "C2s":
        (scenes, cams), shade = small_c2(), "splitsum"
    elif case == "ONE_TILE":
        (scenes, _), shade = small_multiview(), "albedo"
        cams = [g.look_at_camera(np.array([0.3, -2.8, 0.9]), 16, 16)]
    elif case in ("BIG", "HUGE"):
        (scenes, _), shade = small_multiview(), "albedo"
        side = 2112 if case == "BIG" else 2944
        cams = [g.look_at_camera(np.array([0.3, -2.8, 0.9]), side, side)]
    else:
        (scenes, cams), shade = small_multiview(), "splitsum"
    opts = ss.Options(shade=shade, tile_w=tile[0], tile_h=tile[1], launch=launch)
    r, b, *_ = gpu_run(ss, scenes, cams, opts)
    dbg = r.debug_binning(b)
    zb = dbg["rec_zbits"].cpu().numpy().view(np.uint32)
    rect = dbg["rec_rect"].cpu().numpy()
    keys = dbg["keys"].cpu().numpy().view(np.uint64)
    vals = dbg["vals"].cpu().numpy().view(np.uint32)
    ranges = dbg["ranges"].cpu().numpy().view(np.uint32)
    oo = oracle_options(O, opts)
    ref_k, ref_v = [], []
    rec_base, tile_base = 0, 0
    for cam in cams:
        sc = scenes[cam.scene]
        keep, rz, rr = O.bin_f32(sc, cam, oo)
        n = sc.n
        k = keep.astype(bool)
        gz, grect = zb[rec_base:rec_base + n], rect[rec_base:rec_base + n]
        assert (gz[k] == rz[k]).all(), "z_start bits differ"
        # culled on the GPU <=> culled in the reference (empty rectangle)
        g_keep = (grect[:, 0] <= grect[:, 2]) & (grect[:, 1] <= grect[:, 3])
        assert (g_keep == k).all(), (np.nonzero(g_keep != k)[0][:10])
        tiles_x = -(-cam.width // tile[0])
        tr = np.stack([grect[:, 0] // tile[0], grect[:, 1] // tile[1], grect[:, 2] // tile[0],
                       grect[:, 3] // tile[1]], 1)
        assert (tr[k] == rr[k]).all(), "tile rectangles differ"
        kk, vv = O.sorted_pairs(keep, rz, rr, tiles_x, tile_base=tile_base, rec_base=rec_base)
        ref_k.append(kk)
        ref_v.append(vv)
        rec_base += n
        tile_base += tiles_x * (-(-cam.height // tile[1]))
    ref_k = np.concatenate(ref_k)
    ref_v = np.concatenate(ref_v)
    assert keys.shape == ref_k.shape
    assert (keys == ref_k).all()
    assert (vals == ref_v).all()
    # per-tile ranges
    tiles = (ref_k >> np.uint64(32)).astype(np.int64)
    cnt = np.bincount(tiles, minlength=tile_base)
    ends = np.cumsum(cnt)
    starts = ends - cnt
    nz = cnt > 0
    assert (ranges[nz, 0] == starts[nz]).all() and (ranges[nz, 1] == ends[nz]).all()
    assert (ranges[~nz] == 0).all()


# ---------------------------------------------------------------- forward
def _forward_case(O, ss, scenes, cams, shade, pix_fn, exact_ties=False, **kw):
    opts = ss.Options(shade=shade, **kw)
    maps, lut = oracle_maps(O, scenes, shade)
    pix = [pix_fn(c, v) for v, c in enumerate(cams)]
    # exact ties: a 4-ulp move of the depths would break them, so the conditioning
    # probe does not apply; both sides see the ties exactly
    ref = oracle_forward(O, scenes, cams, opts, pix, maps, lut, conditioning=not exact_ties)
    _, _, img, a, nl, _ = gpu_run(ss, scenes, cams, opts)
    rep, masks = compare_images(cams, pix, ref, img, a, exact_ties)
    print("forward", {k: v for k, v in rep.items() if k != "worst"})
    for v, c in enumerate(cams):
        idx = pixel_index(cams, v, pix[v])
        assert (nl[idx][masks[v]] == ref[v]["n_layers"][masks[v]]).all()
    return rep


def test_forward_parity_albedo_full_image(O, ss):
    w = g.make_config("C1")
    rep = _forward_case(O, ss, w.scenes, w.cameras, "albedo", lambda c, v: all_pix(c))
    assert_image_parity(rep)
    assert rep["total"] == 128 * 128


def test_forward_parity_splitsum_full_image(O, ss):
    scenes, cams = small_c2()
    rep = _forward_case(O, ss, scenes, cams, "splitsum", lambda c, v: all_pix(c))
    assert_image_parity(rep)


def test_forward_parity_multiview_ragged(O, ss):
    scenes, cams = small_multiview()   # 72 x 56: ragged against 16 x 16 tiles
    rep = _forward_case(O, ss, scenes, cams, "splitsum", lambda c, v: all_pix(c))
    assert_image_parity(rep)


@pytest.mark.parametrize("sigma", [0.0, 0.5])
def test_forward_parity_sigma(O, ss, sigma):
    w = g.make_config("C1")
    rep = _forward_case(O, ss, w.scenes, w.cameras, "albedo", lambda c, v: all_pix(c), sigma_f=sigma)
    assert_image_parity(rep)


# ---------------------------------------------------------------- backward
def _backward_case(O, ss, scenes, cams, shade, pix_fn, seed=0, with_alpha=True, exact_ties=False, **kw):
    opts = ss.Options(shade=shade, **kw)
    maps, lut = oracle_maps(O, scenes, shade)
    oo = oracle_options(O, opts)
    pix = [pix_fn(c, v) for v, c in enumerate(cams)]
    ref = oracle_forward(O, scenes, cams, opts, pix, maps, lut, conditioning=False)
    n_pix = sum(c.width * c.height for c in cams)
    rng = np.random.default_rng(seed)
    G = np.zeros((n_pix, 3))
    Ga = np.zeros(n_pix) if with_alpha else None
    per_view = []
    for v, c in enumerate(cams):
        r = ref[v]
        ok = decision_ok(r, exact_ties)
        gv = rng.normal(size=(len(pix[v]), 3)) * ok[:, None]
        gav = rng.normal(size=len(pix[v])) * ok if with_alpha else None
        idx = pixel_index(cams, v, pix[v])
        G[idx] = gv
        if with_alpha:
            Ga[idx] = gav
        per_view.append((gv, gav))
    _, _, img, a, nl, gg = gpu_run(ss, scenes, cams, opts, G, Ga)
    # oracle gradient: sum over views of per-view adjoints (scene-local arrays)
    names = ["position", "normal", "tangent", "scale", "albedo", "roughness", "metallic"]
    ref_g = [{k: np.zeros_like(getattr(s, k), dtype=np.float64) for k in names} for s in scenes]
    ref_maps = [None if maps[i] is None else np.zeros_like(maps[i]) for i in range(len(scenes))]
    for v, c in enumerate(cams):
        sc = scenes[c.scene]
        hw = tuple(np.asarray(sc.envmap).shape[:2]) if maps[c.scene] is not None else (0, 0)
        gr = O.render_grad(sc, c, oo, pix[v], per_view[v][0], per_view[v][1], maps=maps[c.scene],
                           lut=lut, env_hw=hw)
        for k in names:
            ref_g[c.scene][k] += gr[k]
        if ref_maps[c.scene] is not None:
            ref_maps[c.scene] += gr["maps"]
    offs = np.cumsum([0] + [s.n for s in scenes])
    errs = {}
    pos_norm = np.linalg.norm(np.concatenate([rg["position"] for rg in ref_g], axis=-1))
    for k in names:
        got = gg[k]
        want = np.concatenate([rg[k] for rg in ref_g], axis=-1)
        if np.linalg.norm(want) == 0 and shade == "albedo" and k in ("roughness", "metallic"):
            assert np.abs(got).max() == 0
            continue
        if np.linalg.norm(want) < 1e-9 * pos_norm:
            # analytically zero (e.g. the tangent of isotropic surfels): FP32 noise only
            errs[k] = float(np.linalg.norm(got) / pos_norm)
            continue
        errs[k] = rel_l2(got, want)
        ps = per_surfel_report(got, want)
        print(k, "per surfel", ps)
        assert ps["n_over"] == 0, (k, ps)
    if shade == "splitsum":
        for i, sc in enumerate(scenes):
            He, We = np.asarray(sc.envmap).shape[:2]
            dE = O.envmap_adjoint(ref_maps[i], He, We)
            errs[f"envmap{i}"] = rel_l2(gg["envmap"][i], dE)
    print("gradients (relative L2)", errs)
    return errs


# the two walks of the raster backward (options.bwd_walk)
WALKS = ["rows", "records"]


@pytest.mark.parametrize("walk", WALKS)
@pytest.mark.parametrize("tile", [(16, 16), (8, 8)])
def test_backward_parity_albedo_full_image(O, ss, walk, tile):
    w = g.make_config("C1")
    errs = _backward_case(O, ss, w.scenes, w.cameras, "albedo", lambda c, v: all_pix(c), bwd_walk=walk,
                          tile_w=tile[0], tile_h=tile[1])
    assert max(errs.values()) <= GRAD_REL_L2, errs


@pytest.mark.parametrize("walk", WALKS)
def test_backward_parity_splitsum_full_image(O, ss, walk):
    scenes, cams = small_c2()
    errs = _backward_case(O, ss, scenes, cams, "splitsum", lambda c, v: all_pix(c), bwd_walk=walk)
    assert max(errs.values()) <= GRAD_REL_L2, errs


@pytest.mark.parametrize("case", ["C1", "multiview"])
@pytest.mark.parametrize("tile", [(8, 8), (16, 8), (32, 16)])
def test_backward_walks_agree(ss, case, tile):
    """Both walks of the backward sum the same fragment contributions: gradients
    equal to float summation order (relative L2 <= 1e-5 per group)."""
    if case == "C1":
        w = g.make_config("C1")
        scenes, cams, shade = w.scenes, w.cameras, "albedo"
    else:
        scenes, cams = small_multiview()
        shade = "splitsum"
    n_pix = sum(c.width * c.height for c in cams)
    rng = np.random.default_rng(29)
    G, Ga = rng.normal(size=(n_pix, 3)), rng.normal(size=n_pix)
    out = [gpu_run(ss, scenes, cams, ss.Options(shade=shade, bwd_walk=walk, tile_w=tile[0], tile_h=tile[1]),
                   G, Ga)[5] for walk in WALKS]
    pos = np.linalg.norm(out[0]["position"])
    for k in ("position", "normal", "scale", "albedo", "roughness", "metallic"):
        if np.linalg.norm(out[0][k]) <= 1e-6 * pos:
            continue
        assert rel_l2(out[1][k], out[0][k]) <= 1e-5, (k, rel_l2(out[1][k], out[0][k]))
    if shade == "splitsum":
        assert rel_l2(out[1]["envmap"][0], out[0]["envmap"][0]) <= 1e-5


@pytest.mark.parametrize("env_lds", [0, 6144])
def test_backward_parity_splitsum_global_levels(O, ss, env_lds):
    """Environment-level gradients through global atomics for every level (env_lds 0)
    or for every level but the irradiance one (6144 floats): the wave-cooperative
    global scatter of the shading adjoint for all three lookups, against the oracle."""
    scenes, cams = small_c2()
    errs = _backward_case(O, ss, scenes, cams, "splitsum", lambda c, v: all_pix(c), env_lds=env_lds)
    assert max(errs.values()) <= GRAD_REL_L2, errs


@pytest.mark.parametrize("walk", WALKS)
def test_backward_parity_multiview(O, ss, walk):
    scenes, cams = small_multiview()
    errs = _backward_case(O, ss, scenes, cams, "splitsum", lambda c, v: all_pix(c), seed=3, bwd_walk=walk)
    assert max(errs.values()) <= GRAD_REL_L2, errs


# ---------------------------------------------------------------- densification statistic
def _two_scene_views():
    a = g.sphere_scene(41, 3000, scale=0.03, svbrdf=True)
    b = g.torus_scene(42, 8000, scale_mu=math.log(0.02), scale_sigma=0.3)
    a.envmap = g.lognormal_envmap(43, 16, 32)
    b.envmap = g.lognormal_envmap(44, 16, 32)
    cams = [g.look_at_camera(3.0 * d, 64, 48) for d in g.fibonacci_directions(2)]
    cams += [g.look_at_camera(3.0 * d, 56, 72, scene=1) for d in g.fibonacci_directions(3)[1:]]
    return [a, b], cams


@pytest.mark.parametrize("walk", WALKS)
@pytest.mark.parametrize("case", ["C1_sigma0.5", "multiview", "two_scenes"])
def test_screen_grad_parity(O, ss, case, walk):
    """Sec. 3.6.1 statistic (sum over views and pixels of |(dL_p/dT1z, dL_p/dT2z)| T4z)
    and the visible-view count against the oracle; the other gradients are unchanged
    by requesting it."""
    if case == "C1_sigma0.5":
        w = g.make_config("C1")
        scenes, cams, shade, kw = w.scenes, w.cameras, "albedo", dict(sigma_f=0.5)
    elif case == "multiview":
        scenes, cams = small_multiview()
        shade, kw = "splitsum", {}
    else:
        scenes, cams = _two_scene_views()
        shade, kw = "splitsum", {}
    opts = ss.Options(shade=shade, bwd_walk=walk, **kw)
    maps, lut = oracle_maps(O, scenes, shade)
    oo = oracle_options(O, opts)
    pix = [all_pix(c) for c in cams]
    ref = oracle_forward(O, scenes, cams, opts, pix, maps, lut, conditioning=False)
    n_pix = sum(c.width * c.height for c in cams)
    rng = np.random.default_rng(17)
    G = np.zeros((n_pix, 3))
    Ga = np.zeros(n_pix)
    want_abs = [np.zeros(s.n) for s in scenes]
    want_vis = [np.zeros(s.n, np.int64) for s in scenes]
    for v, c in enumerate(cams):
        ok = decision_ok(ref[v])
        gv = rng.normal(size=(len(pix[v]), 3)) * ok[:, None]
        gav = rng.normal(size=len(pix[v])) * ok
        idx = pixel_index(cams, v, pix[v])
        G[idx] = gv
        Ga[idx] = gav
        sc = scenes[c.scene]
        hw = tuple(np.asarray(sc.envmap).shape[:2]) if maps[c.scene] is not None else (0, 0)
        r = O.screen_grad(sc, c, oo, pix[v], gv, gav, maps=maps[c.scene], lut=lut, env_hw=hw)
        want_abs[c.scene] += r["abs"]
        want_vis[c.scene] += r["visible"]
    r = ss.Renderer(opts)
    b = ss.batch_from_scenes(scenes, cams)
    r.forward(b)
    assert r.poll()["status"] == 0
    gt = torch.from_numpy(np.ascontiguousarray(G, np.float32)).cuda()
    ga = torch.from_numpy(np.ascontiguousarray(Ga, np.float32)).cuda()
    with_ss = r.backward(b, gt, ga, want_screen_grad=True)
    plain = r.backward(b, gt, ga)
    torch.cuda.synchronize()
    got_abs = with_ss["screen_grad"].cpu().numpy()
    got_vis = with_ss["visible_views"].cpu().numpy()
    np.testing.assert_array_equal(got_vis, np.concatenate(want_vis))
    wa = np.concatenate(want_abs)
    assert wa.max() > 0 and (got_abs >= 0).all()
    assert rel_l2(got_abs, wa) <= GRAD_REL_L2, rel_l2(got_abs, wa)
    for k in ("position", "normal", "scale", "albedo"):
        assert rel_l2(with_ss[k].cpu().numpy(), plain[k].cpu().numpy()) <= 1e-5, k


# ---------------------------------------------------------------- depth consolidation
@pytest.mark.parametrize("walk", WALKS)
@pytest.mark.parametrize("case", ["C1", "multiview"])
def test_cons_parity(O, ss, case, walk):
    """eq:cons_loss per pixel against the oracle (relative L2 <= 1e-3: the FP32 depth of
    a fragment carries ~2 ulp(z) from T4z = (z_start + z_end)/2, against layer depth
    spreads of ~1e-2), the composited depth (image protocol), the image unchanged by
    the extra statistics, and the gradients of a loss on image, cons and depth
    together (relative L2 <= 1e-3 per group)."""
    if case == "C1":
        w = g.make_config("C1")
        scenes, cams, shade = w.scenes, w.cameras, "albedo"
    else:
        scenes, cams = small_multiview()
        shade = "splitsum"
    # unsplit lists: the forward with depth statistics never splits them, so the
    # image without the statistics is then bit-identical
    opts = ss.Options(shade=shade, depth_stats=True, seg_len=-1, bwd_walk=walk)
    maps, lut = oracle_maps(O, scenes, shade)
    oo = oracle_options(O, opts)
    pix = [all_pix(c) for c in cams]
    ref = oracle_forward(O, scenes, cams, opts, pix, maps, lut, conditioning=False)
    r = ss.Renderer(opts)
    b = ss.batch_from_scenes(scenes, cams)
    img0, a0, _ = r.forward(b)
    img0, a0 = img0.cpu().numpy(), a0.cpu().numpy()
    img, a, nl, aux = r.forward(b, want_layers=True, want_cons=True, want_depth=True)
    assert r.poll()["status"] == 0
    img, a = img.cpu().numpy(), a.cpu().numpy()
    cons, depth = aux["cons"].cpu().numpy(), aux["depth"].cpu().numpy()
    np.testing.assert_array_equal(img, img0)
    np.testing.assert_array_equal(a, a0)
    want, got, want_z, got_z = [], [], [], []
    n_pix = sum(c.width * c.height for c in cams)
    rng = np.random.default_rng(23)
    G = np.zeros((n_pix, 3))
    Dc = np.zeros(n_pix)
    Dz = np.zeros(n_pix)
    per_view = []
    for v, c in enumerate(cams):
        ok = decision_ok(ref[v])
        idx = pixel_index(cams, v, pix[v])
        want.append(ref[v]["cons"][ok])
        got.append(cons[idx][ok])
        want_z.append(ref[v]["depth"][ok])
        got_z.append(depth[idx][ok])
        gv = rng.normal(size=(len(pix[v]), 3)) * ok[:, None]
        dcv = rng.normal(size=len(pix[v])) * ok * 10.0
        dzv = rng.normal(size=len(pix[v])) * ok
        G[idx] = gv
        Dc[idx] = dcv
        Dz[idx] = dzv
        per_view.append((gv, dcv, dzv))
    want, got = np.concatenate(want), np.concatenate(got)
    assert want.max() > 0
    assert rel_l2(got, want) <= 1e-3, rel_l2(got, want)
    # composited depth: the image protocol (relative L2 1e-4, per pixel 1e-4 of max(|ref|, 1e-2 max))
    want_z, got_z = np.concatenate(want_z), np.concatenate(got_z)
    assert rel_l2(got_z, want_z) <= 1e-4, rel_l2(got_z, want_z)
    bound = 1e-4 * np.maximum(np.abs(want_z), 1e-2 * np.abs(want_z).max())
    assert (np.abs(got_z - want_z) <= bound).mean() >= 0.99
    gt = torch.from_numpy(np.ascontiguousarray(G, np.float32)).cuda()
    dct = torch.from_numpy(np.ascontiguousarray(Dc, np.float32)).cuda()
    dzt = torch.from_numpy(np.ascontiguousarray(Dz, np.float32)).cuda()
    gg = r.backward(b, gt, None, d_cons=dct, d_depth=dzt)
    gg = {k: v.cpu().numpy() for k, v in gg.items() if not isinstance(v, list)}
    names = ["position", "normal", "tangent", "scale", "albedo"]
    ref_g = [{k: np.zeros_like(getattr(sc, k), dtype=np.float64) for k in names} for sc in scenes]
    for v, c in enumerate(cams):
        sc = scenes[c.scene]
        hw = tuple(np.asarray(sc.envmap).shape[:2]) if maps[c.scene] is not None else (0, 0)
        gr = O.render_grad(sc, c, oo, pix[v], per_view[v][0], None, maps=maps[c.scene], lut=lut, env_hw=hw,
                           dcons=per_view[v][1], ddepth=per_view[v][2])
        for k in names:
            ref_g[c.scene][k] += gr[k]
    pos_norm = np.linalg.norm(np.concatenate([rg["position"] for rg in ref_g], axis=-1))
    for k in names:
        want_k = np.concatenate([rg[k] for rg in ref_g], axis=-1)
        if np.linalg.norm(want_k) < 1e-9 * pos_norm:
            assert np.linalg.norm(gg[k]) <= 1e-6 * pos_norm, k
            continue
        assert rel_l2(gg[k], want_k) <= GRAD_REL_L2, (k, rel_l2(gg[k], want_k))
    # without a cons forward the cons adjoint is refused
    r.forward(b)
    with pytest.raises(RuntimeError):
        r.backward(b, gt, None, d_cons=dct)


@pytest.mark.parametrize("walk", WALKS)
def test_normal_image_parity(O, ss, walk):
    """Normal image (Sec. 4.2.3): per layer the Shepard mean of the unit normals,
    renormalised, composited like colour; forward with the image protocol and the
    geometric gradients (relative L2 <= 1e-3 per group)."""
    scenes, cams = small_multiview()
    rep = _forward_case(O, ss, scenes, cams, "normal", lambda c, v: all_pix(c))
    assert_image_parity(rep)
    errs = _backward_case(O, ss, scenes, cams, "normal", lambda c, v: all_pix(c), seed=5, bwd_walk=walk)
    errs = {k: e for k, e in errs.items() if k not in ("albedo", "roughness", "metallic")}
    assert max(errs.values()) <= GRAD_REL_L2, errs


# ---------------------------------------------------------------- per-pixel MIP variant
def _per_pixel_case(case):
    if case == "checkerboard":
        w = g.checkerboard_workload(n_side=240, extent=3.0, square=0.15, width=96, height=72,
                                    eye=(0.0, -3.2, 0.35))
        return w.scenes, w.cameras, "albedo", dict(sigma_f=0.1)
    if case == "C1_sigma0.5":
        w = g.make_config("C1")
        return w.scenes, w.cameras, "albedo", dict(sigma_f=0.5)
    scenes, cams = small_multiview()
    return scenes, cams, "splitsum", dict(sigma_f=0.3)


@pytest.mark.parametrize("case", ["checkerboard", "C1_sigma0.5"])
def test_per_pixel_mip_forward_parity(O, ss, case):
    """Sec. 3.3.1 variant (Jacobian at every intersection) against the oracle with the
    image protocol."""
    scenes, cams, shade, kw = _per_pixel_case(case)
    rep = _forward_case(O, ss, scenes, cams, shade, lambda c, v: all_pix(c), mip="pixel", **kw)
    assert_image_parity(rep)


@pytest.mark.parametrize("walk", WALKS)
@pytest.mark.parametrize("case", ["checkerboard", "C1_sigma0.5", "multiview"])
def test_per_pixel_mip_backward_parity(O, ss, case, walk):
    """Adjoint of the per-pixel-Jacobian filter (Sec. 3.3.1): dL/d(record) through the
    pixel's own Sigma_mip and det, against the oracle's tape adjoint (relative L2 per
    group, split-sum and the environment maps included for the multi-view case)."""
    scenes, cams, shade, kw = _per_pixel_case(case)
    errs = _backward_case(O, ss, scenes, cams, shade, lambda c, v: all_pix(c), mip="pixel", bwd_walk=walk, **kw)
    assert max(errs.values()) <= GRAD_REL_L2, errs


# ---------------------------------------------------------------- tables, invariances, edges
def test_brdf_lut_matches_oracle(O, ss):
    lut = ss.make_brdf_lut(64, 64, 1024).cpu().numpy()
    ref = O.brdf_lut(64, 64, 1024)
    # both integrate in FP64; the GPU table is rounded to FP32
    assert np.abs(lut - ref).max() < 1e-6


def test_forward_parity_sampled_pixels(O, ss):
    """Split-sum forward at seeded sampled pixels (the protocol used at full size)."""
    scenes, cams = small_c2()
    rep = _forward_case(O, ss, scenes, cams, "splitsum", lambda c, v: sample_pix(c, 300, 5))
    assert_image_parity(rep)


@pytest.mark.parametrize("variant", [dict(lds_batch=32), dict(lds_batch=256), dict(tile_w=8, tile_h=8),
                                     dict(tile_w=32, tile_h=16), dict(persistent=False),
                                     dict(launch="per_view")])
def test_forward_bit_identical_across_tunables(ss, variant):
    """Unsplit lists: the forward is bit-identical for every tunable.  Split lists
    (the default; this scene's longest lists have ~15k entries): segments start
    at fixed list positions, so the LDS batch and the launch mode still give
    bit-identical images; another tile shape (other lists) or the non-persistent
    launch (no split) changes only the float summation order of layers that span
    a segment boundary -- the layer counts stay identical."""
    scenes, cams = small_multiview()
    base = gpu_run(ss, scenes, cams, ss.Options(shade="splitsum", seg_len=-1))
    other = gpu_run(ss, scenes, cams, ss.Options(shade="splitsum", seg_len=-1, **variant))
    assert np.array_equal(base[2], other[2]) and np.array_equal(base[3], other[3])
    assert np.array_equal(base[4], other[4])
    split = gpu_run(ss, scenes, cams, ss.Options(shade="splitsum"))
    other = gpu_run(ss, scenes, cams, ss.Options(shade="splitsum", **variant))
    assert np.array_equal(split[4], other[4]) and np.array_equal(split[4], base[4])
    if set(variant) <= {"lds_batch", "launch"}:
        assert np.array_equal(split[2], other[2]) and np.array_equal(split[3], other[3])
    else:
        np.testing.assert_allclose(other[2], split[2], rtol=1e-5, atol=1e-7)
        np.testing.assert_allclose(other[3], split[3], rtol=1e-5, atol=1e-7)


def test_per_view_backward_matches_batched(ss):
    scenes, cams = small_multiview()
    n_pix = sum(c.width * c.height for c in cams)
    G = np.random.default_rng(1).normal(size=(n_pix, 3))
    a = gpu_run(ss, scenes, cams, ss.Options(shade="splitsum"), G)[5]
    b = gpu_run(ss, scenes, cams, ss.Options(shade="splitsum", launch="per_view"), G)[5]
    for k in a:
        if k == "envmap":
            assert rel_l2(b[k][0], a[k][0]) < 1e-5
        else:
            assert rel_l2(b[k], a[k]) < 1e-5, k


def test_all_culled_gives_background(ss):
    from conftest import axis_camera, make_scene
    cam = axis_camera(40, 24, 50.0, background=(0.2, 0.4, 0.6))
    sc = make_scene([[0, 0, -2.0], [0.1, 0, -1.0]], [[0, 0, 1.0]] * 2, [[1, 0, 0]] * 2, [[0.05, 0.05]] * 2)
    _, _, img, a, nl, _ = gpu_run(ss, [sc], [cam], ss.Options())
    assert np.allclose(img, np.array([0.2, 0.4, 0.6], np.float32)) and (a == 0).all() and (nl == 0).all()


def test_layer_cap_matches_oracle(O, ss):
    from conftest import axis_camera, make_scene
    cam = axis_camera(40, 40, 100.0)
    pos, nrm, tan, scl, alb = [], [], [], [], []
    rng = np.random.default_rng(0)
    th = np.radians(8.0)
    for k in range(20):
        # lattice not commensurate with the pixel grid (no exact cutoff ties), planes
        # tilted by 8 degrees so that every surfel has a depth extent
        gx, gy = np.meshgrid(np.arange(-4, 5) * 0.0317 + 0.0043 * k, np.arange(-4, 5) * 0.0317 - 0.0029 * k)
        n = gx.size
        pos.append(np.stack([gx.ravel(), gy.ravel() * np.cos(th), 2.0 + 0.05 * k + gy.ravel() * np.sin(th)], 1))
        nrm.append(np.tile([0, -np.sin(th), np.cos(th)], (n, 1)))
        tan.append(np.tile([1.0, 0, 0], (n, 1)))
        scl.append(np.full((n, 2), 0.02))
        alb.append(rng.uniform(0, 1, (n, 3)))
    sc = make_scene(*[np.concatenate(x) for x in (pos, nrm, tan, scl, alb)])
    rep = _forward_case(O, ss, [sc], [cam], "albedo", lambda c, v: all_pix(c))
    assert_image_parity(rep)
    _, _, img, a, nl, _ = gpu_run(ss, [sc], [cam], ss.Options())
    assert nl.max() == 16


def test_stage_profile_counts(ss):
    scenes, cams = small_multiview()
    r = ss.Renderer(ss.Options(shade="splitsum"))
    b = ss.batch_from_scenes(scenes, cams)
    r.forward(b)
    r.profile(True)
    for _ in range(2):
        r.forward(b)
        r.backward(b, torch.ones((b.n_pixels, 3), device="cuda"))
    prof = r.profile_read()
    print(prof)
    for k, (ms, n) in prof.items():
        assert n == 2 and ms > 0, (k, ms, n)


def test_capacity_and_state_errors(ss):
    w = g.make_config("C1")
    r = ss.Renderer(ss.Options(), check_capacity=False)   # the library's own latch, no re-render
    b = ss.batch_from_scenes(w.scenes, w.cameras)
    with pytest.raises(ss.SurfsplatError) as e:
        r.backward(b, torch.zeros((b.n_pixels, 3), device="cuda"))
    assert e.value.status == 4  # SS_ERR_STATE
    r.forward(b)
    d0 = r.poll()
    assert d0["status"] == 0
    # larger surfels with the same shapes: more pairs than the reserved capacity.
    # The forward flags it (every slot below the capacity is still written, so
    # nothing reads past it); after a reserve the same batch renders.
    b.params["scale"].mul_(8.0)
    r.forward(b)
    d1 = r.poll()
    assert d1["status"] == 3 and d1["n_pairs"] > d0["pair_capacity"], (d0, d1)  # SS_ERR_CAPACITY
    r.reserve(b)
    img, a = r.forward(b)[:2]
    d2 = r.poll()
    assert d2["status"] == 0 and d2["n_pairs"] == d1["n_pairs"], (d1, d2)
    assert torch.isfinite(img).all() and torch.isfinite(a).all()


def test_graph_replay_matches_eager(ss):
    """The whole forward+backward step captured once in a HIP graph and replayed: every
    replay, with unrelated eager work and a synchronisation before it, gives the eager
    images bit for bit and the eager gradients to rounding (atomic order)."""
    scenes, cams = small_multiview()
    r = ss.Renderer(ss.Options(shade="splitsum"))
    b = ss.batch_from_scenes(scenes, cams)
    r.reserve(b)
    n_pix = b.n_pixels
    rng = np.random.default_rng(5)
    G = torch.from_numpy(rng.normal(size=(n_pix, 3)).astype(np.float32)).cuda()
    Ga = torch.from_numpy(rng.normal(size=n_pix).astype(np.float32)).cuda()
    img = torch.empty((n_pix, 3), device="cuda")
    alpha = torch.empty((n_pix,), device="cuda")
    nl = torch.empty((n_pix,), device="cuda", dtype=torch.uint8)
    grads = {k: torch.empty_like(b.params[k]) for k in ss.PARAMS}
    grads["envmap"] = [torch.empty_like(e) for e in b.envmaps]

    def step():
        r.forward(b, out=(img, alpha, nl))
        r.backward(b, G, Ga, grads=grads)

    def snapshot():
        out = {"img": img.clone(), "alpha": alpha.clone(), "nl": nl.clone()}
        out.update({k: grads[k].clone() for k in ss.PARAMS})
        out["envmap"] = grads["envmap"][0].clone()
        return out

    step()
    torch.cuda.synchronize()
    assert r.poll()["status"] == 0
    want = snapshot()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        step()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    cg = torch.cuda.CUDAGraph()
    with torch.cuda.graph(cg):
        step()
    other = ss.Renderer(ss.Options())
    w1 = g.make_config("C1")
    b1 = ss.batch_from_scenes(w1.scenes, w1.cameras)
    for rep in range(3):
        # eager work between replays, on the same device: another renderer's forward
        # and plain torch ops, then poison every output the graph must rewrite
        other.forward(b1)
        _ = torch.randn(1 << 20, device="cuda").sum().item()
        img.fill_(float("nan"))
        alpha.fill_(float("nan"))
        nl.fill_(255)
        for k in ss.PARAMS:
            grads[k].fill_(float("nan"))
        grads["envmap"][0].fill_(float("nan"))
        torch.cuda.synchronize()
        cg.replay()
        torch.cuda.synchronize()
        assert r.poll()["status"] == 0
        got = snapshot()
        for k in ("img", "alpha", "nl"):
            assert torch.equal(got[k], want[k]), (rep, k)
        for k in list(ss.PARAMS) + ["envmap"]:
            a, e = got[k].double().cpu().numpy(), want[k].double().cpu().numpy()
            assert np.isfinite(a).all() and rel_l2(a, e) < 1e-5, (rep, k, rel_l2(a, e))
