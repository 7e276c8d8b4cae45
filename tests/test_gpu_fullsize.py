"""Parity at the benchmark's full sizes, in the launch configuration bench.py
times (batched, persistent raster, tile shape from the autotune cache).

The oracle is brute force over every surfel, so outputs are compared on seeded
sampled pixels: the forward at those pixels, and the backward with dL/dimage
and dL/dalpha nonzero only there (every gradient is then exactly the oracle's
adjoint of those pixels).
"""
import numpy as np
import pytest

import scenegen as g
from parity_util import (GRAD_REL_L2, assert_image_parity, compare_images, decision_ok,
                         oracle_forward, oracle_maps, oracle_options, pixel_index, rel_l2)

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


def bench_options(ss, name, shade):
    from paper_2605_05876_amd import autotune
    t = autotune.lookup(name) or {}
    return ss.Options(shade=shade, tile_w=t.get("tile_w", 16), tile_h=t.get("tile_h", 16),
                      lds_batch=t.get("lds_batch", 128))


def sample(cam, k, seed):
    rng = np.random.default_rng(seed)
    xs = rng.integers(int(cam.width * 0.2), int(cam.width * 0.8), k)
    ys = rng.integers(int(cam.height * 0.2), int(cam.height * 0.8), k)
    return np.unique(np.stack([xs, ys], 1), axis=0).astype(np.int32)


@pytest.mark.parametrize("name,k", [("C3", 96), ("C5", 64)])
def test_fullsize_sampled_parity(O, ss, name, k):
    w = g.make_config(name)
    opts = bench_options(ss, name, w.shade)
    cams = w.cameras
    pix = [sample(c, k, 100 + v) for v, c in enumerate(cams)]
    maps, lut = oracle_maps(O, w.scenes, w.shade)
    ref = oracle_forward(O, w.scenes, cams, opts, pix, maps, lut)
    r = ss.Renderer(opts)
    b = ss.batch_from_scenes(w.scenes, cams)
    img, a, nl = r.forward(b, want_layers=True)
    assert r.poll()["status"] == 0
    rep, masks = compare_images(cams, pix, ref, img.cpu().numpy(), a.cpu().numpy())
    print(name, "forward", {k_: v for k_, v in rep.items() if k_ != "worst"})
    assert_image_parity(rep)
    # backward with the gradient concentrated on the compared pixels
    rng = np.random.default_rng(7)
    n_pix = b.n_pixels
    G = np.zeros((n_pix, 3), np.float32)
    Ga = np.zeros(n_pix, np.float32)
    per_view = []
    for v, c in enumerate(cams):
        ok = decision_ok(ref[v])
        gv = rng.normal(size=(len(pix[v]), 3)) * ok[:, None]
        gav = rng.normal(size=len(pix[v])) * ok
        idx = pixel_index(cams, v, pix[v])
        G[idx] = gv
        Ga[idx] = gav
        per_view.append((gv, gav))
    grads = r.backward(b, torch.from_numpy(G).cuda(), torch.from_numpy(Ga).cuda())
    torch.cuda.synchronize()
    oo = oracle_options(O, opts)
    names = ["position", "normal", "tangent", "scale", "albedo", "roughness", "metallic"]
    ref_g = [{n: np.zeros_like(getattr(s, n), dtype=np.float64) for n in names} for s in w.scenes]
    ref_maps = [np.zeros_like(m) for m in maps]
    for v, c in enumerate(cams):
        sc = w.scenes[c.scene]
        gr = O.render_grad(sc, c, oo, pix[v], per_view[v][0], per_view[v][1], maps=maps[c.scene], lut=lut,
                           env_hw=sc.envmap.shape[:2])
        for n in names:
            ref_g[c.scene][n] += gr[n]
        ref_maps[c.scene] += gr["maps"]
    errs = {}
    for n in names:
        errs[n] = rel_l2(grads[n].cpu().numpy(), np.concatenate([rg[n] for rg in ref_g], axis=-1))
    for i, sc in enumerate(w.scenes):
        dE = O.envmap_adjoint(ref_maps[i], *sc.envmap.shape[:2])
        errs[f"envmap{i}"] = rel_l2(grads["envmap"][i].cpu().numpy(), dE)
    print(name, "backward", errs)
    assert max(errs.values()) <= GRAD_REL_L2, errs


@pytest.mark.parametrize("name", ["C3"])
def test_fullsize_binning_properties(O, ss, name):
    """Tile lists at full size, where the oracle's per-record pair listing is too
    slow: z_start bits and tile rectangles against the oracle's FP32 binning
    (exact), then properties that fix the sorted pair list uniquely -- strictly
    increasing (tile, z_start bits, record), every pair's tile inside its
    record's rectangle, and each record's pair count equal to its rectangle's
    tile count -- and per-tile ranges that delimit the runs of equal tiles."""
    w = g.make_config(name)
    opts = bench_options(ss, name, w.shade)
    cams = w.cameras
    r = ss.Renderer(opts)
    b = ss.batch_from_scenes(w.scenes, cams)
    r.forward(b)
    assert r.poll()["status"] == 0
    dbg = r.debug_binning(b)
    zb = dbg["rec_zbits"].cpu().numpy().view(np.uint32)
    keys = dbg["keys"].cpu().numpy().view(np.uint64)
    vals = dbg["vals"].cpu().numpy().view(np.uint32).astype(np.int64)
    ranges = dbg["ranges"].cpu().numpy().view(np.uint32).astype(np.int64)
    oo = oracle_options(O, opts)
    n_rec = sum(w.scenes[c.scene].n for c in cams)
    trect = np.zeros((n_rec, 4), np.int64)
    keep_all = np.zeros(n_rec, bool)
    rec_off, tile_off, tiles_x = [], [], []
    rec_base = tile_base = 0
    for cam in cams:
        sc = w.scenes[cam.scene]
        keep, rz, rr = O.bin_f32(sc, cam, oo)
        k = keep.astype(bool)
        assert (zb[rec_base:rec_base + sc.n][k] == rz[k]).all(), "z_start bits differ"
        trect[rec_base:rec_base + sc.n] = rr
        keep_all[rec_base:rec_base + sc.n] = k
        tx = -(-cam.width // opts.tile_w)
        rec_off.append(rec_base)
        tile_off.append(tile_base)
        tiles_x.append(tx)
        rec_base += sc.n
        tile_base += tx * (-(-cam.height // opts.tile_h))
    n = len(keys)
    tile = (keys >> np.uint64(32)).astype(np.int64)
    z = (keys & np.uint64(0xffffffff)).astype(np.uint32)
    assert (z == zb[vals]).all()
    assert keep_all[vals].all()
    # strictly increasing (key, record): sorted, and no pair listed twice
    dk = keys[1:] > keys[:-1]
    eq = keys[1:] == keys[:-1]
    assert (dk | (eq & (vals[1:] > vals[:-1]))).all()
    # every pair's tile inside its record's tile rectangle
    view = np.searchsorted(np.asarray(rec_off), vals, side="right") - 1
    local = tile - np.asarray(tile_off)[view]
    txs = np.asarray(tiles_x)[view]
    px, py = local % txs, local // txs
    rr = trect[vals]
    assert ((px >= rr[:, 0]) & (px <= rr[:, 2]) & (py >= rr[:, 1]) & (py <= rr[:, 3])).all()
    # as many pairs per record as its rectangle has tiles
    area = np.where(keep_all, (trect[:, 2] - trect[:, 0] + 1) * (trect[:, 3] - trect[:, 1] + 1), 0)
    assert (np.bincount(vals, minlength=n_rec) == area).all()
    assert n == area.sum()
    # ranges
    cnt = np.bincount(tile, minlength=tile_base)
    ends = np.cumsum(cnt)
    starts = ends - cnt
    nz = cnt > 0
    assert (ranges[nz, 0] == starts[nz]).all() and (ranges[nz, 1] == ends[nz]).all()
    assert (ranges[~nz] == 0).all()
    print(name, "pairs", n, "records kept", int(keep_all.sum()), "of", n_rec)
