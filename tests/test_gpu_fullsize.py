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


def bench_options(ss, name, shade):
    from paper_2605_05876_amd import autotune
    t = autotune.lookup(name) or {}
    return ss.Options(shade=shade, tile_w=t.get("tile_w", 16), tile_h=t.get("tile_h", 16),
                      lds_batch=t.get("lds_batch", 128))


def tile_list_lengths(O, scene, cam, opts):
    """Records per tile, from the oracle's FP32 tile rectangles (2-D prefix sums)."""
    keep, _, rect = O.bin_f32(scene, cam, oracle_options(O, opts))
    tx, ty = -(-cam.width // opts.tile_w), -(-cam.height // opts.tile_h)
    r = rect[keep.astype(bool)].astype(np.int64)
    d = np.zeros((ty + 1, tx + 1), np.int64)
    np.add.at(d, (r[:, 1], r[:, 0]), 1)
    np.add.at(d, (r[:, 1], r[:, 2] + 1), -1)
    np.add.at(d, (r[:, 3] + 1, r[:, 0]), -1)
    np.add.at(d, (r[:, 3] + 1, r[:, 2] + 1), 1)
    return d.cumsum(0).cumsum(1)[:ty, :tx]


def sample(O, scene, cam, opts, k, seed):
    """k pixels, seeded: a quarter in the tiles with the longest lists (the
    density clusters, deepest layer walks), a quarter on the image border rows
    and columns (clipped rectangles, ragged tiles), half uniform over the image."""
    rng = np.random.default_rng(seed)
    W, H = cam.width, cam.height
    kc, kb = k // 4, k // 4
    ku = k - kc - kb
    cnt = tile_list_lengths(O, scene, cam, opts)
    top = np.argsort(cnt.ravel())[::-1][:max(4, kc // 4)]
    t = top[rng.integers(0, len(top), kc)]
    tyi, txi = t // cnt.shape[1], t % cnt.shape[1]
    cx = np.minimum(txi * opts.tile_w + rng.integers(0, opts.tile_w, kc), W - 1)
    cy = np.minimum(tyi * opts.tile_h + rng.integers(0, opts.tile_h, kc), H - 1)
    side = rng.integers(0, 4, kb)
    along = rng.random(kb)
    bx = np.where(side == 0, 0, np.where(side == 1, W - 1, (along * W).astype(np.int64)))
    by = np.where(side == 2, 0, np.where(side == 3, H - 1, (along * H).astype(np.int64)))
    ux, uy = rng.integers(0, W, ku), rng.integers(0, H, ku)
    xy = np.stack([np.concatenate([cx, bx, ux]), np.concatenate([cy, by, uy])], 1)
    return np.unique(xy, axis=0).astype(np.int32)


def stratified(cam, cell, seed):
    """One seeded pixel in every cell x cell block of the image (ragged edges kept)."""
    rng = np.random.default_rng(seed)
    ys, xs = np.mgrid[0:cam.height:cell, 0:cam.width:cell]
    x = np.minimum(xs.ravel() + rng.integers(0, cell, xs.size), cam.width - 1)
    y = np.minimum(ys.ravel() + rng.integers(0, cell, ys.size), cam.height - 1)
    return np.stack([x, y], 1).astype(np.int32)


@pytest.mark.parametrize("name,k", [("C2", 0), ("C3", 96), ("C4", 160), ("C5", 64)])
def test_fullsize_sampled_parity(O, ss, name, k):
    """C2 on a stratified grid (one pixel per 4 x 4 block: 16384 of its 262144
    pixels; the whole image would take the oracle minutes), the others on
    cluster + border + uniform samples of every view."""
    w = g.make_config(name)
    opts = bench_options(ss, name, w.shade)
    cams = w.cameras
    if k == 0:
        pix = [stratified(c, 4, 100 + v) for v, c in enumerate(cams)]
    else:
        pix = [sample(O, w.scenes[c.scene], c, opts, k, 100 + v) for v, c in enumerate(cams)]
    maps, lut = oracle_maps(O, w.scenes, w.shade)
    ref = oracle_forward(O, w.scenes, cams, opts, pix, maps, lut)
    r = ss.Renderer(opts)
    b = ss.batch_from_scenes(w.scenes, cams)
    img, a, nl = r.forward(b, want_layers=True)
    assert r.poll()["status"] == 0
    rep, masks = compare_images(cams, pix, ref, img.cpu().numpy(), a.cpu().numpy())
    print(name, "forward", {k_: v for k_, v in rep.items() if k_ != "worst"})
    assert_image_parity(rep)
    # the samples exercise the layer separation (Alg. 1): some pixels composite several layers
    assert max(int(r["n_layers"].max()) for r in ref) >= 2
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
        got, want = grads[n].cpu().numpy(), np.concatenate([rg[n] for rg in ref_g], axis=-1)
        errs[n] = rel_l2(got, want)
        ps = per_surfel_report(got, want)
        print(name, n, "per surfel", ps)
        assert ps["n_over"] == 0, (n, ps)
    for i, sc in enumerate(w.scenes):
        dE = O.envmap_adjoint(ref_maps[i], *sc.envmap.shape[:2])
        errs[f"envmap{i}"] = rel_l2(grads["envmap"][i].cpu().numpy(), dE)
    print(name, "backward", errs)
    assert max(errs.values()) <= GRAD_REL_L2, errs


@pytest.mark.parametrize("name", ["C3", "C4"])
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
