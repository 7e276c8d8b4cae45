"""Helpers shared by the GPU parity tests: run the HIP renderer and the CPU
oracle on the same seeded inputs and compare them with the stated protocol.

Comparison protocol (FP32 GPU against the FP64 oracle):
  * images: relative L2 over the compared pixels <= 1e-4, and per pixel
    |d| <= 1e-4 max(|ref|, 1e-2 max|ref|);
  * pixels whose decision margin is small (cutoff |q - r^2|/r^2 < 1e-6, depth gap
    |z_start - z_max|/z_max < 1e-5) are excluded: FP32 and FP64 may
    legitimately take the other branch there; at most 0.1% of the pixels;
  * a covering fragment (FP64 decisions) that the FP32 binning misses -- its
    surfel culled, or the pixel outside its rectangle -- fails the comparison
    (`viol`); nothing is masked for it;
  * pixels that are ill-conditioned in FP32 -- whose FP64 value moves by more than
    half the per-pixel bound when the FP32 surfel inputs are perturbed by 4 ulps
    (thin, grazing ellipses) -- are held to a wider bound instead:
    |d| <= bound + 2 c, with c the value's shift under that perturbation (an FP32
    evaluation of the same decisions carries input-sized rounding errors, so its
    error is of the order of c); each is reported;
  * gradients: relative L2 <= 1e-3 per parameter group, with dL/dimage zero on
    the excluded pixels; and per surfel, the error of each group's gradient
    vector |d_s| <= 1e-2 |ref_s| + 1e-4 max_s |ref_s| (an FP32 sum over a
    surfel's fragments carries relative errors ~1e-6, amplified where its
    fragments' contributions cancel, hence the floor at a small fraction of the
    largest surfel gradient).
"""
import numpy as np

CUT_MARGIN = 1e-6
GAP_MARGIN = 1e-5
COND_ULPS = 4
COND_WIDEN = 2.0
IMG_REL_L2 = 1e-4
IMG_PIX = 1e-4
GRAD_REL_L2 = 1e-3
MAX_MASKED = 1e-3
SURFEL_REL = 1e-2
SURFEL_FLOOR = 1e-4


def oracle_options(O, opts):
    return O.Options(r_cut=opts.r_cut, gamma=opts.gamma, sigma_f=opts.sigma_f, k_max=opts.k_max,
                     shade=opts.shade, tile_w=opts.tile_w, tile_h=opts.tile_h,
                     mip=getattr(opts, "mip", "centre"), t_min=getattr(opts, "t_min", 0.0),
                     tonemap=getattr(opts, "tonemap", "linear"))


def oracle_maps(O, scenes, shade):
    if shade != "splitsum":
        return [None] * len(scenes), None
    maps = [O.envmap(np.asarray(s.envmap, np.float64)) for s in scenes]
    return maps, O.brdf_lut(64, 64, 1024)


def perturbed(scene, seed, ulps=COND_ULPS):
    """The scene with every geometric float32 input moved by about `ulps` ulps."""
    import copy
    rng = np.random.default_rng(seed)
    sc = copy.copy(scene)
    for k in ("position", "normal", "tangent", "scale"):
        a = np.asarray(getattr(scene, k), np.float32)
        f = 1.0 + ulps * 2.0 ** -24 * rng.choice([-1.0, 1.0], size=a.shape)
        setattr(sc, k, np.ascontiguousarray((a.astype(np.float64) * f).astype(np.float32)))
    return sc


def oracle_forward(O, scenes, cameras, opts, pix_per_view, maps, lut, conditioning=True):
    out = []
    oo = oracle_options(O, opts)
    for v, cam in enumerate(cameras):
        sc = scenes[cam.scene]
        hw = tuple(np.asarray(sc.envmap).shape[:2]) if maps[cam.scene] is not None else (0, 0)
        r = O.render(sc, cam, oo, pix_per_view[v], maps=maps[cam.scene], lut=lut, env_hw=hw)
        if conditioning:
            rp = O.render(perturbed(sc, 1000 + v), cam, oo, pix_per_view[v], maps=maps[cam.scene],
                          lut=lut, env_hw=hw)
            r["cond"] = np.abs(np.concatenate([rp["image"] - r["image"], (rp["alpha"] - r["alpha"])[:, None]], 1))
        out.append(r)
    return out


def decision_ok(r, exact_ties=False):
    """Pixels whose decisions FP32 and FP64 take alike.  exact_ties: the scene's
    depth ties are exact in both precisions (zero-extent intervals at one
    representable depth, identity view), so a zero depth gap is no ambiguity."""
    ok = r["cut_margin"] >= CUT_MARGIN
    return ok if exact_ties else ok & (r["gap_margin"] >= GAP_MARGIN)


def pixel_index(cameras, v, pix):
    off = sum(c.width * c.height for c in cameras[:v])
    return off + pix[:, 1] * cameras[v].width + pix[:, 0]


def compare_images(cameras, pix_per_view, ref, img_gpu, alpha_gpu, exact_ties=False):
    """Returns (report dict, list of per-view boolean 'compared' masks)."""
    img_gpu = np.asarray(img_gpu, np.float64)
    alpha_gpu = np.asarray(alpha_gpu, np.float64)
    refs, gots, masks, conds = [], [], [], []
    n_masked = n_cut = n_gap = n_viol = 0
    n_total = 0
    for v, cam in enumerate(cameras):
        r = ref[v]
        ok = decision_ok(r, exact_ties)
        n_viol += int(r["viol"].sum())
        idx = pixel_index(cameras, v, pix_per_view[v])
        refs.append(np.concatenate([r["image"], r["alpha"][:, None]], 1)[ok])
        gots.append(np.concatenate([img_gpu[idx], alpha_gpu[idx][:, None]], 1)[ok])
        conds.append(r["cond"][ok] if "cond" in r else np.zeros((int(ok.sum()), 4)))
        masks.append(ok)
        n_masked += int((~ok).sum())
        n_cut += int((r["cut_margin"] < CUT_MARGIN).sum())
        n_gap += 0 if exact_ties else int((r["gap_margin"] < GAP_MARGIN).sum())
        n_total += ok.size
    R = np.concatenate(refs)
    G = np.concatenate(gots)
    Cd = np.concatenate(conds)
    d = np.abs(G - R)
    rel_l2 = float(np.linalg.norm(G - R) / max(np.linalg.norm(R), 1e-30))
    bound = IMG_PIX * np.maximum(np.abs(R), 1e-2 * np.abs(R).max())
    well = (Cd <= 0.5 * bound).all(1) if d.size else np.zeros(0, bool)
    n_cond = int((~well).sum())
    # per-pixel bound; ill-conditioned pixels against the wider bound + 2 c
    wide = bound + COND_WIDEN * Cd
    ratio = np.where(well, (d / bound).max(1), (d / wide).max(1)) if d.size else np.zeros(0)
    worst = float(ratio.max()) if d.size else 0.0
    cond_ratio = float(ratio[~well].max()) if n_cond else 0.0
    # details of the worst compared pixels (for failure messages)
    info = []
    if d.size:
        allpix = np.concatenate([p[m] for p, m in zip(pix_per_view, masks)])
        allref = [dict((k, r[k][m]) for k in ("cut_margin", "gap_margin", "n_layers")) for r, m in zip(ref, masks)]
        cm = np.concatenate([a["cut_margin"] for a in allref])
        gm = np.concatenate([a["gap_margin"] for a in allref])
        nl = np.concatenate([a["n_layers"] for a in allref])
        for i in np.argsort(-ratio)[:4]:
            info.append(dict(pix=allpix[i].tolist(), ref=R[i].round(7).tolist(), got=G[i].round(7).tolist(),
                             ratio=round(float(ratio[i]), 3), cut=float(cm[i]), gap=float(gm[i]), nl=int(nl[i])))
    return dict(rel_l2=rel_l2, worst_pixel_ratio=worst, masked=n_masked, total=n_total,
                masked_frac=n_masked / max(n_total, 1), masked_cut=n_cut, masked_gap=n_gap, viol=n_viol,
                cond_pixels=n_cond, cond_frac=n_cond / max(n_total, 1), cond_worst_ratio=cond_ratio,
                worst=info), masks


def assert_image_parity(rep):
    assert rep["viol"] == 0, rep
    assert rep["masked_frac"] <= MAX_MASKED, rep
    assert rep["rel_l2"] <= IMG_REL_L2, rep
    assert rep["worst_pixel_ratio"] <= 1.0, rep


def rel_l2(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def per_surfel_report(got, want):
    """Per surfel (columns of a [C][N] gradient group): the worst ratio of the
    error to the bound SURFEL_REL |ref_s| + SURFEL_FLOOR max |ref|, and the
    surfels over it."""
    got = np.asarray(got, np.float64).reshape(-1, np.shape(got)[-1])
    want = np.asarray(want, np.float64).reshape(-1, np.shape(want)[-1])
    err = np.linalg.norm(got - want, axis=0)
    ref = np.linalg.norm(want, axis=0)
    bound = SURFEL_REL * ref + SURFEL_FLOOR * max(ref.max(), 1e-30)
    ratio = err / bound
    over = np.nonzero(ratio > 1.0)[0]
    return dict(worst=float(ratio.max()) if ratio.size else 0.0, over=over[:10].tolist(), n_over=int(over.size))
