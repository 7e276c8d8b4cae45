"""GPU parity on scenes built to stress single decisions of the method, full
image, forward and backward (image protocol, per-group and per-surfel gradient
bounds of parity_util):

* near plane: surfels straddling znear, partly behind the camera, crossing the
  image border (the cull and the bounding rectangle, App. A.1);
* tie planes: whole planes of equal z_start (the sort's tie-break, Sec. 3.2.1);
  their zero-extent intervals sit at one float32 depth under an identity view,
  so the zero depth gaps are exact in both precisions and are compared;
* occluded planes: an opaque front plane over a second one (eq:compositing);
* thin shell: layers closer than their depth extent merge (Alg. 1, Sec. 5);
* two overlapping spheres: silhouettes and an occlusion edge (Sec. 4.4.3),
  at a reduced resolution;

and invariance under a permutation of the surfels.
"""
import dataclasses
import math

import numpy as np
import pytest

import scenegen as g
from parity_util import GRAD_REL_L2, assert_image_parity, oracle_options, rel_l2
from test_gpu_parity import O, _backward_case, _forward_case, all_pix, ss  # noqa: F401

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _scene(name):
    if name == "near_plane":
        return g.near_plane_workload()
    if name == "tie_planes":
        # the principal point moved off the lattice's symmetry, so no pixel centre
        # sits exactly on a cutoff circle (the ties in depth are untouched)
        w = g.tie_planes_workload()
        c = w.cameras[0]
        w.cameras[0] = dataclasses.replace(c, cx=c.cx + 0.3183, cy=c.cy + 0.2718)
        return w
    if name == "occluded_planes":
        return g.occluded_planes_workload()
    if name == "thin_shell":
        return g.thin_shell_workload()
    return g.two_spheres_workload(n_each=8000, width=200, height=150)


@pytest.mark.parametrize("name", ["near_plane", "tie_planes", "occluded_planes", "thin_shell", "two_spheres"])
def test_scene_parity(O, ss, name):
    w = _scene(name)
    kw = dict(tile_w=16, tile_h=8, exact_ties=(name == "tie_planes"))
    rep = _forward_case(O, ss, w.scenes, w.cameras, w.shade, lambda c, v: all_pix(c), **kw)
    assert_image_parity(rep)
    errs = _backward_case(O, ss, w.scenes, w.cameras, w.shade, lambda c, v: all_pix(c), **kw)
    assert max(errs.values()) <= GRAD_REL_L2, errs


def _permuted(scene, perm):
    return dataclasses.replace(scene, **{k: np.ascontiguousarray(np.asarray(getattr(scene, k))[..., perm])
                                         for k in ("position", "normal", "tangent", "scale", "albedo",
                                                   "roughness", "metallic")})


def _perm_case(name):
    if name == "C1":
        w = g.make_config("C1")
        return w.scenes, w.cameras, w.shade
    if name == "multiview":
        sc = g.superquadric_scene(33, 30_000, scale_mu=math.log(0.012), scale_sigma=0.5)
        sc.envmap = g.lognormal_envmap(33, 16, 32)
        return [sc], [g.look_at_camera(3.0 * d, 72, 56) for d in g.fibonacci_directions(3)], "splitsum"
    w = _scene(name)
    return w.scenes, w.cameras, w.shade


def _tile_ties(keep, zbits, rect):
    """Whether two kept records with equal z_start bits share a tile."""
    k = np.nonzero(keep)[0]
    o = np.argsort(zbits[k], kind="stable")
    ids, z = k[o], zbits[k][o]
    starts = np.nonzero(np.r_[True, z[1:] != z[:-1]])[0]
    ends = np.r_[starts[1:], len(z)]
    for a0, a1 in zip(starts, ends):
        grp = rect[ids[a0:a1]]
        for i in range(len(grp)):
            for j in range(i + 1, len(grp)):
                ri, rj = grp[i], grp[j]
                if ri[0] <= rj[2] and rj[0] <= ri[2] and ri[1] <= rj[3] and rj[1] <= ri[3]:
                    return True
    return False


@pytest.mark.parametrize("name", ["C1", "multiview", "tie_planes"])
def test_permutation_invariance(O, ss, name):
    """The renderer is a function of the set of surfels, not of their order: a
    seeded permutation of every scene's surfels leaves the image unchanged and
    permutes the gradients.  Visiting order is (z_start, index); without equal
    z_start keys in a tile list (checked on the oracle's FP32 binning) every
    per-pixel sequence and every deterministic-mode sum is unchanged, so the
    images and gradients are bit-identical; with ties (the tie planes, a few in
    the multi-view scene) only the order of equal keys moves, so they agree to
    FP32 rounding."""
    scenes, cams, shade = _perm_case(name)
    rng = np.random.default_rng(17)
    perms = [rng.permutation(s.n) for s in scenes]
    pscenes = [_permuted(s, p) for s, p in zip(scenes, perms)]
    opts = ss.Options(shade=shade, deterministic=True)
    oo = oracle_options(O, opts)
    ties = any(_tile_ties(*O.bin_f32(scenes[c.scene], c, oo)) for c in cams)
    assert ties == (name != "C1")     # C1 runs the bit-identical branch
    gen = torch.Generator("cuda").manual_seed(3)
    out = []
    for sc in (scenes, pscenes):
        b = ss.batch_from_scenes(sc, cams)
        r = ss.Renderer(opts)
        img, a, nl = r.forward(b, want_layers=True)
        if not out:
            G = torch.randn((b.n_pixels, 3), device="cuda", generator=gen)
            Ga = torch.randn((b.n_pixels,), device="cuda", generator=gen)
        gr = r.backward(b, G, Ga)
        torch.cuda.synchronize()
        assert r.poll()["status"] == 0
        out.append((img.cpu().numpy(), a.cpu().numpy(), nl.cpu().numpy(), {k: gr[k].cpu().numpy() for k in ss.PARAMS},
                    [e.cpu().numpy() for e in gr["envmap"]] if shade == "splitsum" else []))
    (i0, a0, n0, g0, e0), (i1, a1, n1, g1, e1) = out
    offs = np.cumsum([0] + [s.n for s in scenes])
    order = np.concatenate([offs[i] + p for i, p in enumerate(perms)])
    assert (n0 == n1).all()
    if not ties:
        assert np.array_equal(i0, i1) and np.array_equal(a0, a1)
        for k in ss.PARAMS:
            assert np.array_equal(g1[k], g0[k][..., order]), k
        for x, y in zip(e0, e1):
            assert np.array_equal(x, y)
    else:
        np.testing.assert_allclose(i1, i0, rtol=1e-5, atol=1e-6)
        np.testing.assert_allclose(a1, a0, rtol=1e-5, atol=1e-6)
        pos = np.linalg.norm(g0["position"])
        for k in ss.PARAMS:
            want = g0[k][..., order]
            if np.linalg.norm(want) < 1e-6 * pos:   # analytically zero (isotropic tangent): noise
                assert np.linalg.norm(g1[k] - want) <= 1e-6 * pos, k
            else:
                assert rel_l2(g1[k], want) <= 1e-5, k
