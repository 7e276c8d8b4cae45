"""Pins for the oracle's auxiliary images (Sec. 4.2.3): the normal image (per layer
the Shepard mean of the unit normals, renormalised to unit length, composited
like colour) and the composited depth sum_k T_k alpha_k z_k.

* one flat tilted plane: the normal image is alpha n + (1 - alpha) bg exactly;
* two tilted planes of different orientation, separated (two layers) and as a
  thin shell (one layer, normal = normalize(W_a n_a + W_b n_b)), with weights
  and depths from an independent ray/plane solve per surfel;
* fronto-parallel lattice planes: depth = a1 z1 + (1 - a1) a2 z2 with the
  lattice-sum weights;
* adjoints against dual-number JVPs, JVPs against finite differences.
"""
import math

import numpy as np
import pytest

import scenegen as g
from conftest import axis_camera, make_scene
from test_oracle_cons import _fragments
from test_oracle_pins import KAPPA, concat, f32, lattice, lattice_weights

PARAMS = ["position", "normal", "tangent", "scale", "albedo", "roughness", "metallic"]


def plane(n_side, spacing, s, z0, theta, phi=0.0, seed=0):
    """Square lattice of isotropic surfels on the plane through (0, 0, z0) with
    normal (sin th sin ph, -sin th cos ph, cos th) (facing the camera at -z)."""
    n = np.array([math.sin(theta) * math.sin(phi), -math.sin(theta) * math.cos(phi), math.cos(theta)])
    a = np.cross(n, [0.0, 0.0, 1.0]) if abs(n[2]) < 0.999 else np.array([1.0, 0.0, 0.0])
    a /= np.linalg.norm(a)
    b = np.cross(n, a)
    gr = (np.arange(n_side) - (n_side - 1) / 2.0) * spacing
    U, V = np.meshgrid(gr, gr, indexing="ij")
    pos = np.array([0.0, 0.0, z0]) + U.ravel()[:, None] * a + V.ravel()[:, None] * b
    m = pos.shape[0]
    rng = np.random.default_rng(seed)
    return pos, np.tile(-n, (m, 1)), np.tile(a, (m, 1)), np.full((m, 2), s), rng.uniform(0, 1, (m, 3))


def _unit(v):
    v = f32(v)
    return v / np.linalg.norm(v)


def test_normal_image_flat_plane(oracle_lib):
    O = oracle_lib
    bg = (0.1, 0.2, 0.3)
    cam = axis_camera(64, 64, 100.0, background=bg)
    p = plane(25, 0.05, 0.05, 2.0, math.radians(30), 0.4, seed=1)
    pix = np.array([[32, 32], [30, 35], [36, 29]])
    r = O.render(make_scene(*p), cam, O.Options(sigma_f=0.0, shade="normal"), pix)
    nv = _unit(p[1][0])
    for k, (px, py) in enumerate(pix):
        (w, _), = _fragments(cam, px, py, [p])
        a = 1 - math.exp(-KAPPA * w.sum())
        np.testing.assert_allclose(r["image"][k], a * nv + (1 - a) * f32(bg), rtol=0, atol=1e-12)


def test_normal_image_two_orientations(oracle_lib):
    O = oracle_lib
    cam = axis_camera(64, 64, 100.0)
    opt = O.Options(sigma_f=0.0, shade="normal")
    pa = plane(25, 0.05, 0.05, 2.0, math.radians(30), 0.0, seed=1)
    far = plane(25, 0.05, 0.05, 2.6, math.radians(40), 1.0, seed=2)
    near = plane(25, 0.05, 0.05, 2.01, math.radians(35), 0.2, seed=3)
    pix = np.array([[32, 32], [31, 34]])
    rf = O.render(make_scene(*concat(pa, far)), cam, opt, pix)
    rn = O.render(make_scene(*concat(pa, near)), cam, opt, pix)
    na, nf, nn = _unit(pa[1][0]), _unit(far[1][0]), _unit(near[1][0])
    for k, (px, py) in enumerate(pix):
        (wa, _), (wb, _) = _fragments(cam, px, py, [pa, far])
        a1, a2 = 1 - math.exp(-KAPPA * wa.sum()), 1 - math.exp(-KAPPA * wb.sum())
        assert rf["n_layers"][k] == 2
        np.testing.assert_allclose(rf["image"][k], a1 * na + (1 - a1) * a2 * nf, rtol=0, atol=1e-12)
        (wa, _), (wb, _) = _fragments(cam, px, py, [pa, near])
        Wa, Wb = wa.sum(), wb.sum()
        m = Wa * na + Wb * nn
        al = 1 - math.exp(-KAPPA * (Wa + Wb))
        assert rn["n_layers"][k] == 1
        np.testing.assert_allclose(rn["image"][k], al * m / np.linalg.norm(m), rtol=0, atol=1e-12)


def test_depth_fronto_parallel_planes(oracle_lib):
    O = oracle_lib
    cam = axis_camera(64, 64, 100.0)
    s = 0.05
    front = lattice(int(1.0 / (2 * s)) | 1, 2 * s, s, 2.0, seed=1)
    back = lattice(41, s, s, 2.6, seed=2)
    pix = np.array([[32, 32], [34, 30]])
    r = O.render(make_scene(*concat(front, back)), cam, O.Options(sigma_f=0.0), pix)
    for k, (px, py) in enumerate(pix):
        W1 = lattice_weights(front[0], s, 2.0, cam, px, py, 3.0).sum()
        W2 = lattice_weights(back[0], s, 2.6, cam, px, py, 3.0).sum()
        a1, a2 = 1 - math.exp(-KAPPA * W1), 1 - math.exp(-KAPPA * W2)
        expect = a1 * f32(2.0) + (1 - a1) * a2 * f32(2.6)
        assert abs(r["depth"][k] - expect) <= 1e-13 * expect


def _scene():
    w = g.make_config("C1", n_scale=0.3, res_scale=0.375)
    return w.scenes[0], w.cameras[0]


@pytest.mark.parametrize("what", ["depth", "normal"])
def test_aux_adjoint_matches_dual_jvp(oracle_lib, what):
    O = oracle_lib
    sc, cam = _scene()
    opt = O.Options(sigma_f=0.2, shade="normal" if what == "normal" else "albedo")
    pix = O.all_pixels(cam)
    rng = np.random.default_rng(31)
    G = rng.normal(size=(len(pix), 3))
    dz = rng.normal(size=len(pix)) if what == "depth" else None
    if what == "depth":
        G = 0 * G
    gr = O.render_grad(sc, cam, opt, pix, G, None, ddepth=dz)
    for k in ("position", "normal", "tangent", "scale"):
        v = {k: rng.normal(size=getattr(sc, k).shape)}
        jv = O.render_jvp(sc, cam, opt, pix, v)
        lhs = (G * jv["image_dot"]).sum() + (0.0 if dz is None else (dz * jv["depth_dot"]).sum())
        rhs = (gr[k] * v[k]).sum()
        assert abs(lhs - rhs) <= 1e-10 * max(1e-3, abs(lhs)), (k, lhs, rhs)
    assert np.abs(gr["albedo"]).max() == 0


@pytest.mark.parametrize("what", ["depth", "normal"])
def test_aux_jvp_matches_finite_differences(oracle_lib, what):
    O = oracle_lib
    sc, cam = _scene()
    opt = O.Options(sigma_f=0.1, shade="normal" if what == "normal" else "albedo")
    pix = O.all_pixels(cam)
    rng = np.random.default_rng(8)
    wts = rng.normal(size=len(pix)) if what == "depth" else rng.normal(size=(len(pix), 3))

    def objective():
        r = O.render(sc, cam, opt, pix)
        return (wts * (r["depth"] if what == "depth" else r["image"])).sum()

    if what == "depth":
        r0 = O.render_grad(sc, cam, opt, pix, np.zeros((len(pix), 3)), None, ddepth=wts)
    else:
        r0 = O.render_grad(sc, cam, opt, pix, wts, None)
    live = np.nonzero(np.abs(r0["position"]).sum(0) > 0)[0]
    checked = 0
    for k in ("position", "normal", "scale"):
        arr = getattr(sc, k)
        for trial in range(6):
            i = int(rng.choice(live))
            idx = (int(rng.integers(0, arr.shape[0])), i)
            p = float(arr[idx])
            v = {k: np.zeros(arr.shape)}
            v[k][idx] = 1.0
            jv = O.render_jvp(sc, cam, opt, pix, v)
            d = (wts * (jv["depth_dot"] if what == "depth" else jv["image_dot"])).sum()

            def fd(h):
                hi, lo = np.float32(p + h), np.float32(p - h)
                arr[idx] = hi
                fp = objective()
                arr[idx] = lo
                fm = objective()
                arr[idx] = np.float32(p)
                return (fp - fm) / (float(hi) - float(lo))
            h = 2e-3 * max(abs(p), 0.05)
            f1, f2 = fd(h), fd(h / 2)
            scale = max(abs(d), 1e-3 * np.abs(r0[k]).max(), 1e-8)
            if abs(f1 - f2) > 2e-3 * scale:
                continue
            fr = (4 * f2 - f1) / 3
            assert abs(fr - d) <= 2e-4 * scale + 1e-7, (k, idx, fr, d, f1, f2)
            checked += 1
    assert checked >= 9
