"""Pins for the oracle's depth-consolidation term (eq:cons_loss, Sec. 3.7.1):
per pixel, sum_{i<j} w_i w_j |z_i - z_j| + sum_i w_i^2 sigma_i^2 over the
composited layers, with w_i = T_i alpha_i and z_i, sigma_i^2 the Shepard-weighted
mean and variance of the layer's fragment depths.

* fronto-parallel lattice planes: every fragment of a plane has the plane's
  depth, so the term is w1 w2 |z1 - z2| with W from the lattice sum;
* tilted planes: fragment depths and weights from an independent world-space
  ray/plane solve per surfel; separated planes give two layers, a thin shell
  one merged layer whose variance is W_a W_b (z_a - z_b)^2 / W^2;
* the tape adjoint of the term against dual-number JVPs, and the JVPs against
  central finite differences.
"""
import math

import numpy as np
import pytest

import scenegen as g
from conftest import axis_camera, make_scene
from test_oracle_pins import KAPPA, concat, f32, lattice, lattice_weights, tilted_plane

PARAMS = ["position", "normal", "tangent", "scale", "albedo", "roughness", "metallic"]


def test_fronto_parallel_planes(oracle_lib):
    O = oracle_lib
    cam = axis_camera(64, 64, 100.0)
    s = 0.05
    pix = np.array([[32, 32], [34, 30], [29, 35]])
    front = lattice(int(1.0 / (2 * s)) | 1, 2 * s, s, 2.0, seed=1)
    back = lattice(41, s, s, 2.6, seed=2)
    r1 = O.render(make_scene(*front), cam, O.Options(sigma_f=0.0), pix)
    np.testing.assert_array_equal(r1["cons"], 0.0)      # one flat layer: no spread
    r = O.render(make_scene(*concat(front, back)), cam, O.Options(sigma_f=0.0), pix)
    for k, (px, py) in enumerate(pix):
        W1 = lattice_weights(front[0], s, 2.0, cam, px, py, 3.0).sum()
        W2 = lattice_weights(back[0], s, 2.6, cam, px, py, 3.0).sum()
        a1, a2 = 1 - math.exp(-KAPPA * W1), 1 - math.exp(-KAPPA * W2)
        expect = a1 * (1 - a1) * a2 * (f32(2.6) - f32(2.0))
        assert r["n_layers"][k] == 2
        assert abs(r["cons"][k] - expect) <= 1e-12 * expect


def _fragments(cam, px, py, parts, rcut=3.0):
    """Per plane: (weights, depths) of the surfels reaching pixel (px, py), from a
    ray/plane intersection with each surfel's own FP32 centre and normal."""
    d = np.array([(px + 0.5 - f32(cam.cx)) / f32(cam.fx), (py + 0.5 - f32(cam.cy)) / f32(cam.fy), 1.0])
    out = []
    for pos, nrm, _, scl, _ in parts:
        c = f32(pos)
        n = f32(nrm)
        n = n / np.linalg.norm(n, axis=1, keepdims=True)
        t = (n * c).sum(1) / (n @ d)
        hit = t[:, None] * d[None]
        q = ((hit - c) ** 2).sum(1) / f32(scl[:, 0]) ** 2
        assert np.abs(q - rcut * rcut).min() > 1e-9
        m = q < rcut * rcut
        out.append((np.exp(-0.5 * q[m]), t[m]))
    return out


def _layer(w, z):
    W = w.sum()
    zm = (w * z).sum() / W
    return W, zm, (w * (z - zm) ** 2).sum() / W


def test_tilted_planes_separated_and_thin_shell(oracle_lib):
    O = oracle_lib
    cam = axis_camera(64, 64, 100.0)
    s, th = 0.05, math.radians(30)
    pix = np.array([[32, 32], [30, 33], [36, 28]])
    opt = O.Options(sigma_f=0.0)
    a = tilted_plane(25, s, s, 2.0, th, 1)
    far_b = tilted_plane(25, s, s, 2.6, th, 2)
    near_b = tilted_plane(25, s, s, 2.02, th, 2)
    rf = O.render(make_scene(*concat(a, far_b)), cam, opt, pix)
    rn = O.render(make_scene(*concat(a, near_b)), cam, opt, pix)
    for k, (px, py) in enumerate(pix):
        # separated: two layers, each (nearly) flat
        (wa, za), (wb, zb) = _fragments(cam, px, py, [a, far_b])
        Wa, ma, va = _layer(wa, za)
        Wb, mb, vb = _layer(wb, zb)
        aa, ab = 1 - math.exp(-KAPPA * Wa), 1 - math.exp(-KAPPA * Wb)
        w1, w2 = aa, (1 - aa) * ab
        expect = w1 * w2 * abs(ma - mb) + w1 * w1 * va + w2 * w2 * vb
        assert rf["n_layers"][k] == 2
        assert abs(rf["cons"][k] - expect) <= 1e-10 * expect, (rf["cons"][k], expect)
        # thin shell: one merged layer; variance W_a W_b (z_a - z_b)^2 / W^2
        (wa, za), (wb, zb) = _fragments(cam, px, py, [a, near_b])
        W, zm, var = _layer(np.r_[wa, wb], np.r_[za, zb])
        Wa, Wb = wa.sum(), wb.sum()
        spread = Wa * Wb * (za.mean() - zb.mean()) ** 2 / W ** 2
        assert abs(var - spread) <= 1e-6 * spread      # both planes are flat
        al = 1 - math.exp(-KAPPA * W)
        expect = al * al * var
        assert rn["n_layers"][k] == 1
        assert abs(rn["cons"][k] - expect) <= 1e-9 * expect, (rn["cons"][k], expect)


def _multi_layer_scene():
    w = g.make_config("C1", n_scale=0.3, res_scale=0.375)
    return w.scenes[0], w.cameras[0]


@pytest.mark.parametrize("sigma", [0.0, 0.3])
def test_cons_adjoint_matches_dual_jvp(oracle_lib, sigma):
    O = oracle_lib
    sc, cam = _multi_layer_scene()
    opt = O.Options(sigma_f=sigma)
    pix = O.all_pixels(cam)
    r = O.render(sc, cam, opt, pix)
    assert r["n_layers"].max() >= 2 and (r["cons"] > 0).sum() > 100
    rng = np.random.default_rng(21)
    dc = rng.normal(size=len(pix))
    G = rng.normal(size=(len(pix), 3))
    gr = O.render_grad(sc, cam, opt, pix, 0 * G, None, dcons=dc)
    grG = O.render_grad(sc, cam, opt, pix, G, None, dcons=dc)
    grI = O.render_grad(sc, cam, opt, pix, G, None)
    for k in PARAMS:      # linear in the loss weights
        np.testing.assert_allclose(grG[k], gr[k] + grI[k], rtol=1e-9, atol=1e-12)
    for k in ("position", "normal", "tangent", "scale"):
        v = {k: rng.normal(size=getattr(sc, k).shape)}
        jv = O.render_jvp(sc, cam, opt, pix, v)
        lhs = (dc * jv["cons_dot"]).sum()
        rhs = (gr[k] * v[k]).sum()
        assert abs(lhs - rhs) <= 1e-10 * max(1e-3, abs(lhs)), (k, lhs, rhs)
    assert np.abs(gr["albedo"]).max() == 0      # depth statistics do not see colour


def test_cons_jvp_matches_finite_differences(oracle_lib):
    O = oracle_lib
    sc, cam = _multi_layer_scene()
    opt = O.Options(sigma_f=0.1)
    pix = O.all_pixels(cam)
    rng = np.random.default_rng(4)
    dc = rng.normal(size=len(pix))
    r0 = O.render_grad(sc, cam, opt, pix, np.zeros((len(pix), 3)), None, dcons=dc)
    live = np.nonzero(np.abs(r0["position"]).sum(0) > 0)[0]

    def objective():
        return (dc * O.render(sc, cam, opt, pix)["cons"]).sum()

    checked = 0
    for k in ("position", "normal", "tangent", "scale"):
        arr = getattr(sc, k)
        for trial in range(6):
            i = int(rng.choice(live))
            idx = (int(rng.integers(0, arr.shape[0])), i)
            p = float(arr[idx])
            v = {k: np.zeros(arr.shape)}
            v[k][idx] = 1.0
            d = (dc * O.render_jvp(sc, cam, opt, pix, v)["cons_dot"]).sum()

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
            if abs(f1 - f2) > 2e-3 * scale:       # a decision flipped inside the step
                continue
            fr = (4 * f2 - f1) / 3
            assert abs(fr - d) <= 2e-4 * scale + 1e-7, (k, idx, fr, d, f1, f2)
            checked += 1
    assert checked >= 12
