"""Pins of the oracle's two output options.

* Tone map (the log-space + sRGB transfer applied to HDR images with
  eq:photo_loss, Sec. 3.7.1): a dense constant-colour plane whose linear value
  is known reproduces tabulated sRGB encodings (IEC 61966-2-1: the segment
  joint 0.0031308 -> 0.04045, 18% grey -> 0.46136, 0.5 -> 0.73536, 1 -> 1);
  decoding the tone-mapped image with the standard's inverse and expm1
  recovers the linear render; derivatives through it match dual-number JVPs
  and central differences.
* Early-out t_min: on stacked sparse planes the walk ends after the first
  layer whose transmittance behind it drops below t_min, with the image and
  alpha of that prefix (closed form from lattice sums); t_min = 0 is the exact
  semantics.
"""
import math

import numpy as np
import pytest

from conftest import axis_camera, make_scene
from test_oracle_grad import PARAMS, _objective, small_albedo
from test_oracle_pins import KAPPA, concat, f32, lattice, lattice_weights

# (linear value v of the sRGB encoding, its tabulated encoding)
SRGB_TABLE = [(0.0031308, 0.04045), (0.18, 0.46136), (0.5, 0.73536), (1.0, 1.0)]


def srgb_decode(y):
    """IEC 61966-2-1 decoding (the inverse of the encoding)."""
    y = np.asarray(y, np.float64)
    return np.where(y <= 0.04045, y / 12.92, ((y + 0.055) / 1.055) ** 2.4)


def test_tonemap_tabulated_srgb_values(oracle_lib):
    """log(1 + x) = v: a plane of colour x = e^v - 1 at full coverage gives srgb(v)."""
    O = oracle_lib
    cam = axis_camera(48, 48, 100.0)
    s = 0.05
    pix = np.array([[24, 24], [22, 27]])
    for v, want in SRGB_TABLE:
        x = math.expm1(v)
        sc = make_scene(*lattice(41, s / 3, s, 2.0, color=[x, x, x]))
        r = O.render(sc, cam, O.Options(sigma_f=0.0, tonemap="srgb_log"), pix)
        lin = O.render(sc, cam, O.Options(sigma_f=0.0), pix)
        np.testing.assert_allclose(lin["image"], float(f32(x)), rtol=1e-15)
        # the plane's colour is x rounded to float32: its encoding moves by at
        # most the slope times that rounding, far below the table's 5e-6
        np.testing.assert_allclose(r["image"], want, atol=6e-6)
        np.testing.assert_array_equal(r["alpha"], lin["alpha"])


def test_tonemap_inverts_to_linear_render(oracle_lib):
    O = oracle_lib
    sc, cam, *_ = small_albedo()
    sc.albedo = np.ascontiguousarray(sc.albedo * 3.0, np.float32)   # HDR values above 1
    pix = O.all_pixels(cam)
    lin = O.render(sc, cam, O.Options(), pix)
    tm = O.render(sc, cam, O.Options(tonemap="srgb_log"), pix)
    assert lin["image"].max() > 1.5 and (tm["image"] >= 0).all()
    np.testing.assert_allclose(np.expm1(srgb_decode(tm["image"])), lin["image"], rtol=1e-12, atol=1e-15)
    np.testing.assert_array_equal(tm["alpha"], lin["alpha"])
    np.testing.assert_array_equal(tm["n_layers"], lin["n_layers"])


@pytest.mark.parametrize("opt", [dict(tonemap="srgb_log"), dict(t_min=0.3), dict(t_min=0.3, tonemap="srgb_log")])
def test_adjoint_matches_jvp_with_options(oracle_lib, opt):
    O = oracle_lib
    sc, cam, *_ = small_albedo()
    o = O.Options(**opt)
    pix = O.all_pixels(cam)
    rng = np.random.default_rng(11)
    G = rng.normal(size=(len(pix), 3))
    ga = rng.normal(size=len(pix))
    gr = O.render_grad(sc, cam, o, pix, G, ga)
    for k in ("position", "normal", "scale", "albedo"):
        v = {k: rng.normal(size=getattr(sc, k).shape)}
        jv = O.render_jvp(sc, cam, o, pix, v)
        lhs = (G * jv["image_dot"]).sum() + (ga * jv["alpha_dot"]).sum()
        rhs = (gr[k] * v[k]).sum()
        assert abs(lhs - rhs) <= 1e-10 * max(1.0, abs(lhs)), (k, lhs, rhs)


def test_tonemap_jvp_matches_finite_differences(oracle_lib):
    O = oracle_lib
    sc, cam, *_ = small_albedo()
    o = O.Options(tonemap="srgb_log")
    pix = O.all_pixels(cam)
    rng = np.random.default_rng(5)
    G = rng.normal(size=(len(pix), 3))
    ga = np.zeros(len(pix))
    r0 = O.render_grad(sc, cam, o, pix, G, ga)
    live = np.nonzero(np.abs(r0["position"]).sum(0) > 0)[0]
    checked = 0
    for k in ("position", "albedo", "scale"):
        arr = getattr(sc, k)
        for trial in range(6):
            i = int(rng.choice(live))
            row = int(rng.integers(0, arr.shape[0]))
            p = float(arr[row, i])
            v = {k: np.zeros(arr.shape)}
            v[k][row, i] = 1.0
            jv = O.render_jvp(sc, cam, o, pix, v)
            d = (G * jv["image_dot"]).sum()

            def fd(h):
                hi, lo = np.float32(p + h), np.float32(p - h)
                arr[row, i] = hi
                fp = _objective(O, sc, cam, o, pix, G, ga, None, None, (0, 0))
                arr[row, i] = lo
                fm = _objective(O, sc, cam, o, pix, G, ga, None, None, (0, 0))
                arr[row, i] = np.float32(p)
                return (fp - fm) / (float(hi) - float(lo))
            h = 2e-3 * max(abs(p), 0.05)
            f1, f2 = fd(h), fd(h / 2)
            scale = max(abs(d), 1e-3 * np.abs(r0[k]).max(), 1e-8)
            if abs(f1 - f2) > 2e-3 * scale:
                continue
            fr = (4 * f2 - f1) / 3
            assert abs(fr - d) <= 2e-4 * scale + 1e-7, (k, row, i, fr, d)
            checked += 1
    assert checked >= 9


@pytest.mark.parametrize("t_min", [0.0, 0.5, 0.05, 1e-3])
def test_early_out_on_stacked_planes(oracle_lib, t_min):
    """Sparse planes (spacing 2 s, alpha ~ 0.4 each) one behind the other: the walk
    composites layers while the transmittance in front of the next one stays at or
    above t_min, and the background keeps the transmittance left at that point."""
    O = oracle_lib
    bg = (0.1, 0.2, 0.3)
    cam = axis_camera(64, 64, 100.0, background=bg)
    s = 0.05
    planes = [lattice(7, 2 * s, s, 2.0 + 0.05 * k, seed=30 + k) for k in range(12)]
    sc = make_scene(*concat(*planes))
    pix = np.array([[32, 32], [30, 33]])
    r = O.render(sc, cam, O.Options(sigma_f=0.0, t_min=t_min), pix)
    for k, (px, py) in enumerate(pix):
        T, C, K = 1.0, np.zeros(3), 0
        for j in range(12):
            z = 2.0 + 0.05 * j
            w = lattice_weights(planes[j][0], s, z, cam, px, py, 3.0)
            a = 1 - math.exp(-KAPPA * w.sum())
            C += T * a * (w[:, None] * f32(planes[j][4])).sum(0) / w.sum()
            T *= 1 - a
            K += 1
            if T < t_min:
                break
        assert r["n_layers"][k] == K, (t_min, r["n_layers"][k], K)
        np.testing.assert_allclose(r["image"][k], C + T * f32(bg), rtol=1e-12)
        np.testing.assert_allclose(r["alpha"][k], 1 - T, rtol=1e-12)
        if t_min == 0.0:
            assert K == 12
        elif t_min == 0.5:
            assert K <= 2
