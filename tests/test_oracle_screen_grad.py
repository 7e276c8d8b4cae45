"""Pins for the oracle's densification statistic (Sec. 3.6.1, eq:ss_grad):
per pixel p and surfel i, g = (dL_p/dT1z, dL_p/dT2z) T4z, accumulated as sum |g|.

* closed form for a fronto-parallel isotropic surfel, where the statistic is the
  gradient of L_p with respect to the projected centre (the MIP filter does not
  depend on T1z, T2z there);
* finite differences through the camera translation for tilted anisotropic
  surfels with the MIP filter on: T1z = fx c'_x + cx c'_z and T2z = fy c'_y +
  cy c'_z, so dT1z/dt_x = fx, dT2z/dt_y = fy, and t moves no other T entry;
* for overlapping surfels, the plain vector sum over pixels satisfies
  sum_i vec_x[i] fx / T4z_i = dL/dt_x (all surfels move with the camera), and
  sum |g| >= |sum g| per surfel.
"""
import math

import numpy as np
import pytest

from conftest import axis_camera, make_scene

KAPPA = float(np.float32(2 * math.pi)) / (2 * math.pi)


def f32(x):
    return np.asarray(x, np.float32).astype(np.float64)


@pytest.mark.parametrize("sigma", [0.0, 0.1, 0.7])
def test_fronto_parallel_closed_form(oracle_lib, sigma):
    """One fronto-parallel isotropic surfel: image = a c + (1 - a) bg, a = 1 - e^{-kw},
    w = n_f exp(-d^2 / (2 m^2 (1+phi))), so dL_p/dx0 = dL_p/dw * w (x - x0)/(m^2 (1+phi))
    and g = dL_p/d(x0, y0) since x0 = T1z/T4z."""
    O = oracle_lib
    bg = (0.1, 0.2, 0.3)
    cam = axis_camera(64, 64, 100.0, background=bg)
    c = np.array([0.013, -0.021, 2.0])
    s = 0.05
    alb = np.array([0.2, 0.5, 0.9])
    sc = make_scene(c, [0, 0, -1], [1, 0, 0], [s, s], alb=alb)
    pix = O.all_pixels(cam)
    rng = np.random.default_rng(5)
    G = rng.standard_normal((pix.shape[0], 3))
    ga = rng.standard_normal(pix.shape[0])
    r = O.screen_grad(sc, cam, O.Options(sigma_f=sigma), pix, G, ga)
    cc = f32(c)
    z = cc[2]
    x0 = f32(cam.fx) * cc[0] / z + f32(cam.cx)
    y0 = f32(cam.fy) * cc[1] / z + f32(cam.cy)
    dx = pix[:, 0] + 0.5 - x0
    dy = pix[:, 1] + 0.5 - y0
    m = f32(cam.fx) * f32(s) / z
    phi = f32(sigma) / m ** 2
    v = m * m * (1 + phi)
    q = (dx * dx + dy * dy) / v
    assert np.abs(q - 9.0).min() > 1e-6
    w = np.where(q < 9.0, np.exp(-0.5 * q) / (1 + phi), 0.0)
    e = np.exp(-KAPPA * w)
    dLdw = KAPPA * e * (G @ (f32(alb) - f32(bg)) + ga)
    gx = dLdw * w * dx / v
    gy = dLdw * w * dy / v
    assert r["visible"][0]
    np.testing.assert_allclose(r["abs"][0], np.hypot(gx, gy).sum(), rtol=1e-12)
    np.testing.assert_allclose(r["vec"][:, 0], [gx.sum(), gy.sum()], rtol=1e-10, atol=1e-12)


def _isolated_scene(rng, n_side=3, spacing=0.5, z=2.0):
    """A grid of tilted anisotropic surfels whose footprints do not overlap."""
    pos, nrm, tan, scl = [], [], [], []
    for a in range(n_side):
        for b in range(n_side):
            pos.append([(a - (n_side - 1) / 2) * spacing, (b - (n_side - 1) / 2) * spacing,
                        z + rng.uniform(-0.3, 0.3)])
            th = rng.uniform(0.3, 1.1)
            ph = rng.uniform(0, 2 * np.pi)
            nrm.append([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), -np.cos(th)])
            tan.append(rng.standard_normal(3))
            scl.append(rng.uniform(0.02, 0.05, 2))
    return np.array(pos), np.array(nrm), np.array(tan), np.array(scl)


def _render(O, sc, cam, opt, pix, G, ga):
    r = O.render(sc, cam, opt, pix)
    return (r["image"] * G).sum(1) + r["alpha"] * ga, r


@pytest.mark.parametrize("sigma", [0.0, 0.5])
def test_tilted_surfels_match_camera_fd(oracle_lib, sigma):
    O = oracle_lib
    rng = np.random.default_rng(11 + int(10 * sigma))
    pos, nrm, tan, scl = _isolated_scene(rng)
    alb = rng.uniform(0, 1, (pos.shape[0], 3))
    sc = make_scene(pos, nrm, tan, scl, alb=alb)
    bg = (0.3, 0.1, 0.2)
    cam = axis_camera(96, 96, 120.0, background=bg)
    opt = O.Options(sigma_f=sigma)
    pix = O.all_pixels(cam)
    r_all = O.render(sc, cam, opt, pix)
    assert r_all["n_layers"].max() == 1   # footprints do not overlap
    # pixels whose cutoff decision the FD step cannot flip (the step moves
    # rho^2 by well under 1% of r^2)
    pix = pix[r_all["cut_margin"] > 0.02]
    G = rng.standard_normal((pix.shape[0], 3))
    ga = rng.standard_normal(pix.shape[0])
    sg = O.screen_grad(sc, cam, opt, pix, G, ga)
    L0, r0 = _render(O, sc, cam, opt, pix, G, ga)
    # per-pixel owner: the surfel whose fragment covers the pixel
    owner = np.full(pix.shape[0], -1)
    for k in np.nonzero(r0["n_layers"])[0]:
        owner[k] = O.pixel_fragments(sc, cam, opt, int(pix[k, 0]), int(pix[k, 1]))["idx"][0]

    def dL(axis, h):
        out = []
        for sgn in (1, -1):
            t = np.zeros(3, np.float32)
            t[axis] = sgn * h
            c2 = axis_camera(96, 96, 120.0, t=t, background=bg)
            out.append(_render(O, sc, c2, opt, pix, G, ga)[0])
        return (out[0] - out[1]) / (2 * h)

    h = 2.0 ** -13
    # Richardson: (4 D(h) - D(2h)) / 3 removes the h^2 term
    fdx = (4 * dL(0, h) - dL(0, 2 * h)) / 3
    fdy = (4 * dL(1, h) - dL(1, 2 * h)) / 3
    T4z = f32(pos)[:, 2]   # camera at the origin, R = I: c'_z = c_z
    for i in range(pos.shape[0]):
        mine = owner == i
        assert mine.sum() > 20
        gx = fdx[mine] * T4z[i] / f32(cam.fx)
        gy = fdy[mine] * T4z[i] / f32(cam.fy)
        ref_abs = np.hypot(gx, gy).sum()
        assert sg["visible"][i]
        assert abs(sg["abs"][i] - ref_abs) <= 1e-6 * ref_abs, (i, sg["abs"][i], ref_abs)
        np.testing.assert_allclose(sg["vec"][:, i], [gx.sum(), gy.sum()], rtol=1e-5,
                                   atol=1e-6 * ref_abs)


def test_overlapping_surfels_vector_sum(oracle_lib):
    """Dense overlapping scene (several layers per pixel): the camera-translation
    derivative of the total loss equals sum_i vec[i] f / T4z_i, and |sum g| <= sum |g|."""
    O = oracle_lib
    rng = np.random.default_rng(3)
    n = 60
    pos = np.c_[rng.uniform(-0.25, 0.25, (n, 2)), rng.uniform(1.8, 2.4, n)]
    nrm = np.c_[rng.uniform(-0.5, 0.5, (n, 2)), -np.ones(n)]
    tan = rng.standard_normal((n, 3))
    scl = rng.uniform(0.03, 0.08, (n, 2))
    alb = rng.uniform(0, 1, (n, 3))
    sc = make_scene(pos, nrm, tan, scl, alb=alb)
    bg = (0.2, 0.2, 0.2)
    cam = axis_camera(48, 48, 60.0, background=bg)
    opt = O.Options(sigma_f=0.3)
    pix = O.all_pixels(cam)
    pix = pix[O.render(sc, cam, opt, pix)["cut_margin"] > 0.01]   # no cutoff flips under the FD step
    G = rng.standard_normal((pix.shape[0], 3))
    ga = rng.standard_normal(pix.shape[0])
    sg = O.screen_grad(sc, cam, opt, pix, G, ga)
    L0, r0 = _render(O, sc, cam, opt, pix, G, ga)
    assert r0["n_layers"].max() >= 3

    def dL(axis, h):
        out = []
        for sgn in (1, -1):
            t = np.zeros(3, np.float32)
            t[axis] = sgn * h
            c2 = axis_camera(48, 48, 60.0, t=t, background=bg)
            out.append(_render(O, sc, c2, opt, pix, G, ga)[0].sum())
        return (out[0] - out[1]) / (2 * h)

    T4z = f32(pos)[:, 2]
    for axis, f in ((0, f32(cam.fx)), (1, f32(cam.fy))):
        h = 2.0 ** -16
        fd = (4 * dL(axis, h) - dL(axis, 2 * h)) / 3
        ad = (sg["vec"][axis] * f / T4z).sum()
        assert abs(fd - ad) <= 1e-5 * max(abs(ad), 1e-3 * np.abs(sg["abs"] * f / T4z).sum()), (axis, fd, ad)
    norms = np.hypot(sg["vec"][0], sg["vec"][1])
    assert (norms <= sg["abs"] * (1 + 1e-12) + 1e-300).all()
    assert (sg["abs"][~sg["visible"]] == 0).all()
    assert (norms < 0.9 * sg["abs"]).any()    # cancellation happens: the statistic is not |sum g|
