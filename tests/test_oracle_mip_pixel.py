"""Pins for the oracle's per-pixel-Jacobian MIP variant (Sec. 3.3.1): the filter
Sigma_mip = I + sigma_f J J^T with J = d(u,v)/d(x,y) taken at each pixel's
ray-surfel intersection instead of the surfel centre (Sec. 3.3.2).

* under an affine projection of the surfel (fronto-parallel: J is the same at
  every pixel) the two variants agree;
* for tilted surfels, J by central differences of an independent world-space
  ray/plane solve at every pixel gives the same weights (inside the binning
  rectangle, which the variant keeps as its support);
* the variant's adjoint equals its dual-number JVPs.
"""
import math

import numpy as np
import pytest

import scenegen as g
from conftest import axis_camera, make_scene
from test_oracle_pins import KAPPA, _frame, _ray_uv, _rot, concat, f32, lattice


@pytest.mark.parametrize("sigma", [0.1, 0.7])
def test_fronto_parallel_equals_centre(oracle_lib, sigma):
    O = oracle_lib
    cam = axis_camera(64, 64, 100.0, background=(0.1, 0.2, 0.3))
    s = 0.02
    sc = make_scene(*concat(lattice(15, 2.2 * s, s, 2.0, seed=1), lattice(21, 1.5 * s, s, 2.4, seed=2)))
    pix = O.all_pixels(cam)
    rc = O.render(sc, cam, O.Options(sigma_f=sigma), pix)
    rp = O.render(sc, cam, O.Options(sigma_f=sigma, mip="pixel"), pix)
    assert (rc["n_layers"] == rp["n_layers"]).all() and rc["n_layers"].max() == 2
    np.testing.assert_allclose(rp["image"], rc["image"], rtol=0, atol=1e-13)
    np.testing.assert_allclose(rp["alpha"], rc["alpha"], rtol=0, atol=1e-13)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_tilted_surfel_per_pixel_jacobian(oracle_lib, seed):
    O = oracle_lib
    rng = np.random.default_rng(100 + seed)
    R = _rot(rng)
    t = rng.uniform(-0.5, 0.5, 3)
    cam = axis_camera(48, 40, 90.0, R=R, t=t)
    c_cam = np.array([rng.uniform(-0.1, 0.1), rng.uniform(-0.1, 0.1), rng.uniform(1.6, 2.4)])
    Rf, tf = f32(cam.R), f32(cam.t)
    c = np.linalg.solve(Rf, c_cam - tf)
    n_cam = np.array([rng.uniform(-1.5, 1.5), rng.uniform(-1.5, 1.5), -1.0])   # strongly tilted
    nrm = np.linalg.solve(Rf, n_cam)
    tan = rng.normal(size=3)
    scl = rng.uniform(0.01, 0.04, 2)
    sc = make_scene(c, nrm, tan, scl)
    n_, u_, v_ = _frame(f32(nrm), f32(tan))
    tu, tv, cc = f32(scl)[0] * u_, f32(scl)[1] * v_, f32(c)
    pix = O.all_pixels(cam)
    sigma = 0.5
    r = O.render(sc, cam, O.Options(sigma_f=sigma, mip="pixel"), pix)
    rcen = O.render(sc, cam, O.Options(sigma_f=sigma), pix)
    pr = O.pixel_rects(sc, cam, O.Options(sigma_f=sigma))[0]
    h = 1e-4
    exp_a = np.zeros(len(pix))
    ok = np.ones(len(pix), bool)
    for k, (px, py) in enumerate(pix):
        x, y = px + 0.5, py + 0.5
        u, v, lam = _ray_uv(cam, x, y, cc, tu, tv)
        J = np.zeros((2, 2))
        for j, (dx, dy) in enumerate([(h, 0), (0, h)]):
            up = _ray_uv(cam, x + dx, y + dy, cc, tu, tv)
            um = _ray_uv(cam, x - dx, y - dy, cc, tu, tv)
            J[:, j] = [(up[0] - um[0]) / (2 * h), (up[1] - um[1]) / (2 * h)]
        S = np.eye(2) + sigma * J @ J.T
        uv = np.array([u, v])
        q = uv @ np.linalg.solve(S, uv)
        ok[k] = abs(q - 9.0) > 1e-6
        inside = pr[0] <= px <= pr[1] and pr[2] <= py <= pr[3]
        if q < 9.0 and lam > 0 and inside:
            exp_a[k] = 1 - math.exp(-KAPPA * math.exp(-0.5 * q) / math.sqrt(np.linalg.det(S)))
    assert (exp_a > 0).sum() > 20
    np.testing.assert_allclose(r["alpha"][ok], exp_a[ok], rtol=0, atol=1e-8)
    # the variant differs from the centre filter on this surfel (the test has teeth)
    assert np.abs(r["alpha"] - rcen["alpha"]).max() > 1e-4


def test_per_pixel_adjoint_matches_jvp(oracle_lib):
    O = oracle_lib
    w = g.make_config("C1", n_scale=0.3, res_scale=0.375)
    sc, cam = w.scenes[0], w.cameras[0]
    opt = O.Options(sigma_f=0.4, mip="pixel")
    pix = O.all_pixels(cam)
    rng = np.random.default_rng(2)
    G = rng.normal(size=(len(pix), 3))
    gr = O.render_grad(sc, cam, opt, pix, G, None)
    for k in ("position", "normal", "tangent", "scale", "albedo"):
        v = {k: rng.normal(size=getattr(sc, k).shape)}
        jv = O.render_jvp(sc, cam, opt, pix, v)
        lhs = (G * jv["image_dot"]).sum()
        rhs = (gr[k] * v[k]).sum()
        assert abs(lhs - rhs) <= 1e-10 * max(1e-3, abs(lhs)), (k, lhs, rhs)


def test_per_pixel_support_reading_drops_little_weight(oracle_lib):
    """The per-pixel filter's own acceptance region is unbounded: where a ray meets a
    surfel plane near its vanishing line, J grows without bound and
    u^T (I + sigma_f J J^T)^{-1} u falls below r_cut^2 far from the surfel.  The
    reading restricts its support to the centre filter's binning rectangle; the
    oracle counts what that removes.  The removed weight is a small fraction of the
    kept weight on these scenes (it is < 1e-3 per fragment on average)."""
    import scenegen as g
    O = oracle_lib
    cases = [(g.checkerboard_workload(n_side=240, extent=3.0, square=0.15, width=96, height=72,
                                      eye=(0.0, -3.2, 0.35)), 0.1),
             (g.make_config("C1"), 0.5), (g.near_plane_workload(), 0.5)]
    for w, sig in cases:
        sc, cam = w.scenes[0], w.cameras[0]
        r = O.render(sc, cam, O.Options(sigma_f=sig, mip="pixel"), O.all_pixels(cam))
        kept = -np.log(np.maximum(1.0 - r["alpha"], 1e-300)) / (O.Options().gamma / (2 * np.pi))
        dropped = r["pp_drop_w"].sum()
        assert r["pp_drop"].sum() > 0
        assert dropped / kept.sum() < 3e-3, (w.name, dropped, kept.sum())
        assert dropped / r["pp_drop"].sum() < 1e-3


def test_per_pixel_jvp_matches_finite_differences(oracle_lib):
    """Directional derivatives of the per-pixel variant against central differences
    of its FP64 forward (Richardson-extrapolated; coordinates whose step flips a
    decision are skipped)."""
    from test_oracle_grad import _objective
    O = oracle_lib
    w = g.make_config("C1", n_scale=0.3, res_scale=0.375)
    sc, cam = w.scenes[0], w.cameras[0]
    opt = O.Options(sigma_f=0.4, mip="pixel")
    pix = O.all_pixels(cam)
    rng = np.random.default_rng(9)
    G = rng.normal(size=(len(pix), 3))
    ga = np.zeros(len(pix))
    r0 = O.render_grad(sc, cam, opt, pix, G, None)
    live = np.nonzero(np.abs(r0["position"]).sum(0) > 0)[0]
    checked = 0
    for k in ("position", "normal", "scale", "albedo"):
        arr = getattr(sc, k)
        for trial in range(6):
            i = int(rng.choice(live))
            row = int(rng.integers(0, arr.shape[0]))
            p = float(arr[row, i])
            v = {k: np.zeros(arr.shape)}
            v[k][row, i] = 1.0
            d = (G * O.render_jvp(sc, cam, opt, pix, v)["image_dot"]).sum()

            def fd(h):
                hi, lo = np.float32(p + h), np.float32(p - h)
                arr[row, i] = hi
                fp = _objective(O, sc, cam, opt, pix, G, ga, None, None, (0, 0))
                arr[row, i] = lo
                fm = _objective(O, sc, cam, opt, pix, G, ga, None, None, (0, 0))
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
    assert checked >= 12
