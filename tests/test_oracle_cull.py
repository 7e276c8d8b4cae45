"""Pins of the oracle's cull and of the bounding-rectangle check.

Reading of the bounding rectangle (App. A.1, "scaled by r_cut relative to the
T-matrix half-extents"): a surfel is kept when its MIP acceptance ellipse
{u^T Sigma_mip^{-1} u < r_cut^2} lies entirely beyond the near plane, and the
pixel rectangle must contain every pixel centre the ellipse covers.  The oracle
takes the cull in FP64 from its own records (minimum depth over the ellipse,
c'_z - r_cut sqrt(t_z^T Sigma_mip t_z)) and counts, per pixel, covering
fragments that the FP32 binning (the decision the GPU shares bit for bit)
culls or leaves outside its rectangle.  The tests below pin that FP64 cull by
brute force and require zero such fragments on scenes that stress the near
plane, the image border, grazing silhouettes and the MIP widening.
"""
import numpy as np
import pytest

import scenegen as g


def _scenes():
    return {
        "near_plane": g.near_plane_workload(),
        "two_spheres": g.two_spheres_workload(n_each=3000, width=96, height=72),
        "C1": g.make_config("C1"),
        "C2s": g.make_config("C2", n_scale=0.05, res_scale=0.25),
        "C3s": g.make_config("C3", n_scale=0.03, res_scale=0.1, views=2),
        "thin_shell": g.thin_shell_workload(),
        "occluded": g.occluded_planes_workload(),
    }


def _projective_sigma(T1, T2, T4, sigma, h=1e-5):
    """Sigma_mip = I + sigma_f J J^T with J = M^{-1}, M = d(x, y)/d(u, v) at the
    surfel centre, M by central differences of x = T1.(u,v,1)/T4.(u,v,1),
    y = T2.(u,v,1)/T4.(u,v,1) (Sec. 3.3.2, eq:mip_cov)."""
    def xy(u, v):
        w = np.array([u, v, 1.0])
        return np.array([T1 @ w, T2 @ w]) / (T4 @ w)
    M = np.stack([(xy(h, 0) - xy(-h, 0)) / (2 * h), (xy(0, h) - xy(0, -h)) / (2 * h)], 1)
    J = np.linalg.inv(M)
    return np.eye(2) + sigma * J @ J.T


@pytest.mark.parametrize("sigma", [0.1, 0.5])
def test_sigma_mip_is_the_projection_jacobian(oracle_lib, sigma):
    O = oracle_lib
    w = g.near_plane_workload()
    sc, cam = w.scenes[0], w.cameras[0]
    rec = O.records(sc, cam, O.Options(sigma_f=sigma))
    idx = np.nonzero(rec["keep64"])[0][:200]
    for i in idx:
        S = _projective_sigma(rec["T1"][i], rec["T2"][i], rec["T4"][i], sigma)
        got = np.array([[rec["sig"][i, 0], rec["sig"][i, 1]], [rec["sig"][i, 1], rec["sig"][i, 2]]])
        np.testing.assert_allclose(got, S, rtol=1e-6, atol=1e-9 * np.abs(S).max())


@pytest.mark.parametrize("sigma", [0.0, 0.1, 0.5])
def test_cull_is_minimum_depth_over_the_acceptance_ellipse(oracle_lib, sigma):
    """The kept surfels are exactly those whose acceptance ellipse lies beyond
    znear, found by sampling the ellipse boundary u = r_cut L (cos t, sin t)
    (Sigma_mip = L L^T) and taking the minimum camera depth T4.(u, v, 1)."""
    O = oracle_lib
    w = g.near_plane_workload()
    sc, cam = w.scenes[0], w.cameras[0]
    rec = O.records(sc, cam, O.Options(sigma_f=sigma))
    t = np.linspace(0.0, 2 * np.pi, 20001)
    circle = np.stack([np.cos(t), np.sin(t)])
    z = rec["T4"][:, 2]
    checked = culled_in_front = 0
    for i in np.nonzero(z > cam.znear)[0]:
        S = _projective_sigma(rec["T1"][i], rec["T2"][i], rec["T4"][i], sigma)
        L = np.linalg.cholesky(S)
        uv = 3.0 * L @ circle
        zmin = (rec["T4"][i, 0] * uv[0] + rec["T4"][i, 1] * uv[1] + z[i]).min()
        # sampling error of the minimum: (dt)^2 / 2 of the depth amplitude
        amp = z[i] - zmin
        np.testing.assert_allclose(rec["margin"][i] * z[i] + cam.znear, zmin, rtol=0,
                                   atol=1e-6 * max(amp, 1.0))
        if abs(zmin - cam.znear) > 1e-6 * z[i]:
            assert rec["keep64"][i] == (zmin > cam.znear), i
            checked += 1
            culled_in_front += int(not rec["keep64"][i])
    # the scene exercises the rule: many surfels whose centre is beyond znear are
    # culled because their ellipse reaches it
    assert checked > 2000 and culled_in_front > 100, (checked, culled_in_front)


@pytest.mark.parametrize("sigma", [0.0, 0.1, 0.5])
def test_fp32_cull_matches_the_fp64_rule(oracle_lib, sigma):
    """The FP32 binning's cull (stages 0-2) is the FP64 rule, away from its margin;
    its remaining rejections are empty rectangles (stage 3)."""
    O = oracle_lib
    for name, w in _scenes().items():
        for v, cam in enumerate(w.cameras):
            sc = w.scenes[cam.scene]
            rec = O.records(sc, cam, O.Options(sigma_f=sigma))
            cull32 = rec["stage32"] <= 2
            differ = cull32 == rec["keep64"]
            assert (np.abs(rec["margin"][differ]) < 1e-5).all(), (name, v, np.nonzero(differ)[0][:5])
            assert (rec["keep32"] == (rec["stage32"] == 4)).all()


@pytest.mark.parametrize("sigma", [0.0, 0.1, 0.5])
def test_no_covered_pixel_outside_the_fp32_binning(oracle_lib, sigma):
    """Every fragment the FP64 brute force finds covering a pixel belongs to a
    surfel the FP32 binning keeps, and the pixel lies inside its FP32 rectangle
    (counted per pixel by the oracle: `viol`)."""
    O = oracle_lib
    tot_cov = 0
    for name, w in _scenes().items():
        for v, cam in enumerate(w.cameras):
            sc = w.scenes[cam.scene]
            r = O.render(sc, cam, O.Options(sigma_f=sigma), O.all_pixels(cam))
            assert r["viol"].sum() == 0, (name, v, int(r["viol"].sum()))
            tot_cov += int((r["n_layers"] > 0).sum())
    assert tot_cov > 30000


def test_viol_counts_a_planted_rectangle_miss(oracle_lib):
    """The violation count is live: a camera of half the width (same intrinsics)
    clamps every FP32 rectangle to the left half, so the covered pixels of the
    right half, rendered through it, must all report violations."""
    O = oracle_lib
    w = g.make_config("C1")
    sc, cam = w.scenes[0], w.cameras[0]
    import copy
    small = copy.copy(cam)
    small.width, small.height = cam.width // 2, cam.height
    pix = O.all_pixels(cam)
    right = pix[pix[:, 0] >= small.width]
    r = O.render(sc, small, O.Options(), right)
    assert r["viol"].sum() > 100
