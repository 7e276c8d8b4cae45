"""Pins of the oracle's derivatives.

* the reverse-mode adjoint against exact forward-mode (dual-number) JVPs:
  <G, J v> = <J^T G, v> for random directions over every parameter group and
  the environment maps;
* the JVP against central finite differences of the FP64 forward, one float32
  input coordinate at a time, rejecting coordinates whose perturbation flips a
  discrete decision (cutoff, gap, cull) -- detected as an FD that is not stable
  under halving the step;
* the environment-map adjoint against the prefilter (a linear map).
"""
import math

import numpy as np
import pytest

import scenegen as g

PARAMS = ["position", "normal", "tangent", "scale", "albedo", "roughness", "metallic"]


def small_albedo():
    w = g.make_config("C1", n_scale=0.3, res_scale=0.375)
    return w.scenes[0], w.cameras[0], "albedo", None, None, (0, 0)


def small_splitsum(oracle):
    sc = g.torus_scene(12, 2500, scale_mu=math.log(0.03), scale_sigma=0.3)
    E = g.lognormal_envmap(12, 16, 32)
    cam = g.look_at_camera((0.0, -2.6, 1.5), 40, 40)
    maps = oracle.envmap(E.astype(np.float64))
    lut = oracle.brdf_lut(16, 16, 128)
    return sc, cam, "splitsum", maps, lut, (16, 32)


def _setup(oracle_lib, kind):
    return small_albedo() if kind == "albedo" else small_splitsum(oracle_lib)


@pytest.mark.parametrize("kind", ["albedo", "splitsum"])
def test_adjoint_matches_dual_jvp(oracle_lib, kind):
    O = oracle_lib
    sc, cam, shade, maps, lut, hw = _setup(O, kind)
    opt = O.Options(shade=shade)
    pix = O.all_pixels(cam)
    rng = np.random.default_rng(7)
    G = rng.normal(size=(len(pix), 3))
    ga = rng.normal(size=len(pix))
    gr = O.render_grad(sc, cam, opt, pix, G, ga, maps=maps, lut=lut, env_hw=hw)
    for trial in range(2):
        v = {k: rng.normal(size=getattr(sc, k).shape) for k in PARAMS}
        vm = rng.normal(size=maps.shape) if maps is not None else None
        jv = O.render_jvp(sc, cam, opt, pix, v, maps=maps, dmaps=vm, lut=lut, env_hw=hw)
        lhs = (G * jv["image_dot"]).sum() + (ga * jv["alpha_dot"]).sum()
        rhs = sum((gr[k] * v[k]).sum() for k in PARAMS)
        if vm is not None:
            rhs += (gr["maps"] * vm).sum()
        assert abs(lhs - rhs) <= 1e-10 * max(1.0, abs(lhs)), (lhs, rhs)
        # and per parameter group, so that a wrong group cannot hide behind another
        for k in PARAMS:
            vk = {k: v[k]}
            jk = O.render_jvp(sc, cam, opt, pix, vk, maps=maps, lut=lut, env_hw=hw)
            l = (G * jk["image_dot"]).sum() + (ga * jk["alpha_dot"]).sum()
            r = (gr[k] * v[k]).sum()
            assert abs(l - r) <= 1e-10 * max(1.0, abs(l)), (k, l, r)


def _objective(O, sc, cam, opt, pix, G, ga, maps, lut, hw):
    r = O.render(sc, cam, opt, pix, maps=maps, lut=lut, env_hw=hw)
    return (G * r["image"]).sum() + (ga * r["alpha"]).sum()


@pytest.mark.parametrize("kind", ["albedo", "splitsum"])
def test_jvp_matches_finite_differences(oracle_lib, kind):
    O = oracle_lib
    sc, cam, shade, maps, lut, hw = _setup(O, kind)
    opt = O.Options(shade=shade)
    pix = O.all_pixels(cam)
    rng = np.random.default_rng(3)
    G = rng.normal(size=(len(pix), 3))
    ga = rng.normal(size=len(pix))
    base = O.render(sc, cam, opt, pix, maps=maps, lut=lut, env_hw=hw)
    # coordinates of surfels that reach the image
    r0 = O.render_grad(sc, cam, opt, pix, G, ga, maps=maps, lut=lut, env_hw=hw)
    live = np.nonzero(np.abs(r0["position"]).sum(0) > 0)[0]
    groups = PARAMS if shade == "splitsum" else ["position", "normal", "tangent", "scale", "albedo"]
    checked = 0
    for k in groups:
        arr = getattr(sc, k)
        for trial in range(6):
            i = int(rng.choice(live))
            row = int(rng.integers(0, arr.shape[0])) if arr.ndim == 2 else None
            idx = (row, i) if row is not None else (i,)
            p = float(arr[idx])
            v = {k: np.zeros(arr.shape)}
            v[k][idx] = 1.0
            jv = O.render_jvp(sc, cam, opt, pix, v, maps=maps, lut=lut, env_hw=hw)
            d = (G * jv["image_dot"]).sum() + (ga * jv["alpha_dot"]).sum()

            def fd(h):
                hi, lo = np.float32(p + h), np.float32(p - h)
                arr[idx] = hi
                fp = _objective(O, sc, cam, opt, pix, G, ga, maps, lut, hw)
                arr[idx] = lo
                fm = _objective(O, sc, cam, opt, pix, G, ga, maps, lut, hw)
                arr[idx] = np.float32(p)
                return (fp - fm) / (float(hi) - float(lo))
            h = 2e-3 * max(abs(p), 0.05)
            f1, f2 = fd(h), fd(h / 2)
            scale = max(abs(d), 1e-3 * np.abs(r0[k]).max(), 1e-8)
            if abs(f1 - f2) > 2e-3 * scale:       # a decision flipped inside the step
                continue
            # Richardson extrapolation of the central difference
            fr = (4 * f2 - f1) / 3
            # FD round-off floor: ~1e-16 |objective| / h
            assert abs(fr - d) <= 2e-4 * scale + 1e-7, (k, idx, fr, d, f1, f2)
            checked += 1
    assert checked >= 3 * len(groups)


def test_envmap_adjoint_is_transpose(oracle_lib):
    O = oracle_lib
    He, We = 8, 16
    rng = np.random.default_rng(0)
    vE = rng.normal(size=(He, We, 3))
    dm = rng.normal(size=O.map_size(He, We))
    lhs = (dm * O.envmap(vE)).sum()
    rhs = (O.envmap_adjoint(dm, He, We) * vE).sum()
    assert abs(lhs - rhs) <= 1e-11 * abs(lhs)


def test_isotropic_scale_gives_zero_tangent_gradient(oracle_lib):
    """With s_u = s_v the kernel is rotation invariant in the tangent plane, so the
    tangent direction cannot change the image (albedo shading)."""
    O = oracle_lib
    sc, cam, shade, maps, lut, hw = small_albedo()
    pix = O.all_pixels(cam)
    rng = np.random.default_rng(1)
    G = rng.normal(size=(len(pix), 3))
    gr = O.render_grad(sc, cam, O.Options(), pix, G)
    assert np.abs(gr["tangent"]).max() <= 1e-9 * np.abs(gr["position"]).max()
