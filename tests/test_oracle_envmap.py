"""Pins of the environment prefilter's specular levels (eq:ibl, Sec. 3.4.2) by an
independent 1-D integral.

Reading (split-sum prefilter with n = v = R): level l = 1..5 has GGX roughness
alpha_l = (l/5)^2, resolution max(H_e >> l, 4) x max(W_e >> l, 8), and
Spec_l(R) = sum_t E_t K(R, t) / sum_t K(R, t) with
K(R, t) = D(R . h_t; alpha_l) max(0, R . d_t) dOmega_t, h_t = normalize(R + d_t).

For E(d) = d_z the normalised lobe is symmetric about R, so
Spec_l(R) = R_z m1(alpha_l) with m1 the lobe's mean cosine, and for E(d) = d_z^2,
Spec_l(R) = R_z^2 c2 + (1 - R_z^2)(1 - c2)/2 with c2 the mean squared cosine.
With theta the angle between R and d, R . h = cos(theta / 2), so
    m1 = int cos^2 D sin / int cos D sin,  c2 = int cos^3 D sin / int cos D sin
over theta in [0, pi/2] (D at cos(theta/2)).  These are scipy quadratures; the
map's texel quadrature converges to them with resolution.  The same holds for
the irradiance of E(d) = d_z: Irr(d) = (1/pi) int d'_z max(0, d . d') dOmega'
= (2/3) d_z.

A wrong lobe (alpha_l = l/5, or D taken at R . d instead of R . h), wrong level
sizes or wrong texel directions change these values by far more than the
quadrature error, which the test checks explicitly for the first two.
"""
import math

import numpy as np
import pytest
from scipy import integrate


def _D(mu, a):
    a2 = a * a
    t = mu * mu * (a2 - 1.0) + 1.0
    return a2 / (math.pi * t * t)


def lobe_moments(alpha, half_vector=True):
    f = (lambda th: _D(math.cos(th / 2), alpha)) if half_vector else (lambda th: _D(math.cos(th), alpha))
    kw = dict(limit=400, points=[min(4 * alpha, 1.0)])
    den = integrate.quad(lambda th: f(th) * math.cos(th) * math.sin(th), 0, math.pi / 2, **kw)[0]
    m1 = integrate.quad(lambda th: f(th) * math.cos(th) ** 2 * math.sin(th), 0, math.pi / 2, **kw)[0] / den
    c2 = integrate.quad(lambda th: f(th) * math.cos(th) ** 3 * math.sin(th), 0, math.pi / 2, **kw)[0] / den
    return m1, c2


def texel_dirs(H, W):
    th = np.pi * (np.arange(H) + 0.5) / H
    ph = 2 * np.pi * (np.arange(W) + 0.5) / W
    T, P = np.meshgrid(th, ph, indexing="ij")
    return np.stack([np.sin(T) * np.cos(P), np.sin(T) * np.sin(P), np.cos(T)], -1)


def _levels(O, E):
    He, We = E.shape[:2]
    m = O.envmap(E)
    out = []
    off = He * We * 3
    for l in range(1, 6):
        h, w = max(He >> l, 4), max(We >> l, 8)
        out.append(m[off:off + h * w * 3].reshape(h, w, 3))
        off += h * w * 3
    irr = m[off:off + 32 * 64 * 3].reshape(32, 64, 3)
    assert off + 32 * 64 * 3 == m.size
    return out, irr


def _errors(O, He, We):
    d = texel_dirs(He, We)
    lin, irr = _levels(O, np.repeat(d[..., 2:3], 3, -1))
    quad, _ = _levels(O, np.repeat(d[..., 2:3] ** 2, 3, -1))
    e_lin, e_quad = [], []
    for l in range(1, 6):
        m1, c2 = lobe_moments((l / 5) ** 2)
        h, w = lin[l - 1].shape[:2]
        Rz = texel_dirs(h, w)[..., 2:3]
        e_lin.append(np.abs(lin[l - 1] - Rz * m1).max())
        e_quad.append(np.abs(quad[l - 1] - (Rz ** 2 * c2 + (1 - Rz ** 2) * (1 - c2) / 2)).max())
    e_irr = np.abs(irr - (2.0 / 3.0) * texel_dirs(32, 64)[..., 2:3]).max()
    return np.array(e_lin), np.array(e_quad), e_irr


def test_specular_levels_match_the_lobe_moments(oracle_lib):
    O = oracle_lib
    lin32, quad32, irr32 = _errors(O, 32, 64)
    lin64, quad64, irr64 = _errors(O, 64, 128)
    # second-order convergence of the texel quadrature: the finer map is closer
    assert (lin64 < lin32).all() and (quad64 < quad32).all() and irr64 < irr32
    assert lin64.max() < 4e-4 and quad64.max() < 6e-4 and irr64 < 2e-4, (lin64, quad64, irr64)
    # the readings that this pin rules out differ by far more than that
    tol = 4e-4
    for l in range(1, 5):
        m1, c2 = lobe_moments((l / 5) ** 2)
        m1_lin_alpha, _ = lobe_moments(l / 5)
        m1_no_half, _ = lobe_moments((l / 5) ** 2, half_vector=False)
        assert abs(m1 - m1_lin_alpha) > 10 * tol, l
        assert abs(m1 - m1_no_half) > 10 * tol, l


def test_lobe_moments_closed_form_at_alpha_one():
    """alpha = 1 makes D constant (1/pi): m1 = 2/3, c2 = 1/2 exactly (cosine-weighted
    hemisphere moments), a check of the quadrature itself."""
    m1, c2 = lobe_moments(1.0)
    assert abs(m1 - 2.0 / 3.0) < 1e-12 and abs(c2 - 0.5) < 1e-12
