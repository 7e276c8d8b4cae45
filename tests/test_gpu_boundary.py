"""GPU tests of the boundary's state and option handling, through the C ABI:
forward generation numbers, recovery from (and poisoning after) a pair-capacity
overflow, the transmittance early-out and the tone-map epilogue against the
oracle, the work counters, input validation and the library-picked LDS batch."""
import numpy as np
import pytest

import scenegen as g
from parity_util import GRAD_REL_L2, assert_image_parity, decision_ok, oracle_options, rel_l2
from test_gpu_parity import O, _backward_case, _forward_case, all_pix, small_c2, ss  # noqa: F401

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _c1_small():
    w = g.make_config("C1", n_scale=0.5, res_scale=0.5)   # 2048 surfels, 64 x 64
    return w.scenes, w.cameras


def test_generation_guards_backward(ss):
    scenes, cams = _c1_small()
    r = ss.Renderer(ss.Options())
    b = ss.batch_from_scenes(scenes, cams)
    r.forward(b)
    g1 = r.last_generation
    r.forward(b)
    g2 = r.last_generation
    assert g1 >= 1 and g2 == g1 + 1 and r.poll()["generation"] == g2
    G = torch.ones((b.n_pixels, 3), device="cuda")
    with pytest.raises(ss.SurfsplatError) as e:
        r.backward(b, G, generation=g1)
    assert e.value.status == ss.SS_ERR_STATE
    r.backward(b, G, generation=g2)
    # through autograd: two renders through one renderer, then the first's backward
    params = {k: b.params[k].clone().requires_grad_(True) for k in ss.PARAMS}
    offs = [0, scenes[0].n]
    img1, _ = ss.render(r, params, offs, cams)
    img2, _ = ss.render(r, params, offs, cams)
    with pytest.raises(Exception, match="out of order"):
        img1.sum().backward()
    img2.sum().backward()
    assert params["position"].grad is not None and torch.isfinite(params["position"].grad).all()


def test_capacity_overflow_rerenders_or_poisons(ss):
    w = g.make_config("C1")
    b = ss.batch_from_scenes(w.scenes, w.cameras)
    r = ss.Renderer(ss.Options())            # polls after each forward and reserves again
    r.forward(b)
    cap = r.poll()["pair_capacity"]
    b.params["scale"].mul_(4.0)              # several times the reserved pairs
    img, a, nl = r.forward(b, want_layers=True)
    d = r.poll()
    assert d["status"] == 0 and d["n_pairs"] > cap and d["pair_capacity"] > d["n_pairs"], (d, cap)
    fresh = ss.Renderer(ss.Options())
    img2, a2, nl2 = fresh.forward(b, want_layers=True)
    assert torch.equal(img, img2) and torch.equal(a, a2) and torch.equal(nl, nl2)
    # without the check the overflow is latched and every output is NaN
    b.params["scale"].div_(4.0)
    r2 = ss.Renderer(ss.Options(), check_capacity=False)
    r2.forward(b)
    b.params["scale"].mul_(4.0)
    img3, a3, _ = r2.forward(b)
    d = r2.poll()
    assert d["device_status"] == ss.SS_ERR_CAPACITY and d["n_pairs"] > d["pair_capacity"], d
    assert torch.isnan(img3).all() and torch.isnan(a3).all()
    gr = r2.backward(b, torch.ones_like(img3))
    torch.cuda.synchronize()
    for k in ("position", "normal", "scale", "albedo"):
        assert torch.isnan(gr[k]).all(), k


@pytest.mark.parametrize("t_min", [0.5, 0.05])
def test_early_out_parity(O, ss, t_min):
    """t_min: the walk of a pixel ends once the transmittance in front of the next
    layer is below t_min; layer counts, image and gradients against the oracle."""
    w = g.make_config("C1")
    rep = _forward_case(O, ss, w.scenes, w.cameras, "albedo", lambda c, v: all_pix(c), t_min=t_min)
    assert_image_parity(rep)
    errs = _backward_case(O, ss, w.scenes, w.cameras, "albedo", lambda c, v: all_pix(c), t_min=t_min)
    assert max(errs.values()) <= GRAD_REL_L2, errs
    # it removes layers
    r0, r1 = ss.Renderer(ss.Options()), ss.Renderer(ss.Options(t_min=t_min))
    b = ss.batch_from_scenes(w.scenes, w.cameras)
    nl0 = r0.forward(b, want_layers=True)[2].float().mean().item()
    nl1 = r1.forward(b, want_layers=True)[2].float().mean().item()
    assert nl1 < nl0, (nl0, nl1)


@pytest.mark.parametrize("case", ["C1", "C2s"])
def test_tonemap_parity(O, ss, case):
    """Fused log-space + sRGB epilogue (eq:photo_loss transfer): image and
    gradients of a loss on the tone-mapped image against the oracle."""
    if case == "C1":
        w = g.make_config("C1")
        scenes, cams, shade = w.scenes, w.cameras, "albedo"
    else:
        (scenes, cams), shade = small_c2(), "splitsum"
    rep = _forward_case(O, ss, scenes, cams, shade, lambda c, v: all_pix(c), tonemap="srgb_log")
    assert_image_parity(rep)
    errs = _backward_case(O, ss, scenes, cams, shade, lambda c, v: all_pix(c), tonemap="srgb_log")
    assert max(errs.values()) <= GRAD_REL_L2, errs


def test_counters(O, ss):
    """Work counters of the raster forward: the composited layers equal the sum of
    the layer counts, the accumulated fragments the oracle's count (unique given
    the decisions), and the summed layer weights -log(1 - alpha) / kappa per pixel."""
    w = g.make_config("C1")
    opts = ss.Options(counters=True)
    r = ss.Renderer(opts)
    b = ss.batch_from_scenes(w.scenes, w.cameras)
    img, a, nl = r.forward(b, want_layers=True)
    d = r.poll()
    nl = nl.cpu().numpy().astype(np.int64)
    assert d["n_layers"] == int(nl.sum()) > 0, d
    cam = w.cameras[0]
    ref = O.render(w.scenes[0], cam, oracle_options(O, opts), all_pix(cam))
    ok = decision_ok(ref)
    want_f = int(ref["n_frag"].sum())
    # pixels next to a decision may differ by a fragment or a layer
    assert abs(d["n_fragments"] - want_f) <= 16 * int((~ok).sum()), (d["n_fragments"], want_f, int((~ok).sum()))
    assert d["n_evaluated"] >= d["n_fragments"] > 0
    kappa = opts.gamma / (2 * np.pi)
    want_w = float(-np.log1p(-ref["alpha"]).sum() / kappa)   # T_{K+1} = exp(-kappa sum_k W_k)
    assert abs(d["sum_layer_weight"] - want_w) <= 1e-3 * want_w, (d["sum_layer_weight"], want_w)
    plain = ss.Renderer(ss.Options())
    plain.forward(b)
    dp = plain.poll()
    assert dp["n_fragments"] == 0 and dp["n_evaluated"] == 0


def test_validate_counts_nonfinite(ss):
    scenes, cams = _c1_small()
    b = ss.batch_from_scenes(scenes, cams)
    b.params["position"][0, 5] = float("nan")
    b.params["albedo"][1, 7] = float("inf")
    r = ss.Renderer(ss.Options(validate=True))
    r.forward(b)
    assert r.poll()["n_nonfinite"] == 2
    G = torch.ones((b.n_pixels, 3), device="cuda")
    G[3, 1] = float("nan")
    Ga = torch.zeros(b.n_pixels, device="cuda")
    Ga[10] = float("-inf")
    r.backward(b, G, Ga)
    assert r.poll()["n_nonfinite"] == 4
    r0 = ss.Renderer(ss.Options())
    r0.forward(b)
    assert r0.poll()["n_nonfinite"] == 0


def test_library_picked_lds_batch(ss):
    """lds_batch = 0: the reserve picks the batch; the forward is bit-identical to
    any fixed batch and the gradients agree to float-sum order."""
    w = g.make_config("C1")
    b = ss.batch_from_scenes(w.scenes, w.cameras)
    ra, rb = ss.Renderer(ss.Options(lds_batch=0)), ss.Renderer(ss.Options(lds_batch=128))
    ia, aa, _ = ra.forward(b)
    ib, ab, _ = rb.forward(b)
    assert torch.equal(ia, ib) and torch.equal(aa, ab)
    G = torch.randn((b.n_pixels, 3), device="cuda", generator=torch.Generator("cuda").manual_seed(5))
    ga, gb = ra.backward(b, G), rb.backward(b, G)
    for k in ("position", "normal", "scale", "albedo"):
        assert rel_l2(ga[k].cpu().numpy(), gb[k].cpu().numpy()) <= 1e-5, k


def _det_case(case):
    import math
    if case == "C1":
        w = g.make_config("C1")
        return w.scenes, w.cameras, "albedo", {}
    if case == "multiview":
        sc = g.superquadric_scene(33, 30_000, scale_mu=math.log(0.012), scale_sigma=0.5)
        sc.envmap = g.lognormal_envmap(33, 16, 32)
        cams = [g.look_at_camera(3.0 * d, 72, 56) for d in g.fibonacci_directions(3)]
        return [sc], cams, "splitsum", {}
    scenes, cams = small_c2()
    return scenes, cams, "splitsum", dict(launch="per_view")


@pytest.mark.parametrize("walk", ["rows", "records"])
@pytest.mark.parametrize("case", ["C1", "multiview", "per_view"])
def test_deterministic_backward_is_bitwise_reproducible(O, ss, case, walk):
    """options.deterministic: two backward passes (and a second renderer) give
    bit-identical gradients of every parameter group, the environment maps and the
    densification statistic; and they pass the oracle bar."""
    scenes, cams, shade, kw = _det_case(case)
    kw["bwd_walk"] = walk
    opts = ss.Options(shade=shade, deterministic=True, **kw)
    b = ss.batch_from_scenes(scenes, cams)
    gen = torch.Generator("cuda").manual_seed(11)
    G = torch.randn((b.n_pixels, 3), device="cuda", generator=gen)
    Ga = torch.randn((b.n_pixels,), device="cuda", generator=gen)
    runs = []
    for r in (ss.Renderer(opts), ss.Renderer(opts)):
        for _ in range(2):
            r.forward(b)
            gr = r.backward(b, G, Ga, want_screen_grad=True)
            torch.cuda.synchronize()
            runs.append({k: ([e.clone() for e in v] if isinstance(v, list) else v.clone()) for k, v in gr.items()})
    for other in runs[1:]:
        for k, v in runs[0].items():
            if isinstance(v, list):
                for a, c in zip(v, other[k]):
                    assert torch.equal(a, c), k
            else:
                assert torch.equal(v, other[k]), k
    errs = _backward_case(O, ss, scenes, cams, shade, lambda c, v: all_pix(c), deterministic=True, **kw)
    assert max(errs.values()) <= GRAD_REL_L2, errs
