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
  at a reduced resolution.
"""
import dataclasses

import pytest

import scenegen as g
from parity_util import GRAD_REL_L2, assert_image_parity
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
    print(name, {k: v for k, v in rep.items() if k != "worst"})
    assert_image_parity(rep)
    errs = _backward_case(O, ss, w.scenes, w.cameras, w.shade, lambda c, v: all_pix(c), **kw)
    print(name, "gradients", errs)
    assert max(errs.values()) <= GRAD_REL_L2, errs
