"""The C ABI library loads and exports every entry point its header declares;
host-side argument checks answer without touching the device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "surfsplat.h")


def declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:ss_status|const char\*)\s+(ss_\w+)\s*\(", txt, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    import paper_2605_05876_amd as m
    return m.load_library()


def test_header_declares_entry_points():
    names = declared()
    for n in ("ss_create", "ss_render", "ss_render_backward", "ss_reserve", "ss_poll", "ss_brdf_lut"):
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    for n in declared():
        assert hasattr(lib, n), n


def test_python_binding_names_match_header():
    from paper_2605_05876_amd import surfsplat
    assert sorted(surfsplat.EXPORTED) == declared()


def test_struct_layout_matches_header(tmp_path):
    """ctypes mirrors of the ABI structs have the size and field offsets the C
    compiler gives the header's definitions."""
    import subprocess
    from paper_2605_05876_amd import surfsplat as s
    structs = {"ss_options": s.ss_options, "ss_camera": s.ss_camera, "ss_batch": s.ss_batch,
               "ss_outputs": s.ss_outputs, "ss_grad_in": s.ss_grad_in, "ss_grads": s.ss_grads,
               "ss_diag": s.ss_diag}
    lines = ['#include "surfsplat.h"', "#include <stddef.h>", "#include <stdio.h>", "int main(void){"]
    for n, t in structs.items():
        lines.append(f'printf("{n} %zu\\n", sizeof({n}));')
        for f, _ in t._fields_:
            lines.append(f'printf("{n}.{f} %zu\\n", offsetof({n}, {f}));')
    lines.append("return 0;}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = dict(l.split() for l in subprocess.run([str(exe)], capture_output=True, text=True,
                                                 check=True).stdout.splitlines())
    for n, t in structs.items():
        assert int(got[n]) == ctypes.sizeof(t), n
        for f, _ in t._fields_:
            assert int(got[f"{n}.{f}"]) == getattr(t, f).offset, (n, f)


def test_host_argument_checks(lib):
    from paper_2605_05876_amd import surfsplat as s
    o = s.ss_options()
    assert lib.ss_default_options(ctypes.byref(o)) == 0
    assert (o.r_cut, o.k_max, o.tile_w, o.tile_h, o.env_lds) == (3.0, 16, 16, 16, -1)
    assert (o.t_min, o.deterministic, o.validate, o.counters, o.tonemap, o.seg_len, o.bwd_walk) == (0.0,) + (0,) * 6
    ctx = ctypes.c_void_p()
    bad = s.ss_options.from_buffer_copy(o)
    bad.tile_w = 12
    assert lib.ss_create(ctypes.byref(bad), ctypes.byref(ctx)) == s.SS_ERR_UNSUPPORTED
    bad = s.ss_options.from_buffer_copy(o)
    bad.k_max = 17
    assert lib.ss_create(ctypes.byref(bad), ctypes.byref(ctx)) == s.SS_ERR_INVALID_ARG
    bad = s.ss_options.from_buffer_copy(o)
    bad.env_lds = -2
    assert lib.ss_create(ctypes.byref(bad), ctypes.byref(ctx)) == s.SS_ERR_INVALID_ARG
    bad = s.ss_options.from_buffer_copy(o)
    bad.lds_batch = 100
    assert lib.ss_create(ctypes.byref(bad), ctypes.byref(ctx)) == s.SS_ERR_UNSUPPORTED
    for field, value, want in (("t_min", -0.1, s.SS_ERR_INVALID_ARG), ("t_min", 1.0, s.SS_ERR_INVALID_ARG),
                               ("validate", 2, s.SS_ERR_INVALID_ARG), ("tonemap", 3, s.SS_ERR_INVALID_ARG),
                               ("counters", -1, s.SS_ERR_INVALID_ARG), ("seg_len", 100, s.SS_ERR_INVALID_ARG),
                               ("seg_len", 65536, s.SS_ERR_INVALID_ARG), ("seg_len", -2, s.SS_ERR_INVALID_ARG),
                               ("bwd_walk", 3, s.SS_ERR_INVALID_ARG), ("bwd_walk", -1, s.SS_ERR_INVALID_ARG)):
        bad = s.ss_options.from_buffer_copy(o)
        setattr(bad, field, value)
        assert lib.ss_create(ctypes.byref(bad), ctypes.byref(ctx)) == want, field
    ok = s.ss_options.from_buffer_copy(o)
    ok.lds_batch, ok.t_min, ok.validate, ok.counters, ok.tonemap, ok.seg_len, ok.bwd_walk = 0, 0.01, 1, 1, 1, 512, 2
    assert lib.ss_create(ctypes.byref(ok), ctypes.byref(ctx)) == 0
    assert lib.ss_destroy(ctx) == 0
    assert lib.ss_create(None, ctypes.byref(ctx)) == s.SS_ERR_INVALID_ARG
    assert lib.ss_create(ctypes.byref(o), ctypes.byref(ctx)) == 0
    # null batch / outputs are rejected before any device work
    assert lib.ss_render(ctx, None, None, None) == s.SS_ERR_INVALID_ARG
    assert lib.ss_render_static(ctx, None, None, None) == s.SS_ERR_INVALID_ARG
    assert lib.ss_render_backward(ctx, None, None, None, None) == s.SS_ERR_INVALID_ARG
    b = s.ss_batch()
    b.n_scenes = 1
    offs = (ctypes.c_int64 * 2)(0, 10)
    b.surfel_offset = offs
    b.n_views = 0
    out = s.ss_outputs(1, 1, None)
    assert lib.ss_render(ctx, ctypes.byref(b), ctypes.byref(out), None) == s.SS_ERR_INVALID_ARG
    cam = (s.ss_camera * 1)()
    cam[0].width, cam[0].height, cam[0].fx, cam[0].fy, cam[0].znear = 8, 8, 10.0, 10.0, 0.01
    cam[0].scene = 3
    b.n_views = 1
    b.cameras = cam
    assert lib.ss_render(ctx, ctypes.byref(b), ctypes.byref(out), None) == s.SS_ERR_INVALID_ARG
    # backward without a forward is a state error (checked before device work)
    cam[0].scene = 0
    for k in ("position", "normal", "tangent", "scale", "albedo", "roughness", "metallic"):
        setattr(b, k, 1)
    gin = s.ss_grad_in(1, None)
    gr = s.ss_grads()
    assert lib.ss_render_backward(ctx, ctypes.byref(b), ctypes.byref(gin), ctypes.byref(gr), None) == s.SS_ERR_STATE
    assert lib.ss_destroy(ctx) == 0
    assert lib.ss_status_str(3).decode().startswith("pair capacity")
    assert "ss_render_static" in lib.ss_status_str(7).decode()
