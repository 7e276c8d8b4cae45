"""MI355X-native differentiable EWA surfel rasterizer (3D Surface Splatting hot path).

The rendering path is the HIP library libsurfsplat.so (C ABI in
include/surfsplat.h); `surfsplat` is its ctypes binding and the
torch.autograd.Function around it.
"""
from .surfsplat import (Batch, Options, Renderer, SurfsplatError, SurfelRenderFunction,  # noqa: F401
                        load_library, make_brdf_lut, render, PARAMS, SS_OK, SS_ERR_INVALID_ARG, SS_ERR_HIP,
                        SS_ERR_CAPACITY, SS_ERR_STATE, SS_ERR_UNSUPPORTED, SS_ERR_NOMEM,
                        SS_ERR_STATIC_LIMIT, STATIC_SCRATCH_BYTES)


def batch_from_scenes(scenes, cameras, device="cuda", with_envmap=None):
    """Concatenate scenes (objects with [C][N] float32 numpy attributes named as in
    PARAMS and an optional `envmap`) into a device Batch."""
    import numpy as np
    import torch
    params = {}
    for k in PARAMS:
        arrs = [np.asarray(getattr(s, k), np.float32) for s in scenes]
        a = np.concatenate(arrs, axis=-1)
        params[k] = torch.from_numpy(np.ascontiguousarray(a)).to(device)
    offs = [0]
    for s in scenes:
        offs.append(offs[-1] + int(np.asarray(s.position).shape[1]))
    if with_envmap is None:
        with_envmap = all(getattr(s, "envmap", None) is not None for s in scenes)
    envs = None
    if with_envmap:
        envs = [torch.from_numpy(np.ascontiguousarray(s.envmap, np.float32)).to(device) for s in scenes]
    return Batch(params, offs, cameras, envs)
