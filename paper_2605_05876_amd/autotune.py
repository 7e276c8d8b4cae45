"""Tile size / LDS batch / backward walk autotuner for the raster kernels.

Sweeps tile shapes, surfels-per-LDS-batch and the two walks of the raster
backward on a workload, times one forward + backward step per candidate and
keeps the fastest in a JSON cache keyed by device architecture and workload
name.  The forward image is bit-identical across candidates (the per-pixel
fragment sequence and its FP32 arithmetic do not depend on them), and the
gradients agree to float summation order, so the choice is free of accuracy
effects.
"""
import json
import os

CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "autotune_cache.json")
TILES = [(8, 8), (16, 8), (16, 16), (32, 8), (32, 16)]
BATCHES = [32, 64, 128, 256]
WALKS = ["rows", "records"]


def _arch():
    try:
        import torch
        return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:
        return "gfx950"


def lookup(workload: str, arch: str = None):
    try:
        with open(CACHE) as f:
            data = json.load(f)
    except (OSError, ValueError):
        return None
    return data.get(f"{arch or _arch()}/{workload}")


def tune(workload_name, batch, make_step, steps=5, tiles=TILES, batches=BATCHES, walks=WALKS, log=print):
    """make_step(tile_w, tile_h, lds_batch, bwd_walk) -> callable running one fwd+bwd
    step.  Returns the best {tile_w, tile_h, lds_batch, bwd_walk, ms} and stores it in
    the cache."""
    import torch
    results = []
    for tw, th in tiles:
        for lb in batches:
            for wk in walks:
                step = make_step(tw, th, lb, wk)
                step()
                torch.cuda.synchronize()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                for _ in range(steps):
                    step()
                e1.record()
                torch.cuda.synchronize()
                ms = e0.elapsed_time(e1) / steps
                results.append({"tile_w": tw, "tile_h": th, "lds_batch": lb, "bwd_walk": wk, "ms": ms})
                log(f"[autotune] {tw}x{th} batch {lb} {wk}: {ms:.3f} ms")
    best = min(results, key=lambda r: r["ms"])
    try:
        with open(CACHE) as f:
            data = json.load(f)
    except (OSError, ValueError):
        data = {}
    data[f"{_arch()}/{workload_name}"] = {**best, "candidates": results}
    with open(CACHE, "w") as f:
        json.dump(data, f, indent=1)
    return best
