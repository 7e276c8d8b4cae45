#!/usr/bin/env python3
"""Forward + backward throughput of the EWA surfel rasterizer on one MI355X.

One step = one pass of the whole path over one batch: environment levels,
preprocess + shade, binning (scan, emission, radix sort, ranges), raster
forward, raster backward, preprocess/shade adjoint, environment adjoint, for
every view of the workload.  Inputs are resident in HBM before timing.

Default workload: 1M surfels on a union of 5 superquadrics, 8 views of
800 x 800, split-sum shading with a 128 x 256 HDR environment, batched
launches captured in a HIP graph.  Also reported: the same work as per-view
launches, per-stage times, the dominant kernel against the HBM roofline, and
the CPU oracle on a bounded sample.  Prints one JSON line.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3   # MI355X vector FP32 (256 CUs at 2.4 GHz)
# Algorithmic FP32 operations per covering fragment, the workload model's
# per-unit figures: about 45 for the forward (evaluation, cutoff, weight,
# compositing) and 130 for the backward (the evaluation again, the layer
# coefficients, the 11 record values through the chain rule and their sums);
# the two transcendentals per fragment are not counted.
FLOPS_PER_FRAGMENT = {"raster_forward": 45, "raster_backward": 130}
# A tighter count of what these kernels' formulation needs (an FMA counts 2,
# each reciprocal or exponential 1): the evaluation (pixel offset, perspective
# denominator, quadratic form, cutoff, weight: 20 + 2), the layer state (2), and
# in the backward the gradient of the 11 record values (39 + 1) plus their
# per-record sums (11).  Reported beside the model's figure.
FLOPS_PER_FRAGMENT_TIGHT = {"raster_forward": 30, "raster_backward": 75}
WORKLOAD_DESC = {
    "C1": "4,096 surfels on the unit sphere, albedo shading, 1 view 128x128",
    "C2": "200k surfels on a displaced torus, split-sum, envmap 64x128, 1 view 512x512",
    "C3": "1M surfels on 5 superquadrics, split-sum, envmap 128x256, 8 views 800x800",
    "C4": "3M density-clustered surfels on a displaced sphere, split-sum, envmap 128x256, 1 view 1920x1080",
    "C5": "4 scenes (50k, 300k, 1M, 2M surfels), 16 views 256^2..1024^2, split-sum, envmaps 128x256",
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def algorithmic_bytes(stage, n_pairs, n_rec_vis, n_pix, mean_layers, n_surf):
    """Algorithmic HBM bytes of one launch of a raster kernel:
    per pair a 4-byte sorted id and the 64-byte record; per pixel the image,
    alpha and layer count (forward writes, backward reads dL/dimage, dL/dalpha),
    16 bytes per composited layer; backward adds a read-modify-write of the 11
    record gradients of every record that reaches a pixel."""
    per_pair = 4 + 64
    if stage == "raster_forward":
        return n_pairs * per_pair + n_pix * (12 + 4 + 1 + 16 * mean_layers)
    if stage == "raster_backward":
        return n_pairs * per_pair + n_pix * (12 + 4 + 1 + 16 * mean_layers) + n_rec_vis * 11 * 4 * 2
    return None


def raster_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in ("paper_2605_05876_amd/csrc/raster.hip", "paper_2605_05876_amd/csrc/common.h"):
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def committed_record(name, workload, tile, lds_batch):
    """The JSON record at the end of profiles/<name>, if it was taken on this
    workload and tile setup with the current raster sources (else None)."""
    try:
        text = open(os.path.join(ROOT, "profiles", name)).read()
        rec = json.loads(text.rsplit("```json", 1)[1].split("```", 1)[0])
    except (OSError, IndexError, ValueError):
        return None
    if (rec.get("source_sha256") != raster_source_hash() or rec.get("workload") != workload
            or rec.get("tile") != tile or rec.get("lds_batch") != lds_batch):
        return None
    return rec


def measured_traffic(kernel, workload, tile, lds_batch):
    """HBM bytes per launch of a raster kernel from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE summary (None when stale)."""
    rec = committed_record("hbm_traffic_raster_c3.md", workload, tile, lds_batch)
    return rec[kernel]["bytes_per_launch"] if rec and kernel in rec else None


def measured_valu_busy(kernel, workload, tile, lds_batch):
    """VALU issue fraction of a raster kernel from the committed instruction
    counters (None when stale)."""
    rec = committed_record("counters_raster_c3.md", workload, tile, lds_batch)
    return rec[kernel]["valu_issue_busy"] if rec and kernel in rec else None


def step_algorithmic_bytes(n_surf, n_rec, n_pairs, n_pix):
    """HBM bytes one fwd+bwd step must move at least: parameters read twice and
    their gradients written (192 per surfel), per (surfel, view) record its write,
    its gradient write and read back (200), per pair the emission, sort, sorted id
    and two reads of id + record (180), per pixel-view the image and alpha, their
    gradients and the re-read state (56)."""
    return 192 * n_surf + 200 * n_rec + 180 * n_pairs + 56 * n_pix


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(workload, opts_shade, budget_s=20.0):
    """The oracle (FP64 brute force) on a bounded sample: view 0, a seeded set
    of pixels, every surfel; forward + backward including the environment
    prefilter and its adjoint.  Mpixel-views/s over the sampled pixels."""
    import numpy as np
    import oracle as O
    sc, cam = workload.scenes[0], workload.cameras[0]
    opt = O.Options(shade=opts_shade)
    rng = np.random.default_rng(0)
    t0 = time.perf_counter()
    maps = lut = None
    hw = (0, 0)
    if opts_shade == "splitsum":
        maps = O.envmap(np.asarray(sc.envmap, np.float64))
        lut = O.brdf_lut(64, 64, 1024)
        hw = sc.envmap.shape[:2]
    t_env = time.perf_counter() - t0
    # calibrate the pixel count so that the sample takes ~budget_s: the cost of one
    # call is a fixed part (per-surfel preprocessing) plus a per-pixel part, so
    # time two probe sizes and solve for both
    def probe(n):
        pp = np.stack([rng.integers(0, cam.width, n), rng.integers(0, cam.height, n)], 1).astype(np.int32)
        t = time.perf_counter()
        O.render(sc, cam, opt, pp, maps=maps, lut=lut, env_hw=hw)
        O.render_grad(sc, cam, opt, pp, np.ones((n, 3)), np.ones(n), maps=maps, lut=lut, env_hw=hw)
        return time.perf_counter() - t
    t_a, t_b = probe(16), probe(256)
    per_px = max((t_b - t_a) / 240.0, 1e-7)
    fixed = max(t_a - 16 * per_px, 0.0)
    k = int(max(64, min(200000, (budget_s - t_env - fixed) / per_px)))
    pix = np.stack([rng.integers(0, cam.width, k), rng.integers(0, cam.height, k)], 1).astype(np.int32)
    t2 = time.perf_counter()
    if opts_shade == "splitsum":
        maps = O.envmap(np.asarray(sc.envmap, np.float64))
    O.render(sc, cam, opt, pix, maps=maps, lut=lut, env_hw=hw)
    gr = O.render_grad(sc, cam, opt, pix, rng.normal(size=(k, 3)), rng.normal(size=k), maps=maps,
                       lut=lut, env_hw=hw)
    if opts_shade == "splitsum":
        O.envmap_adjoint(gr["maps"], *hw)
    dt = time.perf_counter() - t2
    cores = O.set_threads()
    # the same per-pixel work on one thread, on a smaller sample (~budget/4)
    O.set_threads(1)
    k1 = int(max(16, min(k, (budget_s / 4) / max(per_px * cores, 1e-9))))
    pix1 = pix[:k1]
    t3 = time.perf_counter()
    O.render(sc, cam, opt, pix1, maps=maps, lut=lut, env_hw=hw)
    O.render_grad(sc, cam, opt, pix1, np.ones((k1, 3)), np.ones(k1), maps=maps, lut=lut, env_hw=hw)
    dt1 = time.perf_counter() - t3
    O.set_threads(cores)
    return {"value": k / dt / 1e6, "unit": "Mpixel-views/s", "cores": cores, "kind": "oracle",
            "cpu": cpu_model(), "value_1thread": k1 / dt1 / 1e6,
            "sample": f"view 0 of the workload, {k} seeded pixels, all {sc.n} surfels, FP64 forward + "
                      f"adjoint incl. environment prefilter and its adjoint; {dt:.1f} s on {cores} threads; "
                      f"1 thread: {k1} of those pixels (forward + adjoint, no environment) in {dt1:.1f} s"}


def check_status(renderer, what):
    """Polls the device status (synchronising); a latched error (a pair-capacity
    overflow in a timed step) makes the run fail instead of reporting a rate of
    truncated work."""
    d = renderer.poll()
    if d["device_status"] != 0 or d["status"] != 0:
        raise RuntimeError(f"device status after {what}: {d}")
    return d


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", default="C3", choices=list(WORKLOAD_DESC))
    ap.add_argument("--tile", default=None, help="WxH, e.g. 16x16 (default: autotune cache or 16x16)")
    ap.add_argument("--lds-batch", type=int, default=None)
    ap.add_argument("--bwd-walk", default=None, choices=["auto", "rows", "records"],
                    help="walk of the raster backward (default: autotune cache or auto)")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-per-view", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile-only", action="store_true", help="eager steps only (for rocprofv3)")
    ap.add_argument("--autotune", action="store_true",
                    help="sweep tile shape x LDS batch on --config, store the best in the autotune cache "
                         "(and print the sweep as one JSON line)")
    ap.add_argument("--mip-ablation", action="store_true",
                    help="forward time of the 4M-surfel checkerboard at 800x600 with no MIP filter, the "
                         "centre-precomputed filter, the per-pixel Jacobian and 4x supersampling")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "runs on one GPU only; the multi-GPU path (split the views, one "
                                   "all-reduce of the surfel gradients) is not implemented",
                                   "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2605_05876_amd as ss
    import scenegen as g
    from paper_2605_05876_amd import autotune

    torch.cuda.set_device(0)
    if args.mip_ablation:
        return mip_ablation(args)
    if args.autotune:
        return run_autotune(args)
    t0 = time.perf_counter()
    w = g.make_config(args.config)
    log(f"[bench] workload {args.config}: {w.n_surfels} surfels, {len(w.cameras)} views, "
        f"{w.pixel_views} pixel-views ({time.perf_counter() - t0:.1f} s to generate)")
    tune = autotune.lookup(args.config)
    tw, th = (16, 16)
    lb = 128
    walk = "auto"
    if tune:
        tw, th, lb = tune["tile_w"], tune["tile_h"], tune["lds_batch"]
        walk = tune.get("bwd_walk", "auto")
    if args.tile:
        tw, th = (int(x) for x in args.tile.lower().split("x"))
    if args.lds_batch:
        lb = args.lds_batch
    if args.bwd_walk:
        walk = args.bwd_walk
    opts = ss.Options(shade=w.shade, tile_w=tw, tile_h=th, lds_batch=lb, bwd_walk=walk)
    batch = ss.batch_from_scenes(w.scenes, w.cameras)
    n_pix = batch.n_pixels
    rng = np.random.default_rng(0)
    G = torch.from_numpy(rng.normal(size=(n_pix, 3)).astype(np.float32)).cuda()
    Ga = torch.from_numpy(rng.normal(size=n_pix).astype(np.float32)).cuda()

    def make(launch):
        # no poll inside timed steps: the device status is checked after each timed loop
        r = ss.Renderer(ss.Options(**{**opts.__dict__, "launch": launch}), check_capacity=False)
        ws = r.reserve(batch)
        img = torch.empty((n_pix, 3), device="cuda")
        alpha = torch.empty((n_pix,), device="cuda")
        nl = torch.empty((n_pix,), device="cuda", dtype=torch.uint8)
        grads = {k: torch.empty_like(batch.params[k]) for k in ss.PARAMS}
        if batch.envmaps is not None:
            grads["envmap"] = [torch.empty_like(e) for e in batch.envmaps]

        def step():
            r.forward(batch, out=(img, alpha, nl))
            r.backward(batch, G, Ga, grads=grads)
        return r, step, ws, (img, alpha, nl, grads)

    def timed(step, n, graph):
        if graph:
            s = torch.cuda.Stream()
            s.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(s):
                for _ in range(2):
                    step()
            torch.cuda.current_stream().wait_stream(s)
            torch.cuda.synchronize()
            cg = torch.cuda.CUDAGraph()
            with torch.cuda.graph(cg):
                step()
            run = cg.replay
        else:
            run = step
        for _ in range(args.warmup):
            run()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t = time.perf_counter()
        e0.record()
        for _ in range(n):
            run()
        e1.record()
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t) / n * 1e3
        return max(wall, e0.elapsed_time(e1) / n)

    r, step, ws, bufs = make("batched")
    step()
    torch.cuda.synchronize()
    diag = r.poll()
    if diag["status"] != 0:
        raise RuntimeError(f"device status {diag}")
    log(f"[bench] reserved {ws / 2**30:.2f} GiB; pairs {diag['n_pairs']}, records {diag['n_records']}")
    use_graph = not args.no_graph and not args.profile_only
    if args.profile_only:
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        # a plain copy of known size, to calibrate the HBM byte counters
        src = torch.empty(256 * 2**20 // 4, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] profile-only run done (+ one {src.numel() * 4} byte device copy)")
        return
    ms = timed(step, args.steps, use_graph)
    value = n_pix / (ms * 1e-3) / 1e6
    log(f"[bench] batched{'+graph' if use_graph else ''}: {ms:.3f} ms/step, {value:.1f} Mpixel-views/s")
    check_status(r, "batched timed steps")

    # per-stage times (eager, HIP events on the library's stream)
    r.profile(True)
    for _ in range(max(3, min(args.steps, 10))):
        step()
    prof = r.profile_read()
    r.profile(False)
    log(f"[bench] raw stage profile: {prof}")
    stages = {k: (v[0] / v[1] if v[1] else 0.0) for k, v in prof.items()}
    per_step = {k: v[0] / max(1, max(3, min(args.steps, 10))) for k, v in prof.items()}
    log("[bench] stage ms/launch: " + ", ".join(f"{k} {v:.3f}" for k, v in stages.items()))
    check_status(r, "stage-profiled steps")
    dom = max(("raster_forward", "raster_backward"), key=lambda k: per_step[k])
    nl_mean = float(bufs[2].float().mean().item())
    # the work of one step, counted by the raster forward (options.counters)
    rc = ss.Renderer(ss.Options(**{**opts.__dict__, "counters": True}), check_capacity=False)
    rc.forward(batch)
    dc = check_status(rc, "counted forward")
    del rc
    work = {"P_pairs": diag["n_pairs"], "F_fragments": dc["n_fragments"], "E_evaluated": dc["n_evaluated"],
            "layers": dc["n_layers"], "W_mean": round(dc["sum_layer_weight"] / max(dc["n_layers"], 1), 3),
            "layers_per_pixel": round(dc["n_layers"] / n_pix, 4),
            "E_over_F": round(dc["n_evaluated"] / max(dc["n_fragments"], 1), 2)}
    log(f"[bench] work: {work}")
    t_dom = stages[dom] * 1e-3
    alg = algorithmic_bytes(dom, diag["n_pairs"], diag["n_records"], n_pix, nl_mean, w.n_surfels)
    hbm_achieved = alg / t_dom / 1e9 if t_dom > 0 else 0.0
    flops = FLOPS_PER_FRAGMENT[dom] * dc["n_fragments"]
    alu_achieved = flops / t_dom / 1e12 if t_dom > 0 else 0.0
    traffic = measured_traffic(dom, args.config, f"{tw}x{th}", lb)
    valu_busy = measured_valu_busy(dom, args.config, f"{tw}x{th}", lb)
    # the binding resource: VALU issue (counters) against HBM (measured traffic,
    # else the algorithmic bytes)
    hbm_use = (traffic if traffic else alg) / t_dom / 1e9 / HBM_PEAK_GBS if t_dom > 0 else 0.0
    alu_use = valu_busy if valu_busy is not None else alu_achieved / FP32_PEAK_TFLOPS
    bound = "alu" if alu_use >= hbm_use else "hbm"
    if bound == "alu":
        roof = {"kernel": dom, "bound": "alu", "achieved": round(alu_achieved, 3), "peak": FP32_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": round(alu_achieved / FP32_PEAK_TFLOPS, 5)}
    else:
        roof = {"kernel": dom, "bound": "hbm", "achieved": round(hbm_achieved, 2), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(hbm_achieved / HBM_PEAK_GBS, 5)}
    roof.update({"traffic": traffic, "valu_issue_busy": valu_busy,
                 "alu": {"algorithmic_flops_per_launch": int(flops),
                         "flops_per_fragment": FLOPS_PER_FRAGMENT[dom],
                         "tight_flops_per_fragment": FLOPS_PER_FRAGMENT_TIGHT[dom],
                         "tight_frac": round(FLOPS_PER_FRAGMENT_TIGHT[dom] * dc["n_fragments"] / t_dom / 1e12
                                             / FP32_PEAK_TFLOPS, 5) if t_dom > 0 else 0.0,
                         "achieved_TFLOPs": round(alu_achieved, 3),
                         "frac": round(alu_achieved / FP32_PEAK_TFLOPS, 5)},
                 "hbm": {"algorithmic_bytes_per_launch": int(alg), "achieved_GBps": round(hbm_achieved, 2),
                         "frac": round(hbm_achieved / HBM_PEAK_GBS, 5)},
                 "launch_ms": round(stages[dom], 4), "n_pairs": diag["n_pairs"],
                 "mean_layers": round(nl_mean, 3)})
    if traffic:
        roof["traffic_over_algorithmic"] = round(traffic / alg, 3)
        roof["traffic_GBps"] = round(traffic / t_dom / 1e9, 1)
    b_step = step_algorithmic_bytes(w.n_surfels, diag["n_records"], diag["n_pairs"], n_pix)
    step_roof = {"algorithmic_bytes": int(b_step), "achieved_GBps": round(b_step / (ms * 1e-3) / 1e9, 1),
                 "hbm_frac": round(b_step / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 5),
                 "hbm_ceiling_Mpixel_views_s": round(n_pix / (b_step / (HBM_PEAK_GBS * 1e9)) / 1e6, 1)}

    out = {"metric": "fwd+bwd Mpixel-views/s", "value": round(value, 2), "unit": "Mpixel-views/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": f"{args.config}: {WORKLOAD_DESC[args.config]}",
                      "launch": "batched" + ("+hipgraph" if use_graph else ""),
                      "tile": f"{tw}x{th}", "lds_batch": lb,
                      "bwd_walk": walk if walk != "auto" else ("records" if lb >= 256 else "rows"),
                      "pixel_views": n_pix, "surfels": w.n_surfels},
           "roofline": roof,
           "step_roofline": step_roof,
           "work": work,
           "stages_ms_per_step": {k: round(v, 4) for k, v in per_step.items()}}
    del r, step, bufs
    torch.cuda.empty_cache()

    if not args.no_per_view:
        # plain per-view launches (one launch chain per view, eager), and the same
        # captured in a graph
        rp, stepp, _, bp = make("per_view")
        stepp()
        torch.cuda.synchronize()
        msp = timed(stepp, args.steps, False)
        check_status(rp, "per-view timed steps")
        out["per_view"] = {"value": round(n_pix / (msp * 1e-3) / 1e6, 2), "ms_per_step": round(msp, 4),
                           "launch": "per-view, eager", "speedup_batched": round(msp / ms, 3)}
        log(f"[bench] per-view eager: {msp:.3f} ms/step")
        # where the per-view time goes: the same stages, summed over the views
        rp.profile(True)
        n_prof = max(3, min(args.steps, 10))
        for _ in range(n_prof):
            stepp()
        pprof = rp.profile_read()
        rp.profile(False)
        out["per_view"]["stages_ms_per_step"] = {k: round(v[0] / n_prof, 4) for k, v in pprof.items()}
        out["per_view"]["stage_launches_per_step"] = {k: v[1] // n_prof for k, v in pprof.items()}
        log(f"[bench] per-view stages ms/step: {out['per_view']['stages_ms_per_step']}")
        if use_graph:
            msg = timed(stepp, args.steps, True)
            check_status(rp, "per-view graph steps")
            out["per_view"]["graph_ms_per_step"] = round(msg, 4)
            log(f"[bench] per-view+graph: {msg:.3f} ms/step")
        del rp, stepp, bp
        torch.cuda.empty_cache()

    if not args.no_cpu_baseline:
        log("[bench] CPU oracle baseline ...")
        out["cpu_baseline"] = cpu_baseline(w, w.shade)
    print(json.dumps(out), flush=True)


def run_autotune(args):
    """Time one fwd+bwd step per (tile, LDS batch) candidate; keep the fastest."""
    import numpy as np
    import torch

    import paper_2605_05876_amd as ss
    import scenegen as g
    from paper_2605_05876_amd import autotune

    w = g.make_config(args.config)
    batch = ss.batch_from_scenes(w.scenes, w.cameras)
    n = batch.n_pixels
    rng = np.random.default_rng(0)
    G = torch.from_numpy(rng.normal(size=(n, 3)).astype(np.float32)).cuda()
    Ga = torch.from_numpy(rng.normal(size=n).astype(np.float32)).cuda()
    keep = []

    def make_step(tw, th, lb, walk):
        keep.clear()
        torch.cuda.empty_cache()
        r = ss.Renderer(ss.Options(shade=w.shade, tile_w=tw, tile_h=th, lds_batch=lb, bwd_walk=walk))
        r.reserve(batch)
        out = (torch.empty((n, 3), device="cuda"), torch.empty(n, device="cuda"), None)
        grads = {k: torch.empty_like(batch.params[k]) for k in ss.PARAMS}
        if batch.envmaps is not None:
            grads["envmap"] = [torch.empty_like(e) for e in batch.envmaps]
        keep.append((r, out, grads))

        def step():
            r.forward(batch, out=out)
            r.backward(batch, G, Ga, grads=grads)
        return step
    best = autotune.tune(args.config, batch, make_step, steps=max(3, args.steps), log=log)
    print(json.dumps({"autotune": args.config, "best": best,
                      "cache": autotune.lookup(args.config)}), flush=True)


def mip_ablation(args):
    """Anti-aliasing comparison of Sec. 4.4.2 on its synthetic scene: forward time per
    frame of a 4M-surfel checkerboard plane at 800x600 with (a) no MIP filter
    (sigma_f = 0), (b) the centre-precomputed filter, (c) the per-pixel Jacobian and
    (d) 4x supersampling (1600x1200 without the filter, then a 2x2 box filter)."""
    import torch
    import torch.nn.functional as F

    import paper_2605_05876_amd as ss
    import scenegen as g

    t0 = time.perf_counter()
    w = g.checkerboard_workload()
    big = g.checkerboard_workload(width=1600, height=1200)
    log(f"[mip] checkerboard: {w.n_surfels} surfels ({time.perf_counter() - t0:.1f} s to generate)")
    batch = ss.batch_from_scenes(w.scenes, w.cameras)
    batch_big = ss.batch_from_scenes(big.scenes, big.cameras)
    sigma = 0.1
    cases = {"none": (batch, dict(sigma_f=0.0)), "centre": (batch, dict(sigma_f=sigma)),
             "per_pixel": (batch, dict(sigma_f=sigma, mip="pixel")), "ssaa4x": (batch_big, dict(sigma_f=0.0))}
    out = {"metric": "forward ms/frame, 4M-surfel checkerboard plane, 800x600", "unit": "ms",
           "higher_is_better": False, "dtype": "f32", "data": "synthetic", "steps": args.steps,
           "config": {"workload": "ground plane 2000^2 lattice over [-10,10]^2, checker 0.2, camera at "
                                  "(0,-10.6,0.45) looking at the origin, 45 deg vertical FOV",
                      "sigma_f": sigma},
           "paper_ms_context": {"none": 42, "centre": 50, "per_pixel": 65, "ssaa4x": 87}}
    images = {}
    for name, (b, kw) in cases.items():
        r = ss.Renderer(ss.Options(shade="albedo", **kw))
        r.reserve(b)
        img = torch.empty((b.n_pixels, 3), device="cuda")
        alpha = torch.empty((b.n_pixels,), device="cuda")
        cam = b.cameras[0]

        def step():
            r.forward(b, out=(img, alpha, None))
            if name == "ssaa4x":
                x = img.view(cam.height, cam.width, 3).permute(2, 0, 1)[None]
                return F.avg_pool2d(x, 2)
            return img
        step()
        torch.cuda.synchronize()
        assert r.poll()["status"] == 0
        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.steps):
            res = step()
        e1.record()
        torch.cuda.synchronize()
        out[name] = round(e0.elapsed_time(e1) / args.steps, 3)
        res = res.reshape(3, -1).t() if name == "ssaa4x" else res
        images[name] = res.reshape(-1, 3).float().cpu()
        log(f"[mip] {name}: {out[name]:.3f} ms/frame")
        del r
        torch.cuda.empty_cache()
    # how far each filtered image is from the supersampled one (a quality context)
    ref = images["ssaa4x"]
    out["rms_vs_ssaa4x"] = {k: round(float((v - ref).pow(2).mean().sqrt()), 5) for k, v in images.items()
                            if k != "ssaa4x"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
