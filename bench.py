"""Benchmark: path samples/s at 1080p with HDR-NIF lighting on one MI355X.

Workload: the small-BVH scene (displaced icosphere, 81,920 + 2 triangles) at
1920x1080, 32 spp, max depth 6, lit by the HDR-NIF in FP16 on MFMA after
on-device training (batch 65,536, 2^24 samples).  A step is one full render
(camera rays, traversal + shading, NIF on every escaped ray, accumulation).
Prints one JSON line.  Also reported: the same render with the plain
environment-map lookup (rate and image difference at equal seeds), NIF
queries/s and MFMA utilisation, the trace kernel's roofline from live HIP
events and counted algorithmic bytes, and the CPU oracle timed on a row
sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "path samples/s at 1080p; NIF rays/s + MFMA util vs env-map lookup at equal RMSE"
HBM_PEAK_GBS = 8000.0
MFMA_PEAK_TFLOPS = {"fp16": 2500.0, "bf16": 2500.0, "fp8": 5000.0, "fp32": 157.3}
NIF_FLOP_PER_QUERY = 2 * (64 * 96 + 4 * 96 * 96 + 96 * 3)  # 86,592
# algorithmic bytes of the trace kernel: ray in 48 B, one node
# per BVH node fetched (64 B two-wide, 112 B four-wide), 48 B per primitive
# slot tested, 80 B per hit (slot re-read + material), 32 B per escaped ray
# (environment queue), 48 B per survivor
B_RAY, B_PRIM, B_HIT, B_ESC, B_OUT = 48, 48, 80, 32, 48
B_NODE = {2: 64, 4: 112}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_trace_small_bvh_1080p_traffic.json")


def _parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=5)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--width", type=int, default=1920)
    p.add_argument("--height", type=int, default=1080)
    p.add_argument("--spp", type=int, default=32)
    p.add_argument("--depth", type=int, default=6)
    p.add_argument("--train-samples", type=int, default=1 << 24)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-envmap", action="store_true")
    p.add_argument("--calibrate-copy", action="store_true",
                   help="run one 1 GiB device copy (rocprof counter calibration)")
    p.add_argument("--cpu-seconds", type=float, default=15.0)
    return p.parse_args()


def _kernel_sha():
    h = hashlib.sha256()
    for f in ("k_render.hip", "npt_device.h", "npt_shared.h"):
        h.update(open(os.path.join(ROOT, "paper_2305_20061_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def _traffic_per_launch():
    """HBM bytes per trace launch from committed rocprofv3 counters, if they
    were taken on the current kernel source."""
    try:
        t = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if t.get("kernel_sha") != _kernel_sha():
        return None
    return t.get("bytes_per_launch")


def _oracle_rows(args):
    """Worker: oracle render of a row subset; returns path samples traced."""
    scene_cfg, rows, W, H, spp, depth, seed, params = args
    import oracle as O
    from paper_2305_20061_amd import synth
    sc = synth.scene_for(scene_cfg)
    S = O.Scene(sc, accel=1)
    cam = O.make_camera(**sc["camera"])
    rd = O.render_desc(W, H, spp, depth, seed, nif_params=params, nif=O.nif_shape())
    out = np.zeros((H, W, 3))
    n = 0
    t0 = time.perf_counter()
    for y in rows:
        n += O.lib().or_render_rows(S.h, O.C.byref(cam), O.C.byref(rd), y, H + 1,
                                    out.ctypes.data_as(O.C.POINTER(O.C.c_double)))
    return n, time.perf_counter() - t0


def cpu_baseline(W, H, spp, depth, seed, seconds):
    """The oracle (single-threaded C, FP64 NIF) on a bounded row sample, run as
    one process per host core over disjoint rows."""
    from paper_2305_20061_amd import synth
    params = synth.nif_init(3).astype(np.float32).astype(np.float16).astype(np.float64)
    cores = max(1, min(16, os.cpu_count() or 1))
    # calibrate one row on one core
    n1, t1 = _oracle_rows((3, [H // 2], W, H, spp, depth, seed, params))
    per_row = t1
    rows_total = max(cores, int(seconds * cores / max(per_row, 1e-3)))
    rows_total = min(rows_total, H)
    step = max(1, H // rows_total)
    rows = list(range(0, H, step))[:rows_total]
    chunks = [rows[i::cores] for i in range(cores)]
    t0 = time.perf_counter()
    with mp.get_context("spawn").Pool(cores) as pool:
        res = pool.map(_oracle_rows, [(3, c, W, H, spp, depth, seed, params) for c in chunks if c])
    wall = time.perf_counter() - t0
    paths = sum(r[0] for r in res)
    return {"value": paths / wall, "unit": "path samples/s", "cores": cores, "kind": "oracle",
            "sample": f"{len(rows)} of {H} rows (every {step}th), {W} px x {spp} spp each, "
                      f"depth {depth}, FP64 NIF; {paths} path samples in {wall:.1f} s"}


def main():
    args = _parse()
    if args.gpus != 1:
        print(json.dumps({"error": "one GPU only: this build measures a single MI355X; "
                                   "the multi-GPU sharding is described in DESIGN.md"}))
        sys.exit(2)
    import torch

    from paper_2305_20061_amd import npt, synth

    torch.cuda.set_device(0)
    W, H, spp, depth, seed = args.width, args.height, args.spp, args.depth, 1
    scene = synth.scene_for(3)
    env = synth.env_map()
    ctx = npt.npt_create(0)
    extra = {}
    try:
        t0 = time.perf_counter()
        # 4-wide BVH, leaf size 2, no LDS-staged levels: fastest in the sweep
        npt.npt_load_scene(ctx, scene, max_leaf=2, lds_levels=0, width=4)
        extra["bvh_build_ms"] = 1e3 * (time.perf_counter() - t0)
        extra["bvh"] = npt.npt_bvh_info(ctx)
        npt.npt_env_upload(ctx, env)
        npt.npt_nif_upload(ctx, synth.nif_init(3))
        npt.npt_nif_set_precision(ctx, npt.FP16)
        tr = npt.npt_nif_train(ctx, npt.train_params(batch=65536, samples=args.train_samples, seed=1,
                                                     grad_prec=npt.FP16))
        extra["train"] = {"ms": tr["ms"], "steps": tr["steps"], "first_loss": tr["first_loss"],
                          "last_loss": tr["last_loss"], "grid_eval": npt.npt_nif_eval_grid(ctx, 1024, 512)}
        npt.npt_set_env_mode(ctx, npt.ENV_NIF)
        out = torch.empty(H, W, 3, dtype=torch.float32, device="cuda")

        if args.calibrate_copy:
            # one elementwise kernel reading 1 GiB and writing 1 GiB: the scale
            # for the FETCH_SIZE / WRITE_SIZE counters of the same run
            a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
            b = torch.empty_like(a)
            torch.mul(a, 1.0, out=b)
            torch.cuda.synchronize()
            extra["copy_calibration"] = {"read_bytes": a.numel() * 4, "write_bytes": b.numel() * 4}
            del a, b

        # counting render (outside the timed region): algorithmic bytes
        npt.npt_set_render_options(ctx, rr_start=3, count_visits=1)
        npt.npt_render(ctx, W, H, spp, depth, seed, out)
        cs = npt.npt_get_stats(ctx)
        rays = np.array(cs["rays"], np.float64)
        esc = np.array(cs["escaped"], np.float64)
        visits = np.array(cs["node_visits"], np.float64)
        tests = np.array(cs["prim_tests"], np.float64)
        survivors = np.concatenate([rays[1:], [0.0]])
        hits = rays - esc
        alg_bytes = float(np.sum(B_RAY * rays + B_NODE[extra["bvh"]["width"]] * visits + B_PRIM * tests + B_HIT * hits
                                 + B_ESC * esc + B_OUT * survivors))
        extra["per_ray"] = {"node_visits": float(visits.sum() / rays.sum()),
                            "prim_tests": float(tests.sum() / rays.sum()),
                            "rays_per_path": float(rays.sum() / cs["paths"]),
                            "escaped_per_path": float(esc.sum() / cs["paths"])}

        # timed renders with per-kernel events
        npt.npt_set_render_options(ctx, rr_start=3, kernel_timing=1)
        for _ in range(args.warmup):
            npt.npt_render(ctx, W, H, spp, depth, seed, out)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            npt.npt_render(ctx, W, H, spp, depth, seed, out)
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        st = npt.npt_get_stats(ctx)  # events of the last timed render
        img_nif = out.cpu().numpy().astype(np.float64)
        ms_step = 1e3 * elapsed / args.steps
        value = W * H * spp * args.steps / elapsed

        trace_launch_ms = st["ms_trace"] / max(1, st["trace_launches"])
        achieved = alg_bytes / st["trace_launches"] / (trace_launch_ms * 1e-3) / 1e9
        traffic = _traffic_per_launch()
        nif_tflops = st["env_queries"] * NIF_FLOP_PER_QUERY / (st["ms_env"] * 1e-3) / 1e12
        extra["kernels"] = {"trace_ms_per_render": st["ms_trace"], "trace_launches": st["trace_launches"],
                            "trace_ms_per_launch": trace_launch_ms, "nif_ms_per_render": st["ms_env"],
                            "nif_launches": st["env_launches"], "render_ms_device": st["ms_total"]}
        extra["nif"] = {"precision": "fp16", "queries_per_render": st["env_queries"],
                        "queries_per_s": st["env_queries"] / (st["ms_env"] * 1e-3),
                        "tflops": nif_tflops, "mfma_util": nif_tflops / MFMA_PEAK_TFLOPS["fp16"],
                        "flop_per_query": NIF_FLOP_PER_QUERY}

        if not args.no_envmap:
            npt.npt_set_env_mode(ctx, npt.ENV_MAP)
            npt.npt_render(ctx, W, H, spp, depth, seed, out)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for _ in range(args.steps):
                npt.npt_render(ctx, W, H, spp, depth, seed, out)
            torch.cuda.synchronize()
            e_el = time.perf_counter() - t1
            se = npt.npt_get_stats(ctx)
            img_map = out.cpu().numpy().astype(np.float64)
            rel = float(np.sqrt(np.sum((img_nif - img_map) ** 2) / np.sum(img_map ** 2)))
            extra["env_map"] = {"path_samples_per_s": W * H * spp * args.steps / e_el,
                                "lookup_queries_per_s": se["env_queries"] / (se["ms_env"] * 1e-3),
                                "lookup_ms_per_render": se["ms_env"],
                                "nif_vs_envmap_image_rel_rmse": rel}
            npt.npt_set_env_mode(ctx, npt.ENV_NIF)
    finally:
        npt.npt_destroy(ctx)

    line = {
        "metric": METRIC, "value": value, "unit": "path samples/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32 rays / f16 NIF", "data": "synthetic",
        "config": {"workload": f"small-BVH+NIF: displaced icosphere 81,922 tris, {W}x{H}, {spp} spp, "
                               f"max depth {depth}, FP16 NIF (64-96x5-3) trained on device, seed {seed}",
                   "paths_per_step": W * H * spp},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic, "kernel": "k_trace (traversal + shading)",
                     "alg_bytes_per_launch": alg_bytes / st["trace_launches"]},
    }
    line.update(extra)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(W, H, spp, depth, seed, args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
