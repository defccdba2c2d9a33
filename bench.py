"""Benchmark: path samples/s at 1080p with HDR-NIF lighting on one MI355X.

Workload (default): the large-BVH scene, a 2048 x 2048 fractal terrain
(8,380,418 triangles) plus 256 instanced copies of the displaced icosphere
(81,920 triangles each) through the two-level BVH, at 1920x1080, 64 spp, max
depth 8, every escaped ray lit by the HDR-NIF with FP8 inference on MFMA
after on-device training (batch 65,536, 2^24 samples, FP16 gradients).  A
step is one full render (camera rays, traversal + shading, NIF on every
escaped ray, accumulation).  Prints one JSON line.

Also reported, on the same scene, camera and seeds: the FP16 NIF and the
plain environment-map lookup (path rate, NIF/lookup queries/s, image
difference), NIF throughput at a fixed 2^21-query batch, the trace kernel's
roofline from live HIP events and counted algorithmic bytes, the small-BVH
scene (FP16 NIF, 32 spp, depth 6) rate, and the CPU oracle timed on a row
sample of the same workload.  --config 3 makes the small-BVH scene the
timed workload instead.
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
# FP8 mode runs the first and output layers on FP16 MFMAs: the peak of the
# query's FLOP mix (1 / (f16 share / 2.5 + f8 share / 5.0) PFLOP/s)
_F8_SHARE = 2 * 4 * 96 * 96 / NIF_FLOP_PER_QUERY
MFMA_PEAK_TFLOPS_FP8_MIX = 1.0 / ((1.0 - _F8_SHARE) / 2500.0 + _F8_SHARE / 5000.0)
# algorithmic bytes of the extend kernel (closest hit): ray origin and
# direction in (24 B), one node per BVH node fetched (64 B two-wide, 112 B
# four-wide), 48 B per primitive slot tested, 16 B hit record out; instance
# records (32 B per instance entered) are not counted
B_RAY, B_PRIM, B_HITREC = 24, 48, 16
B_NODE = {2: 64, 4: 112}
# shade kernel per ray: ray and hit record in (64 B); per hit slot + material
# (80 B); per escaped ray the environment queue entry (32 B); per survivor the
# next queue entry (48 B).  Environment lookup per query: queue entry (32 B),
# four texels (64 B), path radiance read-modify-write (32 B)
B_SHADE_RAY, B_SHADE_HIT, B_SHADE_ESC, B_SHADE_OUT, B_LOOKUP = 64, 80, 32, 48, 128
WORKLOADS = {
    4: dict(name="large-BVH", spp=64, depth=8, prec="fp8",
            desc="large-BVH+NIF: 2048^2 terrain 8,380,418 tris + 256 instances x 81,920 tris (two-level BVH4), "
                 "{W}x{H}, {spp} spp, max depth {depth}, FP8 NIF (64-96x5-3) trained on device, seed {seed}",
            traffic="k_extend_large_bvh_1080p_traffic.json", counters="counters_large_bvh_fp8_1080p.json"),
    3: dict(name="small-BVH", spp=32, depth=6, prec="fp16",
            desc="small-BVH+NIF: displaced icosphere 81,922 tris, {W}x{H}, {spp} spp, max depth {depth}, "
                 "FP16 NIF (64-96x5-3) trained on device, seed {seed}",
            traffic="k_extend_small_bvh_1080p_traffic.json", counters="counters_small_bvh_fp16_1080p.json"),
}


def _parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=5)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--config", type=int, default=4, choices=(3, 4))
    p.add_argument("--width", type=int, default=1920)
    p.add_argument("--height", type=int, default=1080)
    p.add_argument("--train-samples", type=int, default=1 << 24)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-envmap", action="store_true", help="skip the FP16-NIF and env-map comparison renders")
    p.add_argument("--no-small", action="store_true", help="skip the small-BVH rate")
    p.add_argument("--calibrate-copy", action="store_true",
                   help="run one 1 GiB device copy (rocprof counter calibration)")
    p.add_argument("--cpu-seconds", type=float, default=15.0)
    p.add_argument("--node-format", choices=("fp32", "fp16-extent", "q8", "fp16-corner"), default="fp16-corner",
                   help="BVH4 node encoding: FP32 boxes (112 B), FP32 lower planes + binary16 extents (96 B), "
                        "8-bit planes on a per-node step (64 B), or binary16 planes on an FP32 node corner (80 B)")
    p.add_argument("--max-leaf", type=int, default=2, help="primitives per BVH leaf (1..8)")
    p.add_argument("--sort-rays", type=int, default=0,
                   help="1: sort every 1024-ray chunk of the secondary queues (direction octant, origin) before tracing")
    p.add_argument("--pool-paths", type=int, default=0,
                   help="upper bound on paths in flight (0: the library default, 2^27); a frame takes "
                        "ceil(paths / pool) passes")
    p.add_argument("--lds-levels", type=int, default=0,
                   help="top BVH levels staged in LDS per workgroup (of the two-level scene: of its top tree)")
    p.add_argument("--nif-sizes", action="store_true",
                   help="instead of the headline run: NIF model size against path rate and PSNR (one JSON line)")
    p.add_argument("--study-budgets", default="24,26,28,30",
                   help="--nif-study: training budgets, log2 of the samples of one continuing run")
    p.add_argument("--study-sun-radii", default="0.5,2,4",
                   help="--nif-study: angular radii (degrees) of the sun disk of the synthetic sky")
    p.add_argument("--nif-study", action="store_true",
                   help="instead of the headline run: the NIF output colour-space comparison (one JSON line)")
    p.add_argument("--spp-sweep", action="store_true",
                   help="instead of the headline run: path rate against samples per pixel on the box scenes "
                        "at 720x720 (one JSON line)")
    return p.parse_args()


def _sha(files):
    h = hashlib.sha256()
    for f in files:
        h.update(open(os.path.join(ROOT, "paper_2305_20061_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def _kernel_sha():
    return _sha(("k_render.hip", "npt_device.h", "npt_shared.h"))


# the sources each committed counter record was taken on
COUNTER_SOURCES = {"k_extend": ("k_render.hip", "npt_device.h", "npt_shared.h"),
                   "nif": ("k_nif.hip", "npt_nif_layout.h", "npt_nif_mma.h", "npt_mfma.h", "npt_device.h"),
                   "training": ("k_train_fused.hip", "npt_train.h", "npt_nif_mma.h", "npt_mfma.h",
                                "npt_nif_layout.h", "npt_device.h")}


def _counters(name):
    """Counter-derived figures of the committed rocprofv3 --pmc record
    profiles/<name>, per kernel, where its kernel source is the current one
    (else that kernel's entry is null)."""
    try:
        t = json.load(open(os.path.join(ROOT, "profiles", name)))
    except (OSError, ValueError):
        return None
    keep = ("mfma_busy", "valu_insts_per_simd_cycle", "valu_per_tile", "mfma_busy_cycles_per_tile",
            "lds_bank_conflict_share", "l2_hit_rate", "l2_request_gbs_128B", "ta_busy", "td_busy",
            "td_stalled_on_l2", "valu_wave_insts_per_64_node_visits", "valu_lane_utilization")
    out = {"source": f"profiles/{name}: rocprofv3 --pmc passes over bench.py on the same kernel sources, "
                     "not measured in this run"}
    for k, v in t.items():
        if not isinstance(v, dict) or "kernel_sha" not in v:
            continue
        group = "k_extend" if k.startswith("k_extend") else "nif" if k.startswith("k_nif") else "training"
        ok = v["kernel_sha"] == _sha(COUNTER_SOURCES[group])
        out[k] = {kk: v[kk] for kk in keep if kk in v} if ok else None
    return out


def _extend_limiter(counters):
    """What holds the extend kernel, in the words of its committed counter
    record (a wave64 FP32 VALU instruction takes 4 SIMD cycles)."""
    k = (counters or {}).get("k_extend")
    if not k:
        return "no counter record for these kernel sources"
    busy = 4.0 * k["valu_insts_per_simd_cycle"]
    lanes = k.get("valu_lane_utilization")
    active = f"{lanes:.2f} of the lanes active" if lanes is not None else "part of the lanes active"
    return (f"VALU issue (the SIMDs {100 * busy:.0f} % busy with wave64 VALU instructions, {active}: "
            f"divergent traversal) and the texture data path (TD busy {k['td_busy']:.2f}), "
            "with the tree in L2/MALL; HBM carries about a quarter of the algorithmic bytes "
            "(rocprofv3 counters, see counters)")


def _traffic_per_launch(name):
    """HBM bytes per extend launch from committed rocprofv3 counters, if they
    were taken on the current kernel source."""
    try:
        t = json.load(open(os.path.join(ROOT, "profiles", name)))
    except (OSError, ValueError):
        return None
    if t.get("kernel_sha") != _kernel_sha():
        return None
    return t.get("bytes_per_launch")


def _oracle_rows(args):
    """Worker: oracle render of a row subset; returns path samples traced."""
    cfg, rows, W, H, spp, depth, seed, prec = args
    import oracle as O
    from paper_2305_20061_amd import synth
    sc = synth.scene_for(cfg)
    S = O.Scene(sc, accel=1)
    cam = O.make_camera(**sc["camera"])
    shape = O.nif_shape()
    params = O.nif_dequantize(shape, synth.nif_init(3).astype(np.float32).astype(np.float64), prec)
    rd = O.render_desc(W, H, spp, depth, seed, nif_params=params, nif=shape, nif_prec=prec)
    out = np.zeros((H, W, 3))
    n = 0
    t0 = time.perf_counter()
    for y in rows:
        n += O.lib().or_render_rows(S.h, O.C.byref(cam), O.C.byref(rd), y, H + 1,
                                    out.ctypes.data_as(O.C.POINTER(O.C.c_double)))
    return n, time.perf_counter() - t0


def cpu_baseline(cfg, W, H, spp, depth, seed, prec, seconds):
    """The oracle (single-threaded C, FP64 sums) on a bounded row sample, run
    as one process per host core over disjoint rows."""
    cores = max(1, min(16, os.cpu_count() or 1))
    with mp.get_context("spawn").Pool(1) as pool:  # one row on one core
        n1, per_row = pool.map(_oracle_rows, [(cfg, [H // 2], W, H, spp, depth, seed, prec)])[0]
    rows_total = min(H, max(cores, int(seconds * cores / max(per_row, 1e-3))))
    step = max(1, H // rows_total)
    rows = list(range(0, H, step))[:rows_total]
    chunks = [rows[i::cores] for i in range(cores)]
    with mp.get_context("spawn").Pool(cores) as pool:
        res = pool.map(_oracle_rows, [(cfg, c, W, H, spp, depth, seed, prec) for c in chunks if c])
    paths = sum(r[0] for r in res)
    wall = max(r[1] for r in res)  # render time of the slowest worker (scene setup excluded)
    return {"value": paths / wall, "unit": "path samples/s", "cores": cores, "kind": "oracle",
            "single_core_value": n1 / per_row,
            "sample": f"{len(rows)} of {H} rows (every {step}th), {W} px x {spp} spp each, depth {depth}, "
                      f"{['FP32', 'FP16', 'BF16', 'FP8'][prec]}-rounded NIF operands with FP64 sums; "
                      f"{paths} path samples, slowest worker {wall:.1f} s"}


def _stage(msg):
    """Progress of the run's stages on stderr (the JSON line stays on stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _timed_renders(npt, torch, ctx, W, H, spp, depth, seed, out, steps, warmup):
    for _ in range(warmup):
        npt.npt_render(ctx, W, H, spp, depth, seed, out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        npt.npt_render(ctx, W, H, spp, depth, seed, out)
    torch.cuda.synchronize()
    return time.perf_counter() - t0, npt.npt_get_stats(ctx)


def _query_rate(npt, torch, ctx, mode, n=1 << 21, reps=20):
    """env queries/s of one mode at a fixed batch (events on the stream the
    library launches on: the null stream, torch's default)."""
    g = torch.Generator(device="cpu").manual_seed(0)
    d = torch.randn(n, 3, generator=g)
    d = (d / d.norm(dim=1, keepdim=True)).cuda()
    out = torch.empty(n, 3, device="cuda")
    npt.npt_env_query(ctx, mode, d, out)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        npt.npt_env_query(ctx, mode, d, out)
    e1.record()
    torch.cuda.synchronize()
    return n * reps / (e0.elapsed_time(e1) * 1e-3)


def _rel(a, b):
    return float(np.sqrt(np.sum((a - b) ** 2) / np.sum(b ** 2)))


# equal-RMSE study: image size divisor and samples of the env-map reference
EQ_DIV, EQ_REF_SPP = 4, 16384


def _equal_rmse(npt, torch, ctx, W, H, spp, depth, seed, precs, sample_s):
    """NIF images against the env map at equal error.  Without light sampling
    the env-map estimate is unbiased but carries the sun's fireflies; the NIF
    (which has not learned the sun) is smooth but biased.  At W/EQ_DIV x
    H/EQ_DIV (per-pixel error depends on the paths, not on the pixel count)
    the study renders an env-map reference of EQ_REF_SPP samples with another
    seed, the env-map image at 1..spp samples and each NIF image at spp.
    Model: squared relative error of an env-map image at s samples is C/s
    against the truth, r = C/EQ_REF_SPP for the reference; with independent
    noise an image X gives e^2 = (a + r)/(1 + r), a = |X - truth|^2/|truth|^2.
    C comes from the env-map curve, a from each NIF image, and the env-map
    sample count of equal error is C/a.  sample_s: device seconds per path
    sample of each mode at full size."""
    w, h, R = W // EQ_DIV, H // EQ_DIV, EQ_REF_SPP
    out = torch.empty(h, w, 3, dtype=torch.float32, device="cuda")

    def render(s, sd):
        npt.npt_render(ctx, w, h, s, depth, sd, out)
        torch.cuda.synchronize()
        return out.cpu().numpy().astype(np.float64)

    nif = {}
    for name, code in precs.items():
        npt.npt_nif_set_precision(ctx, code)
        nif[name] = render(spp, seed)
    npt.npt_set_env_mode(ctx, npt.ENV_MAP)
    ref = render(R, seed + 1000)
    curve, s = {}, 1
    while s <= spp:
        curve[s] = _rel(render(s, seed), ref)
        s *= 2
    # e^2 (1 + C/R) = C (1/s + 1/R)  =>  C = e^2 / (1/s + 1/R - e^2/R), one estimate per s
    cs = np.array([e * e / (1.0 / k + 1.0 / R - e * e / R) for k, e in curve.items()])
    C = float(np.exp(np.mean(np.log(cs))))
    r = C / R
    res = {"size": [w, h], "reference": f"env-map render, {R} spp, seed {seed + 1000}",
           "reference_rel_rmse_vs_truth": float(np.sqrt(r)),
           "env_map_rel_rmse_vs_reference_by_spp": {str(k): v for k, v in curve.items()},
           "env_map_variance_constant_C": C,
           "C_estimates_max_rel_dev": float(np.max(np.abs(cs / C - 1.0))),
           f"env_map_rel_rmse_vs_truth_at_{spp}_spp": float(np.sqrt(C / spp))}
    for name, img in nif.items():
        e = _rel(img, ref)
        a = e * e * (1.0 + r) - r
        row = {"rel_rmse_vs_reference": e, "rel_rmse_vs_truth": float(np.sqrt(max(a, 0.0)))}
        if a > 0:
            s_eq = C / a
            row["env_map_spp_at_equal_rmse"] = s_eq
            row["nif_cost_over_env_map_at_equal_rmse"] = sample_s[name] * spp / (sample_s["map"] * s_eq)
        else:
            row["note"] = "NIF error below the reference's own noise: unresolved"
        res[name] = row
    return res


SWEEP_SPP = [1, 2, 4, 8, 16, 32, 64, 128, 256, 512, 1024]


def spp_sweep(args):
    """Path rate against samples per pixel (the sample-count study of Sec. 4.5) on the
    closed box (area light, no environment, depth 5) and the open box (FP16
    NIF trained on the device, depth 6) at 720x720: where fixed costs per
    render (launches, queue set-up, accumulation) stop mattering.  Device
    time from HIP events around each render on the library's stream."""
    import torch

    from paper_2305_20061_amd import npt, synth

    torch.cuda.set_device(0)
    W = H = 720
    res = {}
    for name, cfg, depth in (("box", 0, 5), ("open_box_nif_fp16", 1, 6)):
        ctx = npt.npt_create(0)
        try:
            npt.npt_load_scene(ctx, synth.scene_for(cfg))
            if cfg == 0:
                npt.npt_set_env_mode(ctx, npt.ENV_NONE)
            else:
                npt.npt_env_upload(ctx, synth.env_map())
                npt.npt_nif_upload(ctx, synth.nif_init(3))
                npt.npt_nif_train(ctx, npt.train_params(batch=65536, samples=args.train_samples, seed=1,
                                                        grad_prec=npt.FP16))
                npt.npt_nif_set_precision(ctx, npt.FP16)
                npt.npt_set_env_mode(ctx, npt.ENV_NIF)
            out = torch.empty(H, W, 3, dtype=torch.float32, device="cuda")
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            rows = {}
            for spp in SWEEP_SPP:
                reps = max(2, min(20, 4096 // spp))
                npt.npt_render(ctx, W, H, spp, depth, 1, out)
                torch.cuda.synchronize()
                e0.record()
                for _ in range(reps):
                    npt.npt_render(ctx, W, H, spp, depth, 1, out)
                e1.record()
                torch.cuda.synchronize()
                ms = e0.elapsed_time(e1) / reps
                st = npt.npt_get_stats(ctx)
                rows[str(spp)] = {"ms_per_render": ms, "path_samples_per_s": W * H * spp / (ms * 1e-3),
                                  "passes": st["passes"]}
            res[name] = rows
        finally:
            npt.npt_destroy(ctx)
    print(json.dumps({"spp_sweep": res, "size": [W, H], "unit": "path samples/s", "data": "synthetic"}))


def _psnr_log(nif_rgb, ref_rgb):
    """PSNRs in the log1p domain: RGB over all channels, luminance (BT.601 Y)
    and chrominance (BT.601 U, V) of the log1p values; the peak is the
    reference's largest log1p value."""
    a, b = np.log1p(np.maximum(nif_rgb, 0.0)), np.log1p(ref_rgb)
    peak = float(b.max())

    def yuv(x):
        y = 0.299 * x[:, 0] + 0.587 * x[:, 1] + 0.114 * x[:, 2]
        return y, np.stack([0.492 * (x[:, 2] - y), 0.877 * (x[:, 0] - y)], 1)

    def psnr(x, z):
        return float(10 * np.log10(peak * peak / np.mean((x - z) ** 2)))

    ya, ca = yuv(a)
    yb, cb = yuv(b)
    return {"psnr_rgb": psnr(a, b), "psnr_luminance": psnr(ya, yb), "psnr_chrominance": psnr(ca, cb)}


def _hue_deg(a, b):
    """Angle in degrees between two RGB vectors (0: the same hue and saturation)."""
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    c = float(np.dot(a, b) / max(np.linalg.norm(a) * np.linalg.norm(b), 1e-30))
    return float(np.degrees(np.arccos(np.clip(c, -1.0, 1.0))))


def _luma(x):
    return float(0.299 * x[0] + 0.587 * x[1] + 0.114 * x[2])


# networks of the colour-space study: the workload's and the paper's own
STUDY_NETS = {"16/96/5": dict(n_freq=16, hidden=96, layers=5, skip=0),
              "10/128/4 skip 2": dict(n_freq=10, hidden=128, layers=4, skip=2)}


def nif_study(args):
    """The output colour-space comparison of Sec. 4.3 on the synthetic sun-lit
    sky (the workload's 0.5-degree sun disk and larger ones, same radiance),
    over a training budget: the network (the workload's 16/96/5 and the
    paper's 10/128/4 with the features again at layer 2) is trained on the
    device (Huber, Adam, batch 65,536, FP16 GEMM operands) with its three
    outputs in YUV, RGB or YCoCg, and evaluated after 2^a, 2^b, ... samples
    of one continuing run.  Reported per point: log-domain PSNRs and MSE of
    the NIF (FP32 inference) against the map at every texel centre; its
    radiance at the sun's centre, the ratio of its luminance to the sun's and
    the angle between the two RGB vectors (the hue error); and for an open-box
    render lit by the NIF (FP16 inference) the relative RMSE against the
    env-map render at equal seeds and the angle between the two images' mean
    colours (the hue of the light).  Then the master-weight precision of
    Sec. 3.2.1: FP32 master weights against binary16 master weights with
    stochastically rounded updates and loss scale 16384."""
    import torch

    from paper_2305_20061_amd import npt, synth

    torch.cuda.set_device(0)
    budgets = sorted(int(x) for x in args.study_budgets.split(","))
    out = {}
    for radius in sorted(float(x) for x in args.study_sun_radii.split(",")):
        out[f"sun_radius_{radius:g}deg"] = _colour_study(args, budgets, synth.env_map(sun_radius_deg=radius),
                                                         f"sun {radius:g} deg", master=radius == synth.SUN_RADIUS_DEG)
    print(json.dumps({"nif_study": {"colour_space": out, "budgets_log2_samples": budgets, "batch": 65536,
                                    "master_train_samples": args.train_samples,
                                    "render": "open box 512x512, 16 spp, depth 6, seed 1",
                                    "grid": "2048x1024 texel centres"}, "data": "synthetic"}))


def _colour_study(args, budgets, env, tag, master):
    import torch

    from paper_2305_20061_amd import npt, synth

    h, w = env.shape[:2]
    ph = 2 * np.pi * (np.arange(w) + 0.5) / w - np.pi
    th = np.pi * (np.arange(h) + 0.5) / h
    dirs = np.stack([np.sin(th)[:, None] * np.cos(ph)[None, :], np.cos(th)[:, None] * np.ones(w)[None, :],
                     np.sin(th)[:, None] * np.sin(ph)[None, :]], -1).reshape(-1, 3).astype(np.float32)
    ref = env.reshape(-1, 3).astype(np.float64)
    log_ref = np.log1p(ref)
    sun_true = [float(x) for x in ref.max(0)]
    d_dirs = torch.from_numpy(dirs).cuda()
    q = torch.empty(dirs.shape[0], 3, dtype=torch.float32, device="cuda")
    sun = torch.tensor(np.asarray(synth.sun_direction(), np.float32)[None, :]).cuda()
    qs = torch.empty(1, 3, dtype=torch.float32, device="cuda")
    RW, RS, RD = 512, 16, 6
    img = torch.empty(RW, RW, 3, dtype=torch.float32, device="cuda")
    ctx = npt.npt_create(0)
    res = {}
    try:
        npt.npt_load_scene(ctx, synth.scene_for(1))
        npt.npt_env_upload(ctx, env)
        npt.npt_set_env_mode(ctx, npt.ENV_MAP)
        npt.npt_render(ctx, RW, RW, RS, RD, 1, img)
        torch.cuda.synchronize()
        img_map = img.cpu().numpy().astype(np.float64)
        mean_map = img_map.reshape(-1, 3).mean(0)
        for net, shape in STUDY_NETS.items():
            for name, colour in (("yuv", npt.COLOUR_YUV), ("rgb", npt.COLOUR_RGB), ("ycocg", npt.COLOUR_YCOCG)):
                npt.npt_nif_upload(ctx, synth.nif_init(3, **shape), colour=colour, **shape)
                done, train_ms = 0, 0.0
                for lb in budgets:
                    tr = npt.npt_nif_train(ctx, npt.train_params(batch=65536, samples=(1 << lb) - done, seed=1,
                                                                 grad_prec=npt.FP16))
                    done, train_ms = 1 << lb, train_ms + tr["ms"]
                    npt.npt_nif_set_precision(ctx, npt.FP32)
                    npt.npt_env_query(ctx, npt.ENV_NIF, d_dirs, q)
                    npt.npt_env_query(ctx, npt.ENV_NIF, sun, qs)
                    torch.cuda.synchronize()
                    pred = q.cpu().numpy().astype(np.float64)
                    sun_rgb = [float(x) for x in qs.cpu().numpy()[0]]
                    row = {"train_ms": train_ms, "steps": tr["step_total"], "last_loss": tr["last_loss"],
                           **_psnr_log(pred, ref),
                           "log_mse": float(np.mean((np.log1p(np.maximum(pred, 0.0)) - log_ref) ** 2)),
                           "sun_centre_rgb": sun_rgb, "sun_true_rgb": sun_true,
                           "sun_luminance_ratio": _luma(sun_rgb) / _luma(sun_true),
                           "sun_hue_error_deg": _hue_deg(sun_rgb, sun_true)}
                    npt.npt_nif_set_precision(ctx, npt.FP16)
                    npt.npt_set_env_mode(ctx, npt.ENV_NIF)
                    npt.npt_render(ctx, RW, RW, RS, RD, 1, img)
                    torch.cuda.synchronize()
                    im = img.cpu().numpy().astype(np.float64)
                    npt.npt_set_env_mode(ctx, npt.ENV_MAP)
                    row["image_rel_rmse_vs_env_map"] = _rel(im, img_map)
                    row["image_mean_ratio_vs_env_map"] = _luma(im.reshape(-1, 3).mean(0)) / _luma(mean_map)
                    row["image_hue_error_deg"] = _hue_deg(im.reshape(-1, 3).mean(0), mean_map)
                    res.setdefault(net, {}).setdefault(name, {})[f"2^{lb}"] = row
                    _stage(f"colour study {tag} {net} {name} 2^{lb}: sun {row['sun_luminance_ratio']:.3g} of true, "
                           f"hue {row['sun_hue_error_deg']:.1f} deg, image relRMSE "
                           f"{row['image_rel_rmse_vs_env_map']:.3f}")
        # master-weight precision (YUV, FP16 GEMMs): FP32 master against the
        # paper's binary16 master with stochastic rounding and loss scale 16384
        npt.npt_set_env_mode(ctx, npt.ENV_MAP)
        masters = (("fp32_master_ls16384", npt.FP32, 16384.0), ("fp16_master_sr_ls16384", npt.FP16, 16384.0))
        for name, mp, ls in masters if master else ():
            npt.npt_nif_upload(ctx, synth.nif_init(3))
            tr = npt.npt_nif_train(ctx, npt.train_params(batch=65536, samples=args.train_samples, seed=1,
                                                         grad_prec=npt.FP16, loss_scale=ls, master_prec=mp))
            npt.npt_nif_set_precision(ctx, npt.FP32)
            npt.npt_env_query(ctx, npt.ENV_NIF, d_dirs, q)
            torch.cuda.synchronize()
            res.setdefault("master_weights", {})[name] = {
                "train_ms": tr["ms"], "last_loss": tr["last_loss"], "grid": npt.npt_nif_eval_grid(ctx, 1024, 512),
                **_psnr_log(q.cpu().numpy().astype(np.float64), ref)}
    finally:
        npt.npt_destroy(ctx)
    return res


# (hidden, layers, skip-concat layer, frequencies): the paper's sweep sizes,
# the workload's network, and the paper's own architecture (40-d features,
# H128, four dense-ReLU layers, the features again after the narrowed second
# one) with and without its 40-d features
NIF_SIZES = [(64, 2, 0, 16), (96, 5, 0, 16), (128, 4, 2, 16), (128, 4, 2, 10), (256, 4, 0, 16), (1024, 8, 0, 16)]
# shapes with an LDS-resident inference kernel (hidden, layers, skip, frequencies)
RESIDENT = [(96, 5, 0, 16), (128, 4, 2, 10), (128, 4, 2, 16), (64, 2, 0, 16)]


def nif_sizes(args):
    """Model size against path rate and PSNR (Sec. 4.6): the spheres scene
    (1024x1024, 16 spp, depth 8) lit by NIFs of several sizes, each trained
    on the device (2^24 samples, batch 65,536, FP16 GEMMs) and run with FP16
    operands on the layer-serial GEMM path.  Reported per size: parameters, FLOP per query,
    training time, log-domain PSNRs against the map (FP32 inference), path
    samples/s, NIF time and TFLOP/s per render, and the image relRMSE
    against the env-map render at equal seeds; shapes with an LDS-resident
    kernel are rendered again on it, in FP16 and FP8."""
    import torch

    from paper_2305_20061_amd import npt, synth

    torch.cuda.set_device(0)
    env = synth.env_map()
    h, w = env.shape[:2]
    ph = 2 * np.pi * (np.arange(w) + 0.5) / w - np.pi
    th = np.pi * (np.arange(h) + 0.5) / h
    dirs = np.stack([np.sin(th)[:, None] * np.cos(ph)[None, :], np.cos(th)[:, None] * np.ones(w)[None, :],
                     np.sin(th)[:, None] * np.sin(ph)[None, :]], -1).reshape(-1, 3).astype(np.float32)
    ref = env.reshape(-1, 3).astype(np.float64)
    d_dirs = torch.from_numpy(dirs).cuda()
    q = torch.empty(dirs.shape[0], 3, dtype=torch.float32, device="cuda")
    W = H = 1024
    spp, depth = 16, 8
    out = torch.empty(H, W, 3, dtype=torch.float32, device="cuda")
    ctx = npt.npt_create(0)
    rows = []
    try:
        npt.npt_load_scene(ctx, synth.scene_for(2), max_leaf=2, lds_levels=0, width=4)
        npt.npt_env_upload(ctx, env)
        npt.npt_set_env_mode(ctx, npt.ENV_MAP)
        npt.npt_render(ctx, W, H, spp, depth, 1, out)
        torch.cuda.synchronize()
        img_map = out.cpu().numpy().astype(np.float64)
        for hidden, layers, skip, nf in NIF_SIZES:
            npt.npt_nif_set_precision(ctx, npt.FP16)
            npt.npt_nif_upload(ctx, synth.nif_init(3, nf, hidden, layers, skip), n_freq=nf, hidden=hidden,
                               layers=layers, layered=1, skip=skip)
            tr = npt.npt_nif_train(ctx, npt.train_params(batch=65536, samples=args.train_samples, seed=1,
                                                         grad_prec=npt.FP16))
            npt.npt_nif_set_precision(ctx, npt.FP32)
            npt.npt_env_query(ctx, npt.ENV_NIF, d_dirs, q)
            torch.cuda.synchronize()
            psnr = _psnr_log(q.cpu().numpy().astype(np.float64), ref)
            n_params = npt.nif_param_count(hidden, layers, skip, nf)
            trained = npt.npt_nif_download(ctx, n_params)
            F = 4 * nf
            # MACs: first layer, hidden layers (the one before a skip-concat
            # is hidden - F wide), output layer
            flop = 2 * (F * hidden + (layers - 1) * hidden * hidden + 3 * hidden - (F * hidden if skip else 0))
            # the layer-serial path; then, for shapes with an LDS-resident
            # kernel, the same trained weights on it in FP16 and FP8
            runs = [(1, npt.FP16)] + ([(0, npt.FP16), (0, npt.FP8)] if (hidden, layers, skip, nf) in RESIDENT else [])
            for layered, prec in runs:
                npt.npt_nif_set_precision(ctx, npt.FP16)
                npt.npt_nif_upload(ctx, trained, n_freq=nf, hidden=hidden, layers=layers, layered=layered,
                                   skip=skip)
                npt.npt_nif_set_precision(ctx, prec)
                npt.npt_set_env_mode(ctx, npt.ENV_NIF)
                npt.npt_set_render_options(ctx, rr_start=3, kernel_timing=1, sort_rays=args.sort_rays,
                                           pool_paths=args.pool_paths)
                el, st = _timed_renders(npt, torch, ctx, W, H, spp, depth, 1, out, 2, 1)
                npt.npt_set_render_options(ctx, rr_start=3, sort_rays=args.sort_rays, pool_paths=args.pool_paths)
                rows.append({"hidden": hidden, "layers": layers, "skip": skip, "features": F,
                             "path": "layered GEMMs" if layered else "LDS-resident",
                             "prec": {npt.FP16: "fp16", npt.FP8: "fp8"}[prec],
                             "params": n_params, "flop_per_query": flop,
                             "train_ms": tr["ms"], "last_loss": tr["last_loss"], **psnr,
                             "path_samples_per_s": W * H * spp * 2 / el, "nif_ms_per_render": st["ms_env"],
                             "nif_tflops": st["env_queries"] * flop / (st["ms_env"] * 1e-3) / 1e12,
                             "image_rel_rmse_vs_env_map": _rel(out.cpu().numpy().astype(np.float64), img_map)})
                npt.npt_set_env_mode(ctx, npt.ENV_MAP)
                print(json.dumps(rows[-1]), flush=True)
    finally:
        npt.npt_destroy(ctx)
    print(json.dumps({"nif_sizes": rows, "render": f"spheres {W}x{H}, {spp} spp, depth {depth}, seed 1, FP16 NIF",
                      "train_samples": args.train_samples, "data": "synthetic"}))


def main():
    args = _parse()
    if args.gpus != 1:
        print(json.dumps({"error": "one GPU only: this build measures a single MI355X; "
                                   "the multi-GPU sharding is described in DESIGN.md"}))
        sys.exit(2)
    if args.spp_sweep:
        return spp_sweep(args)
    if args.nif_study:
        return nif_study(args)
    if args.nif_sizes:
        return nif_sizes(args)
    import torch

    from paper_2305_20061_amd import npt, synth

    torch.cuda.set_device(0)
    wl = WORKLOADS[args.config]
    W, H, spp, depth, seed = args.width, args.height, wl["spp"], wl["depth"], 1
    prec_name = wl["prec"]
    prec = {"fp8": npt.FP8, "fp16": npt.FP16}[prec_name]
    env = synth.env_map()
    extra = {}
    t0 = time.perf_counter()
    scene = synth.scene_for(args.config)
    extra["scene_gen_ms"] = 1e3 * (time.perf_counter() - t0)
    ctx = npt.npt_create(0)
    try:
        t0 = time.perf_counter()
        # 4-wide BVH, leaf size 2, no LDS-staged levels: fastest in the sweep
        fmt_code = {"fp32": npt.NODES_FP32, "fp16-extent": npt.NODES_FP16_EXTENT, "q8": npt.NODES_Q8,
                    "fp16-corner": npt.NODES_FP16_CORNER}[args.node_format]
        npt.npt_load_scene(ctx, scene, max_leaf=args.max_leaf, lds_levels=args.lds_levels, width=4,
                           node_format=fmt_code)
        extra["bvh_build_ms"] = 1e3 * (time.perf_counter() - t0)
        _stage(f"scene and BVH ready ({extra['bvh_build_ms']:.0f} ms build)")
        extra["bvh"] = {**npt.npt_bvh_info(ctx), "node_format": args.node_format, "lds_levels": args.lds_levels,
                        "max_leaf": args.max_leaf, "sort_rays": args.sort_rays,
                        "node_bytes": {"fp32": B_NODE[4], "fp16-extent": 96, "q8": 64,
                                       "fp16-corner": 80}[args.node_format]}
        del scene
        npt.npt_env_upload(ctx, env)
        npt.npt_nif_upload(ctx, synth.nif_init(3))
        tr = npt.npt_nif_train(ctx, npt.train_params(batch=65536, samples=args.train_samples, seed=1,
                                                     grad_prec=npt.FP16))
        npt.npt_nif_set_precision(ctx, prec)
        _stage(f"NIF trained: {tr['steps']} steps in {tr['ms']:.1f} ms")
        # training FLOP: forward, backward-data and weight-gradient products,
        # 3 x the forward's 86,592 per sample
        train_tflops = 3 * NIF_FLOP_PER_QUERY * tr["steps"] * 65536 / (tr["ms"] * 1e-3) / 1e12
        extra["train"] = {"ms": tr["ms"], "steps": tr["steps"], "ms_per_step": tr["ms"] / max(1, tr["steps"]),
                          "tflops": train_tflops, "mfma_frac": train_tflops / MFMA_PEAK_TFLOPS["fp16"],
                          "first_loss": tr["first_loss"], "last_loss": tr["last_loss"],
                          "grid_eval": npt.npt_nif_eval_grid(ctx, 1024, 512)}
        trained = npt.npt_nif_download(ctx)
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
        npt.npt_set_render_options(ctx, rr_start=3, count_visits=1, sort_rays=args.sort_rays,
                                   pool_paths=args.pool_paths)
        npt.npt_render(ctx, W, H, spp, depth, seed, out)
        cs = npt.npt_get_stats(ctx)
        rays = np.array(cs["rays"], np.float64)
        esc = np.array(cs["escaped"], np.float64)
        visits = np.array(cs["node_visits"], np.float64)
        tests = np.array(cs["prim_tests"], np.float64)
        alg_bytes = float(np.sum((B_RAY + B_HITREC) * rays + extra["bvh"]["node_bytes"] * visits
                                 + B_PRIM * tests))
        survivors = np.concatenate([rays[1:], [0.0]])
        shade_bytes = float(np.sum(B_SHADE_RAY * rays + B_SHADE_HIT * (rays - esc) + B_SHADE_ESC * esc
                                   + B_SHADE_OUT * survivors))
        extra["per_ray"] = {"node_visits": float(visits.sum() / rays.sum()),
                            "prim_tests": float(tests.sum() / rays.sum()),
                            "rays_per_path": float(rays.sum() / cs["paths"]),
                            "escaped_per_path": float(esc.sum() / cs["paths"])}

        # the timed workload, with per-kernel events
        _stage("counting render done; timed renders")
        npt.npt_set_render_options(ctx, rr_start=3, kernel_timing=1, sort_rays=args.sort_rays,
                                   pool_paths=args.pool_paths)
        elapsed, st = _timed_renders(npt, torch, ctx, W, H, spp, depth, seed, out, args.steps, args.warmup)
        _stage(f"timed renders done: {1e3 * elapsed / args.steps:.2f} ms per frame")
        img = {prec_name: out.cpu().numpy().astype(np.float64)}
        ms_step = 1e3 * elapsed / args.steps
        value = W * H * spp * args.steps / elapsed

        trace_launch_ms = st["ms_trace"] / max(1, st["trace_launches"])
        achieved = alg_bytes / st["trace_launches"] / (trace_launch_ms * 1e-3) / 1e9
        traffic = _traffic_per_launch(wl["traffic"])

        def nif_stats(s, name):
            tf = s["env_queries"] * NIF_FLOP_PER_QUERY / (s["ms_env"] * 1e-3) / 1e12
            # each depth's real batch (the escaped rays of that depth, over the passes)
            per_depth = []
            for k, (q, ms) in enumerate(zip(s["escaped"], s["ms_env_depth"])):
                if q > 0 and ms > 0:
                    tfk = q * NIF_FLOP_PER_QUERY / (ms * 1e-3) / 1e12
                    per_depth.append({"depth": k + 1, "queries": q, "ms": ms, "queries_per_s": q / (ms * 1e-3),
                                      "mfma_util": tfk / MFMA_PEAK_TFLOPS[name]})
            r = {"precision": name, "queries_per_render": s["env_queries"],
                 "queries_per_s": s["env_queries"] / (s["ms_env"] * 1e-3), "ms_per_render": s["ms_env"],
                 "launches": s["env_launches"], "tflops": tf, "mfma_util": tf / MFMA_PEAK_TFLOPS[name],
                 "flop_per_query": NIF_FLOP_PER_QUERY, "per_depth": per_depth}
            if name == "fp8":  # against the peak of its FP16 / E4M3 mix
                r["mfma_util_mixed_peak"] = tf / MFMA_PEAK_TFLOPS_FP8_MIX
                r["mixed_peak_tflops"] = MFMA_PEAK_TFLOPS_FP8_MIX
            return r

        extra["kernels"] = {"extend_ms_per_render": st["ms_trace"], "extend_launches": st["trace_launches"],
                            "extend_ms_per_launch": trace_launch_ms, "shade_ms_per_render": st["ms_shade"],
                            "nif_ms_per_render": st["ms_env"], "render_ms_device": st["ms_total"]}
        extra["nif"] = nif_stats(st, prec_name)
        # roofline fraction of every kernel of the step, and their time-weighted sum
        fr = {"extend": (st["ms_trace"], alg_bytes / (st["ms_trace"] * 1e-3) / 1e9 / HBM_PEAK_GBS),
              "shade": (st["ms_shade"], shade_bytes / (st["ms_shade"] * 1e-3) / 1e9 / HBM_PEAK_GBS),
              "nif": (st["ms_env"], extra["nif"]["mfma_util"])}
        tot = sum(v[0] for v in fr.values())
        extra["kernel_roofline_fractions"] = {
            **{k: {"ms_per_render": v[0], "frac": v[1], "peak": "MFMA " + prec_name if k == "nif" else "HBM"}
               for k, v in fr.items()},
            "time_weighted": sum(v[0] * v[1] for v in fr.values()) / tot}
        extra["nif"]["fixed_batch_2^21_queries_per_s"] = _query_rate(npt, torch, ctx, npt.ENV_NIF)

        if not args.no_envmap:
            _stage("comparison renders (FP16 NIF, env map) and the equal-RMSE study")
            modes = {}
            frame_s = {prec_name: ms_step * 1e-3}
            if prec_name != "fp16":
                npt.npt_nif_set_precision(ctx, npt.FP16)
                el, s16 = _timed_renders(npt, torch, ctx, W, H, spp, depth, seed, out, args.steps, 1)
                frame_s["fp16"] = el / args.steps
                img["fp16"] = out.cpu().numpy().astype(np.float64)
                modes["nif_fp16"] = {"path_samples_per_s": W * H * spp * args.steps / el,
                                     **nif_stats(s16, "fp16"),
                                     "fixed_batch_2^21_queries_per_s": _query_rate(npt, torch, ctx, npt.ENV_NIF)}
                npt.npt_nif_set_precision(ctx, prec)
            npt.npt_set_env_mode(ctx, npt.ENV_MAP)
            el, se = _timed_renders(npt, torch, ctx, W, H, spp, depth, seed, out, args.steps, 1)
            img["map"] = out.cpu().numpy().astype(np.float64)
            modes["env_map"] = {"path_samples_per_s": W * H * spp * args.steps / el,
                                "lookup_queries_per_s": se["env_queries"] / (se["ms_env"] * 1e-3),
                                "lookup_hbm_frac": se["env_queries"] * B_LOOKUP / (se["ms_env"] * 1e-3) / 1e9
                                / HBM_PEAK_GBS,
                                "lookup_ms_per_render": se["ms_env"],
                                "fixed_batch_2^21_queries_per_s": _query_rate(npt, torch, ctx, npt.ENV_MAP)}
            # image error of each NIF precision against the map render at equal seeds
            modes["image_rel_rmse_vs_env_map"] = {k: _rel(v, img["map"]) for k, v in img.items() if k != "map"}
            if "fp16" in img and prec_name != "fp16":
                modes["image_rel_rmse_fp8_vs_fp16"] = _rel(img[prec_name], img["fp16"])
            paths = W * H * spp
            sample_s = {k: v / paths for k, v in frame_s.items()}
            sample_s["map"] = el / args.steps / paths
            precs = {prec_name: prec}
            if prec_name != "fp16":
                precs["fp16"] = npt.FP16
            npt.npt_set_env_mode(ctx, npt.ENV_NIF)
            modes["equal_rmse"] = _equal_rmse(npt, torch, ctx, W, H, spp, depth, seed, precs, sample_s)
            npt.npt_nif_set_precision(ctx, prec)
            extra["compare"] = modes
            npt.npt_set_env_mode(ctx, npt.ENV_NIF)
    finally:
        npt.npt_destroy(ctx)

    if args.config == 4 and not args.no_small:
        _stage("small-BVH rate")
        # the small-BVH scene with the same trained network in FP16
        c3 = WORKLOADS[3]
        ctx = npt.npt_create(0)
        try:
            npt.npt_load_scene(ctx, synth.scene_for(3), max_leaf=2, lds_levels=0, width=4,
                               node_format=fmt_code)
            npt.npt_nif_upload(ctx, trained)
            npt.npt_nif_set_precision(ctx, npt.FP16)
            npt.npt_set_env_mode(ctx, npt.ENV_NIF)
            npt.npt_set_render_options(ctx, rr_start=3, kernel_timing=1, sort_rays=args.sort_rays,
                                       pool_paths=args.pool_paths)
            el, s3 = _timed_renders(npt, torch, ctx, W, H, c3["spp"], c3["depth"], seed, out, args.steps, 1)
            extra["small_bvh_fp16"] = {"path_samples_per_s": W * H * c3["spp"] * args.steps / el,
                                       "ms_per_render": 1e3 * el / args.steps, "extend_ms_per_render": s3["ms_trace"],
                                       "shade_ms_per_render": s3["ms_shade"], "nif_ms_per_render": s3["ms_env"],
                                       "spp": c3["spp"], "max_depth": c3["depth"]}
        finally:
            npt.npt_destroy(ctx)

    counters = _counters(wl["counters"])
    line = {
        "metric": METRIC, "value": value, "unit": "path samples/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": f"f32 rays / {prec_name} NIF", "data": "synthetic",
        "config": {"workload": wl["desc"].format(W=W, H=H, spp=spp, depth=depth, seed=seed),
                   "paths_per_step": W * H * spp},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic, "kernel": "k_extend (BVH traversal + primitive tests)",
                     "alg_bytes_per_launch": alg_bytes / st["trace_launches"],
                     "achieved_is": "algorithmic bytes (ray, hit record, nodes fetched, primitive slots tested) "
                                    "per launch / launch time: what a traversal without caches would move",
                     "traffic_source": f"profiles/{wl['traffic']}: rocprofv3 FETCH_SIZE + WRITE_SIZE of this kernel "
                                       "source, copy-calibrated; not measured in this run",
                     "hbm_frac_measured": (traffic / (trace_launch_ms * 1e-3) / 1e9 / HBM_PEAK_GBS
                                           if traffic else None),
                     "limiter": _extend_limiter(counters)},
        "counters": counters,
    }
    line.update(extra)
    if not args.no_cpu_baseline:
        _stage("CPU oracle baseline")
        line["cpu_baseline"] = cpu_baseline(args.config, W, H, spp, depth, seed, prec, args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
