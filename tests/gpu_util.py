"""Helpers shared by the GPU tests: build a context from a synth scene, run
the GPU path through the C ABI, and run the oracle on the same inputs."""
import numpy as np

import oracle as O
from paper_2305_20061_amd import npt


def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU test without a GPU"
    return torch


def make_ctx(scene, env=None, lds_levels=6, max_leaf=4, node_format=0):
    ctx = npt.npt_create(0)
    npt.npt_load_scene(ctx, scene, lds_levels=lds_levels, max_leaf=max_leaf, node_format=node_format)
    if env is not None:
        npt.npt_env_upload(ctx, env)
    else:
        npt.npt_set_env_mode(ctx, npt.ENV_NONE)
    return ctx


def gpu_render(ctx, W, H, spp, depth, seed):
    torch = torch_cuda()
    out = torch.empty(H, W, 3, dtype=torch.float32, device="cuda")
    npt.npt_render(ctx, W, H, spp, depth, seed, out)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.float64)


def gpu_primary(ctx, W, H, sample, seed):
    torch = torch_cuda()
    prim = torch.empty(W * H, dtype=torch.int32, device="cuda")
    inst = torch.empty(W * H, dtype=torch.int32, device="cuda")
    t = torch.empty(W * H, dtype=torch.float32, device="cuda")
    n = torch.empty(W * H, 3, dtype=torch.float32, device="cuda")
    npt.npt_trace_primary(ctx, W, H, sample, seed, prim=prim, inst=inst, t=t, normal=n)
    torch.cuda.synchronize()
    return (prim.cpu().numpy().view(np.uint32), inst.cpu().numpy().view(np.uint32), t.cpu().numpy(),
            n.cpu().numpy())


def oracle_scene(scene, accel=1):
    return O.Scene(scene, accel=accel), O.make_camera(**scene["camera"])


def rel_rmse(g, o):
    g = np.asarray(g, np.float64)
    o = np.asarray(o, np.float64)
    return float(np.sqrt(np.sum((g - o) ** 2)) / np.sqrt(np.sum(o ** 2)))
