"""npt_render_noalloc (the render on the library's fixed device scratch)
against npt_render through the C ABI: the same image bit for bit, on two
calls in a row (the second smaller, so leftovers of the first in the shared
array would show), with the NIF and with the environment map; and the
errors it gives for an image that does not fit and for a layer-serial NIF."""
import numpy as np
import pytest

from paper_2305_20061_amd import npt, synth

from gpu_util import make_ctx, torch_cuda

pytestmark = pytest.mark.gpu


def _both(ctx, W, H, spp, depth, seed):
    torch = torch_cuda()
    a = torch.full((H, W, 3), -1.0, dtype=torch.float32, device="cuda")
    b = torch.full((H, W, 3), -2.0, dtype=torch.float32, device="cuda")
    npt.npt_render(ctx, W, H, spp, depth, seed, a)
    torch.cuda.synchronize()
    npt.npt_render_noalloc(ctx, W, H, spp, depth, seed, b)
    torch.cuda.synchronize()
    st = npt.npt_get_stats(ctx)
    return a.cpu().numpy(), b.cpu().numpy(), st


@pytest.mark.parametrize("mode", ["nif", "map"])
def test_noalloc_render_equals_render_on_two_calls(mode, small_sky):
    scene = synth.scene_for(1)
    ctx = make_ctx(scene, env=small_sky)
    try:
        if mode == "nif":
            npt.npt_nif_upload(ctx, synth.nif_init(3))
            npt.npt_nif_set_precision(ctx, npt.FP16)
            npt.npt_set_env_mode(ctx, npt.ENV_NIF)
        else:
            npt.npt_set_env_mode(ctx, npt.ENV_MAP)
        npt.npt_set_render_options(ctx, rr_start=3)
        for W, H, spp, depth, seed in ((320, 240, 8, 6, 3), (160, 96, 3, 5, 11)):
            print(f"noalloc {mode}: {W}x{H} {spp} spp depth {depth} seed {seed}", flush=True)
            a, b, st = _both(ctx, W, H, spp, depth, seed)
            print(f"  {st['passes']} passes of {st['samples_per_pass']} samples; mean {a.mean():.5f}")
            assert st["paths"] == W * H * spp
            assert np.isfinite(a).all() and a.mean() > 0.0
            assert np.array_equal(a, b)
    finally:
        npt.npt_destroy(ctx)


def test_noalloc_render_rejects_what_it_cannot_do(small_sky):
    torch = torch_cuda()
    ctx = make_ctx(synth.scene_for(1), env=small_sky)
    try:
        # 1024 x 1024 pixels need about 176 MiB at one sample per pass
        out = torch.empty(1024, 1024, 3, dtype=torch.float32, device="cuda")
        with pytest.raises(npt.NptError) as e:
            npt.npt_render_noalloc(ctx, 1024, 1024, 1, 4, 1, out)
        assert e.value.code == npt.NPT_E["INVALID_ARG"]
        # the layer-serial NIF allocates its activations
        npt.npt_nif_upload(ctx, synth.nif_init(3), layered=1)
        npt.npt_set_env_mode(ctx, npt.ENV_NIF)
        small = torch.empty(32, 32, 3, dtype=torch.float32, device="cuda")
        with pytest.raises(npt.NptError) as e:
            npt.npt_render_noalloc(ctx, 32, 32, 1, 4, 1, small)
        assert e.value.code == npt.NPT_E["UNSUPPORTED"]
        # the context still renders
        npt.npt_set_env_mode(ctx, npt.ENV_MAP)
        npt.npt_render_noalloc(ctx, 32, 32, 2, 4, 1, small)
        torch.cuda.synchronize()
        assert np.isfinite(small.cpu().numpy()).all()
    finally:
        npt.npt_destroy(ctx)
