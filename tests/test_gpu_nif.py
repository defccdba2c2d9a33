"""HDR-NIF on the GPU vs the CPU oracle (Sec. 3.2, 3.3): MFMA inference in
FP32/FP16/BF16/FP8 against the oracle's forward pass with the same operand
rounding (weights rounded once, each layer input rounded to its operand
format, exact sums); NIF-lit renders; training gradients and an Adam step
(Sec. 3.2.1) against the oracle's FP64 backward pass."""
import numpy as np
import pytest

import oracle as O
from paper_2305_20061_amd import npt, synth

from gpu_util import gpu_render, make_ctx, oracle_scene, rel_rmse, torch_cuda

pytestmark = pytest.mark.gpu
SHAPE = O.nif_shape(16, 96, 5)
PRECS = [npt.FP32, npt.FP16, npt.BF16, npt.FP8]
# oracle precision codes are the library's
assert (O.PREC_FP32, O.PREC_FP16, O.PREC_BF16, O.PREC_FP8) == (npt.FP32, npt.FP16, npt.BF16, npt.FP8)

# relative-RMSE bounds of the radiance of one query batch against the oracle
# with the same operand rounding: what is left is FP32 accumulation order
# and the FP32 features, which move an operand across a rounding boundary now
# and then (one unit in its last place: 2^-11 FP16, 2^-8 BF16, 2^-4 E4M3).
# FP16 at 1e-3 is the image gate of the FP16-NIF configurations.
QUERY_TOL = {npt.FP32: 5e-5, npt.FP16: 1e-3, npt.BF16: 1e-2, npt.FP8: 2e-2}


def _weights(seed=3):
    p = synth.nif_init(seed).astype(np.float32)
    p[-3:] = (0.6, 0.05, -0.05)  # output bias: Y 0.6, small chroma -> positive radiance
    return p


def _dequant(p, prec):
    return O.nif_dequantize(SHAPE, np.asarray(p, np.float64), prec)


def _dirs(n, seed=0):
    rng = np.random.default_rng(seed)
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return d.astype(np.float32)


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("n", [1, 37, 4096 + 29])
def test_nif_query_matches_oracle(prec, n):
    torch = torch_cuda()
    p = _weights()
    ctx = npt.npt_create(0)
    try:
        npt.npt_nif_upload(ctx, p)
        npt.npt_nif_set_precision(ctx, prec)
        d = _dirs(n)
        dt = torch.from_numpy(d).cuda()
        out = torch.full((n, 3), -1.0, dtype=torch.float32, device="cuda")
        npt.npt_env_query(ctx, npt.ENV_NIF, dt, out)
        torch.cuda.synchronize()
        g = out.cpu().numpy().astype(np.float64)
        dq = npt.npt_nif_get_dequantized(ctx)
    finally:
        npt.npt_destroy(ctx)
    ref_p = _dequant(p, prec)
    assert np.array_equal(dq.astype(np.float64), ref_p)  # the library multiplies the same rounded weights
    o = np.array([O.nif_radiance_q(SHAPE, ref_p, prec, *O.dir_to_uv(x)) for x in d])
    r = rel_rmse(g, o)
    print(f"prec {prec} n {n}: relRMSE {r:.3e}")
    assert np.all(g >= 0)
    assert r <= QUERY_TOL[prec]


# One more ray than 256 workgroups take in one round of the inference
# kernel's tile loop, plus a ragged tail: 512 rays per workgroup and round in
# FP8 (16 waves, one tile each) and FP16 / BF16 (8 waves, two tiles each),
# 256 in FP32, so every precision wraps around the grid at least once.
N_WRAP = 256 * 512 + 29


@pytest.mark.parametrize("prec", PRECS)
def test_nif_query_wraps_the_grid(prec):
    torch = torch_cuda()
    p = _weights()
    ctx = npt.npt_create(0)
    try:
        npt.npt_nif_upload(ctx, p)
        npt.npt_nif_set_precision(ctx, prec)
        d = _dirs(N_WRAP, seed=5)
        dt = torch.from_numpy(d).cuda()
        out = torch.full((N_WRAP, 3), -1.0, dtype=torch.float32, device="cuda")
        npt.npt_env_query(ctx, npt.ENV_NIF, dt, out)
        torch.cuda.synchronize()
        g = out.cpu().numpy().astype(np.float64)
    finally:
        npt.npt_destroy(ctx)
    assert np.all(g >= 0)  # every query written (radiance is clamped at 0; the fill is -1)
    # sampled against the oracle: the first and last tiles, both sides of the
    # first wrap, and a seeded spread
    idx = np.unique(np.concatenate([np.arange(64), np.arange(N_WRAP - 96, N_WRAP),
                                    np.arange(256 * 512 - 32, N_WRAP),
                                    np.random.default_rng(9).integers(0, N_WRAP, 400)]))
    ref_p = _dequant(p, prec)
    o = np.array([O.nif_radiance_q(SHAPE, ref_p, prec, *O.dir_to_uv(d[i])) for i in idx])
    r = rel_rmse(g[idx], o)
    print(f"prec {prec} n {N_WRAP}: {idx.size} sampled, relRMSE {r:.3e}")
    assert r <= QUERY_TOL[prec]


def test_nif_render_matches_oracle_fp32(small_sky):
    scene = synth.scene_for(1)
    p = _weights()
    ctx = make_ctx(scene, env=small_sky)
    try:
        npt.npt_nif_upload(ctx, p)
        npt.npt_nif_set_precision(ctx, npt.FP32)
        npt.npt_set_env_mode(ctx, npt.ENV_NIF)
        g = gpu_render(ctx, 48, 48, 2, 6, 9)
    finally:
        npt.npt_destroy(ctx)
    osc, cam = oracle_scene(scene)
    o = O.render(osc, cam, O.render_desc(48, 48, 2, 6, 9, nif_params=p.astype(np.float64), nif=SHAPE))
    r = rel_rmse(g, o)
    print(f"NIF FP32 render relRMSE {r:.3e}")
    assert r <= 1e-3


@pytest.mark.parametrize("prec", [npt.FP16, npt.BF16, npt.FP8])
def test_nif_render_matches_oracle_low_precision(prec, small_sky):
    scene = synth.scene_for(1)
    p = _weights()
    ctx = make_ctx(scene, env=small_sky)
    try:
        npt.npt_nif_upload(ctx, p)
        npt.npt_nif_set_precision(ctx, prec)
        npt.npt_set_env_mode(ctx, npt.ENV_NIF)
        g = gpu_render(ctx, 48, 48, 2, 6, 9)
    finally:
        npt.npt_destroy(ctx)
    osc, cam = oracle_scene(scene)
    o = O.render(osc, cam, O.render_desc(48, 48, 2, 6, 9, nif_params=_dequant(p, prec), nif=SHAPE,
                                         nif_prec=prec))
    r = rel_rmse(g, o)
    print(f"NIF prec {prec} render relRMSE {r:.3e}")
    assert r <= QUERY_TOL[prec]


# Training gradients: against the oracle whose GEMM operands are rounded as
# the trainer's (same loss scale; FP32 summation order and FP32 features
# are what is left), and against the FP64 gradient without rounding; bounds
# are the measured errors with a margin of about 3x (measured at batch 2048:
# gradients 1.0e-6 / 1.8e-6 / 2.6e-5 against the rounded oracle, 1.0e-6 /
# 1.2e-3 / 4.1e-3 against FP64; losses 2e-7 / 3e-7 / 4e-7 against the
# rounded oracle, 2e-7 / 7.3e-5 / 1.1e-4 against FP64)
LOSS_SCALE = {npt.FP32: 1.0, npt.FP16: 16384.0, npt.BF16: 1.0}  # the trainer's defaults
GRAD_TOL_Q = {npt.FP32: 3e-6, npt.FP16: 6e-6, npt.BF16: 8e-5}
LOSS_TOL_Q = {npt.FP32: 1e-6, npt.FP16: 1e-6, npt.BF16: 2e-6}
GRAD_TOL = {npt.FP32: 3e-6, npt.FP16: 4e-3, npt.BF16: 1.2e-2}
LOSS_TOL = {npt.FP32: 1e-6, npt.FP16: 2.5e-4, npt.BF16: 4e-4}


# FP16 takes the fused step by default; the layer-by-layer one is covered too
@pytest.mark.parametrize("prec,path", [(npt.FP32, npt.TRAIN_AUTO), (npt.FP16, npt.TRAIN_AUTO),
                                       (npt.FP16, npt.TRAIN_LAYERED), (npt.BF16, npt.TRAIN_AUTO)])
def test_training_gradient_matches_oracle(prec, path, small_sky):
    torch = torch_cuda()
    p = synth.nif_init(11)
    B, seed, step = 2048, 5, 2
    ctx = npt.npt_create(0)
    try:
        npt.npt_env_upload(ctx, small_sky)
        npt.npt_nif_upload(ctx, p)
        grad = torch.zeros(43779, dtype=torch.float32, device="cuda")
        loss = torch.zeros(1, dtype=torch.float32, device="cuda")
        tp = npt.train_params(batch=B, seed=seed, grad_prec=prec, path=path)
        npt.npt_nif_train_grad(ctx, tp, step, grad, loss)
        torch.cuda.synchronize()
        g = grad.cpu().numpy().astype(np.float64)
        lg = float(loss.cpu()[0])
    finally:
        npt.npt_destroy(ctx)
    uv, tg = O.nif_train_batch(small_sky, seed, step, B)
    lo, go = O.nif_loss_grad(SHAPE, p.astype(np.float64), uv, tg, 1e-3)
    lq, gq = O.nif_loss_grad_q(SHAPE, p.astype(np.float64), prec, LOSS_SCALE[prec], uv, tg, 1e-3)
    r, rq = rel_rmse(g, go), rel_rmse(g, gq)
    print(f"grad prec {prec} path {path}: relRMSE {rq:.3e} (rounded oracle), {r:.3e} (FP64); loss {lg:.7e} vs {lq:.7e} "
          f"(rounded), {lo:.7e} (FP64)")
    assert abs(lg - lq) <= LOSS_TOL_Q[prec] * abs(lq)
    assert rq <= GRAD_TOL_Q[prec]
    assert abs(lg - lo) <= LOSS_TOL[prec] * abs(lo)
    assert r <= GRAD_TOL[prec]


def test_adam_step_matches_oracle(small_sky):
    p = synth.nif_init(13)
    B, seed = 2048, 21
    ctx = npt.npt_create(0)
    try:
        npt.npt_env_upload(ctx, small_sky)
        npt.npt_nif_upload(ctx, p)
        st = npt.npt_nif_train(ctx, npt.train_params(batch=B, samples=B, seed=seed, grad_prec=npt.FP32))
        q = npt.npt_nif_download(ctx).astype(np.float64)
    finally:
        npt.npt_destroy(ctx)
    ref = p.astype(np.float64).copy()
    m, v = np.zeros_like(ref), np.zeros_like(ref)
    lo = O.nif_train_step(SHAPE, ref, m, v, small_sky, seed, 0, B)
    assert st["steps"] == 1 and abs(st["first_loss"] - lo) <= 1e-4 * lo
    dg, do = q - p.astype(np.float32).astype(np.float64), ref - p
    # the first Adam step is -lr g / (|g| + eps): lr (1e-3) times the sign of
    # g wherever |g| >> eps = 1e-7, less where |g| is near eps.  Measured: the
    # largest difference 4.3e-5 lr over all weights (FP32 weight rounding and
    # the FP32 gradient's error), 9.8e-6 lr among the full-size steps
    lr = 1e-3
    full = np.abs(do) > 0.5 * lr
    err = np.abs(dg - do)
    print(f"Adam step: {full.mean():.4f} of steps full size; max error there {err[full].max() / lr:.2e} lr; "
          f"{np.count_nonzero(err > 1e-3 * lr)} weights beyond 1e-3 lr, max {err.max() / lr:.2e} lr")
    assert full.mean() > 0.8
    assert err[full].max() <= 3e-5 * lr
    assert err.max() <= 1.5e-4 * lr


def test_training_beats_untrained_network(sky_map):
    """The learned part earns its keep: training on the device cuts the
    log-radiance error of the NIF against the map it compresses by a wide
    margin (the untrained network is the method without learning)."""
    ctx = npt.npt_create(0)
    try:
        npt.npt_env_upload(ctx, sky_map)
        npt.npt_nif_upload(ctx, synth.nif_init(3))
        npt.npt_nif_set_precision(ctx, npt.FP16)
        before = npt.npt_nif_eval_grid(ctx, 512, 256)
        st = npt.npt_nif_train(ctx, npt.train_params(batch=65536, samples=1 << 22, seed=1, grad_prec=npt.FP16))
        after = npt.npt_nif_eval_grid(ctx, 512, 256)
    finally:
        npt.npt_destroy(ctx)
    print(f"log-MSE {before['log_mse']:.4e} -> {after['log_mse']:.4e}; loss {st['first_loss']:.3e} -> "
          f"{st['last_loss']:.3e} in {st['steps']} steps, {st['ms']:.1f} ms")
    assert st["last_loss"] < 0.2 * st["first_loss"]
    assert after["log_mse"] < 0.05 * before["log_mse"]


def test_fp8_weight_scales_follow_each_layer():
    # scaling one hidden layer by 2^k moves its E4M3 codes by exactly k in
    # the exponent: the dequantised weights scale by 2^k as well
    p = _weights()
    q = p.copy()
    lo = 64 * 96 + 96 + 96 * 96 + 96  # layer 2 (hidden-to-hidden)
    q[lo:lo + 96 * 96] *= 2.0 ** -7
    outs = []
    for w in (p, q):
        ctx = npt.npt_create(0)
        try:
            npt.npt_nif_upload(ctx, w)
            npt.npt_nif_set_precision(ctx, npt.FP8)
            outs.append(npt.npt_nif_get_dequantized(ctx).astype(np.float64))
        finally:
            npt.npt_destroy(ctx)
    a, b = outs
    assert np.array_equal(b[lo:lo + 96 * 96], a[lo:lo + 96 * 96] * 2.0 ** -7)
    assert np.array_equal(np.delete(a, np.s_[lo:lo + 96 * 96]), np.delete(b, np.s_[lo:lo + 96 * 96]))


COLOURS = [npt.COLOUR_RGB, npt.COLOUR_YCOCG]
assert (O.COLOUR_YUV, O.COLOUR_RGB, O.COLOUR_YCOCG) == (npt.COLOUR_YUV, npt.COLOUR_RGB, npt.COLOUR_YCOCG)


@pytest.mark.parametrize("colour", COLOURS)
@pytest.mark.parametrize("prec", [npt.FP32, npt.FP16, npt.FP8])
def test_nif_query_other_colour_spaces(colour, prec):
    # the output colour matrix (Sec. 4.3) is applied after the last layer:
    # same bounds as the default YUV space
    torch = torch_cuda()
    shape = O.nif_shape(16, 96, 5, colour)
    p = _weights()
    p[-3:] = (0.6, 0.4, 0.5) if colour == npt.COLOUR_RGB else (0.6, 0.05, -0.05)
    n = 4096 + 29
    ctx = npt.npt_create(0)
    try:
        npt.npt_nif_upload(ctx, p, colour=colour)
        npt.npt_nif_set_precision(ctx, prec)
        d = _dirs(n, seed=4)
        out = torch.full((n, 3), -1.0, dtype=torch.float32, device="cuda")
        npt.npt_env_query(ctx, npt.ENV_NIF, torch.from_numpy(d).cuda(), out)
        torch.cuda.synchronize()
        g = out.cpu().numpy().astype(np.float64)
    finally:
        npt.npt_destroy(ctx)
    ref_p = _dequant(p, prec)
    o = np.array([O.nif_radiance_q(shape, ref_p, prec, *O.dir_to_uv(x)) for x in d])
    r = rel_rmse(g, o)
    print(f"colour {colour} prec {prec}: relRMSE {r:.3e}")
    assert r <= QUERY_TOL[prec]


@pytest.mark.parametrize("colour", COLOURS)
def test_training_gradient_other_colour_spaces(colour, small_sky):
    # the head's gradient goes back through M^T of the chosen colour matrix
    torch = torch_cuda()
    shape = O.nif_shape(16, 96, 5, colour)
    p = synth.nif_init(11)
    B, seed, step = 2048, 5, 2
    ctx = npt.npt_create(0)
    try:
        npt.npt_env_upload(ctx, small_sky)
        npt.npt_nif_upload(ctx, p, colour=colour)
        grad = torch.zeros(43779, dtype=torch.float32, device="cuda")
        loss = torch.zeros(1, dtype=torch.float32, device="cuda")
        npt.npt_nif_train_grad(ctx, npt.train_params(batch=B, seed=seed, grad_prec=npt.FP32), step, grad, loss)
        torch.cuda.synchronize()
        g = grad.cpu().numpy().astype(np.float64)
        lg = float(loss.cpu()[0])
    finally:
        npt.npt_destroy(ctx)
    uv, tg = O.nif_train_batch(small_sky, seed, step, B)
    lo, go = O.nif_loss_grad(shape, p.astype(np.float64), uv, tg, 1e-3)
    r = rel_rmse(g, go)
    print(f"colour {colour} grad: relRMSE {r:.3e}, loss {lg:.6e} vs {lo:.6e}")
    assert abs(lg - lo) <= LOSS_TOL[npt.FP32] * abs(lo)
    assert r <= GRAD_TOL[npt.FP32]


# FP16 GEMM operands take the fused step; its oracle step takes the
# rounded-operand gradient (against the FP64 gradient, which differs by about
# 1e-3 relative, only 0.956 of the weights came out identical: the update of
# weights with |g| near Adam's eps moves).  Measured identical: 0.99995 (FP32
# gradients), 0.99977 (FP16, fused step)
FP16_MASTER_SAME = {npt.FP32: 0.999, npt.FP16: 0.999}


@pytest.mark.parametrize("grad_prec", [npt.FP32, npt.FP16])
def test_fp16_master_adam_step_matches_oracle(grad_prec, small_sky):
    # one Adam step with binary16 master weights and stochastically rounded
    # updates (Sec. 3.2.1): every weight stays a binary16 value and takes the
    # oracle's neighbour, except where the GPU's FP32 update and the oracle's
    # FP64 update (rounded to FP32) fall on different sides of the decision;
    # there the two differ by one binary16 step
    p = synth.nif_init(13)
    B, seed = 2048, 21
    ctx = npt.npt_create(0)
    try:
        npt.npt_env_upload(ctx, small_sky)
        npt.npt_nif_upload(ctx, p)
        st = npt.npt_nif_train(ctx, npt.train_params(batch=B, samples=B, seed=seed, grad_prec=grad_prec,
                                                     master_prec=npt.FP16))
        q = npt.npt_nif_download(ctx).astype(np.float64)
    finally:
        npt.npt_destroy(ctx)
    ref = p.astype(np.float64).copy()
    m, v = np.zeros_like(ref), np.zeros_like(ref)
    if grad_prec == npt.FP32:
        lo = O.nif_train_step(SHAPE, ref, m, v, small_sky, seed, 0, B, fp16_master=True)
    else:
        ref = ref.astype(np.float16).astype(np.float64)  # the master is rounded to binary16 first
        uv, tg = O.nif_train_batch(small_sky, seed, 0, B)
        lo, g = O.nif_loss_grad_q(SHAPE, ref, npt.FP16, LOSS_SCALE[npt.FP16], uv, tg, 1e-3)
        O.adam_step_fp16_master(ref, g, m, v, 1, seed)
    assert st["steps"] == 1 and abs(st["first_loss"] - lo) <= 1e-4 * lo
    assert np.array_equal(q.astype(np.float16).astype(np.float64), q)
    same = q == ref
    print(f"FP16 master, grad prec {grad_prec}: {same.mean():.6f} of weights identical, {np.count_nonzero(~same)} differ")
    assert same.mean() >= FP16_MASTER_SAME[grad_prec]
    qh, rh = q[~same].astype(np.float16), ref[~same].astype(np.float16)
    assert np.array_equal(np.nextafter(qh, rh), rh)
    # the update really moved the weights (not a rounding back to the start)
    assert np.mean(q != np.float16(p).astype(np.float64)) > 0.5


def test_per_depth_environment_times_add_up(small_sky):
    # kernel timing: the per-depth environment (NIF) times sum to the total;
    # every depth up to the maximum has its launch (one per pass), none beyond
    torch = torch_cuda()
    ctx = make_ctx(synth.scene_for(1), env=small_sky)
    try:
        npt.npt_nif_upload(ctx, _weights())
        npt.npt_nif_set_precision(ctx, npt.FP8)
        npt.npt_set_env_mode(ctx, npt.ENV_NIF)
        npt.npt_set_render_options(ctx, rr_start=3, kernel_timing=1, samples_per_pass=2)
        out = torch.empty(64, 64, 3, device="cuda")
        npt.npt_render(ctx, 64, 64, 4, 6, 3, out)
        torch.cuda.synchronize()
        st = npt.npt_get_stats(ctx)
    finally:
        npt.npt_destroy(ctx)
    per_depth = np.array(st["ms_env_depth"], np.float64)
    print(f"env ms {st['ms_env']:.4f} over {st['env_launches']} launches; per depth {per_depth[:6]}")
    assert st["passes"] == 2 and st["env_launches"] == 2 * 6
    assert abs(per_depth.sum() - st["ms_env"]) <= 1e-4 * st["ms_env"] + 1e-6
    assert np.all(per_depth[:6] > 0.0) and np.all(per_depth[6:] == 0.0)
    assert sum(st["escaped"]) == st["env_queries"] > 0


@pytest.mark.parametrize("master", [npt.FP32, npt.FP16])
def test_training_resumes_from_saved_state(master, small_sky):
    # four steps straight, against two steps, the training state saved,
    # restored into a new context (whose own weights differ) and two more
    # steps: the same master weights, moments and step count bit for bit --
    # the batches, Adam's bias correction and the stochastic rounding all
    # follow the restored step count
    B = 4096

    def tp(steps):
        return npt.train_params(batch=B, samples=steps * B, seed=3, grad_prec=npt.FP16, master_prec=master)

    def ctx_with(p):
        c = npt.npt_create(0)
        npt.npt_env_upload(c, small_sky)
        npt.npt_nif_upload(c, p)
        return c

    p = synth.nif_init(17)
    states = {}
    for name, steps in (("full", 4), ("mid", 2)):
        c = ctx_with(p)
        try:
            npt.npt_nif_train(c, tp(steps))
            states[name] = npt.npt_nif_get_state(c)
        finally:
            npt.npt_destroy(c)
    c = ctx_with(synth.nif_init(99))
    try:
        npt.npt_nif_set_state(c, *states["mid"])
        back = npt.npt_nif_get_state(c)
        st = npt.npt_nif_train(c, tp(2))
        resumed = npt.npt_nif_get_state(c)
    finally:
        npt.npt_destroy(c)
    assert back[3] == states["mid"][3] == 2
    assert all(np.array_equal(x, y) for x, y in zip(back[:3], states["mid"][:3]))
    assert st["step_total"] == resumed[3] == states["full"][3] == 4
    for x, y in zip(resumed[:3], states["full"][:3]):
        assert np.array_equal(x, y)
    assert not np.array_equal(states["mid"][0], states["full"][0])  # the two later steps moved the weights
