"""On-device NIF training at the benchmarked batch (Sec. 3.2.1: 65,536
samples per step) against the oracle, for the workload's 16/96/5 network and
the paper's 10/128/4 network with the skip-concat at layer 2.

Two step implementations are covered.  The layer-by-layer path (FP32, BF16,
and FP16 when asked for): at this batch its weight gradients run over 128
split-K chunks whose partial sums go through the fixed-order reduction
(eight waves per 64 parameters, four interleaved running sums each).  The
fused path (FP16 on these shapes by default): forward, backward and the
weight-gradient sums of 128 samples per workgroup in one kernel, the 512
workgroups' sums reduced in a fixed order and Adam in a second.

Gradients are compared with the oracle's loss and gradient whose GEMM
operands are rounded as the trainer's are (or_nif_loss_grad_q: weights,
layer inputs and back-propagated gradients rounded to the operand format,
the same loss scale, exact sums), so what is left is FP32 summation order
and the FP32 features; the FP64 gradient without rounding is checked too,
at the distance the rounding itself puts between the two.  A four-step Adam
trajectory is compared step by step with the oracle's steps."""
import numpy as np
import pytest

import oracle as O
from paper_2305_20061_amd import npt, synth

from gpu_util import rel_rmse, torch_cuda

pytestmark = pytest.mark.gpu

B = 65536
DELTA = 1e-3
THREADS = 8
# (n_freq, hidden, layers, skip): the workload's network and the paper's
NETS = [(16, 96, 5, 0), (10, 128, 4, 2)]
# the trainer's default loss scale per GEMM operand precision
LOSS_SCALE = {npt.FP32: 1.0, npt.FP16: 16384.0, npt.BF16: 1.0}

# Bounds against the rounded-operand oracle, from the measured error with a
# margin of about 3x: relative RMSE of the gradient (measured 3.5e-6 /
# 2.4e-5 / 2.7e-5 for FP32 / FP16 / BF16 operands, the larger of the two
# networks) and relative loss error (3.0e-7 / 5.5e-7 / 6.6e-7)
GRAD_TOL_Q = {npt.FP32: 1e-5, npt.FP16: 7e-5, npt.BF16: 8e-5}
LOSS_TOL_Q = {npt.FP32: 1e-6, npt.FP16: 2e-6, npt.BF16: 2e-6}
# ... and against the FP64 gradient without any rounding (3.5e-6 / 4.5e-4 /
# 2.9e-3)
GRAD_TOL_64 = {npt.FP32: 1e-5, npt.FP16: 1.5e-3, npt.BF16: 9e-3}


def _shape(nf, hidden, layers, skip):
    return O.nif_shape(nf, hidden, layers, O.COLOUR_YUV, skip)


def _upload(ctx, p, nf, hidden, layers, skip):
    npt.npt_nif_upload(ctx, p, n_freq=nf, hidden=hidden, layers=layers, skip=skip)


# (operand precision, step implementation): the default path of each
# precision, and the layer-by-layer path where FP16 defaults to the fused one
PATHS = [(npt.FP32, npt.TRAIN_AUTO), (npt.FP16, npt.TRAIN_AUTO), (npt.FP16, npt.TRAIN_LAYERED),
         (npt.BF16, npt.TRAIN_AUTO)]


@pytest.mark.parametrize("net", NETS)
@pytest.mark.parametrize("prec,path", PATHS)
def test_full_batch_gradient_matches_oracle(net, prec, path, small_sky):
    torch = torch_cuda()
    nf, hidden, layers, skip = net
    shape = _shape(*net)
    p = synth.nif_init(11, nf, hidden, layers, skip)
    seed, step = 5, 3
    print(f"full-batch gradient: net {net} prec {prec} path {path} B {B}", flush=True)
    ctx = npt.npt_create(0)
    try:
        npt.npt_env_upload(ctx, small_sky)
        _upload(ctx, p, *net)
        grad = torch.zeros(p.size, dtype=torch.float32, device="cuda")
        loss = torch.zeros(1, dtype=torch.float32, device="cuda")
        npt.npt_nif_train_grad(ctx, npt.train_params(batch=B, seed=seed, grad_prec=prec, path=path), step, grad,
                               loss, n_params=p.size)
        torch.cuda.synchronize()
        g = grad.cpu().numpy().astype(np.float64)
        lg = float(loss.cpu()[0])
    finally:
        npt.npt_destroy(ctx)
    uv, tg = O.nif_train_batch(small_sky, seed, step, B)
    p64 = p.astype(np.float64)
    lq, gq = O.nif_loss_grad_q(shape, p64, prec, LOSS_SCALE[prec], uv, tg, DELTA, threads=THREADS)
    l64, g64 = O.nif_loss_grad(shape, p64, uv, tg, DELTA, threads=THREADS)
    rq, r64 = rel_rmse(g, gq), rel_rmse(g, g64)
    eq = abs(lg - lq) / abs(lq)
    print(f"net {net} prec {prec} path {path}: grad relRMSE {rq:.3e} (rounded oracle), {r64:.3e} (FP64); "
          f"loss rel err {eq:.3e} ({lg:.7e} vs {lq:.7e})")
    assert rq <= GRAD_TOL_Q[prec]
    assert eq <= LOSS_TOL_Q[prec]
    assert r64 <= GRAD_TOL_64[prec]


# Adam trajectory: relative RMSE of the accumulated update (weights after k
# steps minus the initial weights) against the oracle's, and the loss of
# each step's batch; bounds from the measured error over the four steps
# with a margin of about 3x (updates 2.4e-5 FP32, 1.0e-3 FP16; losses
# 1.8e-7, 1.9e-5)
TRAJ_UPDATE_TOL = {npt.FP32: 7e-5, npt.FP16: 3e-3}
TRAJ_LOSS_TOL = {npt.FP32: 1e-6, npt.FP16: 6e-5}


@pytest.mark.parametrize("prec,path", [(npt.FP32, npt.TRAIN_AUTO), (npt.FP16, npt.TRAIN_AUTO),
                                       (npt.FP16, npt.TRAIN_LAYERED)])
def test_four_adam_steps_match_oracle(prec, path, small_sky):
    net = NETS[0]
    nf, hidden, layers, skip = net
    shape = _shape(*net)
    p0 = synth.nif_init(13, nf, hidden, layers, skip).astype(np.float32).astype(np.float64)
    seed, steps = 21, 4
    print(f"Adam trajectory: prec {prec} path {path}, {steps} steps of {B}", flush=True)
    gpu_w, gpu_loss = [], []
    ctx = npt.npt_create(0)
    try:
        npt.npt_env_upload(ctx, small_sky)
        _upload(ctx, p0, *net)
        for k in range(steps):
            st = npt.npt_nif_train(ctx, npt.train_params(batch=B, samples=B, seed=seed, grad_prec=prec,
                                                         path=path))
            assert st["steps"] == 1 and st["step_total"] == k + 1
            gpu_loss.append(st["first_loss"])
            gpu_w.append(npt.npt_nif_download(ctx).astype(np.float64))
    finally:
        npt.npt_destroy(ctx)
    # the oracle's steps: the batch of step k, the rounded-operand gradient,
    # Adam (Kingma & Ba, Alg. 1) in FP64 on FP32 master weights
    w = p0.astype(np.float64).copy()
    m, v = np.zeros_like(w), np.zeros_like(w)
    for k in range(steps):
        uv, tg = O.nif_train_batch(small_sky, seed, k, B)
        lo, g = O.nif_loss_grad_q(shape, w, prec, LOSS_SCALE[prec], uv, tg, DELTA, threads=THREADS)
        O.adam_step(w, g, m, v, k + 1, 1e-3, 0.9, 0.999, 1e-7)
        w = w.astype(np.float32).astype(np.float64)  # FP32 master weights
        du, do = gpu_w[k] - p0, w - p0
        ru = rel_rmse(du, do)
        el = abs(gpu_loss[k] - lo) / lo
        moved = np.mean(np.sign(du) == np.sign(do))
        print(f"prec {prec} path {path} step {k + 1}: update relRMSE {ru:.3e}, sign agreement {moved:.6f}, "
              f"loss rel err {el:.3e}")
        assert ru <= TRAJ_UPDATE_TOL[prec]
        assert el <= TRAJ_LOSS_TOL[prec]


@pytest.mark.parametrize("net", NETS + [(16, 128, 4, 2), (16, 64, 2, 0)])
def test_fused_and_layered_steps_agree(net, small_sky):
    """The fused FP16 step against the layer-by-layer FP16 step on the same
    batch: same rounding points, so only FP32 summation order (and the FP16
    roundings it tips over) separates them; the fused step is deterministic.
    All four shapes with a fused kernel."""
    torch = torch_cuda()
    nf, hidden, layers, skip = net
    p = synth.nif_init(17, nf, hidden, layers, skip)
    res = {}
    ctx = npt.npt_create(0)
    try:
        npt.npt_env_upload(ctx, small_sky)
        _upload(ctx, p, *net)
        for name, path in (("fused", npt.TRAIN_AUTO), ("fused again", npt.TRAIN_AUTO),
                           ("layered", npt.TRAIN_LAYERED)):
            print(f"fused vs layered: net {net} {name}", flush=True)
            grad = torch.zeros(p.size, dtype=torch.float32, device="cuda")
            loss = torch.zeros(1, dtype=torch.float32, device="cuda")
            npt.npt_nif_train_grad(ctx, npt.train_params(batch=B, seed=9, grad_prec=npt.FP16, path=path), 2,
                                   grad, loss, n_params=p.size)
            torch.cuda.synchronize()
            res[name] = (grad.cpu().numpy().astype(np.float64), float(loss.cpu()[0]))
    finally:
        npt.npt_destroy(ctx)
    assert np.array_equal(res["fused"][0], res["fused again"][0]) and res["fused"][1] == res["fused again"][1]
    r = rel_rmse(res["fused"][0], res["layered"][0])
    el = abs(res["fused"][1] - res["layered"][1]) / res["layered"][1]
    print(f"net {net}: fused vs layered grad relRMSE {r:.3e}, loss rel err {el:.3e}")
    assert r <= GRAD_TOL_Q[npt.FP16] and el <= LOSS_TOL_Q[npt.FP16]
