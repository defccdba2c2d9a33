"""LDS-resident NIF inference for the network shapes other than the default
that have their own kernel (Sec. 3.2, 4.6): the paper's H128 network (four
dense-ReLU layers, the second narrowed so that the features concatenated to
its output make 128 inputs; 40-d and 64-d features) and the small H64 L2
network.  Queries in FP32/FP16/BF16/FP8 against the oracle's
forward pass with the same operand rounding, the dequantised weights bit for
bit, a NIF-lit render, the grid evaluation against the layer-serial path, and
which shapes accept FP8."""
import numpy as np
import pytest

import oracle as O
from paper_2305_20061_amd import npt, synth

from gpu_util import gpu_render, make_ctx, oracle_scene, rel_rmse, torch_cuda

pytestmark = pytest.mark.gpu
# (hidden, layers, skip-concat layer, frequencies)
ARCHS = [(128, 4, 2, 10), (128, 4, 2, 16), (64, 2, 0, 16)]
PRECS = [npt.FP32, npt.FP16, npt.BF16, npt.FP8]
# as for the default network: accumulation order, and FP32 features that move
# an operand across a rounding boundary now and then
QUERY_TOL = {npt.FP32: 5e-5, npt.FP16: 1e-3, npt.BF16: 1e-2, npt.FP8: 2e-2}


def _weights(hidden, layers, skip, nf, seed=3):
    p = synth.nif_init(seed, nf, hidden, layers, skip).astype(np.float32)
    p[-3:] = (0.6, 0.05, -0.05)
    return p


def _dirs(n, seed=0):
    rng = np.random.default_rng(seed)
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return d.astype(np.float32)


def _upload(ctx, p, arch, layered=0):
    hidden, layers, skip, nf = arch
    npt.npt_nif_upload(ctx, p, n_freq=nf, hidden=hidden, layers=layers, skip=skip, layered=layered)


@pytest.mark.parametrize("arch", ARCHS)
@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("n", [1, 4096 + 29])
def test_resident_query_matches_oracle(arch, prec, n):
    torch = torch_cuda()
    hidden, layers, skip, nf = arch
    shape = O.nif_shape(nf, hidden, layers, O.COLOUR_YUV, skip)
    p = _weights(*arch)
    ctx = npt.npt_create(0)
    try:
        _upload(ctx, p, arch)
        npt.npt_nif_set_precision(ctx, prec)
        d = _dirs(n)
        out = torch.full((n, 3), -1.0, dtype=torch.float32, device="cuda")
        npt.npt_env_query(ctx, npt.ENV_NIF, torch.from_numpy(d).cuda(), out)
        torch.cuda.synchronize()
        g = out.cpu().numpy().astype(np.float64)
        dq = npt.npt_nif_get_dequantized(ctx, p.size).astype(np.float64)
    finally:
        npt.npt_destroy(ctx)
    ref_p = O.nif_dequantize(shape, p.astype(np.float64), prec)
    assert np.array_equal(dq, ref_p)  # the kernel multiplies the oracle's rounded weights
    o = np.array([O.nif_radiance_q(shape, ref_p, prec, *O.dir_to_uv(x)) for x in d])
    r = rel_rmse(g, o)
    print(f"resident H{hidden} L{layers} skip {skip} freq {nf} prec {prec} n {n}: relRMSE {r:.3e}")
    assert np.all(g >= 0)
    assert r <= QUERY_TOL[prec]


@pytest.mark.parametrize("prec", [npt.FP16, npt.FP8])
def test_paper_network_render_matches_oracle(prec, small_sky):
    arch = ARCHS[0]
    hidden, layers, skip, nf = arch
    shape = O.nif_shape(nf, hidden, layers, O.COLOUR_YUV, skip)
    scene = synth.scene_for(1)
    p = _weights(*arch)
    ctx = make_ctx(scene, env=small_sky)
    try:
        _upload(ctx, p, arch)
        npt.npt_nif_set_precision(ctx, prec)
        npt.npt_set_env_mode(ctx, npt.ENV_NIF)
        g = gpu_render(ctx, 48, 48, 2, 6, 9)
    finally:
        npt.npt_destroy(ctx)
    osc, cam = oracle_scene(scene)
    dq = O.nif_dequantize(shape, p.astype(np.float64), prec)
    o = O.render(osc, cam, O.render_desc(48, 48, 2, 6, 9, nif_params=dq, nif=shape, nif_prec=prec))
    r = rel_rmse(g, o)
    print(f"paper network prec {prec} render relRMSE {r:.3e}")
    assert r <= QUERY_TOL[prec]


def test_resident_and_layered_grid_evaluations_agree(small_sky):
    # the same network and FP16 operands on both inference paths: log-MSE
    # against the map on a grid agrees to the FP16 rounding of the operands
    arch = ARCHS[0]
    p = _weights(*arch)
    res = []
    for layered in (0, 1):
        ctx = npt.npt_create(0)
        try:
            npt.npt_env_upload(ctx, small_sky)
            npt.npt_nif_set_precision(ctx, npt.FP16)
            _upload(ctx, p, arch, layered=layered)
            res.append(npt.npt_nif_eval_grid(ctx, 256, 128)["log_mse"])
        finally:
            npt.npt_destroy(ctx)
    m0, m1 = res
    print(f"grid log-MSE resident {m0:.6e} layered {m1:.6e}")
    assert abs(m0 - m1) <= 1e-3 * m1


def test_fp8_needs_a_resident_shape():
    ctx = npt.npt_create(0)
    try:
        arch = ARCHS[0]
        _upload(ctx, _weights(*arch), arch)
        npt.npt_nif_set_precision(ctx, npt.FP8)  # resident: accepted
        other = (128, 3, 0, 16)
        with pytest.raises(npt.NptError) as e:
            _upload(ctx, _weights(*other), other)  # no resident kernel, FP8 still selected
        assert e.value.code == npt.NPT_E["UNSUPPORTED"]
        npt.npt_nif_set_precision(ctx, npt.FP16)
        _upload(ctx, _weights(*other), other)
        with pytest.raises(npt.NptError) as e:
            npt.npt_nif_set_precision(ctx, npt.FP8)
        assert e.value.code == npt.NPT_E["UNSUPPORTED"]
    finally:
        npt.npt_destroy(ctx)
