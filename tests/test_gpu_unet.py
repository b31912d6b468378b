"""The U-Net's MFMA kernels against the FP64 oracle on the same BF16-rounded
inputs and weights."""
import numpy as np
import pytest

from oracle import unet

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def kvs():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_2607_28414_amd import kvs as k
    k.lib()
    return k


def say(*a):
    print(*a, flush=True)


PAIRS = [(16, 32, 1, False), (32, 64, 1, False), (64, 64, 2, False), (64, 64, 8, False), (64, 32, 1, False),
         (32, 16, 1, True), (16, 16, 1, True), (32, 32, 1, True), (8, 16, 3, False)]


@pytest.mark.parametrize("ci,co,dil,skip", PAIRS)
def test_conv_kernel_matches_oracle(kvs, ci, co, dil, skip):
    """BF16 outputs equal the oracle's FP64 conv rounded to BF16, except
    where FP32 accumulation lands on the other side of a rounding boundary
    (under 1% of outputs).  Every output is within half a BF16 ulp of the
    exact sum plus the FP32 accumulation bound n eps32 sum|w x|."""
    say(f"case conv {ci}->{co} dil {dil} skip {skip}")
    rng = np.random.default_rng(ci * 100 + co + dil)
    dims = (37, 21, 19)  # ragged: 37*21*19 is not a multiple of 16 voxels
    nx, ny, nz = dims
    A = unet.bf16_round(rng.standard_normal((nz, ny, nx, ci)))
    cz, cy, cx = unet.coarse_shape((nz, ny, nx))
    B = unet.bf16_round(rng.standard_normal((cz, cy, cx, ci))) if skip else None
    W = unet.bf16_round(rng.standard_normal((co, 27, ci)) / np.sqrt(27 * ci))
    kp = kvs.kvs_unet_conv_kpad(ci)
    Wp = np.zeros((co, kp))
    Wp[:, :27 * ci] = W.reshape(co, 27 * ci)
    out = kvs.kvs_unet_conv_check(ci, co, dil, unet.to_bits(A), None if B is None else unet.to_bits(B), dims,
                                  unet.to_bits(Wp))
    got = unet.from_bits(out).reshape(nz, ny, nx, co)
    x = A if B is None else unet.bf16_round(np.float32(A) + np.float32(unet.up(B, (nz, ny, nx))))
    exact = unet.conv3(x, W, dil)
    ref = unet.bf16_round(exact)
    diff = got != ref
    frac = diff.mean()
    assert frac < 0.01, frac
    S = unet.conv3(np.abs(x), np.abs(W), dil)
    bound = np.abs(exact) * 2.0 ** -8 + 27 * ci * 2.0 ** -24 * S
    assert np.all(np.abs(got - exact) <= 1.0001 * bound), np.max(np.abs(got - exact) / bound)
    assert np.linalg.norm(got - exact) / np.linalg.norm(exact) < 4e-3


def test_network_forward_matches_oracle(kvs):
    import torch
    say("case unet forward")
    rng = np.random.default_rng(7)
    net = kvs.kvs_unet_create((16, 32, 64), 4)
    try:
        n = kvs.kvs_unet_num_weights(net)
        shapes = unet.layer_shapes(16, 32, 64, 4)
        w = np.concatenate([rng.standard_normal(27 * ci * co) / np.sqrt(27 * ci) for ci, co, _ in shapes])
        assert w.size == n
        kvs.kvs_unet_set_weights(net, w.astype(np.float32))
        assert np.array_equal(kvs.kvs_unet_get_weights(net), w.astype(np.float32))
        nz, ny, nx = 22, 18, 26
        r = np.zeros((nz, ny, nx))
        r[1:-1, 1:-1, 1:-1] = rng.standard_normal((nz - 2, ny - 2, nx - 2))
        rd = torch.from_numpy(r).cuda()
        zd = torch.full_like(rd, np.nan)
        kvs.kvs_unet_forward(net, rd.data_ptr(), 0.5, 3.0, zd.data_ptr(), (nx, ny, nz),
                             torch.cuda.current_stream().cuda_stream)
        torch.cuda.synchronize()
        z = zd.cpu().numpy()
    finally:
        kvs.kvs_unet_destroy(net)
    zo = unet.forward(r, 0.5, 3.0, w.astype(np.float32).astype(np.float64), nbott=4)
    err = np.linalg.norm(z - zo) / np.linalg.norm(zo)
    say(f"forward rel L2 {err:.2e}")
    assert not z[0].any() and not z[:, 0].any() and np.isfinite(z).all()
    assert err < 2e-2
