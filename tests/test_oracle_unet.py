"""Pins of the U-Net oracle (CPU): BF16 rounding, convolution, pooling and
upsampling against independent library routines (torch CPU) and hand
values."""
import numpy as np
import pytest
import torch

from oracle import unet


def test_bf16_round_hand_values_and_torch():
    # 1 + 2^-8 is a tie between 1 and 1 + 2^-7: ties go to even (1.0);
    # 1 + 3 * 2^-8 is a tie between 1 + 2^-7 and 1 + 2^-6 ... -> 1 + 2^-6
    vals = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, -2.5, 3.14159, 1e-20, 65504.0], dtype=np.float32)
    r = unet.bf16_round(vals)
    assert r[0] == 1.0 and r[1] == 1.0 and r[2] == 1 + 2 ** -6
    ref = torch.from_numpy(vals).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(r, ref)
    x = np.random.default_rng(0).standard_normal(10000).astype(np.float32) * 10.0 ** np.random.default_rng(1).uniform(-8, 8, 10000).astype(np.float32)
    np.testing.assert_array_equal(unet.bf16_round(x), torch.from_numpy(x).to(torch.bfloat16).double().numpy())
    np.testing.assert_array_equal(unet.from_bits(unet.to_bits(unet.bf16_round(x))), unet.bf16_round(x))


@pytest.mark.parametrize("dil", [1, 2, 3])
def test_conv3_matches_torch_conv3d(dil):
    rng = np.random.default_rng(dil)
    Z, Y, X, CI, CO = 7, 9, 11, 5, 4
    x = rng.standard_normal((Z, Y, X, CI))
    W = rng.standard_normal((CO, 27, CI))
    ours = unet.conv3(x, W, dil)
    xt = torch.from_numpy(x).permute(3, 0, 1, 2)[None]            # [1][CI][Z][Y][X]
    wt = torch.from_numpy(W.reshape(CO, 3, 3, 3, CI)).permute(0, 4, 1, 2, 3)  # taps (dz, dy, dx)
    ref = torch.nn.functional.conv3d(xt, wt, padding=dil, dilation=dil)[0].permute(1, 2, 3, 0).numpy()
    np.testing.assert_allclose(ours, ref, rtol=1e-12, atol=1e-12)


def test_tap_order_hand_case():
    """tap = 9 (dz + 1) + 3 (dy + 1) + (dx + 1): a single weight on tap
    9*1 + 3*1 + 2 = 14 (dx = +1) reads the right neighbour."""
    x = np.zeros((3, 3, 5, 1))
    x[1, 1, 3, 0] = 2.0
    W = np.zeros((1, 27, 1))
    W[0, 14, 0] = 0.5
    out = unet.conv3(x, W)
    assert out[1, 1, 2, 0] == 1.0 and np.count_nonzero(out) == 1


def test_pool_and_up_against_torch_and_hand_values():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((6, 8, 10, 3))
    ref = torch.nn.functional.avg_pool3d(torch.from_numpy(x).permute(3, 0, 1, 2)[None], 2)[0].permute(1, 2, 3, 0)
    np.testing.assert_allclose(unet.pool(x), ref.numpy(), rtol=1e-14)
    # odd sizes: the last coarse cell averages only the children that exist
    y = np.arange(3, dtype=float).reshape(1, 1, 3, 1)
    p = unet.pool(y)
    assert p.shape == (1, 1, 2, 1) and p[0, 0, 0, 0] == 0.5 and p[0, 0, 1, 0] == 2.0
    # trilinear upsampling: torch's cell-centred trilinear interpolation at
    # scale 2 (edges clamped), cropped to odd fine sizes
    c = rng.standard_normal((3, 4, 5, 2))
    ct = torch.from_numpy(c).permute(3, 0, 1, 2)[None].requires_grad_(True)
    up_t = torch.nn.functional.interpolate(ct, scale_factor=2, mode="trilinear", align_corners=False)
    full = up_t[0].permute(1, 2, 3, 0).detach().numpy()
    np.testing.assert_allclose(unet.up(c, (6, 8, 10)), full, rtol=0, atol=1e-14)
    np.testing.assert_allclose(unet.up(c, (5, 7, 9)), full[:5, :7, :9], rtol=0, atol=1e-14)
    # hand values in 1-D: interior cells 3/4 : 1/4, edge cells clamped
    line = unet.up(np.array([0.0, 4.0, 8.0]).reshape(1, 1, 3, 1), (1, 1, 6))[0, 0, :, 0]
    np.testing.assert_allclose(line, [0.0, 1.0, 3.0, 5.0, 7.0, 8.0])
    # adjoint: torch's gradient of the same interpolation, and <P c, f> = <c, P^T f>
    f = rng.standard_normal((6, 8, 10, 2))
    up_t.backward(torch.from_numpy(f).permute(3, 0, 1, 2)[None])
    np.testing.assert_allclose(unet.up_adjoint(f, (3, 4, 5)), ct.grad[0].permute(1, 2, 3, 0).numpy(), atol=1e-13)
    f2 = rng.standard_normal((5, 7, 9, 2))
    lhs = np.vdot(unet.up(c, (5, 7, 9)), f2)
    rhs = np.vdot(c, unet.up_adjoint(f2, (3, 4, 5)))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_forward_is_linear_and_masked():
    rng = np.random.default_rng(4)
    shapes = unet.layer_shapes(16, 32, 64, 3)
    n = sum(unet.layer_size(*sh) for sh in shapes)
    w = rng.standard_normal(n) * 0.05
    r = np.zeros((10, 12, 14))
    r[1:-1, 1:-1, 1:-1] = rng.standard_normal((8, 10, 12))
    z = unet.forward(r, 1.0, 2.0, w, nbott=3)
    assert not z[0].any() and not z[:, :, -1].any() and np.abs(z).max() > 0
    z2 = unet.forward(r, 1.0, 4.0, w, nbott=3)
    np.testing.assert_allclose(z2, 2 * z)


def test_backward_matches_finite_differences():
    """In exact arithmetic the gradient of L(w) = <dz, y(w)> (y = raw network
    output) returned by the oracle's backward pass equals the central finite
    difference of L along random weight directions."""
    rng = np.random.default_rng(11)
    nb = 3
    shapes = unet.layer_shapes(16, 32, 64, nb)
    w = np.concatenate([rng.standard_normal(unet.layer_size(ci, co, dl)) / np.sqrt(unet.layer_taps(dl) * ci)
                        for ci, co, dl in shapes])
    shp = (9, 10, 12)
    r = np.zeros(shp)
    r[1:-1, 1:-1, 1:-1] = rng.standard_normal((7, 8, 10))
    dz = np.zeros(shp)
    dz[1:-1, 1:-1, 1:-1] = rng.standard_normal((7, 8, 10))
    g = unet.backward(r, 0.7, w, dz, 1.3, nbott=nb, exact=True)
    assert g.shape == w.shape

    def L(wv):
        return 1.3 * np.sum(dz * unet.forward(r, 0.7, 1.0, wv, nbott=nb, exact=True))

    # all layers at once: L is a polynomial of degree (number of layers) in
    # w, so the central difference carries an O(eps^2) term
    for trial in range(2):
        d = rng.standard_normal(w.size)
        eps = 1e-5
        fd = (L(w + eps * d) - L(w - eps * d)) / (2 * eps)
        assert np.dot(g, d) == pytest.approx(fd, rel=1e-6)
    # one layer at a time L is linear in the perturbation: exact to rounding
    off = 0
    for li, (ci, co, dl) in enumerate(shapes):
        n = unet.layer_size(ci, co, dl)
        d = np.zeros(w.size)
        d[off:off + n] = rng.standard_normal(n)
        fd = (L(w + 1e-3 * d) - L(w - 1e-3 * d)) / 2e-3
        assert np.dot(g, d) == pytest.approx(fd, rel=1e-9), li
        off += n


def test_shift_beyond_the_grid_is_zero_padding():
    """A tap farther than the grid extent reads only padding: a dilated conv
    on an axis shorter than its dilation keeps just the in-grid taps (brute
    force over every voxel and tap)."""
    rng = np.random.default_rng(4)
    x = rng.standard_normal((3, 2, 5, 2))
    W = rng.standard_normal((3, 27, 2))
    got = unet.conv3(x, W, dil=4)
    Z, Y, X = x.shape[:3]
    ref = np.zeros((Z, Y, X, 3))
    for z in range(Z):
        for y in range(Y):
            for xx in range(X):
                for t, (dz, dy, dx) in enumerate(unet.taps()):
                    p = (z + 4 * dz, y + 4 * dy, xx + 4 * dx)
                    if 0 <= p[0] < Z and 0 <= p[1] < Y and 0 <= p[2] < X:
                        ref[z, y, xx] += W[:, t, :] @ x[p]
    np.testing.assert_allclose(got, ref, rtol=1e-13, atol=1e-13)
