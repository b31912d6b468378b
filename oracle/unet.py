"""FP64 CPU oracle of the U-Net preconditioner (test infrastructure only).

Plain numpy on BF16-rounded values: each activation is rounded to BF16 (round
to nearest even) exactly where the GPU stores it, each convolution is an FP64
sum over the 27 taps and input channels, so GPU and oracle differ only by the
GPU's FP32 accumulation order.

Network (linear, no biases): e0 = conv(r; 1->C0); e1 = conv(pool(e0));
bottleneck convs at 1/4 resolution (dilations 1, 2, 4, ..., then 1);
g1 = conv(e1 + up(b)); g0 = conv(e0 + up(g1)); z = conv(g0; C0->1) on the
interior.  conv = 3x3x3 cross-correlation with zero padding; pool = mean of
the existing children; up = nearest neighbour.  Arrays are channels-last
[z][y][x][C].
"""
from __future__ import annotations

import numpy as np


def bf16_round(x):
    """Round float32 values to the nearest BF16 (ties to even); returns float64."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64).reshape(f.shape)


def to_bits(x):
    """BF16 bit patterns (uint16) of float values that are already BF16."""
    return (np.ascontiguousarray(np.asarray(x, dtype=np.float32)).view(np.uint32) >> 16).astype(np.uint16)


def from_bits(b):
    return (np.asarray(b, dtype=np.uint32) << 16).view(np.float32).astype(np.float64)


def taps():
    """(dz, dy, dx) for tap = 9 dz' + 3 dy' + dx', each of dz', dy', dx' in 0..2."""
    return [(t // 9 - 1, (t // 3) % 3 - 1, t % 3 - 1) for t in range(27)]


def shift(a, dz, dy, dx):
    """out[z, y, x] = a[z + dz, y + dy, x + dx], zero outside (first 3 axes)."""
    out = np.zeros_like(a)
    Z, Y, X = a.shape[:3]

    def rng(n, d):
        return slice(max(0, -d), min(n, n - d)), slice(max(0, d), min(n, n + d))

    (oz, iz), (oy, iy), (ox, ix) = rng(Z, dz), rng(Y, dy), rng(X, dx)
    out[oz, oy, ox] = a[iz, iy, ix]
    return out


def conv3(x, W, dil=1):
    """x: [Z][Y][X][CI]; W: [CO][27][CI]; returns FP64 [Z][Y][X][CO]."""
    out = np.zeros(x.shape[:3] + (W.shape[0],))
    for t, (dz, dy, dx) in enumerate(taps()):
        xs = shift(x, dil * dz, dil * dy, dil * dx)
        out += xs @ W[:, t, :].T
    return out


def coarse_shape(shape):
    return tuple((n + 1) // 2 for n in shape)


def pool(x):
    """Mean of the existing 2x2x2 children of every coarse voxel."""
    Z, Y, X, C = x.shape
    cz, cy, cx = coarse_shape((Z, Y, X))
    s = np.zeros((cz, cy, cx, C))
    cnt = np.zeros((cz, cy, cx, 1))
    for dz in range(2):
        for dy in range(2):
            for dx in range(2):
                sub = x[dz::2, dy::2, dx::2]
                s[:sub.shape[0], :sub.shape[1], :sub.shape[2]] += sub
                cnt[:sub.shape[0], :sub.shape[1], :sub.shape[2]] += 1
    return s / cnt


def up(c, shape):
    """Nearest-neighbour copy of a coarse field onto `shape` (first 3 axes)."""
    Z, Y, X = shape
    return c[np.arange(Z) // 2][:, np.arange(Y) // 2][:, :, np.arange(X) // 2]


def layer_shapes(c0=16, c1=32, c2=64, nbott=4):
    """(ci, co, dil) of every layer in order, as the GPU network builds them."""
    L = [(1, c0, 1), (c0, c1, 1), (c1, c2, 1)]
    dil = 2
    for _ in range(nbott - 2):
        L.append((c2, c2, dil))
        dil *= 2
    L += [(c2, c1, 1), (c1, c0, 1), (c0, c0, 1), (c0, 1, 1)]
    return L


def split_weights(flat, shapes):
    """Flat master weights ([co][27*ci] per layer) -> list of [co][27][ci]."""
    out, off = [], 0
    for ci, co, _ in shapes:
        n = co * 27 * ci
        out.append(np.asarray(flat[off:off + n], dtype=np.float64).reshape(co, 27, ci))
        off += n
    return out


def forward(r, in_scale, out_scale, flat_w, c0=16, c1=32, c2=64, nbott=4):
    """Network output z (FP64 [Z][Y][X]) for the residual r [Z][Y][X]."""
    shapes = layer_shapes(c0, c1, c2, nbott)
    Ws = [bf16_round(w) for w in split_weights(flat_w, shapes)]
    x = bf16_round(np.float32(in_scale * np.asarray(r, dtype=np.float64)))[..., None]
    e0 = bf16_round(conv3(x, Ws[0]))
    e1 = bf16_round(conv3(bf16_round(pool(e0)), Ws[1]))
    b = bf16_round(pool(e1))
    for li in range(2, 2 + nbott):
        b = bf16_round(conv3(b, Ws[li], shapes[li][2]))
    i1 = bf16_round(np.float32(e1) + np.float32(up(b, e1.shape[:3])))
    g1 = bf16_round(conv3(i1, Ws[2 + nbott]))
    i0 = bf16_round(np.float32(e0) + np.float32(up(g1, e0.shape[:3])))
    g0 = bf16_round(conv3(i0, Ws[3 + nbott]))
    z = out_scale * conv3(g0, Ws[4 + nbott])[..., 0]
    m = np.zeros_like(z)
    m[1:-1, 1:-1, 1:-1] = 1.0
    return z * m
