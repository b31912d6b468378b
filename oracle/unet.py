"""FP64 CPU oracle of the U-Net preconditioner (test infrastructure only).

Plain numpy on BF16-rounded values: each activation is rounded to BF16 (round
to nearest even) exactly where the GPU stores it, each convolution is an FP64
sum over the 27 taps and input channels, so GPU and oracle differ only by the
GPU's FP32 accumulation order.

Network (linear, no biases): e0 = conv(r; 1->C0); e1 = conv(pool(e0));
bottleneck convs at 1/4 resolution (dilations 1, 2, 4, ..., then 1);
g1 = conv(e1 + up(b); C1->C0); gz = g1 . wp (pointwise C0->1) at 1/2
resolution; z = conv(e0; C0->1) + up(gz) on the interior: a local stencil
of r plus the interpolated coarse correction.  e0 itself is never rounded:
the pool and the output conv take it in full precision (only the copy kept
for the output weights' gradient is BF16).
conv = 3x3x3 cross-correlation with zero padding; pool = mean of the
existing children; up = cell-centred trilinear interpolation (per axis a
fine cell takes 3/4 of its parent and 1/4 of the parent's neighbour on its
side, the neighbour index clamped to the coarse grid).  Arrays are
channels-last [z][y][x][C].
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
    if abs(dz) >= Z or abs(dy) >= Y or abs(dx) >= X:
        return out  # shifted entirely outside: zero padding

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


def _repeat(c, shape):
    """Nearest-neighbour copy of a coarse field onto `shape` (first 3 axes)."""
    Z, Y, X = shape
    return c[np.arange(Z) // 2][:, np.arange(Y) // 2][:, :, np.arange(X) // 2]


def _interp_index(n, nc):
    """Parent I and side neighbour J (clamped) of fine cells 0..n-1."""
    i = np.arange(n)
    I = i // 2
    J = np.clip(np.where(i % 2 == 0, I - 1, I + 1), 0, nc - 1)
    return I, J


def up(c, shape):
    """Trilinear (cell-centred, factor 2) interpolation of a coarse field onto
    `shape`, one axis after the other: f[i] = 3/4 c[I] + 1/4 c[J]."""
    out = np.asarray(c, dtype=np.float64)
    for ax in range(3):
        I, J = _interp_index(shape[ax], out.shape[ax])
        out = 0.75 * np.take(out, I, axis=ax) + 0.25 * np.take(out, J, axis=ax)
    return out


def layer_shapes(c0=16, c1=32, c2=64, nbott=4):
    """(ci, co, dil) of every layer in order, as the GPU network builds them;
    dil = 0 marks the pointwise projection (one tap)."""
    L = [(1, c0, 1), (c0, c1, 1), (c1, c2, 1)]
    dil = 2
    for _ in range(nbott - 2):
        L.append((c2, c2, dil))
        dil *= 2
    L += [(c2, c1, 1), (c1, c0, 1), (c0, 1, 0), (c0, 1, 1)]
    return L


def layer_taps(dil):
    return 27 if dil > 0 else 1


def layer_size(ci, co, dil):
    return co * layer_taps(dil) * ci


def split_weights(flat, shapes):
    """Flat master weights ([co][taps*ci] per layer) -> list of [co][taps][ci]."""
    out, off = [], 0
    for ci, co, dil in shapes:
        n = layer_size(ci, co, dil)
        out.append(np.asarray(flat[off:off + n], dtype=np.float64).reshape(co, layer_taps(dil), ci))
        off += n
    return out


def _identity(x):
    return np.asarray(x, dtype=np.float64)


def forward(r, in_scale, out_scale, flat_w, c0=16, c1=32, c2=64, nbott=4, exact=False, keep=False):
    """Network output z (FP64 [Z][Y][X]) for the residual r [Z][Y][X].
    exact=True drops every BF16 rounding (for finite-difference checks);
    keep=True also returns the stored activations for the backward pass."""
    rnd = _identity if exact else bf16_round
    shapes = layer_shapes(c0, c1, c2, nbott)
    Ws = [rnd(w) for w in split_weights(flat_w, shapes)]
    x = rnd(np.float32(in_scale * np.asarray(r, dtype=np.float64)) if not exact else in_scale * np.asarray(r))[..., None]
    e0_out = conv3(x, Ws[0])  # pooled and used by the output conv unrounded
    e0 = rnd(e0_out)          # the activation kept for the output weights' gradient
    p0 = rnd(pool(e0_out))
    e1 = rnd(conv3(p0, Ws[1]))
    b = rnd(pool(e1))
    bins = []
    for li in range(2, 2 + nbott):
        bins.append(b)
        b = rnd(conv3(b, Ws[li], shapes[li][2]))
    i1 = rnd(np.float32(e1) + np.float32(up(b, e1.shape[:3])) if not exact else e1 + up(b, e1.shape[:3]))
    g1 = rnd(conv3(i1, Ws[2 + nbott]))
    f32 = _identity if exact else (lambda a: np.asarray(np.float32(a), dtype=np.float64))
    gz = f32(g1 @ Ws[3 + nbott][0, 0, :])[..., None]
    z = out_scale * (conv3(e0_out, Ws[4 + nbott])[..., 0] + up(gz, e0.shape[:3])[..., 0])
    m = np.zeros_like(z)
    m[1:-1, 1:-1, 1:-1] = 1.0
    z = z * m
    if keep:
        return z, dict(x=x, e0=e0, p0=p0, e1=e1, bins=bins, i1=i1, g1=g1, gz=gz, Ws=Ws, shapes=shapes)
    return z


def conv3_adjoint(dy, W, dil=1):
    """Adjoint of conv3 in its input: dx[v][ci] = sum W[co][t][ci] dy[v - t][co]."""
    dx = np.zeros(dy.shape[:3] + (W.shape[2],))
    for t, (dz, dyy, dx_) in enumerate(taps()):
        dx += shift(dy, -dil * dz, -dil * dyy, -dil * dx_) @ W[:, t, :]
    return dx


def conv3_weight_grad(x, dy, dil=1):
    """dW[co][t][ci] = sum_v x(v + dil t)[ci] dy[v][co]."""
    co, ci = dy.shape[3], x.shape[3]
    g = np.zeros((co, 27, ci))
    for t, (dz, dyy, dx_) in enumerate(taps()):
        xs = shift(x, dil * dz, dil * dyy, dil * dx_)
        g[:, t, :] = dy.reshape(-1, co).T @ xs.reshape(-1, ci)
    return g


def up_adjoint(df, cshape):
    """Adjoint of the trilinear interpolation: each fine value is returned to
    its parent with weight 3/4 and to the side neighbour with weight 1/4."""
    out = np.asarray(df, dtype=np.float64)
    for ax in (2, 1, 0):
        I, J = _interp_index(out.shape[ax], cshape[ax])
        shp = list(out.shape)
        shp[ax] = cshape[ax]
        acc = np.zeros(shp)
        for src, w in ((I, 0.75), (J, 0.25)):
            moved = np.moveaxis(acc, ax, 0)
            np.add.at(moved, src, w * np.moveaxis(out, ax, 0))
        out = acc
    return out


def pool_adjoint(dc, fshape):
    """Adjoint of the children mean: each child gets dc / (children of its parent)."""
    Z, Y, X = fshape
    cnt = np.zeros(dc.shape[:3] + (1,))
    for dz in range(2):
        for dy in range(2):
            for dx in range(2):
                cnt[:len(range(dz, Z, 2)), :len(range(dy, Y, 2)), :len(range(dx, X, 2))] += 1
    return _repeat(dc / cnt, (Z, Y, X))


def backward(r, in_scale, flat_w, dz, dz_scale, c0=16, c1=32, c2=64, nbott=4, exact=False):
    """Flat weight gradient for the gradient dz_scale * dz of the raw network
    output (dz zero outside the interior), mirroring the GPU: FP32 gradient of
    the output, activation gradients rounded to BF16 where they feed a
    transposed convolution, and the output weights' gradient taken against the
    kept BF16 e0 (not in exact mode)."""
    rnd = _identity if exact else bf16_round
    f32 = _identity if exact else (lambda a: np.asarray(np.float32(a), dtype=np.float64))
    _, A = forward(r, in_scale, 1.0, flat_w, c0, c1, c2, nbott, exact=exact, keep=True)
    Ws, shapes = A["Ws"], A["shapes"]
    grads = [None] * len(shapes)
    dzf = f32(dz_scale * np.asarray(dz, dtype=np.float64))[..., None]
    lo, lp, ld1 = len(shapes) - 1, len(shapes) - 2, len(shapes) - 3
    # z = conv(e0; W_out) + up(gz), gz = g1 . wp
    grads[lo] = conv3_weight_grad(A["e0"], dzf)
    de0 = conv3_adjoint(dzf, Ws[lo])
    dgz = up_adjoint(dzf, A["g1"].shape[:3])
    grads[lp] = (A["g1"].reshape(-1, A["g1"].shape[3]).T @ dgz.reshape(-1)).reshape(1, 1, -1)
    dg1 = dgz * Ws[lp][0, 0, :]
    grads[ld1] = conv3_weight_grad(A["i1"], dg1)
    de1 = conv3_adjoint(rnd(dg1), Ws[ld1])
    dcur = up_adjoint(de1, A["bins"][-1].shape[:3])
    for li in range(ld1 - 1, 1, -1):
        xin = A["bins"][li - 2]
        grads[li] = conv3_weight_grad(xin, dcur, shapes[li][2])
        dcur = conv3_adjoint(rnd(dcur), Ws[li], shapes[li][2])
    de1 = de1 + pool_adjoint(dcur, A["e1"].shape[:3])
    grads[1] = conv3_weight_grad(A["p0"], de1)
    dp0 = conv3_adjoint(rnd(de1), Ws[1])
    de0 = de0 + pool_adjoint(dp0, A["e0"].shape[:3])
    grads[0] = conv3_weight_grad(A["x"], de0)
    return np.concatenate([g.reshape(-1) for g in grads])
