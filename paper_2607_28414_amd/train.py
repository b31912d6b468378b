"""Training of the learned preconditioner on samples the solver generates.

A sample is a pair (b, x) with b = A x, A = -lap on the interior of a
unit-spacing grid, both scaled so that b has unit RMS; the loss is the
relative A-norm error (z - x)^T A (z - x) / x^T A x of the network output
z = U(b).  Sample kinds:

* ``force``: x is the potential phi of the projection of a random focal
  push times a random-phase modulation (the force patterns a time-varying
  radiation force produces), b = A phi;
* ``cg``: x is the error after k Jacobi-PCG iterations on such a force,
  b the residual (late residuals carry the long wavelengths);
* ``fpcg``: the same with k flexible-PCG iterations using the current
  network, i.e. the residuals the preconditioner actually meets;
* ``white``: x white noise on the interior (the short wavelengths).

Everything runs in the library's kernels (sample generation, forward,
backward, Adam); this module only orchestrates.  Torch provides the
device buffers.
"""
from __future__ import annotations

import time

import numpy as np

from . import kvs


def focal_force(shape, rng):
    """[3][nz][ny][nx] force on a unit grid: a Gaussian push along a random
    axis (lateral sigma 3-8 cells, axial 10-25 cells, focus within the
    central half) times 1 + 0.5 / sqrt(8) * sum of 8 plane waves with
    wavelengths of 4-20 cells, random directions and phases."""
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz) - nz / 2, np.arange(ny) - ny / 2, np.arange(nx) - nx / 2, indexing="ij")
    c = rng.uniform(-0.25, 0.25, 3) * np.array([nz, ny, nx])
    axis = int(rng.integers(0, 3))
    d = [z - c[0], y - c[1], x - c[2]]
    sl, sa = rng.uniform(3, 8), rng.uniform(10, 25)
    r2 = sum(d[a] ** 2 for a in range(3) if a != axis)
    g = np.exp(-r2 / (2 * sl ** 2) - d[axis] ** 2 / (2 * sa ** 2))
    m = np.ones_like(g)
    for _ in range(8):
        k = 2 * np.pi / rng.uniform(4, 20)
        u = rng.standard_normal(3)
        u /= np.linalg.norm(u)
        m += 0.5 / np.sqrt(8) * np.cos(k * (u[0] * z + u[1] * y + u[2] * x) + rng.uniform(0, 2 * np.pi))
    F = np.zeros((3,) + tuple(shape))
    F[2 - axis] = g * m  # component along the push axis ([0] = x)
    return F


class Trainer:
    """Sample set and Adam loop for one network on n^3 unit grids."""

    def __init__(self, net, n=64, seed=0):
        import torch
        self.torch = torch
        self.net, self.n = net, int(n)
        self.rng = np.random.default_rng(seed)
        self.samples = []  # (kind, b, x) device tensors
        self.train_seconds = 0.0

    def _pair(self):
        t = self.torch
        b = t.zeros((self.n,) * 3, dtype=t.float64, device="cuda")
        return b, t.zeros_like(b)

    def add_force_samples(self, count, snapshots=(0,), precond=kvs.KVS_PC_JACOBI):
        """`count` random forces; for each, one sample per entry of
        `snapshots` (0: the potential itself, k > 0: the error after k
        iterations of the solver with `precond`)."""
        t0 = time.perf_counter()
        n = self.n
        grid = (n, n, n, 1.0, 1.0, 1.0)
        for _ in range(count):
            ctx = kvs.kvs_create(grid)
            try:
                kvs.kvs_set_force(ctx, focal_force((n, n, n), self.rng))
                if precond == kvs.KVS_PC_UNET:
                    kvs.kvs_set_preconditioner(ctx, self.net)
                for k in snapshots:
                    b, x = self._pair()
                    kvs.kvs_unet_make_sample(ctx, k, b.data_ptr(), x.data_ptr(), precond=precond if k else kvs.KVS_PC_JACOBI)
                    kind = "force" if k == 0 else ("fpcg" if precond == kvs.KVS_PC_UNET else "cg")
                    self.samples.append((f"{kind}{k or ''}", b, x))
            finally:
                kvs.kvs_destroy(ctx)
        self.torch.cuda.synchronize()
        self.train_seconds += time.perf_counter() - t0

    def add_white(self, count):
        t0 = time.perf_counter()
        n = self.n
        for _ in range(count):
            xh = np.zeros((n, n, n))
            xh[1:-1, 1:-1, 1:-1] = self.rng.standard_normal((n - 2,) * 3)
            b, x = self._pair()
            x.copy_(self.torch.from_numpy(xh))
            kvs.kvs_unet_sample_from_x(x.data_ptr(), b.data_ptr(), (n, n, n),
                                       self.torch.cuda.current_stream().cuda_stream)
            self.samples.append(("white", b, x))
        self.train_seconds += time.perf_counter() - t0

    def fit(self, iters, lr, lr_floor=0.1, log=None):
        """`iters` Adam steps over the whole sample set (gradients averaged),
        cosine learning rate from lr down to lr_floor * lr.  Returns the mean
        loss per kind at the last step."""
        t0 = time.perf_counter()
        st = self.torch.cuda.current_stream().cuda_stream
        n = self.n
        last = {}
        for it in range(iters):
            per = {}
            for q, (kind, b, x) in enumerate(self.samples):
                loss = kvs.kvs_unet_train_sample(self.net, b.data_ptr(), x.data_ptr(), (n, n, n), q > 0, st)
                per.setdefault(kind.rstrip("0123456789"), []).append(loss)
            f = lr_floor + (1 - lr_floor) * 0.5 * (1 + np.cos(np.pi * it / max(iters, 1)))
            kvs.kvs_unet_adam_step(self.net, lr * f, len(self.samples), st)
            last = {k: float(np.mean(v)) for k, v in per.items()}
            if log and (it % max(1, iters // 4) == 0 or it == iters - 1):
                log(f"  step {it}: " + " ".join(f"{k} {v:.3e}" for k, v in last.items()))
        self.torch.cuda.synchronize()
        self.train_seconds += time.perf_counter() - t0
        return last


def init_weights(net, rng, scale=0.3):
    """Random weights with standard deviation scale / sqrt(fan-in) per layer
    (the network starts near zero: every iteration falls back to Jacobi)."""
    w = np.concatenate([scale * rng.standard_normal(co * taps * ci) / np.sqrt(taps * ci)
                        for ci, co, _, taps in kvs.kvs_unet_layers(net)])
    kvs.kvs_unet_set_weights(net, w.astype(np.float32))


def train_default(net, n=64, seed=0, rounds=4, lr=2e-3, forces=6, base_steps=200, round_steps=120, log=None):
    """The training recipe: base samples (`forces` random forces with their
    potentials and the errors after 20 and 60 Jacobi-PCG iterations, 4
    white-noise fields), `base_steps` Adam steps at learning rate lr; then
    `rounds` times: `forces` more forces with the errors after 3, 10 and 30
    flexible-PCG iterations with the current network, `round_steps` steps at
    lr / 2.  Returns the Trainer (train_seconds: the
    whole time, sample generation included)."""
    tr = Trainer(net, n=n, seed=seed)
    init_weights(net, tr.rng)
    tr.add_force_samples(forces, snapshots=(0, 20, 60))
    tr.add_white(4)
    tr.fit(base_steps, lr, log=log)
    for _ in range(rounds):
        tr.add_force_samples(forces, snapshots=(3, 10, 30), precond=kvs.KVS_PC_UNET)
        tr.fit(round_steps, lr / 2, log=log)
    return tr
