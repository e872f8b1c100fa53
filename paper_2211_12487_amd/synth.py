"""Seeded synthetic tensor streams shaped like the paper's workloads.

The paper compresses ATARI gameplay frames and gel simulations (Sec. 4.2);
neither dataset is available, so these generators stand in for them with
streams of the same order, sizes and kind of structure.  This module holds
no TT-ICE arithmetic: it only draws inputs, and both the GPU library and the
CPU oracle are fed the very same arrays.

Every generator is a pure function of its arguments (NumPy PCG64 seeded
with ``seed``), returns C-ordered arrays of shape ``(N, n_1, ..., n_d)``,
and yields the stream one increment at a time.

Streams
-------
``smooth_separable``  sum of separable products of random cosines plus
                      Gaussian noise (16x16x3, one tensor per increment).
``video``             240x320x3 frames: a fixed separable background plus
                      Gaussian blobs moving on reflected linear paths plus
                      noise (video-shaped, like the gameplay frames).
``fourier_field``     64^3 x 3 snapshots of a random Fourier field whose
                      phases advance linearly in time (simulation-shaped).
``tt_lowrank``        an exactly low-rank stream: random TT-cores with given
                      TT-ranks, the last core supplying one column per tensor
                      (the synthetic stream of the TT-FOA comparison, App. B).
``graded``            sums of rank-1 terms whose weights fall geometrically
                      (a spectrum spanning many decades, for tolerances far
                      below the square root of the unit roundoff).
"""
from __future__ import annotations

import math
from typing import Iterator, Sequence

import numpy as np

__all__ = [
    "cosine_factor",
    "smooth_separable_stream",
    "video_stream",
    "fourier_field_stream",
    "device_separable",
    "tt_lowrank_stream",
    "graded_stream",
    "serving_trace",
    "CONFIGS",
]


def cosine_factor(rng: np.random.Generator, n: int) -> np.ndarray:
    """A smooth random 1-D profile cos(pi*w*t/(n-1) + phi), w~U(0,3), phi~U(0,2pi)."""
    w = rng.uniform(0.0, 3.0)
    phi = rng.uniform(0.0, 2.0 * math.pi)
    t = np.arange(n, dtype=np.float64)
    return np.cos(math.pi * w * t / max(n - 1, 1) + phi)


def _separable_sum(rng: np.random.Generator, dims: Sequence[int], terms: int) -> np.ndarray:
    out = np.zeros(tuple(dims), dtype=np.float64)
    for _ in range(terms):
        w = rng.standard_normal()
        term = np.asarray(w, dtype=np.float64)
        for n in dims:
            term = np.multiply.outer(term, cosine_factor(rng, n))
        out += term
    return out


def smooth_separable_stream(
    n_tensors: int = 100,
    dims: Sequence[int] = (16, 16, 3),
    terms: int = 5,
    noise: float = 1e-3,
    batch: int = 1,
    seed: int = 0,
    dtype=np.float64,
) -> Iterator[np.ndarray]:
    """Each tensor: sum of ``terms`` separable products of cosine profiles
    (weights N(0,1), factors redrawn for every tensor) plus N(0, noise^2)."""
    rng = np.random.default_rng(seed)
    done = 0
    while done < n_tensors:
        nb = min(batch, n_tensors - done)
        out = np.empty((nb,) + tuple(dims), dtype=np.float64)
        for b in range(nb):
            out[b] = _separable_sum(rng, dims, terms)
            out[b] += noise * rng.standard_normal(tuple(dims))
        done += nb
        yield out.astype(dtype, copy=False)


def _reflect(p: np.ndarray, length: float) -> np.ndarray:
    """Fold positions onto [0, length] (a ball bouncing between the borders)."""
    q = np.mod(p, 2.0 * length)
    return np.where(q > length, 2.0 * length - q, q)


def video_stream(
    n_frames: int = 2048,
    batch: int = 32,
    height: int = 240,
    width: int = 320,
    channels: int = 3,
    background_terms: int = 8,
    blobs: int = 4,
    blob_sigma: float = 12.0,
    noise: float = 1e-2,
    seed: int = 0,
    dtype=np.float32,
) -> Iterator[np.ndarray]:
    """Video-shaped frames (H, W, C): fixed rank-``background_terms`` separable
    background, ``blobs`` Gaussian blobs (std ``blob_sigma`` px, colour ~N(0,1)^C)
    moving with speed ~U(0.5, 2) px/frame in a uniform direction and bouncing
    off the borders, plus N(0, noise^2) pixel noise."""
    rng = np.random.default_rng(seed)
    bg = _separable_sum(rng, (height, width, channels), background_terms)
    colour = rng.standard_normal((blobs, channels))
    p0 = np.stack([rng.uniform(0, height - 1, blobs), rng.uniform(0, width - 1, blobs)], 1)
    speed = rng.uniform(0.5, 2.0, blobs)
    ang = rng.uniform(0.0, 2.0 * math.pi, blobs)
    vel = np.stack([speed * np.cos(ang), speed * np.sin(ang)], 1)
    xs = np.arange(height, dtype=np.float64)
    ys = np.arange(width, dtype=np.float64)
    done = 0
    while done < n_frames:
        nb = min(batch, n_frames - done)
        out = np.empty((nb, height, width, channels), dtype=np.float64)
        for b in range(nb):
            t = float(done + b)
            frame = bg.copy()
            cx = _reflect(p0[:, 0] + vel[:, 0] * t, height - 1)
            cy = _reflect(p0[:, 1] + vel[:, 1] * t, width - 1)
            for m in range(blobs):
                gx = np.exp(-0.5 * ((xs - cx[m]) / blob_sigma) ** 2)
                gy = np.exp(-0.5 * ((ys - cy[m]) / blob_sigma) ** 2)
                frame += np.multiply.outer(np.multiply.outer(gx, gy), colour[m])
            out[b] = frame
        out += noise * rng.standard_normal(out.shape)
        done += nb
        yield out.astype(dtype, copy=False)


def _fourier_modes(rng, n_modes, kmax, components):
    ks = []
    while len(ks) < n_modes:
        k = rng.integers(-kmax, kmax + 1, size=3)
        if np.any(k != 0):
            ks.append(k)
    ks = np.array(ks, dtype=np.int64)
    amp = rng.standard_normal((n_modes, components))
    omega = rng.uniform(-0.05, 0.05, n_modes)
    phase = rng.uniform(0.0, 2.0 * math.pi, (n_modes, components))
    return ks, amp, omega, phase


def fourier_field_stream(
    n_snapshots: int = 1000,
    batch: int = 16,
    grid: int = 64,
    components: int = 3,
    n_modes: int = 512,
    kmax: int = 8,
    decay: float = 2.0,
    seed: int = 0,
    dtype=np.float32,
) -> Iterator[np.ndarray]:
    """Simulation-shaped snapshots u_c(x, t) on a grid^3 periodic box:
    sum over ``n_modes`` integer wave vectors k in [-kmax, kmax]^3 \\ {0} of
    a_{m,c} |k|^-decay cos(2 pi k.x/grid + omega_m t + phi_{m,c}) with
    a ~ N(0,1), omega ~ U(-0.05, 0.05) rad/snapshot, phi ~ U(0, 2pi).
    Shape of one snapshot: (grid, grid, grid, components); for
    ``components == 1`` the trailing axis is dropped.  Evaluated exactly with
    an inverse FFT of the sparse spectrum."""
    rng = np.random.default_rng(seed)
    ks, amp, omega, phase = _fourier_modes(rng, n_modes, kmax, components)
    kn = np.sqrt((ks.astype(np.float64) ** 2).sum(1)) ** (-decay)
    idx = tuple((ks % grid).T)
    done = 0
    while done < n_snapshots:
        nb = min(batch, n_snapshots - done)
        shape = (nb, grid, grid, grid, components)
        out = np.empty(shape, dtype=np.float64)
        for b in range(nb):
            t = float(done + b)
            for c in range(components):
                spec = np.zeros((grid, grid, grid), dtype=np.complex128)
                coef = amp[:, c] * kn * np.exp(1j * (omega * t + phase[:, c]))
                np.add.at(spec, idx, coef)
                out[b, ..., c] = np.real(np.fft.ifftn(spec)) * grid ** 3
        done += nb
        if components == 1:
            out = out[..., 0]
        yield out.astype(dtype, copy=False)


class DeviceFourierField:
    """The field of ``fourier_field_stream`` (same seeded modes, same closed
    form) evaluated on a torch device, for streams too large to draw on the
    host: ``snapshots(t0, n)`` returns snapshots t0 .. t0+n-1 as a
    (n, grid, grid, grid[, components]) tensor of ``dtype`` on ``device``,
    computed as the host generator does (FP64 inverse FFT of the sparse
    spectrum, then rounded to ``dtype``).  It agrees with the host generator
    to FP64 rounding (FFT orderings differ), not bit for bit."""

    def __init__(self, grid=64, components=3, n_modes=512, kmax=8, decay=2.0, seed=0, device="cuda"):
        import torch
        rng = np.random.default_rng(seed)
        ks, amp, omega, phase = _fourier_modes(rng, n_modes, kmax, components)
        kn = np.sqrt((ks.astype(np.float64) ** 2).sum(1)) ** (-decay)
        self.grid, self.components, self.device = grid, components, device
        self.idx = tuple(torch.from_numpy(np.ascontiguousarray(a)).to(device) for a in (ks % grid).T)
        self.ak = torch.from_numpy(amp * kn[:, None]).to(device)          # (modes, components)
        self.omega = torch.from_numpy(omega).to(device)
        self.phase = torch.from_numpy(phase).to(device)

    def snapshots(self, t0, n, dtype=None):
        import torch
        dtype = torch.float32 if dtype is None else dtype
        g, C = self.grid, self.components
        out = torch.empty((n, g, g, g, C), dtype=dtype, device=self.device)
        spec = torch.zeros((g, g, g), dtype=torch.complex128, device=self.device)
        for b in range(n):
            t = float(t0 + b)
            for c in range(C):
                spec.zero_()
                coef = self.ak[:, c] * torch.exp(1j * (self.omega * t + self.phase[:, c]))
                spec.index_put_(self.idx, coef, accumulate=True)
                out[b, ..., c] = (torch.fft.ifftn(spec).real * g ** 3).to(dtype)
        return out[..., 0] if C == 1 else out


def device_separable(dims, n, generator, terms=5, noise=1e-3, dtype=None):
    """``n`` tensors of shape ``dims`` (3-way) drawn on the generator's torch
    device: each a sum of ``terms`` separable products of cosine profiles
    cos(pi w t + phi) (w ~ U[0, 3), phi ~ U[0, 2 pi), t on [0, 1]) with N(0,1)
    weights, plus N(0, noise^2); the serving mix's tensors."""
    import torch
    dtype = torch.float32 if dtype is None else dtype
    dev = generator.device
    parts = []
    for nn in dims:
        t = torch.arange(nn, device=dev, dtype=torch.float32) / max(nn - 1, 1)
        w = torch.rand((n, terms, 1), device=dev, generator=generator) * 3.0
        ph = torch.rand((n, terms, 1), device=dev, generator=generator) * (2 * math.pi)
        parts.append(torch.cos(math.pi * w * t + ph))
    wt = torch.randn((n, terms), device=dev, generator=generator)
    Y = (wt[:, :, None, None, None] * parts[0][:, :, :, None, None] * parts[1][:, :, None, :, None]
         * parts[2][:, :, None, None, :]).sum(1)
    Y += noise * torch.randn(Y.shape, device=dev, generator=generator)
    return Y.to(dtype)


def tt_lowrank_stream(
    dims: Sequence[int] = (10, 15, 20),
    ranks: Sequence[int] = (2, 3, 5),
    n_tensors: int = 500,
    batch: int = 1,
    seed: int = 0,
    dtype=np.float64,
) -> Iterator[np.ndarray]:
    """Exactly low-rank stream: random Gaussian TT-cores G_i (r_{i-1}, n_i, r_i)
    with r_0 = 1 and the given inner ranks r_1..r_d, and a Gaussian last core
    (r_d, n_tensors) whose columns generate the tensors one by one."""
    rng = np.random.default_rng(seed)
    d = len(dims)
    rr = [1] + list(ranks)
    cores = [rng.standard_normal((rr[i], dims[i], rr[i + 1])) for i in range(d)]
    last = rng.standard_normal((rr[d], n_tensors))
    basis = cores[0].reshape(dims[0], rr[1])
    for i in range(1, d):
        basis = basis @ cores[i].reshape(rr[i], dims[i] * rr[i + 1])
        basis = basis.reshape(-1, rr[i + 1])
    basis = basis.reshape(tuple(dims) + (rr[d],))
    done = 0
    while done < n_tensors:
        nb = min(batch, n_tensors - done)
        cols = last[:, done:done + nb]
        out = np.moveaxis(np.tensordot(basis, cols, axes=([d], [0])), -1, 0)
        done += nb
        yield np.ascontiguousarray(out).astype(dtype, copy=False)


def graded_stream(
    dims: Sequence[int],
    n_terms: int = 12,
    ratio: float = 1.0 / 30.0,
    n_batches: int = 3,
    batch: int = 2,
    seed: int = 0,
) -> Iterator[np.ndarray]:
    """Sum of n_terms rank-1 terms f_j1 x ... x f_jd (Gaussian factors drawn
    once) with weights ratio**j, each tensor of an increment taking its own
    N(0,1) coefficient per term: every unfolding has a geometrically graded
    spectrum.  FP64."""
    rng = np.random.default_rng(seed)
    terms = []
    for _ in range(n_terms):
        t = rng.standard_normal(dims[0])
        for n in dims[1:]:
            t = np.multiply.outer(t, rng.standard_normal(n))
        terms.append(t)
    for _ in range(n_batches):
        Y = np.zeros((batch,) + tuple(dims))
        for j, t in enumerate(terms):
            a = rng.standard_normal(batch).reshape((batch,) + (1,) * len(dims))
            Y += (ratio ** j) * a * t[None]
        yield Y


def serving_trace(
    n_streams: int = 256,
    rate: float = 2000.0,
    duration: float = 60.0,
    max_increment: int = 64,
    seed: int = 0,
):
    """Arrival trace for the many-stream serving mix: stream shapes drawn from
    {32x32x3, 64x64x3, 128x128x3, 32x32x32}, eps from {0.01, 0.05, 0.1},
    Poisson arrivals at total ``rate`` increments/s, each assigned to a
    uniformly drawn stream, increment sizes uniform on 1..max_increment.
    Returns (streams, arrivals): streams[s] = dict(dims, eps, kind, seed),
    arrivals = list of (time_s, stream_id, n_tensors)."""
    rng = np.random.default_rng(seed)
    shapes = [(32, 32, 3), (64, 64, 3), (128, 128, 3), (32, 32, 32)]
    epss = [0.01, 0.05, 0.1]
    streams = []
    for s in range(n_streams):
        dims = shapes[int(rng.integers(len(shapes)))]
        kind = "separable" if (dims[2] != 3 or rng.uniform() < 0.5) else "video"
        streams.append(dict(dims=dims, eps=epss[int(rng.integers(3))], kind=kind,
                            seed=int(rng.integers(1 << 31))))
    t = 0.0
    arrivals = []
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            break
        arrivals.append((t, int(rng.integers(n_streams)), int(rng.integers(1, max_increment + 1))))
    return streams, arrivals


# Workload table: name -> (dims, eps, stream factory kwargs).  Sizes follow the
# paper's experiments in kind (video frames, 3-D simulation snapshots) with
# the shapes stated for the synthetic stand-ins.
CONFIGS = {
    "separable16": dict(dims=(16, 16, 3), eps=0.05, n=100, batch=1,
                        make=lambda seed=0, n=100, batch=1: smooth_separable_stream(n, (16, 16, 3), 5, 1e-3, batch, seed)),
    "video240": dict(dims=(240, 320, 3), eps=0.1, n=2048, batch=32,
                     make=lambda seed=0, n=2048, batch=32: video_stream(n, batch, seed=seed)),
    "field64": dict(dims=(64, 64, 64, 3), eps=0.01, n=1000, batch=16,
                    make=lambda seed=0, n=1000, batch=16: fourier_field_stream(n, batch, seed=seed)),
}
