"""Seeded slope telemetry of a two-layer frozen-flow atmosphere (input generator).

For training and judging the learned predictor the loop runs on geometric
slopes (no pixels): the slope of a subaperture is the mean phase gradient of
aosim.turbulence.geometric_slopes.  Frozen flow moves each layer's screen
rigidly, so the slope of every possible subaperture position is computed once
per screen (a *slope map*, from cumulative sums of edge phase differences with
the trapezoid weights) and a frame's slopes are gathered from the maps at the
subaperture corners shifted by v t; a shift that is not a whole number of
samples interpolates linearly between the two neighbouring maps' values, which
is the slope of the linearly interpolated phase.

Two layers (ground 8 m/s along +x carrying 70 % of the turbulence, 20 m/s
along +y carrying 30 %), r0 = 0.15 m and L0 = 25 m overall, 1 cm sampling,
1 kHz frames.  Every segment of frames uses its own pair of non-periodic-
looking screens (rectangular periodic FFT screens longer than the travel of a
segment); segments are seeded by (config, segment) so training and test sets
use disjoint seeds.  Runs on a torch device (the GPU when present).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import torch

from .scenario import ROOT_SEED

SEED_KEY = 7           # spawn-key component of telemetry screens


@dataclass(frozen=True)
class Layers:
    speeds: tuple = (8.0, 20.0)          # m/s
    directions: tuple = ((1.0, 0.0), (0.0, 1.0))
    weights: tuple = (0.7, 0.3)
    r0: float = 0.15
    L0: float = 25.0
    delta: float = 0.01                  # m
    rate: float = 1000.0                 # Hz
    noise_px: float = 0.05               # slope measurement noise (px rms)


def screen(ny: int, nx: int, delta: float, r0: float, L0: float, seed: tuple, device) -> torch.Tensor:
    """float32 periodic von Karman screen [ny, nx] (rad), seeded by a spawn key.

    The Gaussian draws come from a generator on ``device`` (seeded from the
    spawn key), so they are reproducible for a given device type and torch
    build."""
    device = torch.device(device)
    g = torch.Generator(device=device)
    g.manual_seed(int(np.random.SeedSequence(ROOT_SEED, spawn_key=seed).generate_state(1)[0]))
    fy = torch.fft.fftfreq(ny, d=delta, dtype=torch.float64, device=device)
    fx = torch.fft.fftfreq(nx, d=delta, dtype=torch.float64, device=device)
    f2 = fy[:, None] ** 2 + fx[None, :] ** 2
    # von Karman phase PSD (as aosim.turbulence.von_karman_psd), evaluated on the device
    psd = 0.023 * r0 ** (-5.0 / 3.0) * (f2 + 1.0 / (L0 * L0)) ** (-11.0 / 6.0)
    psd[0, 0] = 0.0
    amp = torch.sqrt(psd) * math.sqrt(1.0 / (ny * delta) * 1.0 / (nx * delta))
    re = torch.randn((ny, nx), generator=g, dtype=torch.float64, device=device)
    im = torch.randn((ny, nx), generator=g, dtype=torch.float64, device=device)
    c = torch.complex(re * amp, im * amp)
    return (torch.fft.ifft2(c) * (ny * nx)).real.to(torch.float32)


def slope_maps(phi: torch.Tensor, m: int) -> tuple[torch.Tensor, torch.Tensor]:
    """(Gx, Gy) [ny - m, nx - m]: slopes (px) of the subaperture with top-left sample (y0, x0)."""
    p = phi.to(torch.float64)
    dx = p[:, m:] - p[:, :-m]                        # phase difference across a subaperture, along x
    dy = p[m:, :] - p[:-m, :]
    def trap(d, axis):                               # sum_{i=0..m} w_i d[y0 + i], w_0 = w_m = 1/2
        c = torch.cumsum(d, dim=axis)
        z = torch.zeros_like(d.narrow(axis, 0, 1))
        c = torch.cat([z, c], dim=axis)
        n = d.shape[axis] - m
        s = c.narrow(axis, m + 1, n) - c.narrow(axis, 0, n)
        return s - 0.5 * (d.narrow(axis, 0, n) + d.narrow(axis, m, n))
    gx = trap(dx, 0)[:, : dx.shape[1] - m] / (m * math.pi)
    gy = trap(dy, 1)[: dy.shape[0] - m, :] / (m * math.pi)
    return gx.to(torch.float32), gy.to(torch.float32)


class Telemetry:
    """Open-loop slope sequences of a subaperture mask under the two layers."""

    def __init__(self, mask: np.ndarray, pitch: float, config_index: int, layers: Layers = Layers(),
                 device=None):
        self.layers = layers
        self.device = torch.device(device if device is not None else ("cuda" if torch.cuda.is_available() else "cpu"))
        self.m = int(round(pitch / layers.delta))
        sy, sx = np.nonzero(mask)
        self.sy = torch.from_numpy(sy * self.m).to(self.device)
        self.sx = torch.from_numpy(sx * self.m).to(self.device)
        self.n_sub = mask.shape[0]
        self.config_index = config_index

    def segment(self, seg: int, n_frames: int) -> torch.Tensor:
        """float32 [n_frames, 2 n_valid] open-loop slopes (px) of segment `seg` (x block, then y block)."""
        L = self.layers
        span = self.n_sub * self.m + 1
        out = torch.zeros((n_frames, 2 * self.sy.numel()), dtype=torch.float32, device=self.device)
        t = torch.arange(n_frames, dtype=torch.float64, device=self.device)
        for i, (v, d, w) in enumerate(zip(L.speeds, L.directions, L.weights)):
            travel = v / L.rate / L.delta * n_frames
            ny = 1 << max(10, math.ceil(math.log2(span + abs(d[1]) * travel + 2)))
            nx = 1 << max(10, math.ceil(math.log2(span + abs(d[0]) * travel + 2)))
            r0_i = L.r0 * w ** (-3.0 / 5.0)
            phi = screen(ny, nx, L.delta, r0_i, L.L0, (self.config_index, SEED_KEY, seg, i), self.device)
            gx, gy = slope_maps(phi, self.m)
            shift = v / L.rate / L.delta * t                     # samples travelled at frame k
            # the screen moves along +d: the pupil sees it displaced by -d shift
            oy = (abs(d[1]) * travel - d[1] * shift)             # >= 0
            ox = (abs(d[0]) * travel - d[0] * shift)
            for g, blk in ((gx, 0), (gy, 1)):
                y = self.sy[None, :].to(torch.float64) + oy[:, None]
                x = self.sx[None, :].to(torch.float64) + ox[:, None]
                y0, x0 = torch.floor(y), torch.floor(x)
                fy, fx = (y - y0).to(torch.float32), (x - x0).to(torch.float32)
                y0, x0 = y0.long(), x0.long()
                v00 = g[y0, x0]
                v01 = g[y0, x0 + 1]
                v10 = g[y0 + 1, x0]
                v11 = g[y0 + 1, x0 + 1]
                val = (1 - fy) * ((1 - fx) * v00 + fx * v01) + fy * ((1 - fx) * v10 + fx * v11)
                nv = self.sy.numel()
                out[:, blk * nv:(blk + 1) * nv] += val
        return out

    def noise(self, seg: int, n_frames: int, n_slopes: int) -> torch.Tensor:
        """float32 [n_frames, n_slopes] Gaussian slope noise of segment `seg` (device generator)."""
        g = torch.Generator(device=self.device)
        g.manual_seed(int(np.random.SeedSequence(ROOT_SEED, spawn_key=(self.config_index, SEED_KEY + 1, seg))
                          .generate_state(1)[0]))
        return torch.randn((n_frames, n_slopes), generator=g, device=self.device) * self.layers.noise_px


def kl_basis(samples, n_modes: int) -> np.ndarray:
    """float32 [n_modes, n_slopes]: leading eigenvectors (orthonormal rows) of
    the slope covariance of samples [F, n_slopes], from the singular value
    decomposition of the centred samples (float64, host NumPy; offline work)."""
    x = samples.detach().cpu().numpy() if isinstance(samples, torch.Tensor) else np.asarray(samples)
    x = x.astype(np.float64)
    x = x - x.mean(axis=0, keepdims=True)
    _, _, vt = np.linalg.svd(x, full_matrices=False)      # rows: eigenvectors, eigenvalues descending
    return np.ascontiguousarray(vt[:n_modes], dtype=np.float32)
