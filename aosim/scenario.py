"""Seeded synthetic SCAO workloads: the two single-WFS configurations.

``tiny``: 10 x 10 subapertures of 8 x 8 px (80 x 80 frame), D = 2 m, no
obscuration -> 80 subapertures / 160 slopes, 11 x 11 Fried DM -> 97 actuators.

``elt``: 74 x 74 subapertures of 10 x 10 px (740 x 740 frame), D = 39.22 m
(pitch 0.53 m), 28 % central obstruction -> 3972 subapertures / 7944 slopes,
75 x 75 Fried DM -> 4421 actuators; FP32 control matrix 4421 x 7944.

Both: von Karman r0 = 0.15 m (500 nm), L0 = 25 m, frozen flow 10 m/s along +x
at 1 kHz on a 1 cm grid (one sample per frame), 500 photons per subaperture,
Gaussian spots sigma = 1.2 px, read noise 1 e-, dark ~ N(100, 2^2) ADU, flat ~
N(1, 0.02^2), threshold 3 ADU, integrator gain 0.4.

Random streams come from ``numpy.random.SeedSequence(180507254)`` with a
spawn key (config, component[, frame]) so any frame regenerates alone.
"""
from __future__ import annotations

from dataclasses import dataclass
from functools import cached_property

import numpy as np

from . import dm, geometry, shwfs, turbulence

ROOT_SEED = 180507254
_COMPONENT = {"screen": 0, "photon": 1, "read": 2, "dark": 3, "flat": 4, "misc": 5}


@dataclass(frozen=True)
class ScaoConfig:
    name: str
    index: int
    n_sub: int
    n_pix: int
    obscuration: float
    diameter: float          # metres
    samples_per_pitch: int   # phase-screen samples per subaperture pitch (1 cm grid)
    screen_n: int            # periodic screen size (samples)
    r0: float = 0.15
    L0: float = 25.0
    coupling: float = 0.3
    alpha: float = 1e-3
    flux: float = 500.0
    sigma_px: float = 1.2
    read_noise: float = 1.0
    threshold: float = 3.0
    gain: float = 0.4
    leak: float = 1.0
    frames: int = 1000

    @property
    def pitch(self) -> float:
        return self.diameter / self.n_sub

    @property
    def frame_side(self) -> int:
        return self.n_sub * self.n_pix


TINY = ScaoConfig("tiny-scao-10x10", 0, n_sub=10, n_pix=8, obscuration=0.0, diameter=2.0,
                  samples_per_pitch=20, screen_n=2048, frames=1000)
ELT = ScaoConfig("elt-scao-74x74", 1, n_sub=74, n_pix=10, obscuration=0.28, diameter=39.22,
                 samples_per_pitch=53, screen_n=4096, frames=10000)
CONFIGS = {"tiny": TINY, "elt": ELT}


def rng_for(cfg: ScaoConfig, component: str, frame: int | None = None) -> np.random.Generator:
    key = (cfg.index, _COMPONENT[component]) + (() if frame is None else (int(frame),))
    return np.random.default_rng(np.random.SeedSequence(ROOT_SEED, spawn_key=key))


class Scenario:
    """Lazily built geometry, matrices, calibration maps and frames of one config."""

    def __init__(self, cfg: ScaoConfig):
        self.cfg = cfg

    # ---- geometry ---------------------------------------------------------
    @cached_property
    def mask(self) -> np.ndarray:
        return geometry.subaperture_mask(self.cfg.n_sub, self.cfg.obscuration)

    @property
    def n_valid(self) -> int:
        return int(self.mask.sum())

    @cached_property
    def actuators(self) -> np.ndarray:
        return geometry.actuator_positions(self.cfg.n_sub, self.cfg.pitch)

    @property
    def n_act(self) -> int:
        return int(self.actuators.shape[0])

    # ---- matrices ---------------------------------------------------------
    @cached_property
    def interaction(self) -> np.ndarray:
        boxes = geometry.subaperture_boxes(self.mask, self.cfg.pitch)
        w = dm.influence_width(self.cfg.pitch, self.cfg.coupling)
        return dm.interaction_matrix(boxes, self.actuators, w)

    @cached_property
    def control_matrix(self) -> np.ndarray:
        """FP32 ``[n_act, 2 n_valid]`` row-major, the form handed to the controller."""
        return np.ascontiguousarray(dm.tikhonov_control_matrix(self.interaction, self.cfg.alpha)
                                    .astype(np.float32))

    # ---- detector calibration --------------------------------------------
    @cached_property
    def dark(self) -> np.ndarray:
        h = self.cfg.frame_side
        return shwfs.calibration_maps(h, h, rng_for(self.cfg, "dark"))[0]

    @cached_property
    def flat(self) -> np.ndarray:
        h = self.cfg.frame_side
        return shwfs.calibration_maps(h, h, rng_for(self.cfg, "flat"))[1]

    # ---- turbulence --------------------------------------------------------
    @cached_property
    def screen(self) -> np.ndarray:
        a, _ = turbulence.phase_screen_pair(self.cfg.screen_n, self.cfg.pitch / self.cfg.samples_per_pitch,
                                            self.cfg.r0, self.cfg.L0, rng_for(self.cfg, "screen"))
        return a

    def turbulence_slopes(self, k: int) -> np.ndarray:
        """Open-loop slopes (px) of frame k: the screen moved k samples along +x."""
        m = self.cfg.samples_per_pitch
        npts = self.cfg.n_sub * m + 1
        n = self.cfg.screen_n
        cols = (np.arange(npts) - k) % n
        rows = np.arange(npts) % n
        # only the samples on subaperture edges enter the slopes
        edge_cols = self.screen[np.ix_(rows, cols[::m])]
        edge_rows = self.screen[np.ix_(rows[::m], cols)]
        return turbulence.edge_slopes(edge_cols, edge_rows, self.mask, m)

    def residual_slopes(self, k: int, cmd: np.ndarray | None) -> np.ndarray:
        """Turbulence slopes minus the DM's slopes for commands ``cmd`` (None = open loop)."""
        s = self.turbulence_slopes(k)
        if cmd is not None:
            s = s - self.interaction @ np.asarray(cmd, dtype=np.float64)
        return s

    # ---- frames -------------------------------------------------------------
    def frame(self, k: int, slopes_px: np.ndarray) -> np.ndarray:
        """uint16 ``[H, W]`` raw frame for frame index k with the given residual slopes."""
        nv = self.n_valid
        exp = shwfs.spot_expectation(slopes_px[:nv], slopes_px[nv:], self.cfg.n_pix,
                                     self.cfg.sigma_px, self.cfg.flux)
        return shwfs.detector_frame(exp, self.mask, self.cfg.n_pix, self.dark, self.flat,
                                    self.cfg.read_noise, rng_for(self.cfg, "photon", k),
                                    rng_for(self.cfg, "read", k))

    def open_loop_frames(self, k0: int, count: int) -> np.ndarray:
        """uint16 ``[count, H, W]`` open-loop frames k0 .. k0 + count - 1."""
        h = self.cfg.frame_side
        out = np.empty((count, h, h), dtype=np.uint16)
        for i in range(count):
            out[i] = self.frame(k0 + i, self.turbulence_slopes(k0 + i))
        return out
