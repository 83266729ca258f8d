"""Seeded synthetic multi-sensor workloads: several Shack-Hartmann sensors of
uneven size, looking in different directions, reconstructed together onto two
deformable mirrors (ground and altitude) by one control matrix.

``tiny-multi``: D = 2 m; two 10 x 10 sensors of 8 x 8 px and one 4 x 4 sensor
of 6 x 6 px; ground DM 11 x 11 Fried (97 actuators) and a 6 km DM.

``elt-multi``: D = 39.22 m, 28 % obstruction; six 74 x 74 sensors of 10 x 10 px
(3972 subapertures each) on a ring of 45 arcsec and three 16 x 16 sensors of
6 x 6 px (192 subapertures each) on a ring of 60 arcsec: 48,816 slopes.  Ground
DM 75 x 75 Fried (4421 actuators) and an 8 km DM of 26 x 26 pitches over the
metapupil; the control matrix is stored in BF16 by the controller.

Turbulence: two von Karman layers (ground 70 %, altitude 30 % of the r0 = 0.15 m
turbulence), frozen flow at 10 m/s along +x (ground) and 20 m/s along +y
(altitude), 1 cm sampling, periodic screens; a sensor looking in direction
theta sees the altitude layer and the altitude DM shifted by h theta.
Detector model as the single-sensor workloads.  The control matrix is the
Tikhonov inverse of the stacked interaction matrix (sensor rows in order,
each sensor's x block then y block; ground DM columns, then altitude DM
columns).  Seeds: ``SeedSequence(180507254)`` with spawn keys
(config, component, sensor[, frame]).
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from functools import cached_property

import numpy as np

from . import dm, geometry, shwfs, turbulence
from .scenario import ROOT_SEED

ARCSEC = math.pi / (180.0 * 3600.0)
_COMPONENT = {"screen": 0, "photon": 1, "read": 2, "dark": 3, "flat": 4}


@dataclass(frozen=True)
class SensorSpec:
    n_sub: int
    n_pix: int
    obscuration: float
    direction: tuple          # (theta_x, theta_y) in radians
    threshold: float = 3.0
    flux: float = 500.0


@dataclass(frozen=True)
class DmSpec:
    n_sub: int                # Fried grid of n_sub + 1 actuators per side, radius (n_sub + 1) / 2 pitches
    pitch: float              # metres
    altitude: float           # metres


@dataclass(frozen=True)
class MultiConfig:
    name: str
    index: int
    diameter: float
    sensors: tuple
    dms: tuple
    layer_altitudes: tuple = (0.0, None)      # ground, then the altitude DM's conjugate
    layer_weights: tuple = (0.7, 0.3)
    layer_speeds: tuple = ((1, 0), (0, 2))    # samples per frame (x, y) at 1 cm, 1 kHz
    r0: float = 0.15
    L0: float = 25.0
    coupling: float = 0.3
    alpha: float = 1e-3
    sigma_px: float = 1.2
    read_noise: float = 1.0
    gain: float = 0.4
    leak: float = 1.0
    delta: float = 0.01                       # phase-screen sampling, metres
    screen_n: int = 4096
    frames: int = 5000


def _ring(radius_arcsec: float, count: int, start_deg: float = 0.0):
    r = radius_arcsec * ARCSEC
    return tuple((r * math.cos(math.radians(start_deg + 360.0 * i / count)),
                  r * math.sin(math.radians(start_deg + 360.0 * i / count))) for i in range(count))


TINY_MULTI = MultiConfig(
    "tiny-multi", 2, diameter=2.0,
    sensors=tuple(SensorSpec(10, 8, 0.0, d) for d in _ring(20.0, 2)) + (SensorSpec(4, 6, 0.0, (0.0, 0.0)),),
    dms=(DmSpec(10, 0.2, 0.0), DmSpec(6, 0.45, 6000.0)),
    screen_n=1024, frames=200)

ELT_MULTI = MultiConfig(
    "elt-multi", 3, diameter=39.22,
    sensors=tuple(SensorSpec(74, 10, 0.28, d) for d in _ring(45.0, 6))
    + tuple(SensorSpec(16, 6, 0.28, d, flux=2000.0) for d in _ring(60.0, 3, 30.0)),
    dms=(DmSpec(74, 39.22 / 74, 0.0), DmSpec(26, (39.22 + 2 * 8000.0 * 60.0 * ARCSEC) / 26, 8000.0)),
    frames=5000)

MULTI_CONFIGS = {"tiny-multi": TINY_MULTI, "elt-multi": ELT_MULTI}


def rng_for(cfg: MultiConfig, component: str, sensor: int = 0, frame: int | None = None) -> np.random.Generator:
    key = (cfg.index, _COMPONENT[component], int(sensor)) + (() if frame is None else (int(frame),))
    return np.random.default_rng(np.random.SeedSequence(ROOT_SEED, spawn_key=key))


class MultiScenario:
    """Lazily built geometry, matrices, calibration maps and frames of a multi-sensor config."""

    def __init__(self, cfg: MultiConfig):
        self.cfg = cfg

    # ---- geometry ---------------------------------------------------------
    @cached_property
    def masks(self) -> list:
        return [geometry.subaperture_mask(s.n_sub, s.obscuration) for s in self.cfg.sensors]

    @property
    def sensors(self) -> list:
        """(mask, n_pix) per sensor, the form the controller and the oracle take."""
        return [(m, s.n_pix) for m, s in zip(self.masks, self.cfg.sensors)]

    @property
    def n_valid(self) -> list:
        return [int(m.sum()) for m in self.masks]

    @property
    def n_slopes(self) -> int:
        return 2 * sum(self.n_valid)

    def pitch(self, w: int) -> float:
        return self.cfg.diameter / self.cfg.sensors[w].n_sub

    def frame_side(self, w: int) -> int:
        s = self.cfg.sensors[w]
        return s.n_sub * s.n_pix

    @cached_property
    def actuators(self) -> list:
        return [geometry.actuator_positions(d.n_sub, d.pitch) for d in self.cfg.dms]

    @property
    def n_act(self) -> int:
        return sum(a.shape[0] for a in self.actuators)

    @property
    def thresholds(self) -> list:
        return [s.threshold for s in self.cfg.sensors]

    # ---- matrices ---------------------------------------------------------
    @cached_property
    def interaction(self) -> np.ndarray:
        """float64 ``[n_slopes, n_act]``: sensor blocks of rows, DM blocks of columns."""
        rows = []
        for w, (mask, spec) in enumerate(zip(self.masks, self.cfg.sensors)):
            boxes = geometry.subaperture_boxes(mask, self.pitch(w))
            cols = []
            for d, acts in zip(self.cfg.dms, self.actuators):
                shift = np.array([d.altitude * spec.direction[0], d.altitude * spec.direction[1]])
                cols.append(dm.interaction_matrix(boxes, acts - shift[None, :],
                                                  dm.influence_width(d.pitch, self.cfg.coupling)))
            rows.append(np.concatenate(cols, axis=1))
        return np.concatenate(rows, axis=0)

    @cached_property
    def control_matrix(self) -> np.ndarray:
        """FP32 ``[n_act, n_slopes]``."""
        return np.ascontiguousarray(dm.tikhonov_control_matrix(self.interaction, self.cfg.alpha)
                                    .astype(np.float32))

    # ---- detector calibration (frame-set layout) --------------------------
    @cached_property
    def _maps(self) -> list:
        out = []
        for w in range(len(self.cfg.sensors)):
            h = self.frame_side(w)
            dark = shwfs.calibration_maps(h, h, rng_for(self.cfg, "dark", w))[0]
            flat = shwfs.calibration_maps(h, h, rng_for(self.cfg, "flat", w))[1]
            out.append((dark, flat))
        return out

    @property
    def darks(self) -> list:
        return [d for d, _ in self._maps]

    @property
    def flats(self) -> list:
        return [f for _, f in self._maps]

    @property
    def dark_set(self) -> np.ndarray:
        return np.concatenate([d.ravel() for d in self.darks])

    @property
    def flat_set(self) -> np.ndarray:
        return np.concatenate([f.ravel() for f in self.flats])

    # ---- turbulence --------------------------------------------------------
    @cached_property
    def screens(self) -> list:
        out = []
        for i, wgt in enumerate(self.cfg.layer_weights):
            r0_i = self.cfg.r0 * wgt ** (-3.0 / 5.0)
            a, _ = turbulence.phase_screen_pair(self.cfg.screen_n, self.cfg.delta, r0_i, self.cfg.L0,
                                                rng_for(self.cfg, "screen", i))
            out.append(a)
        return out

    def _layer_altitude(self, i: int) -> float:
        h = self.cfg.layer_altitudes[i]
        return self.cfg.dms[-1].altitude if h is None else h

    def turbulence_slopes(self, w: int, k: int) -> np.ndarray:
        """Open-loop slopes (px) of sensor w at frame k, summed over the layers."""
        spec = self.cfg.sensors[w]
        m = int(round(self.pitch(w) / self.cfg.delta))
        npts = spec.n_sub * m + 1
        n = self.cfg.screen_n
        s = np.zeros(2 * self.n_valid[w])
        for i, screen in enumerate(self.screens):
            h = self._layer_altitude(i)
            vx, vy = self.cfg.layer_speeds[i]
            ox = int(round(h * spec.direction[0] / self.cfg.delta)) - vx * k
            oy = int(round(h * spec.direction[1] / self.cfg.delta)) - vy * k
            cols = (np.arange(npts) + ox) % n
            rows = (np.arange(npts) + oy) % n
            s += turbulence.geometric_slopes(screen[np.ix_(rows, cols)], self.masks[w], m)
        # the geometric slope is in pixels of a subaperture of this sensor's pitch
        return s

    def all_turbulence_slopes(self, k: int) -> np.ndarray:
        return np.concatenate([self.turbulence_slopes(w, k) for w in range(len(self.cfg.sensors))])

    def residual_slopes(self, k: int, cmd: np.ndarray | None) -> np.ndarray:
        s = self.all_turbulence_slopes(k)
        if cmd is not None:
            s = s - self.interaction @ np.asarray(cmd, dtype=np.float64)
        return s

    # ---- frames -------------------------------------------------------------
    def frames(self, k: int, slopes_px: np.ndarray) -> list:
        """uint16 frame of every sensor for frame index k with the given concatenated slopes."""
        out, base = [], 0
        for w, spec in enumerate(self.cfg.sensors):
            nv = self.n_valid[w]
            sx, sy = slopes_px[base:base + nv], slopes_px[base + nv:base + 2 * nv]
            base += 2 * nv
            exp = shwfs.spot_expectation(sx, sy, spec.n_pix, self.cfg.sigma_px, spec.flux)
            out.append(shwfs.detector_frame(exp, self.masks[w], spec.n_pix, self.darks[w], self.flats[w],
                                            self.cfg.read_noise, rng_for(self.cfg, "photon", w, k),
                                            rng_for(self.cfg, "read", w, k)))
        return out

    def frame_set(self, k: int, slopes_px: np.ndarray) -> np.ndarray:
        """The sensors' frames of frame k back to back (uint16, one dimension)."""
        return np.concatenate([f.ravel() for f in self.frames(k, slopes_px)])
