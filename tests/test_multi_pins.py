"""Multi-sensor composition (oracle) and the seeded multi-sensor geometry; no GPU."""
import numpy as np
import pytest

import oracle
from aosim import ELT, Scenario, dm, geometry
from aosim.multi import ELT_MULTI, TINY_MULTI, MultiScenario


def _sensor(rng, n_sub, n_pix, level=100.0):
    mask = geometry.subaperture_mask(n_sub, 0.0)
    h = n_sub * n_pix
    frame = rng.integers(90, 400, size=(h, h)).astype(np.uint16)
    dark = np.full((h, h), level, np.float32)
    flat = (1.0 + 0.125 * rng.integers(-2, 3, size=(h, h))).astype(np.float32)
    return mask, n_pix, frame, dark, flat


def test_one_sensor_is_the_single_sensor_frame():
    rng = np.random.default_rng(1)
    mask, n, frame, dark, flat = _sensor(rng, 6, 8)
    nv = int(mask.sum())
    R = rng.standard_normal((7, 2 * nv))
    c0 = rng.standard_normal(7)
    a = oracle.rtc_frame(frame, mask, n, dark, flat, 3.0, R, c0, 0.4, 0.9)
    b = oracle.rtc_frame_multi([frame], [(mask, n)], [dark], [flat], [3.0], R, c0, 0.4, 0.9)
    for k in a:
        assert np.array_equal(a[k], b[k])


def test_sensors_concatenate_their_own_slope_vectors_in_order():
    rng = np.random.default_rng(2)
    s1 = _sensor(rng, 6, 8)
    s2 = _sensor(rng, 3, 6)
    s3 = _sensor(rng, 4, 10)
    sens = [s1, s2, s3]
    nv = [int(s[0].sum()) for s in sens]
    n_s = 2 * sum(nv)
    R = rng.standard_normal((5, n_s))
    ref = rng.standard_normal(n_s).astype(np.float32)
    thr = [3.0, 5.0, 0.0]
    out = oracle.rtc_frame_multi([s[2] for s in sens], [(s[0], s[1]) for s in sens], [s[3] for s in sens],
                                 [s[4] for s in sens], thr, R, np.zeros(5), 0.5, ref=ref)
    parts, counts = [], []
    for (mask, n, frame, dark, flat), T in zip(sens, thr):
        s_w, c_w = oracle.sensor_slopes(frame, mask, n, dark, flat, T)
        # each sensor's own vector: its x block then its y block
        assert s_w.shape == (2 * int(mask.sum()),)
        parts.append(s_w)
        counts.append(c_w)
    s = np.concatenate(parts) - ref.astype(np.float64)
    assert np.array_equal(out["slopes"], s)
    assert np.array_equal(out["counts"], np.concatenate(counts))
    # a = R s by brute force, and the integrator with c0 = 0
    a = np.array([sum(R[r, j] * s[j] for j in range(n_s)) for r in range(5)])
    assert np.allclose(out["recon"], a, rtol=1e-12, atol=1e-12)
    assert np.allclose(out["cmd"], 0.5 * a, rtol=1e-12, atol=1e-12)
    # the second sensor's block sits after the first sensor's 2 nv[0] slopes
    s2_own, _ = oracle.sensor_slopes(s2[2], s2[0], s2[1], s2[3], s2[4], 5.0)
    assert np.array_equal(out["slopes"][2 * nv[0]:2 * nv[0] + 2 * nv[1]],
                          s2_own - ref[2 * nv[0]:2 * nv[0] + 2 * nv[1]].astype(np.float64))


def test_multi_geometry_counts():
    t = MultiScenario(TINY_MULTI)
    assert t.n_valid == [80, 80, 12] and t.n_slopes == 344
    assert [a.shape[0] for a in t.actuators] == [97, 37]
    e = MultiScenario(ELT_MULTI)
    # six 74x74 sensors with the 28 % obstruction (3972 each) and three 16x16 (192 each)
    assert e.n_valid == [3972] * 6 + [192] * 3 and e.n_slopes == 48816
    assert [a.shape[0] for a in e.actuators] == [4421, 577]


def test_on_axis_ground_dm_block_is_the_single_sensor_interaction():
    # a sensor on axis sees the ground DM exactly as the single-sensor model does
    sc = Scenario(ELT)
    boxes = geometry.subaperture_boxes(sc.mask, sc.cfg.pitch)
    D = dm.interaction_matrix(boxes, sc.actuators, dm.influence_width(sc.cfg.pitch, sc.cfg.coupling))
    assert np.array_equal(D, sc.interaction)
    t = MultiScenario(TINY_MULTI)
    D3 = t.interaction[2 * 160:, :97]                 # third sensor (on axis), ground DM columns
    m3 = t.masks[2]
    ref = dm.interaction_matrix(geometry.subaperture_boxes(m3, t.pitch(2)), t.actuators[0],
                                dm.influence_width(TINY_MULTI.dms[0].pitch, TINY_MULTI.coupling))
    assert np.array_equal(D3, ref)


def test_altitude_dm_shift_follows_the_line_of_sight():
    # moving the altitude DM's actuators by h theta is the same as shifting the sensor's boxes by -h theta
    t = MultiScenario(TINY_MULTI)
    w = 0
    d = TINY_MULTI.dms[1]
    theta = np.array(TINY_MULTI.sensors[w].direction)
    boxes = geometry.subaperture_boxes(t.masks[w], t.pitch(w))
    shifted = boxes + np.array([theta[0], theta[0], theta[1], theta[1]]) * d.altitude
    ref = dm.interaction_matrix(shifted, t.actuators[1], dm.influence_width(d.pitch, TINY_MULTI.coupling))
    got = t.interaction[:160, 97:]
    assert np.allclose(got, ref, rtol=0, atol=1e-12)


def test_tiny_multi_closed_loop_converges():
    from _closedloop import oracle_closed_loop_multi
    sc = MultiScenario(TINY_MULTI)
    sets, ref = oracle_closed_loop_multi(sc, 40)
    rms = np.sqrt(np.mean(ref["slopes"] ** 2, axis=1))
    assert sets.shape == (40, sum(sc.frame_side(w) ** 2 for w in range(3)))
    assert rms[-10:].mean() < 0.5 * rms[0]
