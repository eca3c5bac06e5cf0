"""Pins of the source, detector and time-bin set-up, the time step rule and
the paper's printed numbers (Sec. 2.2, Sec. 3.1, Table 1)."""
import json
import math
import os

import numpy as np
import pytest

from oracle import angles, medium, setup, solve
from paper_2105_01028_amd import workloads as W


def test_paper_time_steps(golden_dir):
    """dt = courant * dx / (c0 / n) reproduces the printed steps: 1.3e-4 ns for
    the 1-D vacuum test and 4.0e-4 ns for the phantom, and 3.5 ns of phantom
    time takes the printed ~8680 steps."""
    ref = json.load(open(os.path.join(golden_dir, "paper_numbers.json")))
    for key in ("vacuum_pulse_test", "phantom_run"):
        r = ref[key]
        dx_mm = r["box_cm"] * 10.0 / r["intervals"]
        dt_ps = r["courant"] * medium.time_step(dx_mm, np.array([r["n"]]))
        dt_ns = dt_ps * 1e-3
        assert float(f"{dt_ns:.{r['digits'] - 1}e}") == r["dt_ns"]
    r = ref["phantom_run"]
    dt_ps = r["courant"] * medium.time_step(r["box_cm"] * 10.0 / r["intervals"], np.array([r["n"]]))
    assert abs(r["duration_ns"] * 1e3 / dt_ps - r["steps"]) / r["steps"] < 0.002


def test_table1_phantom_coefficients(golden_dir):
    """Table 1 phantom at 1 mm voxels and Courant one: albedo and the share of
    light that survives one step without absorption."""
    t = json.load(open(os.path.join(golden_dir, "paper_numbers.json")))["phantom_table1"]
    mua, mus, n = t["mua_per_cm"] / 10, t["mus_per_cm"] / 10, t["n"]
    dt = medium.time_step(1.0, np.array([n]))
    a, b, om, ell = medium.collision_coefficients(np.array([mua]), np.array([mus]),
                                                   np.array([n]), dt)
    assert abs(ell[0] - 1.0) < 1e-15                 # Courant one: one voxel per step
    assert abs(om[0] - mus / (mua + mus)) < 1e-15    # Eq. (2)
    assert abs(a[0] - math.exp(-(mua + mus))) < 1e-15
    assert abs(a[0] + b[0] - (1 - (1 - om[0]) * (1 - a[0]))) < 1e-15


def test_detector_geometry_config1(golden_dir):
    ref = json.load(open(os.path.join(golden_dir, "detector_geometry.json")))["config1"]
    p = W.config1()
    assert p.det_face == ref["det_face"]
    assert p.det_i == ref["det_i"]
    assert p.det_j == ref["det_j"]
    d2 = angles.healpix_ring(2)
    assert setup.source_directions(d2, 15.0) == ref["source_dirs_nside2"]
    assert setup.detector_acceptance(d2, 4, 15.0) == ref["accept_top_face_nside2"]
    assert setup.detector_acceptance(d2, 1, 15.0) == ref["accept_xmax_face_nside2"]["indices"]
    assert setup.source_directions(angles.healpix_ring(4), 15.0) == ref["source_dirs_nside4"]
    assert setup.source_directions(angles.healpix_ring(8), 15.0) == ref["source_dirs_nside8"]
    shape = p.shape
    assert setup.detector_voxel(shape, 4, 10, 8) == (0 * 16 + 8) * 16 + 10
    assert setup.detector_voxel(shape, 1, 8, 6) == (6 * 16 + 8) * 16 + 15


def test_pulse_weights():
    dt = 4.6699
    q = setup.pulse_weights(200, dt, 20.0, 10.0, 1.0)
    assert abs(q.sum() - 1.0) < 1e-14
    assert np.all(q >= 0)
    mid = (np.arange(200) + 0.5) * dt
    mean = np.sum(q * mid)
    assert abs(mean - 20.0) < 0.05
    sigma = 10.0 / (2 * math.sqrt(2 * math.log(2)))
    var = np.sum(q * (mid - mean) ** 2)
    assert abs(var - (sigma ** 2 + dt ** 2 / 12)) < 0.2


@pytest.mark.parametrize("dt,bin_ps", [(4.6699, 1.0), (5.0035, 1.0), (0.4, 1.0), (3.0, 3.0)])
def test_rebin(dt, bin_ps):
    steps = 37
    nb = int(math.ceil(steps * dt / bin_ps)) + 2
    W_ = setup.rebin_matrix(steps, dt, bin_ps, nb)
    assert np.allclose(W_.sum(axis=1), 1.0, atol=1e-14)
    rng = np.random.default_rng(0)
    det = rng.uniform(size=(3, steps))
    y = det @ W_
    assert np.allclose(y.sum(axis=1), det.sum(axis=1), rtol=1e-14)
    # a step that lies inside one bin lands there whole
    for m in range(steps):
        j0, j1 = math.floor(m * dt / bin_ps), math.floor(((m + 1) * dt - 1e-12) / bin_ps)
        if j0 == j1:
            assert abs(W_[m, j0] - 1.0) < 1e-12


def test_phase_mode_requires_uniform_index():
    p = W.small_problem(steps=2, advance="phase")
    n = p.n.copy()
    n[0, 0, 0] = 1.0
    with pytest.raises(ValueError):
        solve.build(p.copy(n=n))


def test_time_step_limits_plane_speed():
    p = W.small_problem(steps=2)
    with pytest.raises(ValueError):
        solve.build(p.copy(dt_ps=10.0))
