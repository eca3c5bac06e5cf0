"""Pins of the oracle's angular discretisation: HEALPix directions (Sec. 2.1),
the Henyey-Greenstein phase function (Eq. 11), the discrete phase matrix
(Eq. 12) and the Eq. (9) weights derived from Eqs. (7)-(8)."""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest
from scipy import integrate, optimize

from oracle import angles


@pytest.mark.parametrize("nside", [1, 2, 4, 8, 16])
def test_healpix_count_unit_and_balanced(nside):
    d = angles.healpix_ring(nside)
    assert d.shape == (12 * nside * nside, 3)
    assert np.allclose(np.linalg.norm(d, axis=1), 1.0, atol=1e-15)
    assert np.abs(d.sum(axis=0)).max() < 1e-12


def test_healpix_nside1_matches_hand_worked_centres(golden_dir):
    ref = json.load(open(os.path.join(golden_dir, "healpix_nside1.json")))
    d = angles.healpix_ring(1)
    for k, (z, phi_over_pi) in enumerate(ref["centres"]):
        phi = phi_over_pi * math.pi
        st = math.sqrt(1 - z * z)
        assert np.allclose(d[k], [st * math.cos(phi), st * math.sin(phi), z], atol=1e-15)


def test_healpix_nside2_second_moment_exact(golden_dir):
    ref = json.load(open(os.path.join(golden_dir, "healpix_nside1.json")))["nside2_sum_z2"]
    d = angles.healpix_ring(2)
    assert abs(np.sum(d[:, 2] ** 2) - float(Fraction(ref["num"], ref["den"]))) < 1e-13
    # not a spherical 2-design: <z^2> differs from 1/3
    assert abs(np.mean(d[:, 2] ** 2) * 3 - 0.9757) < 1e-3


@pytest.mark.parametrize("nside", [2, 4, 8])
def test_healpix_equal_area_rings(nside):
    """Equal area: the cap z > 2/3 holds 1/6 of the sphere's area, so N/6
    pixels, counting the ring on z = 2/3 as split evenly by its centre line."""
    d = angles.healpix_ring(nside)
    z = d[:, 2]
    strictly = np.sum(z > 2.0 / 3.0 + 1e-12)
    on = np.sum(np.abs(z - 2.0 / 3.0) < 1e-12)
    assert strictly + on / 2 == len(d) / 6
    # rings: 4i pixels in cap ring i, 4 nside in every belt ring
    zs, counts = np.unique(np.round(z, 12), return_counts=True)
    counts = counts[::-1]
    for i in range(1, nside):
        assert counts[i - 1] == 4 * i
    assert all(c == 4 * nside for c in counts[nside - 1:3 * nside])


@pytest.mark.parametrize("nside", [2, 4])
def test_healpix_symmetries(nside):
    d = angles.healpix_ring(nside)
    key = lambda a: set(map(tuple, np.round(a, 12)))
    base = key(d)
    for M in (np.diag([-1, 1, 1]), np.diag([1, -1, 1]), np.diag([1, 1, -1]),
              np.array([[0, 1, 0], [1, 0, 0], [0, 0, 1]])):
        assert key(d @ M.T) == base


def test_paper_angle_bins(golden_dir):
    ref = json.load(open(os.path.join(golden_dir, "paper_numbers.json")))["angle_bins"]
    assert len(angles.healpix_ring(16)) == ref["fine"]
    assert len(angles.healpix_ring(4)) == ref["coarse"]
    assert ref["fine"] // ref["coarse"] == ref["ratio"]


@pytest.mark.parametrize("g", [0.0, 0.3, 0.62, 0.85, 0.9])
def test_hg_normalised_and_mean_cosine(g):
    """Eq. (11) integrates to one over the sphere and has mean cosine g."""
    norm = 2 * math.pi * integrate.quad(lambda mu: angles.hg(mu, g), -1, 1, epsabs=1e-13,
                                        limit=200)[0]
    mean = 2 * math.pi * integrate.quad(lambda mu: mu * angles.hg(mu, g), -1, 1, epsabs=1e-13,
                                        limit=200)[0]
    assert abs(norm - 1) < 1e-10
    assert abs(mean - g) < 1e-10


@pytest.mark.parametrize("nside,g", [(1, 0.5), (2, 0.9), (4, 0.85), (8, 0.9)])
def test_phase_matrix_doubly_stochastic_symmetric(nside, g):
    d = angles.healpix_ring(nside)
    P = angles.phase_matrix(d, g)
    assert np.all(P >= 0)
    assert np.abs(P - P.T).max() < 1e-15
    assert np.abs(P.sum(axis=0) - 1).max() < 1e-14
    assert np.abs(P.sum(axis=1) - 1).max() < 1e-14
    # P = D K D with D diagonal: P_ij / K_ij factorises as d_i d_j
    K = angles.phase_kernel(d, g)
    L = np.log(P / K)
    dd = np.exp(np.diag(L) / 2)
    assert np.abs(P - dd[:, None] * K * dd[None, :]).max() < 1e-14


def test_phase_matrix_scaling_matches_independent_root_solve():
    """The Sinkhorn fixed point d (K d) = 1 is unique; find it with a generic
    root solver and compare."""
    d = angles.healpix_ring(2)
    K = angles.phase_kernel(d, 0.8)
    sol = optimize.root(lambda x: np.exp(x) * (K @ np.exp(x)) - 1.0, np.zeros(len(d)), tol=1e-15)
    dd = np.exp(sol.x)
    P_ref = dd[:, None] * K * dd[None, :]
    assert np.abs(angles.phase_matrix(d, 0.8) - P_ref).max() < 1e-11


@pytest.mark.parametrize("nside", [1, 2, 4])
def test_isotropic_phase_matrix_is_uniform(nside):
    d = angles.healpix_ring(nside)
    P = angles.phase_matrix(d, 0.0)
    assert np.all(P == P[0, 0])
    assert abs(P[0, 0] - 1.0 / len(d)) < 1e-17


def test_row_normalisation_rows_only():
    d = angles.healpix_ring(2)
    P = angles.phase_matrix(d, 0.9, norm="row")
    assert np.abs(P.sum(axis=1) - 1).max() < 1e-14
    assert np.abs(P.sum(axis=0) - 1).max() > 1e-6


def test_discrete_anisotropy_regression():
    """Point-sampled HG on coarse grids is far more forward-peaked than g."""
    d = angles.healpix_ring(2)
    ge = angles.mean_cosine(angles.phase_matrix(d, 0.9), d)
    assert 0.95 < ge < 0.99


def test_mean_cosine_hand_worked_and_limits():
    """mean_cosine against a hand-worked 2-direction case (60 degrees apart,
    columns = incoming directions: column 0 scatters 0.7 forward and 0.3 at
    60 degrees, column 1 0.2 and 0.8: (0.7 + 0.15 + 0.1 + 0.8) / 2 = 0.875),
    the identity matrix (no deflection: 1), the isotropic g = 0 matrix on
    HEALPix directions (sum of the directions is zero: 0), and convergence to
    the continuum g as the grid refines (within 1 % at nside 16, g = 0.5)."""
    d2 = np.array([[0.0, 0.0, 1.0], [math.sqrt(3) / 2, 0.0, 0.5]])
    P2 = np.array([[0.7, 0.2], [0.3, 0.8]])
    assert abs(angles.mean_cosine(P2, d2) - 0.875) < 1e-15
    d = angles.healpix_ring(4)
    assert abs(angles.mean_cosine(np.eye(len(d)), d) - 1.0) < 1e-14
    assert abs(angles.mean_cosine(angles.phase_matrix(d, 0.0), d)) < 1e-14
    d16 = angles.healpix_ring(16)
    g16 = angles.mean_cosine(angles.phase_matrix(d16, 0.5), d16)
    assert abs(g16 - 0.5) < 0.005, g16


def _eq9_by_quadrature(tau):
    """f0 and f1 straight from Eqs. (7)-(8): the source varies linearly in tau'
    between S0 at the upwind point and S1 at the current one, weighted by
    e^{tau' - tau}."""
    f0 = integrate.quad(lambda t: (1 - t / tau) * math.exp(t - tau), 0, tau, epsabs=1e-15,
                        epsrel=1e-13)[0]
    f1 = integrate.quad(lambda t: (t / tau) * math.exp(t - tau), 0, tau, epsabs=1e-15,
                        epsrel=1e-13)[0]
    return f0, f1


@pytest.mark.parametrize("tau", [1e-6, 1e-3, 0.05, 0.0999, 0.1, 0.5, 1.0, 7.1, 30.0])
def test_eq9_weights_match_formal_solution(tau):
    f0, f1 = angles.eq9_weights(np.array([tau]))
    q0, q1 = _eq9_by_quadrature(tau)
    assert abs(f0[0] - q0) <= 1e-12 * max(1.0, q0) + 1e-12 * q0
    assert abs(f1[0] - q1) <= 1e-12 * max(1.0, q1) + 1e-12 * q1


def test_eq9_reduces_to_constant_source_update():
    """With S0 = S1 the update is I e^-tau + S (1 - e^-tau): f0 + f1 = 1 - e^-tau."""
    tau = np.logspace(-8, math.log10(50.0), 400)
    f0, f1 = angles.eq9_weights(tau)
    assert np.max(np.abs((f0 + f1) - (-np.expm1(-tau))) / -np.expm1(-tau)) < 1e-13
    z0, z1 = angles.eq9_weights(np.array([0.0]))
    assert z0[0] == 0.0 and z1[0] == 0.0
