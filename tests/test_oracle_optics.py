"""Pins of Snell's law (Eq. 13), Fresnel reflectance (Eq. 14) and the
interface interception lists (Sec. 3.3)."""
import math

import numpy as np
import pytest

from oracle import angles, lattice, optics


def _fresnel_amplitudes(n1, n2, t1):
    """Textbook Fresnel equations in amplitude form (cosines only), averaged
    over the two polarisations: an independent form of Eq. (14)."""
    s2 = n1 / n2 * math.sin(t1)
    if s2 >= 1.0:
        return 1.0
    c1, c2 = math.cos(t1), math.sqrt(1 - s2 * s2)
    rs = (n1 * c1 - n2 * c2) / (n1 * c1 + n2 * c2)
    rp = (n2 * c1 - n1 * c2) / (n2 * c1 + n1 * c2)
    return 0.5 * (rs * rs + rp * rp)


@pytest.mark.parametrize("n1,n2", [(1.4, 1.0), (1.0, 1.4), (1.51, 1.0), (1.33, 1.5)])
def test_fresnel_matches_amplitude_form(n1, n2):
    for t1 in np.linspace(1e-4, math.pi / 2 - 1e-4, 400):
        assert abs(optics.fresnel_reflectance(n1, n2, math.cos(t1))
                   - _fresnel_amplitudes(n1, n2, t1)) < 1e-12


def test_fresnel_special_values():
    R0 = optics.fresnel_reflectance(1.4, 1.0, 1.0)
    assert abs(R0 - (0.4 / 2.4) ** 2) < 1e-15
    assert abs(R0 - 0.027778) < 1e-6
    # continuity as theta_1 -> 0
    assert abs(optics.fresnel_reflectance(1.4, 1.0, math.cos(1e-6)) - R0) < 1e-10
    tc = optics.critical_angle(1.4, 1.0)
    assert abs(math.degrees(tc) - 45.584691) < 1e-5
    assert optics.fresnel_reflectance(1.4, 1.0, math.cos(tc + 1e-9)) == 1.0
    assert optics.fresnel_reflectance(1.4, 1.0, math.cos(tc - 1e-7)) > 0.99
    # Brewster angle: p-polarised reflection vanishes, R = R_s / 2
    tb = math.atan(1.0 / 1.4)
    assert abs(math.degrees(tb) - 35.537678) < 1e-5
    s2 = 1.4 * math.sin(tb)
    t2 = math.asin(s2)
    Rs = (math.sin(tb - t2) / math.sin(tb + t2)) ** 2
    assert abs(optics.fresnel_reflectance(1.4, 1.0, math.cos(tb)) - Rs / 2) < 1e-12
    assert abs(Rs / 2 - 0.0526) < 1e-3
    # no index change, no reflection
    assert optics.fresnel_reflectance(1.4, 1.4, 0.3) == 0.0


def test_snell_refracted_direction():
    rng = np.random.default_rng(1)
    for _ in range(200):
        h = rng.normal(size=3)
        h /= np.linalg.norm(h)
        om = rng.normal(size=3)
        om /= np.linalg.norm(om)
        if om @ h < 0:
            om = -om
        n1, n2 = rng.choice([1.0, 1.33, 1.4, 1.51], 2, replace=True)
        t = optics.refract(tuple(om), tuple(h), n1, n2)
        r = optics.reflect(tuple(om), tuple(h))
        assert abs(np.linalg.norm(r) - 1) < 1e-14
        assert abs(np.dot(r, h) + np.dot(om, h)) < 1e-14
        sin1 = np.linalg.norm(np.cross(om, h))
        if t is None:
            assert n1 * sin1 >= n2 - 1e-12
            continue
        t = np.array(t)
        assert abs(np.linalg.norm(t) - 1) < 1e-14
        sin2 = np.linalg.norm(np.cross(t, h))
        assert abs(n1 * sin1 - n2 * sin2) < 1e-14            # Eq. (13)
        assert abs(np.dot(np.cross(om, h), t)) < 1e-14        # coplanar
        assert t @ h > 0


def test_interceptions_on_a_flat_interface():
    """Planar jump at z: normal is +z; every crossing direction reflects to its
    z-mirror and refracts to the nearest pixel of Snell's direction."""
    dirs = angles.healpix_ring(2)
    shape = (6, 5, 5)
    n = np.full(shape, 1.4)
    n[3:] = 1.0
    lat = lattice.RayLattice(dirs, shape)
    ic = optics.interceptions(lat, n)
    assert len(ic) > 0
    for d, v, w, R, dr, dt in ic:
        zv, zw = v // 25, w // 25
        assert {zv, zw} == {2, 3}
        mirror = dirs[d] * np.array([1, 1, -1])
        assert np.allclose(dirs[dr], mirror, atol=1e-12)
        cos1 = abs(dirs[d, 2])
        n1, n2 = (1.4, 1.0) if zv == 2 else (1.0, 1.4)
        assert abs(R - _fresnel_amplitudes(n1, n2, math.acos(cos1))) < 1e-12
        if dt >= 0:
            assert np.sign(dirs[dt, 2]) == np.sign(dirs[d, 2])
