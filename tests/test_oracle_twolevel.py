"""Pins of the two-level angular grid (scattering on a coarser HEALPix grid):
the pixel lookup against the pixel centres and the hierarchy, the parent map,
and the effective scattering matrix."""
import numpy as np
import pytest

from oracle import angles, solve
from paper_2105_01028_amd import workloads as W


@pytest.mark.parametrize("nside", [1, 2, 4, 8, 16])
def test_every_centre_lies_in_its_own_pixel(nside):
    d = angles.healpix_ring(nside)
    assert [angles.healpix_pixel_ring(nside, v) for v in d] == list(range(len(d)))


def test_random_points_fall_in_a_nearby_pixel():
    rng = np.random.default_rng(0)
    for nside in (2, 4, 8):
        d = angles.healpix_ring(nside)
        for _ in range(400):
            v = rng.normal(size=3)
            v /= np.linalg.norm(v)
            j = angles.healpix_pixel_ring(nside, v)
            near = np.argsort(-(d @ v))[:4]
            assert j in near


@pytest.mark.parametrize("nf,nc", [(2, 1), (4, 1), (8, 2), (16, 4), (8, 4)])
def test_children_per_parent(nf, nc):
    par = angles.parents(nf, nc)
    assert np.all(np.bincount(par, minlength=12 * nc * nc) == (nf // nc) ** 2)
    df, dc = angles.healpix_ring(nf), angles.healpix_ring(nc)
    m = np.array([df[par == J].mean(axis=0) for J in range(len(dc))])
    m /= np.linalg.norm(m, axis=1, keepdims=True)
    assert np.min(np.sum(m * dc, axis=1)) > np.cos(np.radians(3.0))


def test_hierarchy_composes():
    """The grid is nested: the parent of a pixel's parent is its grandparent."""
    assert np.array_equal(angles.parents(4, 2)[angles.parents(16, 4)], angles.parents(16, 2))
    assert np.array_equal(angles.parents(2, 1)[angles.parents(8, 2)], angles.parents(8, 1))


def test_two_level_matrix():
    P = angles.two_level_matrix(8, 2, 0.9)
    assert np.allclose(P.sum(axis=0), 1.0, atol=1e-12)
    assert np.allclose(P.sum(axis=1), 1.0, atol=1e-12)
    assert np.allclose(P, P.T, atol=1e-15)
    d = angles.healpix_ring(4)
    assert np.allclose(angles.two_level_matrix(4, 4, 0.8), angles.phase_matrix(d, 0.8), atol=0)
    # children of one coarse bin scatter alike and share every target equally
    par = angles.parents(8, 2)
    kids = np.nonzero(par == 5)[0]
    assert np.allclose(P[:, kids], P[:, kids[:1]], atol=0)


def test_two_level_budget_closes():
    p = W.small_problem(nside=4, nx=7, ny=6, nz=5, steps=12, seed=2).copy(nside_scatter=1)
    r = solve.forward(p)
    inj = r.injected.sum()
    assert abs(inj - r.absorbed.sum() - r.escaped.sum() - r.in_domain[-1]) < 1e-13 * inj
