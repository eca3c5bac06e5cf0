"""Pins of the implicit-source collision (oracle solve.collide_implicit): the
per-voxel solve against the fixed-point iteration of Sec. 2.4 Steps 3-6, the
closed form for isotropic scattering, the total of a column (which P cannot
change, its columns summing to one), exact conservation without absorption,
and the photon budget of whole solves."""
import numpy as np
import pytest

from oracle import angles, medium, solve
from paper_2105_01028_amd import workloads as W


def _setup(g=0.8, mua=0.05, mus=3.0, seed=3, nside=2):
    p = W.small_problem(nside=nside, nx=5, ny=4, nz=3, mua=mua, mus=mus, g=g, steps=1,
                        seed=seed, total_photons=0.0).copy(source="implicit")
    return p, solve.build(p)


def test_solve_is_the_fixed_point_of_steps_3_to_6():
    p, S = _setup()
    rng = np.random.default_rng(1)
    N = rng.uniform(0.0, 1.0, (len(S.dirs), p.nvox))
    Nc, _ = solve.collide_implicit(S, N)
    it = N.copy()
    for _ in range(2000):
        nxt = S.a * N + S.w0 * (S.P @ N) + S.w1 * (S.P @ it)
        if np.abs(nxt - it).max() < 1e-16:
            break
        it = nxt
    assert np.abs(it - Nc).max() < 1e-12 * np.abs(Nc).max()


def test_isotropic_scattering_closed_form():
    p, S = _setup(g=0.0)
    nd = len(S.dirs)
    assert np.allclose(S.P, 1.0 / nd, atol=1e-15)
    rng = np.random.default_rng(2)
    N = rng.uniform(0.0, 1.0, (nd, p.nvox))
    Nc, _ = solve.collide_implicit(S, N)
    tot = N.sum(axis=0)
    tot_c = tot * (S.a + S.w0) / (1.0 - S.w1)
    ref = S.a * N + (S.w0 * tot + S.w1 * tot_c) / nd
    assert np.abs(Nc - ref).max() < 1e-13


@pytest.mark.parametrize("g,mua", [(0.9, 0.05), (0.5, 0.3)])
def test_column_total(g, mua):
    """1^T P = 1^T, so the column total obeys the scalar relation
    T_c = a T + w0 T + w1 T_c whatever the angular distribution."""
    p, S = _setup(g=g, mua=mua)
    rng = np.random.default_rng(3)
    N = rng.uniform(0.0, 1.0, (len(S.dirs), p.nvox))
    Nc, absorbed = solve.collide_implicit(S, N)
    tot = N.sum(axis=0)
    assert np.allclose(Nc.sum(axis=0), tot * (S.a + S.w0) / (1.0 - S.w1), rtol=1e-13)
    assert abs(absorbed - (N.sum() - Nc.sum())) < 1e-13


def test_no_absorption_conserves_light():
    p, S = _setup(mua=0.0, mus=5.0)
    rng = np.random.default_rng(4)
    N = rng.uniform(0.0, 1.0, (len(S.dirs), p.nvox))
    Nc, absorbed = solve.collide_implicit(S, N)
    assert np.allclose(Nc.sum(axis=0), N.sum(axis=0), rtol=1e-14)
    assert abs(absorbed) < 1e-12


def test_weights_are_eq9_parts():
    n = np.full((2, 2, 2), 1.4)
    mua = np.full((2, 2, 2), 0.02)
    mus = np.full((2, 2, 2), 6.0)
    dt = medium.time_step(1.0, n)
    a, w0, w1 = medium.implicit_weights(mua, mus, n, dt)
    a2, b, omega, ell = medium.collision_coefficients(mua, mus, n, dt)
    f0, f1 = angles.eq9_weights((mua + mus) * ell)
    assert np.allclose(a, a2, rtol=0, atol=0)
    assert np.allclose(w0 + w1, b, rtol=1e-15)
    assert np.allclose(w1, omega * f1, rtol=1e-15)


@pytest.mark.parametrize("advance", ["phase", "split"])
def test_budget_closes(advance):
    p = W.small_problem(nside=2, nx=9, ny=8, nz=7, steps=30, seed=5, advance=advance)
    r = solve.forward(p.copy(source="implicit"))
    inj = r.injected.sum()
    assert abs(inj - r.absorbed.sum() - r.escaped.sum() - r.in_domain[-1]) < 1e-13 * inj
