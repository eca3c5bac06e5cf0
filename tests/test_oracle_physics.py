"""Physics pins of the whole oracle step loop: Beer-Lambert attenuation,
photon conservation, linearity, mirror symmetry, the random walk of multiple
scattering and the diffusion limit in a large uniform medium."""
import math

import numpy as np
import pytest

from oracle import angles, physics, solve
from paper_2105_01028_amd import workloads as W


def test_beer_lambert_impulse():
    """mu_s = 0: every photon is multiplied by e^{-mu_a l} at each collision, and
    a photon leaving at step m has collided m + 1 times, so
    det(mu_a)[m] = det(0)[m] e^{-mu_a l (m+1)} exactly."""
    shape = (10, 9, 8)
    base = W.small_problem(nside=2, nx=8, ny=9, nz=10, mua=0.0, mus=0.0, g=0.0, n=1.4,
                           steps=30, total_photons=0.0, det_cone_deg=0.0,
                           dets=([5, 5, 1, 3], [3, 4, 4, 2], [4, 5, 6, 7]))
    S0 = solve.build(base)
    rng = np.random.default_rng(7)
    N0 = np.zeros((48, base.nvox))
    N0[:, rng.integers(0, base.nvox, 6)] = rng.uniform(0.5, 1.0, (48, 6))
    r0 = solve.forward(base, S=S0, state0=N0)
    mua = float(np.float32(0.03))      # the medium arrays are float32
    p = base.copy(mua=np.full(shape, mua, np.float32))
    S1 = solve.build(p)
    r1 = solve.forward(p, S=S1, state0=N0)
    ell = S1.ell[0]
    fac = np.exp(-mua * ell * (np.arange(30) + 1))
    assert r0.det.sum() > 0.1
    assert np.allclose(r1.det, r0.det * fac[None, :], rtol=1e-13, atol=0)
    assert np.allclose(r1.escaped, r0.escaped * fac[:, None], rtol=1e-13, atol=0)


@pytest.mark.parametrize("advance", ["phase", "split"])
def test_abs_exact_impulse_with_scattering(advance):
    """coef="abs_exact" with scattering on: a = e^{-mu_a l} e^{-mu_s l} and
    b = e^{-mu_a l} (1 - e^{-mu_s l}) are the mu_a = 0 coefficients times
    e^{-mu_a l}, so with a uniform mu_a every collision scales the whole field by
    e^{-mu_a l} whatever mu_s does, and for an impulse
    det(mu_a)[m] = det(0)[m] e^{-mu_a l (m+1)} exactly, as without scattering.
    The paper's form b = omega (1 - a) does not factor this way (checked below),
    so a wrong b, a dropped factor or a sign error in either exponent fails."""
    shape = (9, 8, 10)
    n = 1.4
    base = W.small_problem(nside=2, nx=10, ny=8, nz=9, mua=0.0, mus=2.0, g=0.8, n=n,
                           steps=24, total_photons=0.0, det_cone_deg=0.0, seed=17,
                           coef="abs_exact", advance=advance,
                           dets=([4, 4, 1, 3, 5], [3, 6, 4, 2, 5], [4, 5, 6, 7, 3]))
    base = base.copy(mua=np.zeros(shape, np.float32))
    if advance == "split":
        # a second index in a slab: split mode with per-voxel move fractions
        nn = base.n.copy()
        nn[5:] = 1.6
        base = base.copy(n=nn)
    rng = np.random.default_rng(9)
    N0 = np.zeros((48, base.nvox))
    N0[:, rng.integers(0, base.nvox, 8)] = rng.uniform(0.5, 1.0, (48, 8))
    r0 = solve.forward(base, S=solve.build(base), state0=N0)
    mua = float(np.float32(0.04))
    p = base.copy(mua=np.full(shape, mua, np.float32))
    S1 = solve.build(p)
    r1 = solve.forward(p, S=S1, state0=N0)
    # per-voxel path per step (split mode: two indices)
    ell = S1.ell.reshape(-1)
    assert r0.det.sum() > 1e-3 and r0.in_domain[-1] > 1e-3
    if advance == "phase":
        fac = np.exp(-mua * ell[0] * (np.arange(24) + 1))
        assert np.allclose(r1.det, r0.det * fac[None, :], rtol=1e-12, atol=0)
        assert np.allclose(r1.escaped, r0.escaped * fac[:, None], rtol=1e-12, atol=0)
        assert np.allclose(r1.in_domain, r0.in_domain * fac, rtol=1e-12, atol=0)
    else:
        # with two path lengths the factor depends on where the light collided;
        # it lies between the two uniform-path factors, and equals the slower
        # medium's factor where only that medium was ever visited
        lo = np.exp(-mua * ell.max() * (np.arange(24) + 1))
        hi = np.exp(-mua * ell.min() * (np.arange(24) + 1))
        ok = r0.in_domain > 0
        q = r1.in_domain[ok] / r0.in_domain[ok]
        assert np.all(q <= hi[ok] * (1 + 1e-12)) and np.all(q >= lo[ok] * (1 - 1e-12))
    # the paper's coefficient form has no such factorisation
    pp = p.copy(coef="paper")
    rp = solve.forward(pp, S=solve.build(pp), state0=N0)
    rp0 = solve.forward(base.copy(coef="paper"), S=solve.build(base.copy(coef="paper")),
                        state0=N0)
    if advance == "phase":
        assert not np.allclose(rp.in_domain, rp0.in_domain * fac, rtol=1e-6, atol=0)


@pytest.mark.parametrize("advance,coef,mua", [("phase", "paper", 0.0), ("phase", "paper", 0.05),
                                              ("split", "paper", 0.02),
                                              ("phase", "abs_exact", 0.05)])
def test_conservation(advance, coef, mua):
    """Photons injected = in the box + absorbed + escaped, every step."""
    p = W.small_problem(nside=2, nx=9, ny=8, nz=7, mua=mua, mus=3.0, g=0.8, steps=25,
                        advance=advance, coef=coef, seed=3)
    r = solve.forward(p)
    before = np.concatenate([[0.0], r.in_domain[:-1]])
    resid = before + r.injected - r.absorbed - r.escaped.sum(axis=1) - r.in_domain
    assert np.abs(resid).max() < 1e-14
    total = r.injected.sum() - r.absorbed.sum() - r.escaped.sum() - r.in_domain[-1]
    assert abs(total) < 1e-13
    if mua == 0.0:
        assert r.absorbed.max() < 1e-16


def test_conservation_with_refraction():
    """An index jump (air slab inside tissue) reflects and refracts light but
    loses none."""
    p = W.small_problem(nside=2, nx=8, ny=8, nz=12, mua=0.0, mus=2.0, g=0.6, n=1.4, steps=30)
    n = p.n.copy()
    n[5:8] = 1.0
    mus = p.mus.copy()
    mus[5:8] = 0.0
    p2 = p.copy(n=n, mus=mus)
    r = solve.forward(p2)
    assert len(r.setup.icpt) > 100
    total = r.injected.sum() - r.absorbed.sum() - r.escaped.sum() - r.in_domain[-1]
    assert abs(total) < 1e-13


def test_linearity_in_sources():
    """det(alpha s1 + beta s2) = alpha det(s1) + beta det(s2)."""
    p = W.small_problem(nside=2, nx=8, ny=8, nz=8, mua=0.02, mus=2.0, g=0.7, steps=20,
                        total_photons=0.0, seed=11, det_cone_deg=0.0)
    S = solve.build(p)
    rng = np.random.default_rng(5)
    s1 = rng.uniform(0, 1, (48, p.nvox)) * (rng.uniform(size=p.nvox) < 0.05)
    s2 = rng.uniform(0, 1, (48, p.nvox)) * (rng.uniform(size=p.nvox) < 0.05)
    r1 = solve.forward(p, S=S, state0=s1)
    r2 = solve.forward(p, S=S, state0=s2)
    r12 = solve.forward(p, S=S, state0=2.5 * s1 - 0.75 * s2)
    assert np.allclose(r12.det, 2.5 * r1.det - 0.75 * r2.det, rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("cone", [0.0, 15.0])
def test_mirror_symmetry(cone):
    """Source on the 2x2 top-face centre of an even grid and a uniform medium:
    detector patches at mirror images (x -> -x, y -> -y, both) record the same
    light to rounding.  Swapping x and y is only an approximate symmetry: for
    directions with |Omega_x| = |Omega_y| the tie-break picks y as the plane
    axis, which fixes where the z offsets of those rays round."""
    nx = 10
    c = nx // 2
    dets = ([4] * 6, [c + 2, c - 3, c, c, c + 2, c - 3], [c, c, c + 2, c - 3, c - 3, c + 2])
    # pairs: (0,1) x mirror, (2,3) y mirror, (4,5) x and y mirror, (0,2) x <-> y
    p = W.small_problem(nside=2, nx=nx, ny=nx, nz=6, mua=0.01, mus=3.0, g=0.8, steps=40,
                        dets=dets, det_cone_deg=cone)
    p.src_ix = p.src_iy = c - 1
    r = solve.forward(p)
    d = r.det
    assert d[0].sum() > 1e-6
    for i, j in ((0, 1), (2, 3), (4, 5)):
        assert np.abs(d[i] - d[j]).max() <= 1e-12 * np.abs(d[i]).max()
    assert np.abs(d[0] - d[2]).max() <= 0.05 * np.abs(d[0]).max()


def _point_cloud(side, mus, mua, g, steps, nside=2, advance="phase"):
    p = W.small_problem(nside=nside, nx=side, ny=side, nz=side, mua=mua, mus=mus, g=g, n=1.0,
                        steps=steps, total_photons=0.0, advance=advance)
    S = solve.build(p)
    nd = len(S.dirs)
    c = side // 2
    N0 = np.zeros((nd, p.nvox))
    N0[:, (c * side + c) * side + c] = 1.0 / nd
    return p, S, solve.forward(p, S=S, state0=N0)


def test_random_walk_second_moment():
    """g = 0, mu_a = 0, a box no photon can leave in time: each axis' second
    moment of the photon cloud follows the persistent random walk with step l
    and direction correlation a (the unscattered fraction), to the few per cent
    the plane lattice allows."""
    side, steps = 45, 20
    p, S, r = _point_cloud(side, 0.1, 0.0, 0.0, steps)
    assert abs(r.in_domain[-1] - 1.0) < 1e-12
    E = r.state.sum(axis=0).reshape(side, side, side)
    c = side // 2
    z, y, x = np.meshgrid(*(np.arange(side) - c,) * 3, indexing="ij")
    om2 = (S.dirs ** 2).mean(axis=0)
    lam = physics.step_correlation(S.a[0], S.b[0], 0.0)
    for i, X in enumerate((x, y, z)):
        want = physics.persistent_walk_msd(steps, S.ell[0], lam, om2[i])
        got = float((E * X * X).sum())
        assert abs(got / want - 1.0) < 0.03, (i, got, want)


def test_diffusion_limit_decay_rate():
    """Large uniform medium in the diffusive regime (6.4 transport mean free paths,
    mu_s l = 0.2 per step, g = 0, 32 mm side): the late-time decay rate of
    the photons in the box matches diffusion theory, mu_a c + 3 D (pi/L_e)^2
    with D = c / (3 (mu_a + mu_s')), to 5 %."""
    side, steps, mus, mua = 32, 200, 0.2, 0.002
    p, S, r = _point_cloud(side, mus, mua, 0.0, steps)
    y = np.log(r.in_domain)
    m0 = steps // 2
    slope = -np.polyfit(np.arange(m0, steps), y[m0:], 1)[0] / S.dt
    v = S.ell[0] / S.dt
    D = v / (3.0 * (mua + mus))
    L_e = side * p.dx_mm + 4.0 * D / v
    want = mua * v + 3.0 * D * (math.pi / L_e) ** 2
    assert abs(slope / want - 1.0) < 0.05, (slope, want)
    # and the walk-based coefficient of the discrete model itself
    lam = physics.step_correlation(S.a[0], S.b[0], 0.0)
    Dw = physics.walk_diffusion_coefficient(S.ell[0], S.dt, lam)
    want_w = physics.cube_decay_rate(Dw, side * p.dx_mm, v, S.a[0] + S.b[0], S.dt)
    assert abs(slope / want_w - 1.0) < 0.05
