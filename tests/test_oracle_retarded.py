"""Pins of the retarded time stepping below Courant one (oracle retarded).

* Vacuum, one on-axis direction, a whole number of steps per hop: the pulse
  crosses the column with its shape unchanged (the paper's one-dimensional
  test, Sec. 2.2), delayed by exactly D steps per plane.
* A fractional number of steps per hop: each hop spreads the pulse over two
  neighbouring time bins with weights (1 - phi, phi), so after L hops the
  signal is the pulse convolved with Binomial(L, phi), delayed by floor(D) L.
* Absorption without scattering: every hop multiplies by exp(-mu_a dr), and
  the light absorbed over the whole passage is q (1 - e^{-mu_a L dr}).
* With scattering, a constant source drives the field to the fixed point of
  the discrete transport equation N = T(A N) + D q, solved here directly.
* Light is conserved exactly when every direction hops the same distance (the
  eight cube diagonals).  With unequal hops the per-hop source weight
  1 - e^{-dtau_d} of the target direction makes scattering take light out of
  one direction and put it into others at slightly different rates; the
  imbalance per scattering is O(dtau) (its sign depends on the geometry), so in
  the thin limit the total falls four-fold when mu_s halves.
"""
import math

import numpy as np
import pytest

from oracle import medium, retarded, setup
from paper_2105_01028_amd import workloads as W

C0 = medium.C0_MM_PER_PS
ZMAX_FACE = 5   # face = 2 axis + side


def _column(L, D, mua=0.0, t0=8.0, fwhm=5.0, steps=None):
    """A 1 x 1 x L column (1 mm voxels, n = 1) with one direction along +z and
    a time step giving D steps per plane."""
    mu_a, mu_s, n = W.uniform_medium(1, 1, L, mua, 0.0, 1.0)
    dt = 1.0 * 1.0 / (C0 * D)
    p = W.Problem(nx=1, ny=1, nz=L, dx_mm=1.0, nside=1, g=0.0, mua=mu_a, mus=mu_s, n=n,
                  steps=steps or 400, dt_ps=dt, src_ix=0, src_iy=0, src_w=1, t0_ps=t0,
                  fwhm_ps=fwhm, total_photons=1.0)
    S = retarded.build(p, dirs=np.array([[0.0, 0.0, 1.0]]), P=np.array([[1.0]]))
    return p, S


def _pulse(p, S, steps):
    return np.array([setup.pulse_weight(m, S.dt, p.t0_ps, p.fwhm_ps, 1.0)
                     for m in range(steps)])


def test_whole_steps_per_hop_keep_the_pulse_shape():
    L, steps = 6, 400
    p, S = _column(L, 10.0)
    assert S.nlag[0] == 10 and S.phi[0] < 1e-12 and S.H == 11
    res = retarded.forward(p, steps, S)
    q = _pulse(p, S, steps)
    lag = 10 * L - 1
    want = np.zeros(steps)
    want[lag:] = q[:steps - lag]
    got = res.escaped[:, ZMAX_FACE]
    assert np.abs(got - want).max() < 1e-14
    assert np.abs(res.escaped.sum(axis=1) - got).max() == 0.0


@pytest.mark.parametrize("D,L", [(6.3, 5), (7.75, 3), (1.5, 8)])
def test_fractional_delay_is_a_binomial_spread(D, L):
    steps = 300
    p, S = _column(L, D)
    n, phi = int(math.floor(D)), D - math.floor(D)
    res = retarded.forward(p, steps, S)
    q = _pulse(p, S, steps)
    want = np.zeros(steps)
    for m in range(steps):
        s = 0.0
        for j in range(L + 1):
            t = m + 1 - n * L - j
            if 0 <= t < steps:
                s += math.comb(L, j) * phi ** j * (1.0 - phi) ** (L - j) * q[t]
        want[m] = s
    assert np.abs(res.escaped[:, ZMAX_FACE] - want).max() < 1e-14


def test_absorption_per_hop():
    L, steps, mua = 5, 400, 0.2
    p, S = _column(L, 7.5, mua=mua)
    res = retarded.forward(p, steps, S)
    q = _pulse(p, S, steps)
    att = math.exp(-float(p.mua.flat[0]) * L)   # mu_a as stored (float32)
    # two-tap spread with phi = 1/2 (D = 7.5)
    want = np.zeros(steps)
    for m in range(steps):
        for j in range(L + 1):
            t = m + 1 - 7 * L - j
            if 0 <= t < steps:
                want[m] += math.comb(L, j) * 0.5 ** L * q[t]
    assert np.abs(res.escaped[:, ZMAX_FACE] - att * want).max() < 1e-14
    # the pulse has left the column: everything injected is absorbed or out
    assert res.in_domain[-1] < 1e-30
    assert abs(res.absorbed.sum() - q.sum() * (1.0 - att)) < 1e-14
    assert abs(res.injected.sum() - res.absorbed.sum() - res.escaped.sum()) < 1e-14


def _scattering_problem(courant=0.2, seed=4):
    p = W.small_problem(nside=1, nx=4, ny=3, nz=3, mua=0.05, mus=0.8, g=0.5, n=1.3, steps=1,
                        seed=seed, src_w=1, src_ix=1, src_iy=1)
    return p.copy(dt_ps=courant * p.dx_mm * 1.3 / C0)


def test_history_length_at_a_fifth_of_the_crossing_time():
    p = _scattering_problem()
    S = retarded.build(p.copy(nside=4, nx=3, ny=3, nz=3, mua=p.mua[:, :, :3],
                              mus=p.mus[:, :, :3], n=p.n[:, :, :3]))
    # D_d = 5 / |Omega_a| lies in [5, 5 sqrt 3): nine collided fields
    assert 5.0 <= S.D.min() and S.D.max() < 5.0 * math.sqrt(3.0)
    assert S.H == int(np.floor(S.D.max())) + 1 == 9


def test_constant_source_reaches_the_discrete_steady_state():
    p = _scattering_problem()
    S = retarded.build(p)
    nd, nv = S.a.shape
    share = 1.0 / (len(S.src_vox) * len(S.src_dirs))
    N = np.zeros((nd, nv))
    hist = {}
    prev = None
    for m in range(4000):
        for d in S.src_dirs:
            for v in S.src_vox:
                N[d, v] += S.D[d] * share
        hist[m], _ = retarded.collide(S, N)
        hist.pop(m - S.H, None)
        prev = N
        N, _, _ = retarded.transport(S, hist, m, 0)
    # the fixed point after injection: N = T(A N) + D q, assembled from the
    # definitions (T takes each voxel's upwind value, A collides every column)
    n = nd * nv
    A = np.zeros((n, n))
    for d in range(nd):
        for v in range(nv):
            A[d * nv + v, d * nv + v] += S.a[d, v]
            for e in range(nd):
                A[d * nv + v, e * nv + v] += S.b[d, v] * S.P[d, e]
    T = np.zeros((n, n))
    for d in range(nd):
        for v in range(nv):
            u = S.upwind[d][v]
            if u >= 0:
                T[d * nv + v, d * nv + u] = 1.0
    rhs = np.zeros(n)
    for d in S.src_dirs:
        for v in S.src_vox:
            rhs[d * nv + v] = S.D[d] * share
    fixed = np.linalg.solve(np.eye(n) - T @ A, rhs).reshape(nd, nv)
    after_inject = N.copy()
    for d in S.src_dirs:
        for v in S.src_vox:
            after_inject[d, v] += S.D[d] * share
    assert np.abs(prev - after_inject).max() < 1e-12 * fixed.max()
    assert np.abs(after_inject - fixed).max() < 1e-10 * fixed.max()


def test_rejects_varying_index_and_long_steps():
    p = _scattering_problem()
    n2 = p.n.copy()
    n2[0, 0, 0] = 1.0
    with pytest.raises(ValueError):
        retarded.build(p.copy(n=n2))
    with pytest.raises(ValueError):
        retarded.build(p.copy(dt_ps=1.01 * p.dx_mm * 1.3 / C0))


def test_hop_coefficients_are_the_eq9_collision_over_one_hop():
    """a and b of direction d are those of the per-step collision (Eq. 9-10,
    f0 + f1 from Eq. 9) for a step whose path is the hop dr_d."""
    p = _scattering_problem()
    S = retarded.build(p)
    for d in range(len(S.dirs)):
        dt_d = S.hop[d] * float(p.n.flat[0]) / C0   # light at c0/n covers dr_d in dt_d
        a, b, _, ell = medium.collision_coefficients(p.mua, p.mus, p.n, dt_d, "paper")
        assert np.allclose(ell, S.hop[d], rtol=1e-14)
        assert np.abs(S.a[d] - a.ravel()).max() < 1e-15
        assert np.abs(S.b[d] - b.ravel()).max() < 1e-14


def _diagonal_problem(mus, courant):
    mu_a, mu_s, n = W.uniform_medium(7, 6, 5, 0.01, mus, 1.2)
    return W.Problem(nx=7, ny=6, nz=5, dx_mm=1.0, nside=1, g=0.5, mua=mu_a, mus=mu_s, n=n,
                     steps=1, dt_ps=courant * 1.2 / C0, src_ix=3, src_iy=2, src_w=1,
                     t0_ps=5.0, fwhm_ps=3.0, det_face=[4], det_i=[5], det_j=[2])


def test_equal_hops_conserve_light():
    from oracle import angles
    dirs = np.array([[sx, sy, sz] for sz in (1, -1) for sy in (1, -1) for sx in (1, -1)],
                    dtype=np.float64) / math.sqrt(3.0)
    P = angles.phase_matrix(dirs, 0.5)
    p = _diagonal_problem(1.5, 0.37)
    S = retarded.build(p, dirs=dirs, P=P)
    assert np.ptp(S.D) == 0.0 and S.phi[0] > 0.1
    res = retarded.forward(p, 700, S)
    inj = res.injected.sum()
    assert res.in_domain[-1] < 1e-12 * inj
    closure = inj - res.absorbed.sum() - res.escaped.sum() - res.in_domain[-1]
    assert abs(closure) < 1e-13 * inj
    assert res.det.sum() > 0.0


def test_unequal_hops_conserve_light_to_second_order():
    loss = []
    for mus in (1.0 / 16, 1.0 / 32):
        p = W.small_problem(nside=1, nx=8, ny=7, nz=6, mua=0.0, mus=mus, g=0.6, n=1.4,
                            steps=1, seed=3).copy(dt_ps=0.5 * 1.4 / C0, t0_ps=6.0, fwhm_ps=4.0)
        res = retarded.forward(p, 300)
        inj = res.injected.sum()
        assert res.in_domain[-1] < 1e-12 * inj
        loss.append((inj - res.absorbed.sum() - res.escaped.sum()) / inj)
    assert 3.5 < loss[0] / loss[1] < 4.5


def test_two_level_source_uses_the_effective_matrix():
    """With nside_scatter the retarded collision scatters with C P_c A: one
    collision of a random field equals a N + b (P_eff N), and P_eff keeps
    column sums of one, so scattering alone conserves the content."""
    from oracle import angles
    p = W.small_problem(nside=4, nx=5, ny=4, nz=3, mua=0.0, mus=1.5, g=0.7, n=1.2, steps=1,
                        seed=8).copy(nside_scatter=2, dt_ps=0.2 * 1.2 / C0)
    S = retarded.build(p)
    Pe = angles.two_level_matrix(4, 2, p.g, p.hg_norm)
    assert np.abs(S.P - Pe).max() == 0.0
    rng = np.random.default_rng(9)
    N = rng.uniform(0.0, 1.0, (192, p.nvox))
    C, _ = retarded.collide(S, N)
    assert np.abs(C - (S.a * N + S.b * (Pe @ N))).max() < 1e-14
    assert np.allclose(Pe.sum(axis=0), 1.0, atol=1e-13)
