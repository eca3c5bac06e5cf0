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
    assert np.all(S.nlag == 10) and np.all(S.phi < 1e-12) and S.H == 11
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
                N[d, v] += S.D[d, v] * share
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
            rhs[d * nv + v] = S.D[d, v] * share
    fixed = np.linalg.solve(np.eye(n) - T @ A, rhs).reshape(nd, nv)
    after_inject = N.copy()
    for d in S.src_dirs:
        for v in S.src_vox:
            after_inject[d, v] += S.D[d, v] * share
    assert np.abs(prev - after_inject).max() < 1e-12 * fixed.max()
    assert np.abs(after_inject - fixed).max() < 1e-10 * fixed.max()


def test_rejects_long_steps_and_two_level_with_varying_index():
    p = _scattering_problem()
    n2 = p.n.copy()
    n2[0, 0, 0] = 1.0
    with pytest.raises(ValueError):
        retarded.build(p.copy(n=n2, nside=2, nside_scatter=1))
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
    assert np.ptp(S.D) == 0.0 and S.phi[0, 0] > 0.1
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


# ---- varying refractive index -------------------------------------------

def _slab_column(L, z1, z2, n1, n2, dt, t0=4.0, fwhm=3.0):
    """A 1 x 1 x L column along z, index n1 with a slab of n2 in [z1, z2),
    two directions +z and -z, no absorption or scattering."""
    mu_a, mu_s, n = W.uniform_medium(1, 1, L, 0.0, 0.0, n1)
    n[z1:z2] = n2
    p = W.Problem(nx=1, ny=1, nz=L, dx_mm=1.0, nside=1, g=0.0, mua=mu_a, mus=mu_s, n=n,
                  steps=1, dt_ps=dt, src_ix=0, src_iy=0, src_w=1, t0_ps=t0, fwhm_ps=fwhm,
                  total_photons=1.0, src_cone_deg=10.0)
    dirs = np.array([[0.0, 0.0, 1.0], [0.0, 0.0, -1.0]])
    S = retarded.build(p, dirs=dirs, P=np.eye(2))
    return p, S


def _trace_column(L, nvox, dt, R0, steps):
    """Impulse responses of the column by following packets rather than
    fields: a packet (time, voxel, direction) of some flux leaves voxel k
    after D(k) = dx n_k / (c0 dt) steps, split over floor(D) and floor(D) + 1
    steps with weights 1 - phi and phi; at an index jump it splits into a
    transmitted (1 - R0) and a reflected R0 packet, both arriving when the
    transmitted one would; a packet leaving the column is recorded in the
    step before it would arrive.  Packets that meet at one (time, voxel,
    direction) are merged.  Returns the escape per step through the bottom
    (+z end) and the top (-z end) for a unit flux injected at step 0 into
    voxel 0 moving +z."""
    D = [float(nvox[k]) / (C0 * dt) for k in range(L)]
    bottom = np.zeros(steps)
    top = np.zeros(steps)
    live = {(0, 0, +1): 1.0}
    for t in range(steps):
        for (tt, k, s), amp in [(key, a) for key, a in live.items() if key[0] == t]:
            del live[(tt, k, s)]
            n_ = int(math.floor(D[k] + 1e-12))
            ph = D[k] - n_
            for lag, w in ((n_, 1.0 - ph), (n_ + 1, ph)):
                if w <= 0.0:
                    continue
                ta, k2 = t + lag, k + s
                if k2 < 0 or k2 >= L:
                    if ta - 1 < steps:
                        (bottom if s > 0 else top)[ta - 1] += amp * w
                    continue
                outs = ([(k2, s, 1.0 - R0), (k, -s, R0)] if nvox[k2] != nvox[k]
                        else [(k2, s, 1.0)])
                for kk, ss, f in outs:
                    live[(ta, kk, ss)] = live.get((ta, kk, ss), 0.0) + amp * w * f
    return bottom, top


@pytest.mark.parametrize("n2,dfac", [(1.5, 2.0), (1.4, 2.0), (1.5, 2.3)])
def test_slab_timing_and_fresnel_match_a_packet_trace(n2, dfac):
    """Vacuum column (n1 = 1) with a slab of index n2: the light leaving both
    ends equals a packet trace of the same hops, with the pulse delayed by the
    hop durations of each medium and split at each interface by the
    normal-incidence reflectance of Eq. 14, ((n1 - n2)/(n1 + n2))^2.  Two
    index classes with whole (dfac = 2, n2 = 1.5: D = 2 and 3) and fractional
    hop durations."""
    from oracle import optics
    L, z1, z2, steps = 10, 3, 7, 260
    dt = 1.0 / (C0 * dfac)
    p, S = _slab_column(L, z1, z2, 1.0, n2, dt)
    n2 = float(np.float32(n2))           # the medium stores float32 indices
    R0 = ((1.0 - n2) / (1.0 + n2)) ** 2
    assert abs(optics.fresnel_reflectance(1.0, n2, 1.0) - R0) < 1e-15
    assert len(S.icpt) == 4 and all(abs(e[3] - R0) < 1e-15 for e in S.icpt)
    res = retarded.forward(p, steps, S)
    q = _pulse(p, S, steps)
    nvox = np.asarray(p.n).ravel()
    hb, ht = _trace_column(L, nvox, dt, R0, steps)
    want_b = np.convolve(q, hb)[:steps]
    want_t = np.convolve(q, ht)[:steps]
    assert res.escaped[:, 5].sum() > 0.5 and res.escaped[:, 4].sum() > 0.01
    assert np.abs(res.escaped[:, 5] - want_b).max() < 1e-13
    assert np.abs(res.escaped[:, 4] - want_t).max() < 1e-13
    # nothing absorbed, the column empties: every photon leaves
    inj = res.injected.sum()
    assert abs(inj - res.escaped.sum() - res.in_domain[-1]) < 1e-13 * inj
    assert res.in_domain[-1] < 1e-9 * inj


def _air_hole_problem(source, mus=2.0, seed=6, mua=0.02):
    """Tissue (n = 1.4) around an air cylinder (n = 1, no absorption or
    scattering) of radius 2.5 mm along x, voxel noise on mu_a, stepped at a
    fifth of the crossing time of the fastest light."""
    nx, ny, nz = 9, 10, 9
    mu_a, mu_s, n = W.uniform_medium(nx, ny, nz, mua, mus, 1.4)
    rng = np.random.default_rng(seed)
    mu_a = (mu_a * rng.uniform(0.8, 1.2, mu_a.shape)).astype(np.float32)
    z, y = np.meshgrid(np.arange(nz) + 0.5, np.arange(ny) + 0.5, indexing="ij")
    cyl = np.broadcast_to(((y - 5.0) ** 2 + (z - 5.5) ** 2 <= 2.5 ** 2)[:, :, None], n.shape)
    n[cyl], mu_a[cyl], mu_s[cyl] = 1.0, 0.0, 0.0
    return W.Problem(nx=nx, ny=ny, nz=nz, dx_mm=1.0, nside=2, g=0.8, mua=mu_a, mus=mu_s, n=n,
                     steps=1, dt_ps=0.2 * 1.0 / C0, src_ix=3, src_iy=4, src_w=2, t0_ps=6.0,
                     fwhm_ps=4.0, det_face=[4, 4], det_i=[6, 7], det_j=[4, 4],
                     advance="retarded", retarded_source=source)


def test_flux_source_conserves_light_with_interfaces():
    """The flux-weighted source with unequal hops, two indices and Fresnel
    interfaces: every photon injected is absorbed or escapes, to rounding.
    The target-direction form of Eq. 10 on the same medium does not close."""
    p = _air_hole_problem("flux")
    S = retarded.build(p)
    assert len(S.icpt) > 100 and np.unique(S.nlag).size >= 3 and np.unique(S.phi).size > 3
    steps = 1100
    res = retarded.forward(p, steps, S)
    inj = res.injected.sum()
    assert res.in_domain[-1] < 1e-10 * inj
    closure = (inj - res.absorbed.sum() - res.escaped.sum() - res.in_domain[-1]) / inj
    assert abs(closure) < 1e-11, closure
    rt = retarded.forward(p.copy(retarded_source="target"), steps)
    clt = (rt.injected.sum() - rt.absorbed.sum() - rt.escaped.sum() - rt.in_domain[-1]) / inj
    assert abs(clt) > 1e-4


def test_flux_and_target_sources_agree_to_first_order():
    """One collision of the same field with both source weightings: the
    difference is second order in the hop's optical depth (it falls four-fold
    when mu_s halves), and vanishes when every hop has the same length."""
    diffs = []
    for mus in (0.04, 0.02):
        p = _air_hole_problem("flux", mus=mus, mua=0.0)
        S = retarded.build(p)
        St = retarded.build(p.copy(retarded_source="target"))
        rng = np.random.default_rng(4)
        N = rng.uniform(0.0, 1.0, S.a.shape)
        Cf, af = retarded.collide(S, N)
        Ct, at = retarded.collide(St, N)
        assert af == at
        diffs.append(np.abs(Cf - Ct).max() / N.max())
    assert 3.5 < diffs[0] / diffs[1] < 4.5, diffs
    dirs = np.array([[sx, sy, sz] for sz in (1, -1) for sy in (1, -1) for sx in (1, -1)],
                    dtype=np.float64) / math.sqrt(3.0)
    from oracle import angles
    p = _diagonal_problem(1.5, 0.37)
    P = angles.phase_matrix(dirs, 0.5)
    S = retarded.build(p.copy(retarded_source="flux"), dirs=dirs, P=P)
    St = retarded.build(p, dirs=dirs, P=P)
    N = np.random.default_rng(5).uniform(0.0, 1.0, S.a.shape)
    assert np.abs(retarded.collide(S, N)[0] - retarded.collide(St, N)[0]).max() < 1e-14


def test_flux_source_conserves_light_on_the_two_level_grid():
    """The flux-weighted source with the source on a coarser angular grid
    (192 transport, 48 scattering directions, unequal hops): every photon
    injected is absorbed or escapes, to rounding; the target-direction form
    on the same medium does not close."""
    mu_a, mu_s, n = W.uniform_medium(6, 6, 6, 0.02, 1.5, 1.4)
    p = W.Problem(nx=6, ny=6, nz=6, dx_mm=1.0, nside=4, g=0.8, mua=mu_a, mus=mu_s, n=n,
                  steps=1, dt_ps=0.2 * 1.4 / C0, src_ix=2, src_iy=2, src_w=2, t0_ps=6.0,
                  fwhm_ps=4.0, det_face=[4], det_i=[4], det_j=[2], advance="retarded",
                  nside_scatter=2, retarded_source="flux")
    S = retarded.build(p)
    assert np.unique(np.round(S.D[:, 0], 9)).size > 3
    steps = 450
    res = retarded.forward(p, steps, S)
    inj = res.injected.sum()
    assert res.in_domain[-1] < 1e-10 * inj
    closure = (inj - res.absorbed.sum() - res.escaped.sum() - res.in_domain[-1]) / inj
    assert abs(closure) < 1e-11, closure
    rt = retarded.forward(p.copy(retarded_source="target"), steps)
    clt = (rt.injected.sum() - rt.absorbed.sum() - rt.escaped.sum() - rt.in_domain[-1]) / inj
    assert abs(clt) > 1e-4, clt
