"""Pins of the oracle adjoint: transpose identities, finite differences and
the analytic absorption derivative of a non-scattering medium."""
import numpy as np
import pytest

from oracle import adjoint, solve
from paper_2105_01028_amd import workloads as W


def _problem(advance="phase", refract=False, steps=14):
    p = W.small_problem(nside=2, nx=7, ny=6, nz=6, mua=0.05, mus=1.5, g=0.7, n=1.4, steps=steps,
                        seed=21, advance=advance, det_cone_deg=0.0)
    if refract:
        n = p.n.copy()
        n[3:, :, :] = 1.0
        mus = p.mus.copy()
        mus[3:] *= 0.3
        p = p.copy(n=n, mus=mus)
    return p


@pytest.mark.parametrize("advance,refract", [("phase", False), ("split", False), ("split", True)])
def test_transport_transpose_dot_product(advance, refract):
    p = _problem(advance, refract)
    S = solve.build(p)
    rng = np.random.default_rng(2)
    nd, nv = len(S.dirs), p.nvox
    for m in (0, 3):
        x = rng.normal(size=(nd, nv))
        lam = rng.normal(size=(nd, nv))
        Tx, _, _ = solve.transport(S, x, m, len(S.det_vox))
        TtL = adjoint.transport_transpose(S, lam, m)
        assert abs(np.sum(lam * Tx) - np.sum(TtL * x)) < 1e-11 * np.sum(np.abs(lam * Tx))


def test_detector_transpose_dot_product():
    p = _problem("split")
    S = solve.build(p)
    rng = np.random.default_rng(3)
    nd, nv = len(S.dirs), p.nvox
    x = rng.normal(size=(nd, nv))
    g = rng.normal(size=len(S.det_vox))
    _, _, det = solve.transport(S, x, 2, len(S.det_vox))
    Dt = adjoint.detector_transpose(S, g, 2, (nd, nv))
    assert abs(np.dot(g, det) - np.sum(Dt * x)) < 1e-12


@pytest.mark.parametrize("advance,refract", [("phase", False), ("split", True)])
def test_gradient_matches_finite_differences(advance, refract):
    p = _problem(advance, refract)
    ref = p.copy(mua=(p.mua * 1.3).astype(np.float32))
    target = solve.forward(ref).binned(p.bin_ps, p.nbins)
    gmua, gmus, L = adjoint.gradient(p, target)
    assert L > 0
    rng = np.random.default_rng(55)
    vox = rng.choice(p.nvox, 6, replace=False)
    for which, g in (("mua", gmua), ("mus", gmus)):
        fd = adjoint.finite_difference(p, target, vox, 1e-4, which)
        ad = g.ravel()[vox]
        scale = np.abs(ad).max()
        assert scale > 0
        assert np.abs(fd - ad).max() < 1e-6 * scale + 1e-8 * np.abs(g).max(), (which, fd, ad)


def test_absorption_derivative_without_scattering():
    """mu_s = 0, uniform mu_a, a pulse that lies inside the first step: light
    leaving at step m has collided m + 1 times, det[m] = e^{-mu_a l (m+1)} det0[m],
    so dL/dmu_a summed over all voxels equals sum_m dL/ddet[m] (-l (m+1)) det[m]."""
    dets = ([5] * 16, [i for i in range(1, 5) for _ in range(4)], [j for _ in range(4)
                                                                    for j in range(1, 5)])
    p = W.small_problem(nside=2, nx=6, ny=6, nz=5, mua=0.04, mus=0.0, g=0.0, n=1.4, steps=16,
                        det_cone_deg=0.0, dets=dets, t0_ps=1.0, fwhm_ps=0.01)
    res = solve.forward(p)
    target = 0.5 * res.binned(p.bin_ps, p.nbins)
    gmua, gmus, L = adjoint.gradient(p, target)
    _, seed = adjoint.loss_and_seed(res.det, target, res.setup.dt, p.bin_ps, p.nbins)
    ell = res.setup.ell[0]
    m = np.arange(p.steps)
    want = np.sum(seed * res.det * (-ell * (m + 1))[None, :])
    assert res.det.sum() > 0.5
    assert abs(gmua.sum() - want) < 1e-10 * abs(want)


@pytest.mark.parametrize("coef", ["paper", "abs_exact"])
def test_coefficient_derivatives_match_finite_differences(coef):
    """The chain-rule factors da/dmu and db/dmu of both coefficient forms
    against central differences of the coefficients themselves (which the
    impulse pins tie to Eq. 9-10 and to the abs_exact factorisation), over
    thin, moderate and thick voxels, including a voxel without absorption."""
    from oracle import medium
    mua = np.array([0.0, 1e-3, 0.01, 0.05, 0.3, 2.0, 0.02])
    mus = np.array([0.5, 10.0, 8.0, 1.5, 0.0, 3.0, 1e-4])
    n = np.array([1.4, 1.0, 1.5, 1.33, 1.4, 1.6, 1.0])
    dt = 4.67
    an = medium.coefficient_derivatives(mua, mus, n, dt, coef)
    for k, (which, i_a, i_b) in enumerate((("mua", 0, 2), ("mus", 1, 3))):
        h = 1e-5 * np.maximum(mua if which == "mua" else mus, 1e-2)
        def coeffs(delta):
            if which == "mua":
                a, b, _, _ = medium.collision_coefficients(mua + delta, mus, n, dt, coef)
            else:
                a, b, _, _ = medium.collision_coefficients(mua, mus + delta, n, dt, coef)
            return a, b
        ap, bp = coeffs(h)
        am, bm = coeffs(-h)
        fd_a = (ap - am) / (2 * h)
        fd_b = (bp - bm) / (2 * h)
        ok = (mua if which == "mua" else mus) > 0      # central difference stays in mu >= 0
        # truncation ~ h^2, rounding ~ 1e-16 / h: both far below the tolerance
        np.testing.assert_allclose(an[i_a][ok], fd_a[ok], rtol=1e-6, atol=1e-9)
        np.testing.assert_allclose(an[i_b][ok], fd_b[ok], rtol=1e-6, atol=1e-9)


def test_gradient_matches_finite_differences_abs_exact():
    """The whole adjoint with the abs_exact coefficients (db/dmu of that form)
    against central differences of the loss."""
    p = _problem("phase").copy(coef="abs_exact")
    ref = p.copy(mua=(p.mua * 1.3).astype(np.float32))
    target = solve.forward(ref).binned(p.bin_ps, p.nbins)
    gmua, gmus, L = adjoint.gradient(p, target)
    assert L > 0
    rng = np.random.default_rng(56)
    vox = rng.choice(p.nvox, 6, replace=False)
    for which, g in (("mua", gmua), ("mus", gmus)):
        fd = adjoint.finite_difference(p, target, vox, 1e-4, which)
        ad = g.ravel()[vox]
        scale = np.abs(ad).max()
        assert scale > 0
        assert np.abs(fd - ad).max() < 1e-6 * scale + 1e-8 * np.abs(g).max(), (which, fd, ad)
