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
