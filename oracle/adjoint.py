"""Exact transpose of the forward step loop and the gradient of a detector
loss with respect to the per-voxel absorption and scattering coefficients.

The paper itself only runs forward models and names inversion (with machine
learning) as future work (Sec. 4); the gradient is defined here from the
forward operator.  Writing the state before collision at step m as x_m (after
injection), the step is y_m = C x_m, x_{m+1} = T_m y_m, det[:, m] = D_m y_m with
C the per-voxel collision (a_v I + b_v P), T_m the transport and D_m the
detector read-out.  For a loss L(det) with g_m = dL/d det[:, m], the adjoint
runs backwards from lambda_M = 0:
    mu_m     = T_m^T lambda_{m+1} + D_m^T g_m
    lambda_m = C^T mu_m = a mu_m + b (P^T mu_m)
    dL/da_v += sum_d mu_m[d, v] x_m[d, v]
    dL/db_v += sum_d (P^T mu_m)[d, v] x_m[d, v]
and the chain rule through (a, b)(mu_a, mu_s) gives dL/dmu_a, dL/dmu_s.

Test infrastructure only (see the package docstring)."""
import numpy as np

from . import medium, setup
from .solve import forward, move_fraction


def transport_transpose(S, lam, m):
    """T_m^T applied to lam[d, v] (no detector term)."""
    nd, nv = lam.shape
    out = np.zeros_like(lam)
    icpt_by_dv = {(d, v): (w, R, dr, dtt) for (d, v, w, R, dr, dtt) in S.icpt}
    icpt_src = {}
    for (d, v, w, R, dr, dtt) in S.icpt:
        icpt_src.setdefault(d, []).append(v)
    for d in range(nd):
        f = move_fraction(S, d, m) * np.ones(nv)
        dest = S.downwind[d]
        inside = dest >= 0
        if d in icpt_src:
            inside = inside.copy()
            inside[icpt_src[d]] = False
        ahead = np.zeros(nv)
        ahead[inside] = lam[d, dest[inside]]
        out[d] = (1.0 - f) * lam[d] + f * ahead
        for v in icpt_src.get(d, []):
            w, R, dr, dtt = icpt_by_dv[(d, v)]
            val = R * lam[dr, v]
            if dtt >= 0:
                val += (1.0 - R) * lam[dtt, w]
            out[d, v] += f[v] * val
    return out


def detector_transpose(S, g, m, shape_dv):
    """D_m^T g: detector k records f N_c[d, v_k] for accepted d leaving through its face."""
    out = np.zeros(shape_dv)
    for k, v in enumerate(S.det_vox):
        for d in S.det_acc[k]:
            if S.downwind[d][v] < 0 and S.exit_face[d][v] == S.det_face[k]:
                f = move_fraction(S, d, m)
                fv = f[v] if np.ndim(f) else f
                out[d, v] += g[k] * fv
    return out


def loss_and_seed(det, target_binned, dt, bin_ps, nbins):
    """L = sum_k sum_j (y_kj - target_kj)^2 with y = det W (rebinned), and its
    derivative with respect to det[k, m]."""
    W = setup.rebin_matrix(det.shape[1], dt, bin_ps, nbins)
    y = det @ W
    res = y - target_binned
    return float(np.sum(res * res)), 2.0 * res @ W.T


def gradient(prob, target_binned, steps=None, coef=None):
    """dL/dmu_a and dL/dmu_s per voxel (arrays shaped like prob.mua) and L."""
    coef = prob.coef if coef is None else coef
    res = forward(prob, steps=steps, keep_states=True)
    S = res.setup
    steps = res.det.shape[1]
    L, g = loss_and_seed(res.det, target_binned, S.dt, prob.bin_ps, prob.nbins)
    nd, nv = res.state.shape
    lam = np.zeros((nd, nv))
    ga = np.zeros(nv)
    gb = np.zeros(nv)
    for m in range(steps - 1, -1, -1):
        mu = transport_transpose(S, lam, m) + detector_transpose(S, g[:, m], m, (nd, nv))
        z = S.P.T @ mu
        x = res.states[m]
        ga += np.sum(mu * x, axis=0)
        gb += np.sum(z * x, axis=0)
        lam = S.a[None, :] * mu + S.b[None, :] * z
    da_a, da_s, db_a, db_s = medium.coefficient_derivatives(prob.mua, prob.mus, prob.n, S.dt, coef)
    gmua = ga * da_a.ravel() + gb * db_a.ravel()
    gmus = ga * da_s.ravel() + gb * db_s.ravel()
    return gmua.reshape(prob.shape), gmus.reshape(prob.shape), L


def loss(prob, target_binned, steps=None):
    res = forward(prob, steps=steps)
    L, _ = loss_and_seed(res.det, target_binned, res.setup.dt, prob.bin_ps, prob.nbins)
    return L


def finite_difference(prob, target_binned, voxels, rel_h=1e-4, which="mua", steps=None):
    """Central differences of L with respect to mu_a or mu_s at the given flat
    voxel indices, step h = rel_h * mu_v."""
    out = []
    for v in voxels:
        base = getattr(prob, which).astype(np.float64)
        h = rel_h * base.flat[v]
        vals = []
        for sgn in (1.0, -1.0):
            arr = base.copy()
            arr.flat[v] += sgn * h
            p = prob.copy(**{which: arr})
            vals.append(loss(p, target_binned, steps))
        out.append((vals[0] - vals[1]) / (2.0 * h))
    return np.array(out)
