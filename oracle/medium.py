"""Medium: light speed c = c0/n (Sec. 2.1), time step, path per step, and the
collision coefficients of the explicit update.

Test infrastructure only (see the package docstring)."""
import numpy as np

from .angles import eq9_weights

C0_MM_PER_PS = 0.299792458   # vacuum light speed


def reference_index(n):
    """Reading: the time step is set by the slowest-to-cross reference index;
    for a uniform medium that is n itself, otherwise the smallest n (the
    fastest light), so that no voxel moves more than one plane per step."""
    return float(np.min(n))


def time_step(dx_mm, n, dt_ps=0.0):
    """Reading: the Courant-one step dt = dx n_ref / c0 (light at c0/n_ref crosses
    one voxel per step) unless the caller fixes dt.  The paper's own runs use a
    fraction of the crossing time (Sec. 2.2, Sec. 3.1); the configurations here
    state dt = dx n / c."""
    if dt_ps > 0.0:
        return float(dt_ps)
    return dx_mm * reference_index(n) / C0_MM_PER_PS


def path_per_step(n, dt_ps):
    """Distance light travels in one step at c = c0/n (Sec. 2.1)."""
    return C0_MM_PER_PS * dt_ps / np.asarray(n, dtype=np.float64)


def collision_coefficients(mua, mus, n, dt_ps, coef="paper"):
    """Per-voxel (a, b, omega) of the collision update N_c = a N + b (P N).

    Eq. (10) advances intensity along a ray by one segment of optical depth
    dtau = (mu_a + mu_s) dr as I = I0 e^-dtau + S0 f0(dtau) + S1 f1(dtau) with
    f0, f1 from Eq. (9) and the source S = omega sum_j p I_j dOmega of Eq. (12),
    omega = mu_s/(mu_a + mu_s) (Eq. 2).  Reading: the source is taken explicitly
    (S1 := S0 = S at the upwind point and time), so a = e^-dtau and
    b = omega (f0 + f1); dr is the path per step.  A voxel without extinction
    (mu_a = mu_s = 0) has a = 1, b = 0.

    coef="abs_exact" is the alternative b = e^{-mu_a dr} (1 - e^{-mu_s dr}),
    under which absorption acts on scattered light within the step too."""
    mua = np.asarray(mua, dtype=np.float64)
    mus = np.asarray(mus, dtype=np.float64)
    ell = path_per_step(n, dt_ps)
    mut = mua + mus
    tau = mut * ell
    a = np.exp(-tau)
    omega = np.where(mut > 0.0, mus / np.where(mut > 0.0, mut, 1.0), 0.0)
    if coef == "paper":
        f0, f1 = eq9_weights(tau)
        b = omega * (f0 + f1)
    elif coef == "abs_exact":
        b = np.exp(-mua * ell) * (1.0 - np.exp(-mus * ell))
    else:
        raise ValueError(coef)
    return a, b, omega, ell


def implicit_weights(mua, mus, n, dt_ps):
    """Per-voxel (a, w0, w1) of the implicit collision: Eq. (10) with S0 the
    source of the incoming intensity and S1 that of the outgoing one, both by
    Eq. (12) at the voxel, gives for the column of a voxel
        N_c = a N + w0 P N + w1 P N_c,   a = e^-dtau, w0 = omega f0, w1 = omega f1,
    f0, f1 the Eq. (9) weights.  (Sec. 2.4 Steps 3-6 iterate this relation to
    convergence.)"""
    mua = np.asarray(mua, dtype=np.float64)
    mus = np.asarray(mus, dtype=np.float64)
    ell = path_per_step(n, dt_ps)
    mut = mua + mus
    tau = mut * ell
    omega = np.where(mut > 0.0, mus / np.where(mut > 0.0, mut, 1.0), 0.0)
    f0, f1 = eq9_weights(tau)
    return np.exp(-tau), omega * f0, omega * f1


def coefficient_derivatives(mua, mus, n, dt_ps, coef="paper"):
    """Partial derivatives of (a, b) with respect to (mu_a, mu_s), voxel by voxel.

    paper:     a = e^{-mu_t l}, b = (mu_s/mu_t)(1 - a)
               da/dmu_a = da/dmu_s = -l a
               db/dmu_a = -(mu_s/mu_t^2)(1 - a) + (mu_s/mu_t) l a
               db/dmu_s =  (mu_a/mu_t^2)(1 - a) + (mu_s/mu_t) l a
    abs_exact: b = e^{-mu_a l}(1 - e^{-mu_s l})
               db/dmu_a = -l b,  db/dmu_s = l e^{-mu_a l} e^{-mu_s l}
    Voxels with mu_t = 0 get the limits of mu_t -> 0 along mu_a = 0 (b ~ mu_s l)."""
    mua = np.asarray(mua, dtype=np.float64)
    mus = np.asarray(mus, dtype=np.float64)
    ell = path_per_step(n, dt_ps)
    mut = mua + mus
    a = np.exp(-mut * ell)
    da_dmua = -ell * a
    da_dmus = -ell * a
    if coef == "paper":
        safe = np.where(mut > 0.0, mut, 1.0)
        omega = np.where(mut > 0.0, mus / safe, 0.0)
        db_dmua = np.where(mut > 0.0, -(mus / safe ** 2) * (1.0 - a) + omega * ell * a, 0.0)
        db_dmus = np.where(mut > 0.0, (mua / safe ** 2) * (1.0 - a) + omega * ell * a, ell)
    else:
        ea = np.exp(-mua * ell)
        es = np.exp(-mus * ell)
        db_dmua = -ell * ea * (1.0 - es)
        db_dmus = ell * ea * es
    return da_dmua, da_dmus, db_dmua, db_dmus
