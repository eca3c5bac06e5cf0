"""Angular discretisation (Sec. 2.1): HEALPix directions, the Henyey-Greenstein
phase function of Eq. (11) and its discrete form p(Omega_j, Omega) dOmega of
Eq. (12), and the Eq. (9) source weights.

Test infrastructure only (see the package docstring)."""
import math

import numpy as np

FOUR_PI = 4.0 * math.pi


def healpix_ring(nside):
    """Pixel centres of the HEALPix tessellation (Gorski et al. 2005, the
    equal-area hierarchical grid the paper adopts for its angle bins, Sec. 2.1),
    in RING order: rings from the north pole (+z) to the south pole, pixels in
    each ring by increasing azimuth.  N = 12 nside^2 unit vectors.

    Polar caps: ring i (i < nside) has 4i pixels at z = 1 - i^2/(3 nside^2),
    azimuths (pi / 2i)(j - 1/2).  Equatorial belt: ring i (nside <= i <= 3 nside)
    has 4 nside pixels at z = 4/3 - 2i/(3 nside), azimuths (pi / 2 nside)(j - s/2)
    with s = (i - nside + 1) mod 2.  The south cap mirrors the north cap."""
    out = []
    for i in range(1, 4 * nside):
        if i < nside:
            z = 1.0 - i * i / (3.0 * nside * nside)
            phis = [math.pi / (2.0 * i) * (j - 0.5) for j in range(1, 4 * i + 1)]
        elif i <= 3 * nside:
            z = 4.0 / 3.0 - 2.0 * i / (3.0 * nside)
            s = (i - nside + 1) % 2
            phis = [math.pi / (2.0 * nside) * (j - s / 2.0) for j in range(1, 4 * nside + 1)]
        else:
            k = 4 * nside - i
            z = -(1.0 - k * k / (3.0 * nside * nside))
            phis = [math.pi / (2.0 * k) * (j - 0.5) for j in range(1, 4 * k + 1)]
        st = math.sqrt((1.0 - z) * (1.0 + z))
        for phi in phis:
            out.append((st * math.cos(phi), st * math.sin(phi), z))
    return np.array(out, dtype=np.float64)


def hg(mu, g):
    """Henyey-Greenstein phase function of the scattering cosine mu, Eq. (11)."""
    return (1.0 - g * g) / (FOUR_PI * (1.0 + g * g - 2.0 * g * mu) ** 1.5)


def cosine_matrix(dirs):
    """Omega_i . Omega_j, summed in the fixed order x, y, z."""
    c = (dirs[:, None, 0] * dirs[None, :, 0] + dirs[:, None, 1] * dirs[None, :, 1]) \
        + dirs[:, None, 2] * dirs[None, :, 2]
    return np.clip(c, -1.0, 1.0)


def phase_kernel(dirs, g):
    """K_ij = p(Omega_i . Omega_j) dOmega with dOmega = 4 pi / N: the weight that
    the discrete source sum of Eq. (12) gives intensity in direction j when
    forming the source in direction i."""
    n = len(dirs)
    return (FOUR_PI / n) * hg(cosine_matrix(dirs), g)


def phase_matrix(dirs, g, norm="sinkhorn", tol=1e-14, max_iter=200000):
    """Discrete scattering matrix P used in S_i = omega sum_j P_ij I_j.

    The paper normalises the continuous phase function to one over the sphere
    (Sec. 2.1) but says nothing of its discrete sum.  Reading: the point-sampled
    kernel K is scaled to P = D K D (D diagonal, positive) so that every row and
    every column sums to one; then scattering neither creates nor destroys
    photons and P stays symmetric.  The scaling is found by the symmetric
    Sinkhorn iteration d <- sqrt(d / (K d)), whose fixed point satisfies
    d_i (K d)_i = 1.  norm="row" instead divides each row by its sum (rows sum
    to one, columns in general do not)."""
    K = phase_kernel(dirs, g)
    if norm == "row":
        return K / K.sum(axis=1, keepdims=True)
    if norm != "sinkhorn":
        raise ValueError(norm)
    d = np.ones(len(dirs))
    for _ in range(max_iter):
        Kd = K @ d
        if np.max(np.abs(d * Kd - 1.0)) < tol:
            break
        d = np.sqrt(d / Kd)
    else:
        raise RuntimeError("Sinkhorn scaling did not converge")
    return d[:, None] * K * d[None, :]


def mean_cosine(P, dirs):
    """Average over incoming directions of the mean scattering cosine of P
    (the effective anisotropy g of the discrete matrix)."""
    c = cosine_matrix(dirs)
    return float(np.mean(np.sum(P * c, axis=0)))


def eq9_weights(tau):
    """Weights of S0 and S1 in the discretised formal solution, Eq. (9):
    f0 = [1 - (1 + tau) e^-tau] / tau and f1 = [tau - 1 + e^-tau] / tau, for an
    array of optical depths tau >= 0.  Below tau = 0.1 both are evaluated from
    their Taylor series (term n of f0 is (-1)^n (n-1)/n! tau^(n-1), of f1 is
    (-1)^n / n! tau^(n-1), n >= 2) to avoid cancellation; at tau = 0 both are 0."""
    tau = np.asarray(tau, dtype=np.float64)
    f0 = np.zeros_like(tau)
    f1 = np.zeros_like(tau)
    small = tau < 0.1
    big = ~small
    t = tau[big]
    e = np.exp(-t)
    f0[big] = (1.0 - (1.0 + t) * e) / t
    f1[big] = (t - 1.0 + e) / t
    ts = tau[small]
    for nn in range(18, 1, -1):
        fact = math.factorial(nn)
        f0[small] = f0[small] * 1.0 + ((-1) ** nn) * (nn - 1) / fact * ts ** (nn - 1)
        f1[small] = f1[small] * 1.0 + ((-1) ** nn) / fact * ts ** (nn - 1)
    return f0, f1
