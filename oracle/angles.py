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


def healpix_pixel_ring(nside, v):
    """Index, in the order of healpix_ring(nside), of the HEALPix pixel
    (Gorski et al. 2005) that contains the unit vector v.  With z = cos(theta)
    and t = 2 phi / pi in [0, 4):
    equatorial zone |z| <= 2/3: the pixel boundaries are the lines
    nside (1/2 + t) -/+ (3/4) nside z = const, which give the ascending and
    descending edge indices jp, jm, the ring ir = nside + 1 + jp - jm counted
    from z = 2/3, and the pixel ((jp + jm - nside + shift + 1) / 2) mod 4 nside
    counted from azimuth 0 (shift = 1 on even ir).  healpix_ring numbers the
    rings with shift = 1 from azimuth pi / (2 nside) instead (j = 1 .. 4 nside
    in its azimuth formula), one pixel later;
    polar caps: with x = nside sqrt(3 (1 - |z|)) and the fractional part f of t,
    jp = floor(f x), jm = floor((1 - f) x), the ring from the pole is
    ir = jp + jm + 1, and the pixel is floor(t ir) in it."""
    x, y, z = float(v[0]), float(v[1]), float(v[2])
    phi = math.atan2(y, x)
    if phi < 0.0:
        phi += 2.0 * math.pi
    t = (2.0 * phi / math.pi) % 4.0
    za = abs(z)
    npix = 12 * nside * nside
    if za <= 2.0 / 3.0:
        t1 = nside * (0.5 + t)
        t2 = nside * z * 0.75
        jp = int(math.floor(t1 - t2))
        jm = int(math.floor(t1 + t2))
        ir = nside + 1 + jp - jm
        shift = 1 - (ir & 1)
        ip = ((jp + jm - nside + shift + 1) // 2) % (4 * nside)
        if shift:
            ip = (ip - 1) % (4 * nside)
        return 2 * nside * (nside - 1) + (ir - 1) * 4 * nside + ip
    f = t - math.floor(t)
    xx = nside * math.sqrt(3.0 * (1.0 - za))
    jp = int(math.floor(f * xx))
    jm = int(math.floor((1.0 - f) * xx))
    ir = jp + jm + 1
    ip = int(math.floor(t * ir)) % (4 * ir)
    if z > 0.0:
        return 2 * ir * (ir - 1) + ip
    return npix - 2 * ir * (ir + 1) + ip


def parents(nside, nside_scatter):
    """For each direction of the fine grid (nside), the coarse direction
    (nside_scatter) whose pixel contains it.  HEALPix is hierarchical, so each
    coarse pixel holds exactly (nside / nside_scatter)^2 fine pixels."""
    return np.array([healpix_pixel_ring(nside_scatter, v) for v in healpix_ring(nside)])


def two_level_matrix(nside, nside_scatter, g, norm="sinkhorn"):
    """Scattering on a coarser angular grid (Sec. 2.1: the source is computed
    from the mean intensity over the 16 fine bins of each coarse bin).  In
    photon numbers: the photons of a coarse bin are the sum over its children,
    the coarse phase matrix scatters them, and each child of the target bin
    receives an equal share:  P_eff = C P_c A  with A[J][i] = 1 for the parent
    J of i and C[i][J] = 1 / (children per bin)."""
    par = parents(nside, nside_scatter)
    nc = 12 * nside_scatter * nside_scatter
    Pc = phase_matrix(healpix_ring(nside_scatter), g, norm)
    A = np.zeros((nc, len(par)))
    A[par, np.arange(len(par))] = 1.0
    C = A.T / (nside // nside_scatter) ** 2
    return C @ Pc @ A


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
