"""Refraction and reflection at refractive-index boundaries (Sec. 2.1 Eq. 13-14,
Sec. 3.3).

The paper applies Snell's law (Eq. 13) and Fresnel's reflectance (Eq. 14) at
"boundary grids", the voxels next to a region of different n, but does not say
how the reflected and refracted light is routed.  Reading used here: light is
intercepted once, when a move would carry it from voxel v into a downwind voxel
w of different index.  The fraction R goes back into v along the mirror
direction, the fraction 1 - R enters w along the refracted direction; both are
snapped to the nearest discrete direction.  The interface normal is the
direction of the index gradient at v (central differences, edge voxels
repeated), or the move itself where that gradient vanishes, oriented along
the light.

Test infrastructure only (see the package docstring)."""
import math

import numpy as np

SNAP_TIE = 1e-12


def snell_sin(n1, n2, sin1):
    """sin(theta_2) from Eq. (13): n1 / n2 = sin(theta_2) / sin(theta_1)."""
    return n1 / n2 * sin1


def fresnel_reflectance(n1, n2, cos1):
    """Eq. (14): unpolarised reflectance for light going from index n1 into n2
    at incidence angle theta_1 (cos1 = cos theta_1 >= 0):
        R = 1/2 [sin^2(t1 - t2)/sin^2(t1 + t2) + tan^2(t1 - t2)/tan^2(t1 + t2)]
    below the critical angle and R = 1 at and beyond it.  At normal incidence
    both ratios are 0/0; their limit ((n1 - n2)/(n1 + n2))^2 is used."""
    cos1 = min(max(cos1, 0.0), 1.0)
    sin1 = math.sqrt((1.0 - cos1) * (1.0 + cos1))
    sin2 = snell_sin(n1, n2, sin1)
    if sin2 >= 1.0:
        return 1.0
    if sin1 < 1e-9:
        return ((n1 - n2) / (n1 + n2)) ** 2
    t1 = math.acos(cos1)
    t2 = math.asin(sin2)
    rs = math.sin(t1 - t2) ** 2 / math.sin(t1 + t2) ** 2
    rp = math.tan(t1 - t2) ** 2 / math.tan(t1 + t2) ** 2
    return 0.5 * (rs + rp)


def critical_angle(n1, n2):
    return math.asin(n2 / n1) if n2 < n1 else math.pi / 2


def dot3(u, v):
    return (u[0] * v[0] + u[1] * v[1]) + u[2] * v[2]


def reflect(om, h):
    """Mirror direction Omega - 2 (Omega . h) h about the interface with unit normal h."""
    c = dot3(om, h)
    return (om[0] - 2.0 * c * h[0], om[1] - 2.0 * c * h[1], om[2] - 2.0 * c * h[2])


def refract(om, h, n1, n2):
    """Refracted direction (Eq. 13) for unit normal h oriented along the light
    (Omega . h = cos theta_1 > 0):
        Omega_t = (n1/n2) Omega + (cos theta_2 - (n1/n2) cos theta_1) h.
    Returns None beyond the critical angle."""
    cos1 = dot3(om, h)
    eta = n1 / n2
    sin1sq = max(0.0, 1.0 - cos1 * cos1)
    sin2sq = eta * eta * sin1sq
    if sin2sq >= 1.0:
        return None
    cos2 = math.sqrt(1.0 - sin2sq)
    k = cos2 - eta * cos1
    return (eta * om[0] + k * h[0], eta * om[1] + k * h[1], eta * om[2] + k * h[2])


def nearest_direction(dirs, v):
    """Index of the discrete direction closest to v (largest dot product; ties
    within 1e-12 go to the lowest index)."""
    dots = (dirs[:, 0] * v[0] + dirs[:, 1] * v[1]) + dirs[:, 2] * v[2]
    best = np.max(dots)
    return int(np.nonzero(dots >= best - SNAP_TIE)[0][0])


def index_gradient(nidx, x, y, z):
    """Central-difference gradient of n at voxel (x, y, z), with the edge voxel
    repeated outside the box; nidx is indexed [z, y, x]."""
    nz, ny, nx = nidx.shape

    def at(i, j, k):
        return float(nidx[min(max(k, 0), nz - 1), min(max(j, 0), ny - 1), min(max(i, 0), nx - 1)])
    return (0.5 * (at(x + 1, y, z) - at(x - 1, y, z)),
            0.5 * (at(x, y + 1, z) - at(x, y - 1, z)),
            0.5 * (at(x, y, z + 1) - at(x, y, z - 1)))


def intercept(lat, nidx, d, v, w):
    """The interception of direction d's move from voxel v into voxel w, where
    n differs: (R, d_reflected, d_refracted) as described for interceptions()."""
    nz, ny, nx = nidx.shape
    x, y, z = v % nx, (v // nx) % ny, v // (nx * ny)
    wx, wy, wz = w % nx, (w // nx) % ny, w // (nx * ny)
    gx, gy, gz = index_gradient(nidx, x, y, z)
    gn = math.sqrt((gx * gx + gy * gy) + gz * gz)
    if gn > 0.0:
        h = (gx / gn, gy / gn, gz / gn)
    else:
        sx, sy, sz = float(wx - x), float(wy - y), float(wz - z)
        sn = math.sqrt((sx * sx + sy * sy) + sz * sz)
        h = (sx / sn, sy / sn, sz / sn)
    om = tuple(lat.dirs[d])
    if dot3(om, h) < 0.0:
        h = (-h[0], -h[1], -h[2])
    n1, n2 = float(nidx[z, y, x]), float(nidx[wz, wy, wx])
    cos1 = dot3(om, h)
    R = fresnel_reflectance(n1, n2, cos1)
    dr = nearest_direction(lat.dirs, reflect(om, h))
    t = refract(om, h, n1, n2)
    if t is None:
        R = 1.0
    dt = -1 if R >= 1.0 else nearest_direction(lat.dirs, t)
    return R, dr, dt


def interceptions(lat, nidx):
    """All interface crossings of the lattice for index field nidx [z, y, x].

    Returns a list of tuples (d, v, w, R, d_reflected, d_refracted) for every
    direction d and voxel v whose downwind voxel w has a different n:
    R of Eq. (14), d_reflected the direction snapped from the mirror direction
    and d_refracted the one snapped from Snell's direction (-1 under total
    internal reflection)."""
    nflat = np.asarray(nidx, dtype=np.float64).ravel()
    out = []
    for d in range(len(lat.dirs)):
        dest, _ = lat.downwind(d)
        v_all = np.nonzero(dest >= 0)[0]
        diff = v_all[nflat[dest[v_all]] != nflat[v_all]]
        for v in diff:
            v = int(v)
            w = int(dest[v])
            R, dr, dt = intercept(lat, nidx, d, v, w)
            out.append((d, v, w, R, dr, dt))
    return out
