"""Source, detectors, pulse and time bins (Sec. 3.1: a pulse collimated within
15 degrees injected at a surface point, detectors with the same opening angle,
time-resolved signals as in Fig. 9).

Test infrastructure only (see the package docstring)."""
import math

import numpy as np

FACE_NORMALS = {0: (-1.0, 0.0, 0.0), 1: (1.0, 0.0, 0.0), 2: (0.0, -1.0, 0.0),
                3: (0.0, 1.0, 0.0), 4: (0.0, 0.0, -1.0), 5: (0.0, 0.0, 1.0)}


def cone_set(dirs, axis_vec, cone_deg, fallback=4):
    """Directions whose centre lies within cone_deg of axis_vec.  Reading: when
    the angular grid is too coarse to place any centre inside the cone, the
    `fallback` directions nearest to the axis are used (ties by index)."""
    dots = (dirs[:, 0] * axis_vec[0] + dirs[:, 1] * axis_vec[1]) + dirs[:, 2] * axis_vec[2]
    inside = np.nonzero(dots >= math.cos(math.radians(cone_deg)))[0]
    if len(inside) > 0:
        return [int(i) for i in inside]
    order = sorted(range(len(dirs)), key=lambda i: (-dots[i], i))
    return sorted(order[:fallback])


def source_voxels(shape, ix, iy, w):
    """Top-face (z = 0) voxels that receive the pulse: (ix, iy) alone, or the
    2x2 block (ix..ix+1, iy..iy+1), which is centred on a face centre of an
    even grid."""
    nz, ny, nx = shape
    out = []
    for dy in range(w):
        for dx in range(w):
            out.append((0 * ny + iy + dy) * nx + ix + dx)
    return out


def source_directions(dirs, cone_deg):
    """Collimated pulse: directions within cone_deg of the inward normal +z."""
    return cone_set(dirs, (0.0, 0.0, 1.0), cone_deg)


def pulse_weight(m, dt_ps, t0_ps, fwhm_ps, total=1.0):
    """q_m: photons injected during step m = [m dt, (m+1) dt) by a Gaussian pulse
    of the given FWHM centred at t0, i.e. the Gaussian's integral over the step,
    q_m = Phi((t_{m+1} - t0)/sigma) - Phi((t_m - t0)/sigma),
    sigma = FWHM / (2 sqrt(2 ln 2)), scaled so that the pulse after t = 0 holds
    `total` photons."""
    sigma = fwhm_ps / (2.0 * math.sqrt(2.0 * math.log(2.0)))

    def cdf(t):
        return 0.5 * (1.0 + math.erf((t - t0_ps) / (sigma * math.sqrt(2.0))))
    tail = 1.0 - cdf(0.0)
    return (cdf((m + 1) * dt_ps) - cdf(m * dt_ps)) / tail * total


def pulse_weights(steps, dt_ps, t0_ps, fwhm_ps, total=1.0):
    return np.array([pulse_weight(m, dt_ps, t0_ps, fwhm_ps, total) for m in range(steps)])


def detector_voxel(shape, face, i, j):
    """Voxel of a detector patch: face = 2 axis + side, (i, j) the voxel indices
    along the two other axes in increasing axis order."""
    nz, ny, nx = shape
    ext = (nx, ny, nz)
    axis, side = face // 2, face % 2
    p = [0, 0, 0]
    p[axis] = ext[axis] - 1 if side == 1 else 0
    others = [q for q in range(3) if q != axis]
    p[others[0]] = i
    p[others[1]] = j
    return (p[2] * ny + p[1]) * nx + p[0]


def detector_acceptance(dirs, face, cone_deg):
    """Directions a detector records: within cone_deg of the face's outward
    normal (the same opening angle as the source, Sec. 3.1), or all directions
    when cone_deg <= 0."""
    if cone_deg <= 0.0:
        return list(range(len(dirs)))
    return cone_set(dirs, FACE_NORMALS[face], cone_deg)


def rebin_matrix(steps, dt_ps, bin_ps, nbins):
    """W[m, j] = |[m dt, (m+1) dt) intersect [j bin, (j+1) bin)| / dt: the light
    that leaves during step m is spread evenly over that step's interval and
    summed into fixed-width time bins."""
    W = np.zeros((steps, nbins))
    for m in range(steps):
        t0, t1 = m * dt_ps, (m + 1) * dt_ps
        j0 = int(math.floor(t0 / bin_ps))
        j1 = int(math.ceil(t1 / bin_ps))
        for j in range(max(j0, 0), min(j1, nbins)):
            lo = max(t0, j * bin_ps)
            hi = min(t1, (j + 1) * bin_ps)
            if hi > lo:
                W[m, j] = (hi - lo) / dt_ps
    return W
