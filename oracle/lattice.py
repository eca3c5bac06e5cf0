"""Long-characteristic ray lattice (Sec. 2.1, Fig. 1; calculation Step 1).

The paper assigns rays independently of the voxel grid, each running from one
face of the box to the opposite one, and takes a voxel's intensity from the
nearest ray by a single interpolation, so no transverse numerical diffusion
builds up along a ray.  Reading used here: for direction d the box is cut into
planes normal to d's dominant axis a (|Omega_a| largest); the ray through a
voxel advances one plane per move, and at plane k it sits at the voxel nearest
to its exact crossing point, i.e. its transverse offset from the entry plane is
R(k t) with t = Omega_b / |Omega_a|.  Every voxel of plane k then has exactly
one upwind voxel in plane k-1 (shifted by R(k t) - R((k-1) t) in each
transverse axis) and exactly one downwind voxel in plane k+1.  Coefficients at
a crossing are those of the nearest voxel (Sec. 2.1, Eq. 10 text).

Test infrastructure only (see the package docstring)."""
import math

import numpy as np

AXIS_TIE = 1e-12     # axes whose |Omega| is within this of the largest count as tied
ROUND_EPS = 1e-9     # exact half-way offsets round toward zero


def dominant_axis(omega):
    """Index of the axis with the largest |Omega_a|; ties (within 1e-12) are
    broken in favour of z, then y, then x."""
    m = max(abs(omega[0]), abs(omega[1]), abs(omega[2]))
    for ax in (2, 1, 0):
        if abs(omega[ax]) >= m - AXIS_TIE:
            return ax
    raise AssertionError


def transverse_axes(a):
    """The two axes other than a, in increasing order."""
    return {0: (1, 2), 1: (0, 2), 2: (0, 1)}[a]


def nearest_offset(x):
    """Nearest integer to x, exact halves rounded toward zero; odd in x."""
    return int(math.copysign(math.floor(abs(x) + 0.5 - ROUND_EPS), x))


class RayLattice:
    """Per-direction lattice data for a grid of shape (nz, ny, nx).

    axis[d], sign[d]   dominant axis and the sign of Omega along it
    slope[d] = (t_b, t_c)  transverse advance per plane
    offset[d][q][k]    R(k t_q), the ray's transverse offset at plane k (q = 0 for
                       axis b, 1 for axis c), k = 0..n_a
    """

    def __init__(self, dirs, shape):
        self.dirs = np.asarray(dirs, dtype=np.float64)
        self.shape = tuple(shape)                  # (nz, ny, nx)
        self.ext = (shape[2], shape[1], shape[0])  # extent per axis x, y, z
        nd = len(dirs)
        self.axis = np.zeros(nd, dtype=np.int64)
        self.sign = np.zeros(nd, dtype=np.int64)
        self.slope = np.zeros((nd, 2))
        self.offset = []
        for d in range(nd):
            om = self.dirs[d]
            a = dominant_axis(om)
            b, c = transverse_axes(a)
            self.axis[d] = a
            self.sign[d] = 1 if om[a] > 0 else -1
            tb = om[b] / abs(om[a])
            tc = om[c] / abs(om[a])
            self.slope[d] = (tb, tc)
            na = self.ext[a]
            self.offset.append(np.array(
                [[nearest_offset(k * tb) for k in range(na + 1)],
                 [nearest_offset(k * tc) for k in range(na + 1)]], dtype=np.int64))

    def shift_table(self, d):
        """delta[q][k] = R(k t_q) - R((k-1) t_q) for k = 1..n_a (index 0 unused, 0)."""
        off = self.offset[d]
        delta = np.zeros_like(off)
        delta[:, 1:] = off[:, 1:] - off[:, :-1]
        return delta

    def coords(self):
        """Integer coordinates (x, y, z) of every voxel in flat order v = (z ny + y) nx + x."""
        nz, ny, nx = self.shape
        z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
        return [x.ravel(), y.ravel(), z.ravel()]

    def plane_index(self, d, p):
        """Plane k of each voxel for direction d, counted from d's entry face."""
        a = self.axis[d]
        na = self.ext[a]
        return p[a] if self.sign[d] > 0 else (na - 1 - p[a])

    def downwind(self, d):
        """For direction d and every voxel v: the flat index of the next voxel
        along v's ray (plane k+1), or -1 if the ray leaves the box; and the face
        it leaves through (face = 2 axis + side, side 1 for the high-index face),
        or -1.  When a move leaves through several faces at once (an edge or
        corner) the dominant axis counts first, then b, then c."""
        p = self.coords()
        a = self.axis[d]
        b, c = transverse_axes(a)
        s = self.sign[d]
        k = self.plane_index(d, p)
        delta = self.shift_table(d)
        na = self.ext[a]
        nv = p[0].size
        dest = np.full(nv, -1, dtype=np.int64)
        face = np.full(nv, -1, dtype=np.int64)
        last = k + 1 >= na
        face[last] = 2 * a + (1 if s > 0 else 0)
        kk = np.minimum(k + 1, na)
        q = [None, None, None]
        q[a] = p[a] + s
        q[b] = p[b] + delta[0][kk]
        q[c] = p[c] + delta[1][kk]
        for ax, dl in ((b, delta[0][kk]), (c, delta[1][kk])):
            out = (~last) & (face < 0) & ((q[ax] < 0) | (q[ax] >= self.ext[ax]))
            face[out] = 2 * ax + (dl[out] > 0).astype(np.int64)
        ok = face < 0
        nx, ny = self.ext[0], self.ext[1]
        dest[ok] = (q[2][ok] * ny + q[1][ok]) * nx + q[0][ok]
        return dest, face

    def move_fraction_phase(self, nu, m):
        """Phase mode (uniform n): at step m every photon of direction d moves one
        plane iff floor(nu_d (m+1) + 1/2) - floor(nu_d m + 1/2) = 1, so after m
        steps it has advanced floor(nu_d m + 1/2) planes, the nearest lattice
        point to the exact distance travelled."""
        return np.floor(nu * (m + 1) + 0.5) - np.floor(nu * m + 0.5)

    def plane_speed(self, ell_ref, dx):
        """nu_d: planes advanced per step by light that travels ell_ref per step."""
        return np.array([abs(self.dirs[d][self.axis[d]]) for d in range(len(self.dirs))]) \
            * ell_ref / dx
