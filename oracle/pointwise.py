"""One step of the method evaluated at single outputs (voxel, direction), for
grids too large for the whole-field oracle (a 128^3 x 768 field is 12.9 GB in
FP64 and has millions of interface crossings).

Each output of a step follows from the definitions of the whole-field oracle
(solve.collide, solve.transport; Eq. 10 with the explicit source of Eq. 2/12,
the ray lattice of Sec. 2.1 / Fig. 1, and the Eq. 13-14 routing at index jumps
read as in optics.py):

  out[d][v] = (1 - f_d(v)) Nc[d][v]                          light that stays
            + f_d(u) Nc[d][u]            u the upwind voxel of v along d, when
                                         it exists and has the same n as v
            + sum over directions d' whose move from v is intercepted with
              reflected direction d:        R f_d'(v) Nc[d'][v]
            + sum over directions d' whose move from their upwind voxel u'
              into v is intercepted with refracted direction d:
                                            (1 - R) f_d'(u') Nc[d'][u']

with Nc[:, w] = a_w N[:, w] + b_w (P N[:, w]) and f the move fraction of the
advance mode.  With scattering on a coarser angular grid (Sec. 2.1) P is the
effective fine-grid matrix of angles.two_level_matrix; with the implicit
source (Eq. 9-10 with S1 from the outgoing intensity, the fixed point of
Sec. 2.4 Steps 3-6) Nc[:, w] solves (I - w1_w P) Nc = a_w N + w0_w P N, as in
solve.collide_implicit.  Only the columns of N at v and its lattice neighbours
are read.
The lattice neighbours are found from the same per-plane offsets R(k t) that
lattice.RayLattice.downwind uses, one voxel at a time.

Test infrastructure only (see the package docstring)."""
from dataclasses import dataclass
from typing import Callable

import numpy as np

from . import angles, lattice, medium, optics


@dataclass
class LocalSetup:
    dirs: np.ndarray
    P: np.ndarray
    lat: lattice.RayLattice
    a: np.ndarray          # per voxel, flat
    b: np.ndarray
    r: np.ndarray          # n_ref / n per voxel (split mode)
    nu: np.ndarray         # planes per step at the reference path, per direction
    n: np.ndarray          # [nz, ny, nx]
    mode: str
    dt: float
    source: str = "explicit"
    w0: np.ndarray = None      # implicit source: omega f0, omega f1 per voxel, flat
    w1: np.ndarray = None


def build(prob) -> LocalSetup:
    """The per-voxel and per-direction quantities of solve.build, without the
    whole-grid downwind maps and interception list."""
    shape = (prob.nz, prob.ny, prob.nx)
    n = np.asarray(prob.n, dtype=np.float64)
    dirs = angles.healpix_ring(prob.nside)
    ns = getattr(prob, "nside_scatter", 0)
    if ns and ns != prob.nside:
        P = angles.two_level_matrix(prob.nside, ns, prob.g, prob.hg_norm)
    else:
        P = angles.phase_matrix(dirs, prob.g, prob.hg_norm)
    lat = lattice.RayLattice(dirs, shape)
    dt = medium.time_step(prob.dx_mm, n, prob.dt_ps)
    a, b, _, _ = medium.collision_coefficients(prob.mua, prob.mus, n, dt, prob.coef)
    uniform = bool(np.all(n == n.flat[0]))
    mode = prob.advance if prob.advance != "auto" else ("phase" if uniform else "split")
    n_ref = medium.reference_index(n)
    ell_ref = medium.C0_MM_PER_PS * dt / n_ref
    nu = lat.plane_speed(ell_ref, prob.dx_mm)
    source = getattr(prob, "source", "explicit")
    w0 = w1 = None
    if source == "implicit":
        _, w0, w1 = medium.implicit_weights(prob.mua, prob.mus, n, dt)
        w0, w1 = w0.ravel(), w1.ravel()
    return LocalSetup(dirs=dirs, P=P, lat=lat, a=a.ravel(), b=b.ravel(),
                      r=(n_ref / n).ravel(), nu=nu, n=n, mode=mode, dt=dt, source=source,
                      w0=w0, w1=w1)


def _coords(L: LocalSetup, v):
    nz, ny, nx = L.n.shape
    return [v % nx, (v // nx) % ny, v // (nx * ny)]


def _flat(L: LocalSetup, p):
    nz, ny, nx = L.n.shape
    return (p[2] * ny + p[1]) * nx + p[0]


def _plane(L: LocalSetup, d, p):
    a = L.lat.axis[d]
    na = L.lat.ext[a]
    return p[a] if L.lat.sign[d] > 0 else na - 1 - p[a]


def _shift(L: LocalSetup, d, q, k):
    """R(k t_q) - R((k-1) t_q), the ray's transverse step into plane k."""
    off = L.lat.offset[d][q]
    return int(off[k] - off[k - 1])


def downwind_of(L: LocalSetup, d, v):
    """The voxel after v along its ray in direction d, or -1 when the ray leaves
    the box."""
    p = _coords(L, v)
    a = L.lat.axis[d]
    b, c = lattice.transverse_axes(a)
    k = _plane(L, d, p)
    if k + 1 >= L.lat.ext[a]:
        return -1
    q = list(p)
    q[a] = p[a] + int(L.lat.sign[d])
    q[b] = p[b] + _shift(L, d, 0, k + 1)
    q[c] = p[c] + _shift(L, d, 1, k + 1)
    for ax in (b, c):
        if q[ax] < 0 or q[ax] >= L.lat.ext[ax]:
            return -1
    return _flat(L, q)


def upwind_of(L: LocalSetup, d, v):
    """The voxel whose ray in direction d continues into v, or -1 when v's ray
    enters the box at v."""
    p = _coords(L, v)
    a = L.lat.axis[d]
    b, c = lattice.transverse_axes(a)
    k = _plane(L, d, p)
    if k == 0:
        return -1
    q = list(p)
    q[a] = p[a] - int(L.lat.sign[d])
    q[b] = p[b] - _shift(L, d, 0, k)
    q[c] = p[c] - _shift(L, d, 1, k)
    for ax in (b, c):
        if q[ax] < 0 or q[ax] >= L.lat.ext[ax]:
            return -1
    return _flat(L, q)


def move_fraction(L: LocalSetup, d, w, m):
    if L.mode == "phase":
        return float(L.lat.move_fraction_phase(L.nu[d], m))
    return float(L.nu[d] * L.r[w])


def step_outputs(L: LocalSetup, column: Callable[[int], np.ndarray], v, m=0):
    """out[:, v] after one step (collide, then transport) from the state whose
    column at voxel w is column(w) (FP64, one value per direction)."""
    nd = len(L.dirs)
    nflat_v = float(L.n.flat[v])
    cache = {}

    def nc(w):
        if w not in cache:
            x = np.asarray(column(w), dtype=np.float64)
            if L.source == "implicit":
                rhs = L.a[w] * x + L.w0[w] * (L.P @ x)
                cache[w] = np.linalg.solve(np.eye(nd) - L.w1[w] * L.P, rhs)
            else:
                cache[w] = L.a[w] * x + L.b[w] * (L.P @ x)
        return cache[w]

    out = np.zeros(nd)
    for d in range(nd):
        out[d] = (1.0 - move_fraction(L, d, v, m)) * nc(v)[d]
        u = upwind_of(L, d, v)
        if u >= 0 and float(L.n.flat[u]) == nflat_v:
            out[d] += move_fraction(L, d, u, m) * nc(u)[d]
    for dp in range(nd):
        w = downwind_of(L, dp, v)
        if w >= 0 and float(L.n.flat[w]) != nflat_v:
            R, dr, _ = optics.intercept(L.lat, L.n, dp, v, w)
            out[dr] += R * move_fraction(L, dp, v, m) * nc(v)[dp]
        u = upwind_of(L, dp, v)
        if u >= 0 and float(L.n.flat[u]) != nflat_v:
            R, _, dt = optics.intercept(L.lat, L.n, dp, u, v)
            if dt >= 0:
                out[dt] += (1.0 - R) * move_fraction(L, dp, u, m) * nc(u)[dp]
    return out
