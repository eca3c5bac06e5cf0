"""Seeded synthetic workloads for the time-dependent radiative-transfer solve.

This module only *describes* problems: voxel grids of optical properties,
where the pulsed source sits, where the detectors sit, how many steps to run.
It holds none of the method's arithmetic (no directions, no phase matrix, no
time step, no coefficients): both the HIP library and the FP64 oracle derive
those from the numbers stored here, each in its own code.

Media follow the shapes of the paper's phantom studies: a uniform tissue-like
block (Sec. 3.1, Table 1), spherical absorbers with raised mu_a (Sec. 3.2) and
an air-filled cylinder with a different refractive index (Sec. 3.3).  Lengths
are in mm, coefficients in 1/mm, times in ps.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import List, Tuple

import numpy as np

# Face numbering shared by the C-ABI and the tests: face = 2*axis + side, with
# axis 0 = x, 1 = y, 2 = z (z is depth, the top face is z = 0) and side 0 the
# low-index face, side 1 the high-index face.
FACE_TOP = 4
FACE_XMAX = 1


@dataclass
class Problem:
    """One forward solve: medium, source, detectors and step count."""
    nx: int
    ny: int
    nz: int
    dx_mm: float
    nside: int
    g: float
    mua: np.ndarray          # float32 [nz, ny, nx]
    mus: np.ndarray          # float32 [nz, ny, nx]
    n: np.ndarray            # float32 [nz, ny, nx]
    steps: int
    dt_ps: float = 0.0       # 0 => derived from the medium
    hg_norm: str = "sinkhorn"   # "sinkhorn" | "row"
    coef: str = "paper"         # "paper" | "abs_exact"
    advance: str = "auto"       # "auto" | "phase" | "split" | "retarded" (Courant < 1 history)
    precision: str = "fp32"     # "fp32" | "bf16split"
    source: str = "explicit"    # "explicit" | "implicit" (S1 from the new intensity, Eq. 9-10)
    nside_scatter: int = 0      # 0: scatter on the transport directions; else a coarser
                                # HEALPix grid (nside / nside_scatter a power of two)
    transport: str = "auto"     # "auto": phase moves in the collision kernel where it
                                # applies | "sweep": always the separate sweep kernel
    retarded_source: str = "target"   # retarded advance: "target" (the target direction's
                                      # 1 - e^-dtau weights the source) | "flux" (the
                                      # scattered flux of each direction, conservative)
    src_ix: int = 0
    src_iy: int = 0
    src_w: int = 2           # 1 = one top-face voxel, 2 = the 2x2 block at (ix..ix+1, iy..iy+1)
    src_cone_deg: float = 15.0
    t0_ps: float = 20.0
    fwhm_ps: float = 10.0
    total_photons: float = 1.0
    det_face: List[int] = field(default_factory=list)
    det_i: List[int] = field(default_factory=list)
    det_j: List[int] = field(default_factory=list)
    det_cone_deg: float = 15.0   # <= 0 => every direction leaving through the patch
    bin_ps: float = 1.0
    nbins: int = 0
    name: str = ""

    @property
    def shape(self) -> Tuple[int, int, int]:
        return (self.nz, self.ny, self.nx)

    @property
    def nvox(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def ndir(self) -> int:
        return 12 * self.nside * self.nside

    @property
    def ndet(self) -> int:
        return len(self.det_face)

    def copy(self, **kw) -> "Problem":
        out = replace(self, **kw)
        for k in ("mua", "mus", "n"):
            if k not in kw:
                setattr(out, k, getattr(self, k).copy())
        return out


def uniform_medium(nx, ny, nz, mua, mus, n):
    shape = (nz, ny, nx)
    return (np.full(shape, mua, np.float32), np.full(shape, mus, np.float32),
            np.full(shape, n, np.float32))


def surface_line_detectors(nx, nz, dx, cx_mm, cy_mm, distances_mm):
    """Detectors at the given surface distances along +x from (cx, cy) on the
    top face.  A distance that runs past the x = max edge folds over the edge
    onto the x = max face, at depth (distance - remaining top-face length).
    Returns (face, i, j) lists; (i, j) are the in-face voxel indices, the two
    other axes in increasing axis order."""
    faces, ii, jj = [], [], []
    width = nx * dx
    cy = int(np.floor(cy_mm / dx))
    for d in distances_mm:
        x = cx_mm + d
        if x < width:
            faces.append(FACE_TOP)
            ii.append(int(np.floor(x / dx)))
            jj.append(cy)
        else:
            depth = x - width
            faces.append(FACE_XMAX)
            ii.append(cy)
            jj.append(min(int(np.floor(depth / dx)), nz - 1))
    return faces, ii, jj


def config1() -> Problem:
    """16^3 uniform medium, 48 directions, 200 steps, 8 detectors 2-14 mm."""
    nx = ny = nz = 16
    mua, mus, n = uniform_medium(nx, ny, nz, 0.01, 10.0, 1.4)
    f, i, j = surface_line_detectors(nx, nz, 1.0, 8.0, 8.0, np.linspace(2.0, 14.0, 8))
    return Problem(nx=nx, ny=ny, nz=nz, dx_mm=1.0, nside=2, g=0.9, mua=mua, mus=mus, n=n,
                   steps=200, src_ix=7, src_iy=7, src_w=2, det_face=f, det_i=i, det_j=j,
                   nbins=934, name="uniform 16^3, 48 dirs, 200 steps")


def _noise(rng, shape, lo=0.95, hi=1.05):
    return rng.uniform(lo, hi, size=shape)


def config2(seed: int = 2) -> Problem:
    """64^3 phantom-scale medium with +-5% voxel noise, 192 directions, 1000 steps."""
    nx = ny = nz = 64
    rng = np.random.default_rng(seed)
    shape = (nz, ny, nx)
    mua = (0.005 * _noise(rng, shape)).astype(np.float32)
    mus = (8.0 * _noise(rng, shape)).astype(np.float32)
    n = np.full(shape, 1.5, np.float32)
    f, i, j = surface_line_detectors(nx, nz, 1.0, 32.0, 32.0, np.arange(5.0, 41.0, 5.0))
    return Problem(nx=nx, ny=ny, nz=nz, dx_mm=1.0, nside=4, g=0.85, mua=mua, mus=mus, n=n,
                   steps=1000, src_ix=31, src_iy=31, src_w=2, det_face=f, det_i=i, det_j=j,
                   nbins=5004, name="phantom 64^3 +-5% noise, 192 dirs, 1000 steps")


def fiducial101(seed: int = 2) -> Problem:
    """The paper's fiducial phantom run at its own size (Sec. 3.1 and the
    timing of Sec. 4): a 4 cm box at 0.4 mm (101^3 voxels), 3072 transport
    directions with the source on 192, time step 0.4 ps (a fifth of the
    crossing time at n = 1.5), 8680 steps.  The medium takes the values of the
    64^3 phantom (+-5 % voxel noise)."""
    nx = ny = nz = 101
    rng = np.random.default_rng(seed)
    shape = (nz, ny, nx)
    mua = (0.005 * _noise(rng, shape)).astype(np.float32)
    mus = (8.0 * _noise(rng, shape)).astype(np.float32)
    n = np.full(shape, 1.5, np.float32)
    f, i, j = surface_line_detectors(nx, nz, 0.4, 20.0, 20.0, np.arange(5.0, 41.0, 5.0))
    return Problem(nx=nx, ny=ny, nz=nz, dx_mm=0.4, nside=16, nside_scatter=4, g=0.85, mua=mua,
                   mus=mus, n=n, steps=8680, dt_ps=0.4, advance="retarded", src_ix=49,
                   src_iy=49, src_w=2, det_face=f, det_i=i, det_j=j, nbins=3500,
                   name="fiducial phantom 101^3 at 0.4 mm, 3072/192 directions, 0.4 ps")


def _voxel_centres(nx, ny, nz, dx):
    z, y, x = np.meshgrid((np.arange(nz) + 0.5) * dx, (np.arange(ny) + 0.5) * dx,
                          (np.arange(nx) + 0.5) * dx, indexing="ij")
    return x, y, z


def _place_spheres(rng, count, rmin, rmax, box_mm, avoid=None):
    """Rejection-sample sphere centres with a (r + 2 mm) margin to the faces and
    no overlap with the 'avoid' cylinder (axis along x at (y0, z0), radius rc)."""
    out = []
    while len(out) < count:
        r = rng.uniform(rmin, rmax)
        c = rng.uniform(r + 2.0, box_mm - r - 2.0, size=3)
        if avoid is not None:
            y0, z0, rc = avoid
            if np.hypot(c[1] - y0, c[2] - z0) < r + rc:
                continue
        out.append((c, r))
    return out


def config3(seed: int = 3, nx: int = 128) -> Problem:
    """128^3 medium with an air cylinder along x (n = 1.0, no absorption or
    scattering) and three absorbing spheres (mu_a x U[2, 5]); 768 directions."""
    ny = nz = nx
    scale = nx / 128.0
    dx = 1.0
    mua, mus, n = uniform_medium(nx, ny, nz, 0.01, 10.0, 1.4)
    x, y, z = _voxel_centres(nx, ny, nz, dx)
    y0, z0, rc = 64.0 * scale, 32.0 * scale, 6.0 * scale
    rng = np.random.default_rng(seed)
    for c, r in _place_spheres(rng, 3, 4.0 * scale, 8.0 * scale, nx * dx, avoid=(y0, z0, rc)):
        inside = (x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2 <= r * r
        mua[inside] = np.float32(0.01 * rng.uniform(2.0, 5.0))
    cyl = (y - y0) ** 2 + (z - z0) ** 2 <= rc * rc
    mua[cyl] = 0.0
    mus[cyl] = 0.0
    n[cyl] = 1.0
    half = nx * dx / 2.0
    dists = np.arange(5.0, 41.0, 5.0) * scale
    f, i, j = surface_line_detectors(nx, nz, dx, half, half, dists)
    return Problem(nx=nx, ny=ny, nz=nz, dx_mm=dx, nside=8, g=0.9, mua=mua, mus=mus, n=n,
                   steps=2000, src_ix=nx // 2 - 1, src_iy=ny // 2 - 1, src_w=2,
                   det_face=f, det_i=i, det_j=j, nbins=6672,
                   name=f"heterogeneous {nx}^3 with air cylinder, 768 dirs, 2000 steps")


def config5(seed: int = 5, perturbed: bool = False) -> Problem:
    """64^3 adjoint medium: config-2 style noise plus three absorbing spheres of
    radius 2-4 mm.  perturbed=True raises each sphere's mu_a by 20 % (the
    target medium of the gradient study)."""
    nx = ny = nz = 64
    rng = np.random.default_rng(seed)
    shape = (nz, ny, nx)
    mua = 0.005 * _noise(rng, shape)
    mus = 8.0 * _noise(rng, shape)
    x, y, z = _voxel_centres(nx, ny, nz, 1.0)
    for c, r in _place_spheres(rng, 3, 2.0, 4.0, 64.0):
        inside = (x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2 <= r * r
        fac = rng.uniform(2.0, 5.0) * (1.2 if perturbed else 1.0)
        mua[inside] = mua[inside] * fac
    n = np.full(shape, 1.5, np.float32)
    f, i, j = surface_line_detectors(nx, nz, 1.0, 32.0, 32.0, np.arange(5.0, 41.0, 5.0))
    return Problem(nx=nx, ny=ny, nz=nz, dx_mm=1.0, nside=4, g=0.85,
                   mua=mua.astype(np.float32), mus=mus.astype(np.float32), n=n,
                   steps=500, src_ix=31, src_iy=31, src_w=2, det_face=f, det_i=i, det_j=j,
                   nbins=2502, name="adjoint 64^3 with inclusions, 192 dirs, 500 steps")


@dataclass
class Request:
    arrival_s: float
    problem: Problem


def serving_stream(count: int, seed: int = 4, rate_per_s: float = 200.0,
                   sides=(32, 48, 64, 96), steps_range=(500, 1500),
                   sigma: float = 0.2) -> List[Request]:
    """Poisson arrivals of forward solves as a DOT reconstruction would issue
    them: grid side drawn from `sides`, 192 directions, random source voxel and
    8 random detectors on the top face, lognormal per-voxel mu_a and mu_s
    around the phantom medium (mean preserved)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for _ in range(count):
        t += rng.exponential(1.0 / rate_per_s)
        side = int(rng.choice(sides))
        steps = int(rng.integers(steps_range[0], steps_range[1] + 1))
        shape = (side, side, side)
        lm = lambda base: (base * np.exp(sigma * rng.standard_normal(shape) - sigma ** 2 / 2)
                           ).astype(np.float32)
        mua = lm(0.005)
        mus = lm(8.0)
        n = np.full(shape, 1.5, np.float32)
        sx, sy = (int(v) for v in rng.integers(2, side - 2, size=2))
        fi, fj = [], []
        while len(fi) < 8:
            i, j = (int(v) for v in rng.integers(0, side, size=2))
            if np.hypot(i - sx, j - sy) >= 2.0:
                fi.append(i)
                fj.append(j)
        p = Problem(nx=side, ny=side, nz=side, dx_mm=1.0, nside=4, g=0.85, mua=mua, mus=mus,
                    n=n, steps=steps, src_ix=sx, src_iy=sy, src_w=1,
                    det_face=[FACE_TOP] * 8, det_i=fi, det_j=fj,
                    nbins=int(steps * 6), name=f"serving {side}^3, {steps} steps")
        out.append(Request(arrival_s=t, problem=p))
    return out


def small_problem(nside=2, nx=12, ny=10, nz=8, mua=0.02, mus=2.0, g=0.6, n=1.4,
                  steps=40, seed=None, **kw) -> Problem:
    """A small ragged grid for parity tests (non-cubic, sizes that are not tile
    multiples).  With a seed, mu_a and mu_s get +-30 % voxel noise."""
    mu_a, mu_s, nn = uniform_medium(nx, ny, nz, mua, mus, n)
    if seed is not None:
        rng = np.random.default_rng(seed)
        mu_a = (mu_a * rng.uniform(0.7, 1.3, mu_a.shape)).astype(np.float32)
        mu_s = (mu_s * rng.uniform(0.7, 1.3, mu_s.shape)).astype(np.float32)
    dets = kw.pop("dets", None)
    if dets is None:
        f = [FACE_TOP] * 4 + [FACE_XMAX]
        i = [min(nx - 1, nx // 2 + k) for k in (1, 2, 3, 4)] + [ny // 2]
        j = [ny // 2] * 4 + [1]
    else:
        f, i, j = dets
    base = dict(nx=nx, ny=ny, nz=nz, dx_mm=1.0, nside=nside, g=g, mua=mu_a, mus=mu_s, n=nn,
                steps=steps, src_ix=nx // 2 - 1, src_iy=ny // 2 - 1, src_w=2,
                det_face=f, det_i=i, det_j=j, nbins=steps * 6, name="small")
    base.update(kw)
    return Problem(**base)
