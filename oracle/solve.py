"""Forward step loop of the time-dependent solve (Sec. 2.4, Steps 1-7).

State: N[d, v], the number of photons in voxel v travelling in direction d
(Reading: photon number per voxel and direction stands in for the paper's
intensity; the energy density of Figs. 7-8 is then the sum over d).  One step:

  1. injection   the pulse adds q_m photons spread evenly over the source
                 voxels and source directions;
  2. collision   Eq. (10) with the explicit source of Eq. (12):
                 N_c = e^-dtau N + omega (f0 + f1) (P N) per voxel;
  3. transport   along the long-characteristic lattice every direction moves
                 its photons one plane downwind (phase mode: all of them on the
                 steps its phase selects; split mode: the fraction nu_d r_v each
                 step), light leaving the box is absorbed by the boundary
                 (Sec. 3.1) and tallied per face and per detector, and light
                 crossing a refractive-index jump is reflected and refracted
                 (Sec. 3.3, see optics).

Reading: collision then transport in each step (Eq. 10 takes intensity and
source at the upwind point, then moves them), with S1 := S0, without the
per-step iteration of Steps 3-6.

Test infrastructure only (see the package docstring)."""
from dataclasses import dataclass
from typing import List, Optional

import numpy as np

from . import angles, lattice, medium, optics, setup


@dataclass
class Setup:
    dirs: np.ndarray
    P: np.ndarray
    lat: lattice.RayLattice
    dt: float
    a: np.ndarray
    b: np.ndarray
    omega: np.ndarray
    ell: np.ndarray
    nu: np.ndarray
    r: np.ndarray              # path per step relative to the reference (split mode)
    mode: str                  # "phase" | "split"
    downwind: List[np.ndarray]
    exit_face: List[np.ndarray]
    src_vox: List[int]
    src_dirs: List[int]
    pulse: tuple               # (t0, fwhm, total photons)
    det_vox: List[int]
    det_face: List[int]
    det_acc: List[List[int]]
    icpt: list                 # interface interceptions (d, v, w, R, d_r, d_t)
    source: str = "explicit"   # "explicit" | "implicit"
    w0: Optional[np.ndarray] = None   # implicit source: omega f0, omega f1 per voxel
    w1: Optional[np.ndarray] = None


def build(prob, steps=None, coef=None) -> Setup:
    """Everything calculation Step 1 fixes before the time loop."""
    steps = prob.steps if steps is None else steps
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
    a, b, omega, ell = medium.collision_coefficients(prob.mua, prob.mus, n, dt,
                                                     prob.coef if coef is None else coef)
    uniform = bool(np.all(n == n.flat[0]))
    mode = prob.advance if prob.advance != "auto" else ("phase" if uniform else "split")
    if mode == "phase" and not uniform:
        raise ValueError("phase mode needs a uniform refractive index")
    n_ref = medium.reference_index(n)
    ell_ref = medium.C0_MM_PER_PS * dt / n_ref
    nu = lat.plane_speed(ell_ref, prob.dx_mm)
    r = (n_ref / n).ravel()
    if np.max(nu) * np.max(r) > 1.0 + 1e-12:
        raise ValueError("time step moves light more than one plane per step")
    dw, ef = [], []
    for d in range(len(dirs)):
        w, f = lat.downwind(d)
        dw.append(w)
        ef.append(f)
    src_vox = setup.source_voxels(shape, prob.src_ix, prob.src_iy, prob.src_w)
    src_dirs = setup.source_directions(dirs, prob.src_cone_deg)
    det_vox = [setup.detector_voxel(shape, f, i, j)
               for f, i, j in zip(prob.det_face, prob.det_i, prob.det_j)]
    det_acc = [setup.detector_acceptance(dirs, f, prob.det_cone_deg) for f in prob.det_face]
    icpt = optics.interceptions(lat, n) if mode == "split" and not uniform else []
    source = getattr(prob, "source", "explicit")
    w0 = w1 = None
    if source == "implicit":
        _, w0, w1 = medium.implicit_weights(prob.mua, prob.mus, n, dt)
        w0, w1 = w0.ravel(), w1.ravel()
    elif source != "explicit":
        raise ValueError(source)
    return Setup(dirs=dirs, P=P, lat=lat, dt=dt, a=a.ravel(), b=b.ravel(),
                 omega=omega.ravel(), ell=ell.ravel(), nu=nu, r=r, mode=mode,
                 downwind=dw, exit_face=ef, src_vox=src_vox, src_dirs=src_dirs,
                 pulse=(prob.t0_ps, prob.fwhm_ps, prob.total_photons),
                 det_vox=det_vox, det_face=list(prob.det_face), det_acc=det_acc, icpt=icpt,
                 source=source, w0=w0, w1=w1)


def move_fraction(S: Setup, d, m):
    """Fraction of direction d's photons in each voxel that move one plane at step m."""
    if S.mode == "phase":
        return S.lat.move_fraction_phase(S.nu[d], m)
    return S.nu[d] * S.r


def inject(S: Setup, N, m):
    """Step 1 of the step loop: returns the photons added."""
    q = setup.pulse_weight(m, S.dt, *S.pulse)
    share = q / (len(S.src_vox) * len(S.src_dirs))
    for d in S.src_dirs:
        for v in S.src_vox:
            N[d, v] += share
    return q


def collide(S: Setup, N):
    """Collision of Eq. (10) with S1 := S0 and S from Eq. (12): every voxel's
    column N[:, v] becomes a_v N[:, v] + b_v (P N)[:, v].  Returns the new
    state and the photons absorbed, sum_v (1 - a_v - b_v) sum_d N[d, v].
    With the implicit source, collide_implicit."""
    if S.source == "implicit":
        return collide_implicit(S, N)
    J = S.P @ N
    Nc = S.a[None, :] * N + S.b[None, :] * J
    absorbed = float(np.sum((1.0 - S.a - S.b) * N.sum(axis=0)))
    return Nc, absorbed


def collide_implicit(S: Setup, N, chunk=256):
    """Collision with the implicit source: S1 in Eq. (10) is the source of the
    outgoing intensity, so every voxel's column solves
        (I - w1_v P) N_c = a_v N + w0_v P N,
    the fixed point that Sec. 2.4 Steps 3-6 iterate towards; solved here
    directly, voxel by voxel.  Returns the new state and the photons absorbed,
    sum N - sum N_c."""
    nd, nv = N.shape
    rhs = S.a[None, :] * N + S.w0[None, :] * (S.P @ N)
    Nc = np.empty_like(N)
    eye = np.eye(nd)
    for v0 in range(0, nv, chunk):
        v1 = min(nv, v0 + chunk)
        M = eye[None, :, :] - S.w1[v0:v1, None, None] * S.P[None, :, :]
        Nc[:, v0:v1] = np.linalg.solve(M, rhs[:, v0:v1].T[:, :, None])[:, :, 0].T
    absorbed = float(N.sum() - Nc.sum())
    return Nc, absorbed


def transport(S: Setup, Nc, m, ndet):
    """Move every direction's photons along the lattice (Eq. 10, Fig. 1).
    Returns the new state, escape per face and light recorded per detector."""
    nd, nv = Nc.shape
    out = np.zeros_like(Nc)
    escape = np.zeros(6)
    det = np.zeros(ndet)
    icpt_src = {}
    for (d, v, w, R, dr, dtt) in S.icpt:
        icpt_src.setdefault(d, []).append(v)
    held = {}
    for d in range(nd):
        f = move_fraction(S, d, m)
        moving = f * Nc[d]
        out[d] += Nc[d] - moving
        dest = S.downwind[d]
        inside = dest >= 0
        if d in icpt_src:
            inside = inside.copy()
            inside[icpt_src[d]] = False
            for v in icpt_src[d]:
                held[(d, v)] = moving[v]
        out[d, dest[inside]] += moving[inside]
        leaving = np.nonzero(dest < 0)[0]
        faces = S.exit_face[d][leaving]
        for fc in range(6):
            escape[fc] += moving[leaving[faces == fc]].sum()
        for k in range(ndet):
            if d in S.det_acc[k]:
                v = S.det_vox[k]
                if dest[v] < 0 and S.exit_face[d][v] == S.det_face[k]:
                    det[k] += moving[v]
    for (d, v, w, R, dr, dtt) in S.icpt:
        F = held[(d, v)]
        out[dr, v] += R * F
        if dtt >= 0:
            out[dtt, w] += (1.0 - R) * F
    return out, escape, det


@dataclass
class Result:
    det: np.ndarray          # [ndet, steps] light leaving through each detector per step
    injected: np.ndarray     # [steps]
    absorbed: np.ndarray     # [steps]
    escaped: np.ndarray      # [steps, 6] per face
    in_domain: np.ndarray    # [steps] photons in the box after step m
    state: np.ndarray        # final N[d, v]
    setup: Setup
    states: Optional[list] = None   # N after injection, per step (for the adjoint)

    def binned(self, bin_ps, nbins):
        """Detector signals in fixed time bins (Fig. 9 style read-out)."""
        W = setup.rebin_matrix(self.det.shape[1], self.setup.dt, bin_ps, nbins)
        return self.det @ W


def forward(prob, steps=None, S: Optional[Setup] = None, keep_states=False,
            state0=None, start_step=0) -> Result:
    """Run the step loop for `steps` steps (Sec. 2.4 Steps 3-7)."""
    steps = prob.steps if steps is None else steps
    S = build(prob, steps=start_step + steps) if S is None else S
    nd, nv = len(S.dirs), prob.nvox
    ndet = len(S.det_vox)
    N = np.zeros((nd, nv)) if state0 is None else np.array(state0, dtype=np.float64)
    det = np.zeros((ndet, steps))
    inj = np.zeros(steps)
    absb = np.zeros(steps)
    esc = np.zeros((steps, 6))
    dom = np.zeros(steps)
    states = [] if keep_states else None
    for i in range(steps):
        m = start_step + i
        inj[i] = inject(S, N, m)
        if keep_states:
            states.append(N.copy())
        Nc, absb[i] = collide(S, N)
        N, esc[i], det[:, i] = transport(S, Nc, m, ndet)
        dom[i] = N.sum()
    return Result(det=det, injected=inj, absorbed=absb, escaped=esc, in_domain=dom,
                  state=N, setup=S, states=states)
