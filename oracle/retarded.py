"""Time stepping below Courant one with the retarded formal solution
(Sec. 2.1: the retarded form of the formal solution and its evaluation from
the upwind ray point at the retarded time; Sec. 2.2 and Sec. 3.1: time steps
of a tenth and a fifth of the light-crossing time, with the intensity kept
over ten past time bins).

The ray lattice, the directions, P, the source and the detectors are those of
solve.  What changes is time.  Along direction d consecutive planes are dx
apart on the dominant axis, so the hop from the upwind voxel u to voxel v is
dr_d = dx / |Omega_a| long, takes

    D_d = dr_d n / (c0 dt)    steps  (light at c0/n; D_d >= 1 at Courant <= 1)

and has optical depth dtau = mu_t(u) dr_d (coefficients of the nearest voxel,
the hop's start).  The value at v at time t is the upwind value at time
t - D_d, attenuated over the hop, with the source term added (Eq. 10 with the
explicit source S1 := S0, as in solve).

Readings (each one is what the paper leaves open):

  * State: N[d, v] is the photon content of voxel v moving along d, as in
    solve.  A hop moves a voxel's content to the next plane in D_d steps, so
    the light crossing a plane per step is N / D_d.  The source therefore
    puts D_d q into the voxel it feeds with q photons per step, and the
    tallies (escape, detectors, absorption) count content / D_d per step.
  * Collision once per hop: C = a N + b (P N) per voxel with the hop's
    coefficients a = exp(-mu_t dr_d), b = omega (1 - a) (the paper's
    f0 + f1 = 1 - e^-dtau), so a and b depend on the direction through dr_d.
    Every step collides the whole field: each step is a different time slice
    of the light, and every slice is collided once per hop.
  * Retarded time between time bins: linear interpolation.  With
    D_d = n_d + phi_d (n_d integer, 0 <= phi_d < 1)
        N^{m+1}[d, v] = (1 - phi_d) C^{m+1-n_d}[d, u] + phi_d C^{m-n_d}[d, u],
    zero where v has no upwind voxel (vacuum inflow) and C^j = 0 for j < 0.
    The history holds n_max + 1 collided fields (n_max = max_d n_d): nine at
    a fifth of the crossing time, where D_d reaches 5 sqrt(3).
  * A varying refractive index: the hop from u takes D[d, u] = dr_d n_u /
    (c0 dt) steps, the index of the hop's start voxel (the nearest-voxel
    reading of the coefficients), so lag and fraction are per direction and
    voxel.  The light crossing a plane per step is content / D[d, u] (a flux),
    and a move between voxels of the same index copies content.
  * Interfaces (Sec. 3.3, Eq. 13-14): a hop that would carry light from u
    into a voxel w of another index is intercepted, as in solve: of the flux
    F = r / D[d, u] that reaches the interface (r the retarded collided
    content), R F returns into u along the mirror direction d_r and (1 - R) F
    enters w along Snell's direction d_t.  Each becomes content at the flux
    it carries times the hop duration of its new direction and voxel:
    R r D[d_r, u] / D[d, u] and (1 - R) r D[d_t, w] / D[d, u].  Photons are
    then conserved across the interface.
  * Source weighting (prob.retarded_source):
      "target" (default): C = a N + b (P N), b = omega (1 - a), the formal
        solution of Eq. 10 along the target direction's hop with the
        explicit source; the target's own 1 - e^{-dtau} weights the source,
        which the paper prints.  With unequal hops it conserves light only
        to O(dtau) per scattering.
      "flux": C = a N + D (omega P ((1 - a) / D N)) per voxel: the light each
        direction loses to scattering per step, (1 - a_j) omega N_j / D_j,
        is what the others gain per step, so scattering conserves photons
        exactly.  It agrees with "target" to first order in dtau.
  * With the source on a coarser angular grid, P is the effective fine-grid
    matrix of angles.two_level_matrix, and the hop coefficients are those of
    each fine direction (uniform index only).

Test infrastructure only (see the package docstring)."""
from dataclasses import dataclass
from typing import List

import numpy as np

from . import angles, lattice, medium, optics, setup


@dataclass
class RetardedSetup:
    dirs: np.ndarray
    P: np.ndarray
    lat: lattice.RayLattice
    dt: float
    hop: np.ndarray          # dr_d [nd], mm
    D: np.ndarray            # hop duration in steps [nd, nv] (hop from the voxel)
    nlag: np.ndarray         # floor(D) [nd, nv]
    phi: np.ndarray          # D - floor(D) [nd, nv]
    a: np.ndarray            # [nd, nv] hop attenuation
    b: np.ndarray            # [nd, nv] hop source weight
    omega: np.ndarray        # [nv] albedo
    H: int                   # collided fields kept
    downwind: List[np.ndarray]
    exit_face: List[np.ndarray]
    upwind: List[np.ndarray]
    src_vox: List[int]
    src_dirs: List[int]
    pulse: tuple
    det_vox: List[int]
    det_face: List[int]
    det_acc: List[List[int]]
    icpt: list               # interceptions (d, v, w, R, d_r, d_t, w_r, w_t): content weights
    source: str = "target"   # "target" | "flux"


def hop_lengths(lat: lattice.RayLattice, dx):
    """dr_d = dx / |Omega_a|: the distance along direction d between planes."""
    return np.array([dx / abs(lat.dirs[d][lat.axis[d]]) for d in range(len(lat.dirs))])


def hop_coefficients(mua, mus, hop):
    """a[d, v] = exp(-mu_t(v) dr_d) and b[d, v] = omega_v (1 - a[d, v]):
    the explicit-source collision over one hop (Eq. 9-10 with S1 := S0, where
    f0 + f1 = 1 - e^-dtau).  No extinction: a = 1, b = 0."""
    mua = np.asarray(mua, dtype=np.float64).ravel()
    mus = np.asarray(mus, dtype=np.float64).ravel()
    mut = mua + mus
    omega = np.where(mut > 0.0, mus / np.where(mut > 0.0, mut, 1.0), 0.0)
    tau = hop[:, None] * mut[None, :]
    a = np.exp(-tau)
    b = omega[None, :] * (1.0 - a)
    return a, b


def upwind_map(dest, nv):
    """Inverse of a downwind map: u[v] = the voxel whose downwind voxel is v, or -1."""
    u = np.full(nv, -1, dtype=np.int64)
    src = np.nonzero(dest >= 0)[0]
    u[dest[src]] = src
    return u


def build(prob, dirs=None, P=None) -> RetardedSetup:
    """Set-up of the retarded stepping.  dirs and P default to the HEALPix
    grid of prob.nside and its Sinkhorn HG matrix; tests may pass others."""
    shape = (prob.nz, prob.ny, prob.nx)
    n = np.asarray(prob.n, dtype=np.float64)
    uniform = bool(np.all(n == n.flat[0]))
    if dirs is None:
        dirs = angles.healpix_ring(prob.nside)
    ns = getattr(prob, "nside_scatter", 0)
    if ns and ns != prob.nside and not uniform:
        raise ValueError("the two-level source needs a uniform refractive index here")
    if P is None and ns and ns != prob.nside:
        # the source on a coarser angular grid (Sec. 2.1): the effective
        # fine-grid matrix, as in solve.build
        P = angles.two_level_matrix(prob.nside, ns, prob.g, prob.hg_norm)
    if P is None:
        P = angles.phase_matrix(dirs, prob.g, prob.hg_norm)
    source = getattr(prob, "retarded_source", "target")
    if source not in ("target", "flux"):
        raise ValueError(source)
    lat = lattice.RayLattice(dirs, shape)
    dt = medium.time_step(prob.dx_mm, n, prob.dt_ps)
    hop = hop_lengths(lat, prob.dx_mm)
    D = hop[:, None] * n.ravel()[None, :] / (medium.C0_MM_PER_PS * dt)
    if np.min(D) < 1.0 - 1e-12:
        raise ValueError("time step longer than a hop (Courant number above one)")
    nlag = np.floor(D + 1e-12).astype(np.int64)
    phi = np.maximum(D - nlag, 0.0)
    a, b = hop_coefficients(prob.mua, prob.mus, hop)
    mut = np.asarray(prob.mua, dtype=np.float64).ravel() + np.asarray(prob.mus,
                                                                      dtype=np.float64).ravel()
    omega = np.where(mut > 0.0, np.asarray(prob.mus, dtype=np.float64).ravel() /
                     np.where(mut > 0.0, mut, 1.0), 0.0)
    nv = prob.nvox
    dw, ef, uw = [], [], []
    for d in range(len(dirs)):
        w, f = lat.downwind(d)
        dw.append(w)
        ef.append(f)
        uw.append(upwind_map(w, nv))
    icpt = []
    if not uniform:
        for (d, v, w, R, dr, dtt) in optics.interceptions(lat, n):
            wr = R * D[dr, v] / D[d, v]
            wt = (1.0 - R) * D[dtt, w] / D[d, v] if dtt >= 0 else 0.0
            icpt.append((d, v, w, R, dr, dtt, wr, wt))
    return RetardedSetup(
        dirs=np.asarray(dirs, dtype=np.float64), P=np.asarray(P, dtype=np.float64), lat=lat,
        dt=dt, hop=hop, D=D, nlag=nlag, phi=phi, a=a, b=b, omega=omega,
        H=int(nlag.max()) + 1,
        downwind=dw, exit_face=ef, upwind=uw,
        src_vox=setup.source_voxels(shape, prob.src_ix, prob.src_iy, prob.src_w),
        src_dirs=setup.source_directions(dirs, prob.src_cone_deg),
        pulse=(prob.t0_ps, prob.fwhm_ps, prob.total_photons),
        det_vox=[setup.detector_voxel(shape, f, i, j)
                 for f, i, j in zip(prob.det_face, prob.det_i, prob.det_j)],
        det_face=list(prob.det_face),
        det_acc=[setup.detector_acceptance(dirs, f, prob.det_cone_deg) for f in prob.det_face],
        icpt=icpt, source=source)


def inject(S: RetardedSetup, N, m):
    """The pulse's q_m photons of step m, spread evenly over the source pairs;
    a pair (d, v) gets content D[d, v] times its share.  Returns q_m."""
    q = setup.pulse_weight(m, S.dt, *S.pulse)
    share = q / (len(S.src_vox) * len(S.src_dirs))
    for d in S.src_dirs:
        for v in S.src_vox:
            N[d, v] += S.D[d, v] * share
    return q


def collide(S: RetardedSetup, N):
    """The collision of one hop, by the set-up's source weighting (see the
    module docstring); absorbed per step is sum (1 - omega)(1 - a) N / D."""
    if S.source == "flux":
        C = S.a * N + S.D * (S.omega[None, :] * (S.P @ ((1.0 - S.a) / S.D * N)))
    else:
        C = S.a * N + S.b * (S.P @ N)
    absorbed = float(np.sum((1.0 - S.omega[None, :]) * (1.0 - S.a) * N / S.D))
    return C, absorbed


def retarded_value(S: RetardedSetup, hist, d, m):
    """Row d of the collided field at the retarded time m + 1 - D[d, v] of each
    voxel: (1 - phi) C^{m+1-n} + phi C^{m-n}, from hist[j] = C^j (missing =
    zero)."""
    nv = S.a.shape[1]
    r = np.zeros(nv)
    for n in np.unique(S.nlag[d]):
        sel = S.nlag[d] == n
        phi = S.phi[d, sel]
        late = hist.get(m + 1 - int(n))
        early = hist.get(m - int(n))
        if late is not None:
            r[sel] += (1.0 - phi) * late[d, sel]
        if early is not None:
            r[sel] += phi * early[d, sel]
    return r


def transport(S: RetardedSetup, hist, m, ndet):
    """N^{m+1} from the history of collided fields; escape per face and the
    detector records of step m (flux: content / D of what crosses the
    boundary); hops across an index jump are intercepted (module docstring)."""
    nd, nv = S.a.shape
    out = np.zeros((nd, nv))
    escape = np.zeros(6)
    det = np.zeros(ndet)
    held = {}
    cut = {}
    for (d, v, w, R, dr, dtt, wr, wt) in S.icpt:
        cut.setdefault(d, []).append(w)
    for d in range(nd):
        r = retarded_value(S, hist, d, m)
        u = S.upwind[d]
        has = u >= 0
        if d in cut:
            has = has.copy()
            has[cut[d]] = False
        out[d, has] = r[u[has]]
        held[d] = r
        leaving = np.nonzero(S.downwind[d] < 0)[0]
        faces = S.exit_face[d][leaving]
        flux = r[leaving] / S.D[d, leaving]
        for fc in range(6):
            escape[fc] += flux[faces == fc].sum()
        for k in range(ndet):
            v = S.det_vox[k]
            if d in S.det_acc[k] and S.downwind[d][v] < 0 and S.exit_face[d][v] == S.det_face[k]:
                det[k] += r[v] / S.D[d, v]
    for (d, v, w, R, dr, dtt, wr, wt) in S.icpt:
        F = held[d][v]
        out[dr, v] += wr * F
        if dtt >= 0:
            out[dtt, w] += wt * F
    return out, escape, det


@dataclass
class RetardedResult:
    det: np.ndarray
    injected: np.ndarray
    absorbed: np.ndarray
    escaped: np.ndarray
    in_domain: np.ndarray
    state: np.ndarray
    setup: RetardedSetup
    states: list = None


def forward(prob, steps=None, S: RetardedSetup = None, keep_states=False) -> RetardedResult:
    """The step loop: inject, collide (kept in the history), retarded transport."""
    steps = prob.steps if steps is None else steps
    S = build(prob) if S is None else S
    nd, nv = S.a.shape
    ndet = len(S.det_vox)
    N = np.zeros((nd, nv))
    hist = {}
    det = np.zeros((ndet, steps))
    inj = np.zeros(steps)
    absb = np.zeros(steps)
    esc = np.zeros((steps, 6))
    dom = np.zeros(steps)
    states = [] if keep_states else None
    for m in range(steps):
        inj[m] = inject(S, N, m)
        hist[m], absb[m] = collide(S, N)
        hist.pop(m - S.H, None)
        N, esc[m], det[:, m] = transport(S, hist, m, ndet)
        dom[m] = N.sum()
        if keep_states:
            states.append(N.copy())
    return RetardedResult(det=det, injected=inj, absorbed=absb, escaped=esc, in_domain=dom,
                          state=N, setup=S, states=states)
