"""Python binding of libtrinity.so (include/trinity.h): argument marshalling
only.  Every step of the solve runs in the library's HIP kernels; this module
never computes any part of it and fails loudly when the library is missing.

PyTorch, when present, supplies device memory (tensors passed as device
arrays) and the stream the library queues its work on."""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# TRINITY_LIB names another build of the same library (the host-sanitizer test
# loads an AddressSanitizer build this way); by default the in-tree one
LIB_PATH = os.environ.get("TRINITY_LIB") or os.path.join(_HERE, "libtrinity.so")

TR_OK, TR_EINVAL, TR_ENOMEM, TR_EDEVICE, TR_ENUMERIC, TR_ESTATE = 0, -1, -2, -3, -4, -5
STATUS_NAMES = {0: "TR_OK", -1: "TR_EINVAL", -2: "TR_ENOMEM", -3: "TR_EDEVICE",
                -4: "TR_ENUMERIC", -5: "TR_ESTATE"}
HG = {"sinkhorn": 0, "row": 1}
COEF = {"paper": 0, "abs_exact": 1}
ADVANCE = {"auto": 0, "phase": 1, "split": 2, "retarded": 3}
PRECISION = {"fp32": 0, "bf16split": 1}
SOURCE = {"explicit": 0, "implicit": 1}
TRANSPORT = {"auto": 0, "sweep": 1}
RSOURCE = {"target": 0, "flux": 1}
MODE_NAMES = {1: "phase", 2: "split"}
BUDGET_FIELDS = ("injected", "absorbed", "in_domain", "esc0", "esc1", "esc2", "esc3", "esc4",
                 "esc5")


class TrinityError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class GridDesc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("dx_mm", ctypes.c_double), ("nside", ctypes.c_int), ("g", ctypes.c_double),
                ("dt_ps", ctypes.c_double), ("hg_norm", ctypes.c_int), ("coef", ctypes.c_int),
                ("advance", ctypes.c_int), ("precision", ctypes.c_int), ("source", ctypes.c_int),
                ("nside_scatter", ctypes.c_int), ("transport", ctypes.c_int),
                ("retarded_source", ctypes.c_int)]


class Info(ctypes.Structure):
    _fields_ = [("ndir", ctypes.c_int), ("nvox", ctypes.c_int), ("mode", ctypes.c_int),
                ("ninterceptions", ctypes.c_int), ("dt_ps", ctypes.c_double),
                ("steps_done", ctypes.c_longlong), ("device_bytes", ctypes.c_size_t),
                ("history", ctypes.c_int), ("moves_fused", ctypes.c_int)]


class ServerDesc(ctypes.Structure):
    _fields_ = [("nside", ctypes.c_int), ("g", ctypes.c_double), ("hg_norm", ctypes.c_int),
                ("coef", ctypes.c_int), ("budget_bytes", ctypes.c_size_t),
                ("max_slots", ctypes.c_int)]


class Request(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("dx_mm", ctypes.c_double), ("dt_ps", ctypes.c_double),
                ("mua", ctypes.c_void_p), ("mus", ctypes.c_void_p), ("n", ctypes.c_void_p),
                ("src_ix", ctypes.c_int), ("src_iy", ctypes.c_int), ("src_w", ctypes.c_int),
                ("src_cone_deg", ctypes.c_double), ("t0_ps", ctypes.c_double),
                ("fwhm_ps", ctypes.c_double), ("total_photons", ctypes.c_double),
                ("ndet", ctypes.c_int), ("det_face", ctypes.c_void_p),
                ("det_i", ctypes.c_void_p), ("det_j", ctypes.c_void_p),
                ("det_cone_deg", ctypes.c_double), ("bin_ps", ctypes.c_double),
                ("nbins", ctypes.c_int), ("nsteps", ctypes.c_int)]


class RequestInfo(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("steps_done", ctypes.c_longlong),
                ("queued_ms", ctypes.c_double), ("run_ms", ctypes.c_double),
                ("bytes", ctypes.c_size_t)]


REQ_QUEUED, REQ_RUNNING, REQ_DONE, REQ_FAILED, REQ_CANCELLED = 0, 1, 2, 3, 4

_P = ctypes.c_void_p
_I = ctypes.c_int
_D = ctypes.c_double
_PD = ctypes.POINTER(ctypes.c_double)
_PI = ctypes.POINTER(ctypes.c_int)
_PF = ctypes.POINTER(ctypes.c_float)
_SIGS = {
    "tr_create_medium": [ctypes.POINTER(GridDesc), _P, _P, _P, _I, _P, ctypes.POINTER(_P)],
    "tr_bytes_required": [ctypes.POINTER(GridDesc), _I, _I],
    "tr_bytes_required_n": [ctypes.POINTER(GridDesc), _PF, _I, _I],
    "tr_state_bytes": [_P, ctypes.POINTER(ctypes.c_size_t)],
    "tr_save_state": [_P, _P, ctypes.c_size_t],
    "tr_load_state": [_P, _P, ctypes.c_size_t],
    "tr_destroy_medium": [_P],
    "tr_set_source": [_P, _I, _I, _I, _D, _D, _D, _D],
    "tr_set_detectors": [_P, _I, _PI, _PI, _PI, _D, _D, _I],
    "tr_step": [_P, _I],
    "tr_step_noalloc": [_P, _I],
    "tr_solve": [_P, _I],
    "tr_synchronize": [_P],
    "tr_reset": [_P],
    "tr_read_detectors": [_P, _PD, ctypes.c_size_t],
    "tr_read_detector_steps": [_P, _PD, ctypes.c_size_t],
    "tr_read_budget": [_P, _PD, ctypes.c_size_t],
    "tr_read_energy": [_P, _P, _I],
    "tr_get_state": [_P, _P, _I],
    "tr_set_state": [_P, _P, _I],
    "tr_get_info": [_P, ctypes.POINTER(Info)],
    "tr_profile_begin": [_P, _I],
    "tr_solve_checkpointed": [_P, _I, _I],
    "tr_backward": [_P, _PD, _PF, _PF],
    "tr_profile_end": [_P, _PD, _PI],
    "tr_server_create": [ctypes.POINTER(ServerDesc), _P, ctypes.POINTER(_P)],
    "tr_server_destroy": [_P],
    "tr_server_request_bytes": [_P, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_size_t)],
    "tr_server_submit": [_P, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_longlong)],
    "tr_server_advance": [_P, _I, _PI, _PI],
    "tr_server_info": [_P, ctypes.c_longlong, ctypes.POINTER(RequestInfo)],
    "tr_server_result": [_P, ctypes.c_longlong, _PD, ctypes.c_size_t, _PD, ctypes.c_size_t],
    "tr_server_cancel": [_P, ctypes.c_longlong],
    "tr_host_directions": [_I, _PD],
    "tr_host_parents": [_I, _I, _PI],
    "tr_host_phase_matrix": [_I, _D, _I, _PD],
    "tr_host_lattice": [_I, _I, _I, _I, _PI, _PI, _PI],
    "tr_host_move_tables": [_I, _I, _I, _I, _I, _PI, _PI],
    "tr_host_coefficients": [ctypes.POINTER(GridDesc), _PF, _PF, _PF, _PD, _PD, _PD, _PD],
    "tr_host_cone_set": [_I, _D, _D, _D, _D, _PI, _I, _PI],
    "tr_host_pulse": [_D, _D, _D, _D, _I, _I, _PD],
    "tr_host_interceptions": [ctypes.POINTER(GridDesc), _PF, _PI, _PI, _PI, _PD, _PI, _PI, _I,
                              _PI],
    "tr_probe_mfma": [_I, _I, _I, _PD, _PD],
}
EXPORTED = tuple(_SIGS) + ("tr_last_error",)

_lib = None


def lib():
    """Load libtrinity.so once (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2105_01028_amd.build_lib`")
        L = ctypes.CDLL(LIB_PATH)
        for name, args in _SIGS.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = (ctypes.c_size_t if name.startswith("tr_bytes_required")
                          else ctypes.c_int)
        L.tr_last_error.argtypes = []
        L.tr_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _check(status):
    if status != TR_OK:
        raise TrinityError(status, lib().tr_last_error().decode())


def _dptr(a):
    return a.ctypes.data_as(_PD)


def _iptr(a):
    return a.ctypes.data_as(_PI)


def _fptr(a):
    return a.ctypes.data_as(_PF)


def grid_desc(prob) -> GridDesc:
    return GridDesc(prob.nx, prob.ny, prob.nz, float(prob.dx_mm), int(prob.nside), float(prob.g),
                    float(prob.dt_ps), HG[prob.hg_norm], COEF[prob.coef], ADVANCE[prob.advance],
                    PRECISION[prob.precision], SOURCE[getattr(prob, "source", "explicit")],
                    int(getattr(prob, "nside_scatter", 0)),
                    TRANSPORT[getattr(prob, "transport", "auto")],
                    RSOURCE[getattr(prob, "retarded_source", "target")])


def current_stream() -> int:
    """torch's current HIP stream handle (0 = the null stream when torch or the
    GPU is unavailable)."""
    try:
        import torch
        if torch.cuda.is_available():
            return int(torch.cuda.current_stream().cuda_stream)
    except ImportError:
        pass
    return 0


def _is_torch(x):
    return type(x).__module__.startswith("torch")


class Medium:
    """One medium on the device (tr_create_medium ... tr_destroy_medium)."""

    def __init__(self, desc: GridDesc, mua, mus, n, stream: Optional[int] = None):
        L = lib()
        self._h = _P()
        self.desc = desc
        nvox = desc.nx * desc.ny * desc.nz
        if all(_is_torch(a) for a in (mua, mus, n)):
            arrs = [a.contiguous() for a in (mua, mus, n)]
            for a in arrs:
                if a.numel() != nvox or str(a.dtype) != "torch.float32" or not a.is_cuda:
                    raise ValueError("device arrays must be float32 cuda tensors of nvox elements")
            ptrs = [a.data_ptr() for a in arrs]
            on_dev = 1
            self._keep = arrs
        else:
            arrs = [np.ascontiguousarray(a, dtype=np.float32).ravel() for a in (mua, mus, n)]
            for a in arrs:
                if a.size != nvox:
                    raise ValueError("coefficient arrays must hold nx*ny*nz values")
            ptrs = [a.ctypes.data for a in arrs]
            on_dev = 0
        self.stream = current_stream() if stream is None else int(stream)
        _check(L.tr_create_medium(ctypes.byref(desc), ptrs[0], ptrs[1], ptrs[2], on_dev,
                                  self.stream, ctypes.byref(self._h)))
        self.ndet = 0
        self.nbins = 0

    @classmethod
    def from_problem(cls, prob, stream=None, source=True, detectors=True) -> "Medium":
        m = cls(grid_desc(prob), prob.mua, prob.mus, prob.n, stream)
        if source:
            m.set_source(prob.src_ix, prob.src_iy, prob.src_w, prob.src_cone_deg, prob.t0_ps,
                         prob.fwhm_ps, prob.total_photons)
        if detectors:
            m.set_detectors(prob.det_face, prob.det_i, prob.det_j, prob.det_cone_deg,
                            prob.bin_ps, prob.nbins)
        return m

    # ---- life cycle
    def close(self):
        if self._h:
            _check(lib().tr_destroy_medium(self._h))
            self._h = _P()

    destroy_medium = close

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # ---- problem statement
    def set_source(self, ix, iy, w=2, cone_deg=15.0, t0_ps=20.0, fwhm_ps=10.0,
                   total_photons=1.0):
        _check(lib().tr_set_source(self._h, int(ix), int(iy), int(w), float(cone_deg),
                                   float(t0_ps), float(fwhm_ps), float(total_photons)))

    def set_detectors(self, face: Sequence[int], i: Sequence[int], j: Sequence[int],
                      cone_deg=15.0, bin_ps=1.0, nbins=1000):
        f = np.ascontiguousarray(face, dtype=np.int32)
        ii = np.ascontiguousarray(i, dtype=np.int32)
        jj = np.ascontiguousarray(j, dtype=np.int32)
        _check(lib().tr_set_detectors(self._h, len(f), _iptr(f), _iptr(ii), _iptr(jj),
                                      float(cone_deg), float(bin_ps), int(nbins)))
        self.ndet = len(f)
        self.nbins = int(nbins)

    # ---- stepping
    def step(self, nsteps: int):
        _check(lib().tr_step(self._h, int(nsteps)))

    def solve(self, nsteps: int):
        _check(lib().tr_solve(self._h, int(nsteps)))

    def step_noalloc(self, nsteps: int):
        _check(lib().tr_step_noalloc(self._h, int(nsteps)))

    def synchronize(self):
        _check(lib().tr_synchronize(self._h))

    def reset(self):
        _check(lib().tr_reset(self._h))

    # ---- gradients
    def solve_checkpointed(self, nsteps: int, ckpt_every: int = 50):
        _check(lib().tr_solve_checkpointed(self._h, int(nsteps), int(ckpt_every)))

    def backward(self, dL_dbins):
        """dL/d(mu_a), dL/d(mu_s) per voxel for dL/d(binned detector signals)."""
        g = np.ascontiguousarray(dL_dbins, dtype=np.float64).ravel()
        if g.size != self.ndet * self.nbins:
            raise ValueError("dL_dbins must hold ndet * nbins values")
        nv = self.desc.nx * self.desc.ny * self.desc.nz
        dmua = np.zeros(nv, np.float32)
        dmus = np.zeros(nv, np.float32)
        _check(lib().tr_backward(self._h, _dptr(g), _fptr(dmua), _fptr(dmus)))
        shape = (self.desc.nz, self.desc.ny, self.desc.nx)
        return dmua.reshape(shape), dmus.reshape(shape)

    # ---- kernel timing
    KERNELS = ("inject", "collide", "sweep", "gather", "reduce", "coarse_sum", "apply")

    def profile_begin(self, max_steps: int):
        _check(lib().tr_profile_begin(self._h, int(max_steps)))

    def profile_end(self):
        """Summed device ms and launch count per kernel kind since profile_begin."""
        ms = np.zeros(len(self.KERNELS))
        n = np.zeros(len(self.KERNELS), np.int32)
        _check(lib().tr_profile_end(self._h, _dptr(ms), _iptr(n)))
        return {k: (float(ms[i]), int(n[i])) for i, k in enumerate(self.KERNELS)}

    # ---- read-out
    def info(self) -> Info:
        out = Info()
        _check(lib().tr_get_info(self._h, ctypes.byref(out)))
        return out

    def read_detectors(self) -> np.ndarray:
        out = np.zeros(self.ndet * self.nbins)
        _check(lib().tr_read_detectors(self._h, _dptr(out), out.size))
        return out.reshape(self.ndet, self.nbins)

    def read_detector_steps(self) -> np.ndarray:
        steps = self.info().steps_done
        out = np.zeros(max(1, self.ndet * steps))
        _check(lib().tr_read_detector_steps(self._h, _dptr(out), out.size))
        return out[: self.ndet * steps].reshape(self.ndet, steps)

    def read_budget(self) -> np.ndarray:
        steps = self.info().steps_done
        out = np.zeros(max(1, 9 * steps))
        _check(lib().tr_read_budget(self._h, _dptr(out), out.size))
        return out[: 9 * steps].reshape(steps, 9)

    def read_energy(self, out=None):
        inf = self.info()
        if out is not None and _is_torch(out):
            _check(lib().tr_read_energy(self._h, out.data_ptr(), 1))
            return out
        res = np.zeros(inf.nvox, np.float32)
        _check(lib().tr_read_energy(self._h, res.ctypes.data, 0))
        return res

    def get_state(self, out=None):
        inf = self.info()
        if out is not None and _is_torch(out):
            _check(lib().tr_get_state(self._h, out.data_ptr(), 1))
            return out
        res = np.zeros((inf.ndir, inf.nvox), np.float32)
        _check(lib().tr_get_state(self._h, res.ctypes.data, 0))
        return res

    def set_state(self, state):
        if _is_torch(state):
            _check(lib().tr_set_state(self._h, state.contiguous().data_ptr(), 1))
        else:
            s = np.ascontiguousarray(state, dtype=np.float32)
            _check(lib().tr_set_state(self._h, s.ctypes.data, 0))

    def save_state(self) -> np.ndarray:
        """Everything a solve carries between steps (field, history, step index,
        records) as a byte array for load_state."""
        n = ctypes.c_size_t()
        _check(lib().tr_state_bytes(self._h, ctypes.byref(n)))
        buf = np.zeros(n.value, np.uint8)
        _check(lib().tr_save_state(self._h, buf.ctypes.data, buf.size))
        return buf

    def load_state(self, buf):
        b = np.ascontiguousarray(np.frombuffer(buf, np.uint8) if isinstance(buf, (bytes, bytearray))
                                 else buf, dtype=np.uint8)
        _check(lib().tr_load_state(self._h, b.ctypes.data, b.size))


class Server:
    """Continuous-batching server of forward solves (tr_server_* of the C-ABI)."""

    def __init__(self, nside=4, g=0.85, budget_bytes=8 << 30, max_slots=16, hg_norm="sinkhorn",
                 coef="paper", stream: Optional[int] = None):
        self._h = _P()
        self.stream = current_stream() if stream is None else int(stream)
        d = ServerDesc(int(nside), float(g), HG[hg_norm], COEF[coef], int(budget_bytes),
                       int(max_slots))
        _check(lib().tr_server_create(ctypes.byref(d), self.stream, ctypes.byref(self._h)))
        self._shape = {}

    @staticmethod
    def _request(prob):
        keep = [np.ascontiguousarray(a, dtype=np.float32).ravel() for a in (prob.mua, prob.mus,
                                                                            prob.n)]
        dets = [np.ascontiguousarray(a, dtype=np.int32) for a in (prob.det_face, prob.det_i,
                                                                  prob.det_j)]
        r = Request(prob.nx, prob.ny, prob.nz, float(prob.dx_mm), float(prob.dt_ps),
                    keep[0].ctypes.data, keep[1].ctypes.data, keep[2].ctypes.data,
                    int(prob.src_ix), int(prob.src_iy), int(prob.src_w), float(prob.src_cone_deg),
                    float(prob.t0_ps), float(prob.fwhm_ps), float(prob.total_photons),
                    len(dets[0]), dets[0].ctypes.data, dets[1].ctypes.data, dets[2].ctypes.data,
                    float(prob.det_cone_deg), float(prob.bin_ps), int(prob.nbins),
                    int(prob.steps))
        return r, keep + dets

    def request_bytes(self, prob) -> int:
        r, keep = self._request(prob)
        out = ctypes.c_size_t()
        _check(lib().tr_server_request_bytes(self._h, ctypes.byref(r), ctypes.byref(out)))
        return int(out.value)

    def submit(self, prob) -> int:
        r, keep = self._request(prob)
        rid = ctypes.c_longlong()
        _check(lib().tr_server_submit(self._h, ctypes.byref(r), ctypes.byref(rid)))
        self._shape[rid.value] = (len(prob.det_face), int(prob.nbins), int(prob.steps))
        return int(rid.value)

    def advance(self, max_steps=64):
        running, queued = ctypes.c_int(), ctypes.c_int()
        _check(lib().tr_server_advance(self._h, int(max_steps), ctypes.byref(running),
                                       ctypes.byref(queued)))
        return running.value, queued.value

    def info(self, rid) -> RequestInfo:
        out = RequestInfo()
        _check(lib().tr_server_info(self._h, int(rid), ctypes.byref(out)))
        return out

    def result(self, rid):
        ndet, nbins, steps = self._shape[rid]
        det = np.zeros(ndet * nbins)
        bud = np.zeros(9 * steps)
        _check(lib().tr_server_result(self._h, int(rid), _dptr(det), det.size, _dptr(bud),
                                      bud.size))
        return det.reshape(ndet, nbins), bud.reshape(steps, 9)

    def cancel(self, rid):
        _check(lib().tr_server_cancel(self._h, int(rid)))

    def close(self):
        if self._h:
            _check(lib().tr_server_destroy(self._h))
            self._h = _P()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def create_medium(prob, stream=None) -> Medium:
    return Medium.from_problem(prob, stream)


def bytes_required(desc: GridDesc, ndet=8, max_steps=1024) -> int:
    return int(lib().tr_bytes_required(ctypes.byref(desc), int(ndet), int(max_steps)))


def bytes_required_n(desc: GridDesc, n, ndet=8, max_steps=1024) -> int:
    nn = np.ascontiguousarray(n, np.float32).ravel()
    if nn.size != desc.nx * desc.ny * desc.nz:
        raise ValueError("n must hold nx*ny*nz values")
    return int(lib().tr_bytes_required_n(ctypes.byref(desc), _fptr(nn), int(ndet),
                                         int(max_steps)))


# ---- host set-up tables (no device needed) ---------------------------------

def host_directions(nside):
    out = np.zeros(12 * nside * nside * 3)
    _check(lib().tr_host_directions(nside, _dptr(out)))
    return out.reshape(-1, 3)


def host_parents(nside, nside_c):
    out = np.zeros(12 * nside * nside, np.int32)
    _check(lib().tr_host_parents(nside, nside_c, _iptr(out)))
    return out


def host_phase_matrix(nside, g, hg_norm="sinkhorn"):
    n = 12 * nside * nside
    out = np.zeros(n * n)
    _check(lib().tr_host_phase_matrix(nside, float(g), HG[hg_norm], _dptr(out)))
    return out.reshape(n, n)


def host_lattice(nside, nx, ny, nz):
    n = 12 * nside * nside
    me = max(nx, ny, nz)
    axis = np.zeros(n, np.int32)
    sign = np.zeros(n, np.int32)
    off = np.zeros(n * 2 * (me + 1), np.int32)
    _check(lib().tr_host_lattice(nside, nx, ny, nz, _iptr(axis), _iptr(sign), _iptr(off)))
    return axis, sign, off.reshape(n, 2, me + 1)


def host_move_tables(nside, nx, ny, nz, reverse=False):
    n = 12 * nside * nside
    NP = -(-n // 32) * 32
    me = max(nx, ny, nz)
    tab = np.zeros((NP + 1) * me, np.int32)
    dr = np.zeros(NP, np.int32)
    _check(lib().tr_host_move_tables(nside, nx, ny, nz, int(bool(reverse)), _iptr(tab),
                                     _iptr(dr)))
    return tab.reshape(NP + 1, me), dr


def host_coefficients(prob):
    d = grid_desc(prob)
    nv = prob.nvox
    a, b, r = np.zeros(nv), np.zeros(nv), np.zeros(nv)
    dt = ctypes.c_double()
    mua = np.ascontiguousarray(prob.mua, np.float32).ravel()
    mus = np.ascontiguousarray(prob.mus, np.float32).ravel()
    n = np.ascontiguousarray(prob.n, np.float32).ravel()
    _check(lib().tr_host_coefficients(ctypes.byref(d), _fptr(mua), _fptr(mus), _fptr(n),
                                      _dptr(a), _dptr(b), _dptr(r), ctypes.byref(dt)))
    return a, b, r, dt.value


def host_cone_set(nside, axis, cone_deg):
    out = np.zeros(12 * nside * nside, np.int32)
    cnt = ctypes.c_int()
    _check(lib().tr_host_cone_set(nside, float(axis[0]), float(axis[1]), float(axis[2]),
                                  float(cone_deg), _iptr(out), out.size, ctypes.byref(cnt)))
    return out[: cnt.value].tolist()


def host_pulse(dt, t0, fwhm, total, m0, count):
    out = np.zeros(count)
    _check(lib().tr_host_pulse(float(dt), float(t0), float(fwhm), float(total), int(m0),
                               int(count), _dptr(out)))
    return out


def host_interceptions(prob):
    d = grid_desc(prob)
    n = np.ascontiguousarray(prob.n, np.float32).ravel()
    cnt = ctypes.c_int()
    z = np.zeros(1, np.int32)
    _check(lib().tr_host_interceptions(ctypes.byref(d), _fptr(n), _iptr(z), _iptr(z), _iptr(z),
                                       _dptr(np.zeros(1)), _iptr(z), _iptr(z), 0,
                                       ctypes.byref(cnt)))
    c = cnt.value
    dd, vv, ww, rf, rr = (np.zeros(c, np.int32) for _ in range(5))
    R = np.zeros(c)
    _check(lib().tr_host_interceptions(ctypes.byref(d), _fptr(n), _iptr(dd), _iptr(vv), _iptr(ww),
                                       _dptr(R), _iptr(rf), _iptr(rr), c, ctypes.byref(cnt)))
    return list(zip(dd.tolist(), vv.tolist(), ww.tolist(), R.tolist(), rf.tolist(), rr.tolist()))


TR_PROBE_MFMA_F32, TR_PROBE_MFMA_BF16 = 0, 1


def probe_mfma(kind, iters=20000, blocks=1024):
    """tr_probe_mfma: (achieved TFLOP/s, ms) of back-to-back register-operand
    MFMAs, kind TR_PROBE_MFMA_F32 (32x32x2 FP32) or TR_PROBE_MFMA_BF16
    (32x32x16 bf16)."""
    tf, ms = ctypes.c_double(), ctypes.c_double()
    _check(lib().tr_probe_mfma(int(kind), int(iters), int(blocks), ctypes.byref(tf),
                               ctypes.byref(ms)))
    return tf.value, ms.value
