"""The allocation-free step (tr_step_noalloc, through the C-ABI) against
tr_step on the same media: the same kernels with their partial sums in the
per-device workspace instead of the medium's buffers, so the records and the
field must come out bit for bit the same.  Two calls in a row on a larger
medium, then calls on a smaller one (the workspace keeps the previous call's
contents), and the refusals."""
import numpy as np
import pytest

from oracle import solve
from paper_2105_01028_amd import trinity as T
from paper_2105_01028_amd import workloads as W

pytestmark = pytest.mark.gpu


def _stream():
    import torch
    assert torch.cuda.is_available(), "these tests need the GPU"
    return torch.cuda.Stream()


def _run(prob, calls, noalloc, stream):
    import torch
    with torch.cuda.stream(stream):
        m = T.Medium.from_problem(prob)
        for n in calls:
            (m.step_noalloc if noalloc else m.step)(n)
        m.synchronize()
        out = dict(det=m.read_detector_steps(), budget=m.read_budget(), state=m.get_state())
        m.close()
    return out


def _interfaces(p):
    nz, ny, nx = p.shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    n = np.full(p.shape, 1.4, np.float32)
    n[(x - nx / 2) ** 2 + (y - ny / 2) ** 2 + (z - nz / 2) ** 2 < (min(p.shape) / 3) ** 2] = 1.0
    return p.copy(n=n, advance="split")


CASES = [
    # larger medium first: 192 directions, phase advance with the moves in the
    # collision kernel; then a smaller ragged one in split advance with
    # Fresnel interfaces (collide, sweep, gather, tallies)
    ("phase192", lambda: W.small_problem(nside=4, nx=40, ny=36, nz=30, mua=0.02, mus=3.0,
                                         g=0.85, steps=50, seed=4, det_cone_deg=0.0), (20, 30)),
    ("split48", lambda: _interfaces(W.small_problem(nside=2, nx=13, ny=10, nz=9, mua=0.03,
                                                    mus=2.0, g=0.8, steps=25, seed=5,
                                                    det_cone_deg=0.0)), (25,)),
]


def test_noalloc_equals_tr_step_larger_then_smaller():
    s = _stream()
    for name, make, calls in CASES:
        p = make()
        print(f"no-alloc case {name}: grid {p.nx}x{p.ny}x{p.nz}, {p.ndir} directions, "
              f"calls {calls}", flush=True)
        ref = _run(p, (sum(calls),), False, s)
        got = _run(p, calls, True, s)
        for k in ("det", "budget", "state"):
            assert got[k].shape == ref[k].shape, (name, k)
            assert np.array_equal(got[k], ref[k]), (name, k, np.abs(got[k] - ref[k]).max())
        # and the oracle's detector records (the parity bar of the step itself)
        o = solve.forward(p, steps=sum(calls))
        mask = o.det > 1e-6 * o.det.max()
        err = np.linalg.norm(got["det"][mask] - o.det[mask]) / np.linalg.norm(o.det[mask])
        assert err < 1e-4, (name, err)


def test_noalloc_refuses_steps_beyond_the_record_capacity():
    import torch
    p = W.small_problem(nside=2, nx=9, ny=8, nz=7, steps=10, seed=1)
    with torch.cuda.stream(_stream()):
        m = T.Medium.from_problem(p)
        m.step_noalloc(1000)
        with pytest.raises(T.TrinityError) as e:
            m.step_noalloc(100)
        assert e.value.status == T.TR_EINVAL and "capacity" in str(e.value)
        with pytest.raises(T.TrinityError):
            m.step_noalloc(-1)
        m.step_noalloc(0)
        m.synchronize()
        assert m.info().steps_done == 1000
        m.close()
