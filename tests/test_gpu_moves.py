"""Phase stepping with the moves in the collision kernel, through the C-ABI:
against the separate sweep kernel on the same inputs (the same field bits and
detector records, the photon budget up to summation order), and against the
FP64 oracle element by element."""
import numpy as np
import pytest

from oracle import solve
from paper_2105_01028_amd import trinity as T
from paper_2105_01028_amd import workloads as W

pytestmark = pytest.mark.gpu


def _run(prob, steps, state0=None, one_by_one=False):
    import torch
    assert torch.cuda.is_available(), "these tests need the GPU"
    with torch.cuda.stream(torch.cuda.Stream()):
        m = T.Medium.from_problem(prob)
        fused = m.info().moves_fused
        if state0 is not None:
            m.set_state(state0)
        if one_by_one:
            for _ in range(steps):
                m.step(1)
            m.synchronize()
        else:
            m.solve(steps)
        out = dict(state=m.get_state(), det=m.read_detector_steps(), budget=m.read_budget(),
                   energy=m.read_energy(), fused=fused)
        m.close()
    return out


def _problem(nside, shape, steps, **kw):
    """A seeded phase-mode problem whose source and detectors fit any shape,
    one voxel thick included."""
    nx, ny, nz = shape
    dets = ([W.FACE_TOP, W.FACE_TOP, W.FACE_XMAX],
            [min(nx - 1, nx // 2), min(nx - 1, nx // 2 + 1), ny // 2],
            [ny // 2, max(0, ny // 2 - 1), nz // 2])
    return W.small_problem(nside=nside, nx=nx, ny=ny, nz=nz, mua=0.05, mus=2.0, g=0.8,
                           steps=steps, seed=nx + ny + nz, advance="phase",
                           src_ix=max(0, nx // 2 - 1), src_iy=max(0, ny // 2 - 1),
                           src_w=2 if nx >= 2 and ny >= 2 else 1, dets=dets, **kw)


# shapes with one voxel along an axis put every voxel on two faces (the
# per-value face precedence); ragged sizes leave padding columns in the last tile
CASES = [
    (1, "fp32", (9, 7, 5), 23),
    (2, "fp32", (13, 10, 9), 37),
    (4, "fp32", (16, 12, 10), 35),
    (4, "bf16split", (16, 12, 10), 35),
    (2, "bf16split", (21, 14, 11), 33),
    (2, "fp32", (1, 7, 5), 20),
    (2, "fp32", (12, 1, 9), 20),
    (4, "fp32", (20, 13, 1), 20),
    (4, "fp32", (48, 40, 24), 40),
    # more 256-voxel tiles (360) than workgroups: workgroups take several
    # tiles, and the next tile's rows are loaded while the current one runs
    (4, "bf16split", (48, 48, 40), 30),
]


@pytest.mark.parametrize("nside,precision,shape,steps", CASES)
def test_moves_in_collision_equal_separate_sweep(nside, precision, shape, steps):
    nx, ny, nz = shape
    p = _problem(nside, shape, steps, precision=precision)
    rng = np.random.default_rng(nx * ny * nz)
    N0 = rng.uniform(0, 1, (12 * nside * nside, p.nvox)).astype(np.float32)
    a = _run(p, steps, N0)
    b = _run(p.copy(transport="sweep"), steps, N0)
    assert a["fused"] == 1 and b["fused"] == 0
    assert np.array_equal(a["state"], b["state"])
    assert np.array_equal(a["det"], b["det"])
    ba, bb = a["budget"], b["budget"]
    scale = ba[:, 2].max()
    assert np.array_equal(ba[:, 0], bb[:, 0])                # injected
    # absorbed: the same per-tile FP64 partials, summed in another tile order
    assert np.allclose(ba[:, 1], bb[:, 1], rtol=1e-12, atol=1e-15 * ba[:, 1].max())
    # in box, escape: the collision kernel sums 16 values per lane in FP32 before
    # FP64, each partial within 15 * 2^-24 < 1e-6 of itself; the sweep sums in FP64
    assert np.allclose(ba[:, 2:], bb[:, 2:], rtol=1e-6, atol=1e-12 * scale)


@pytest.mark.parametrize("nside,shape", [(2, (13, 10, 9)), (4, (16, 12, 10))])
def test_moves_in_collision_detectors_on_edges_and_corners(nside, shape):
    """Detectors on box edges and corners: their voxels lie on two or three
    faces, where the light that leaves is kept for the read-out and the face
    of each exit follows the sweep's precedence."""
    nx, ny, nz = shape
    dets = ([W.FACE_TOP, W.FACE_TOP, W.FACE_TOP, W.FACE_XMAX, W.FACE_XMAX],
            [0, nx - 1, nx // 2, 0, ny - 1], [0, ny - 1, 0, nz - 1, nz // 2])
    p = W.small_problem(nside=nside, nx=nx, ny=ny, nz=nz, mua=0.05, mus=2.0, g=0.8, steps=30,
                        seed=3, advance="phase", det_cone_deg=60.0, dets=dets)
    rng = np.random.default_rng(nx)
    N0 = rng.uniform(0, 1, (12 * nside * nside, p.nvox)).astype(np.float32)
    a = _run(p, 30, N0)
    b = _run(p.copy(transport="sweep"), 30, N0)
    assert a["fused"] == 1 and b["fused"] == 0
    assert np.array_equal(a["state"], b["state"])
    assert np.array_equal(a["det"], b["det"])
    assert np.abs(a["det"]).max() > 0
    ba, bb = a["budget"], b["budget"]
    assert np.allclose(ba[:, 2:], bb[:, 2:], rtol=1e-6, atol=1e-12 * ba[:, 2].max())


def test_moves_in_collision_graph_replay_equals_single_steps():
    """The field alternates between two buffers by step parity read on the
    device: graph replays of 16 steps and single launches give the same bits."""
    p = W.small_problem(nside=2, nx=12, ny=12, nz=12, steps=40, seed=5, advance="phase")
    a = _run(p, 40)
    b = _run(p, 40, one_by_one=True)
    assert a["fused"] == 1
    assert np.array_equal(a["state"], b["state"])
    assert np.array_equal(a["det"], b["det"])
    assert np.array_equal(a["budget"], b["budget"])


@pytest.mark.parametrize("steps", [1, 2, 17])
def test_moves_in_collision_match_oracle(steps):
    """After odd and even step counts the state read back is the oracle's,
    element by element, and so are the energy and the budget."""
    p = W.small_problem(nside=4, nx=14, ny=11, nz=9, mua=0.05, mus=3.0, g=0.8, steps=steps,
                        seed=13, advance="phase")
    rng = np.random.default_rng(steps)
    N0 = rng.uniform(0, 1, (192, p.nvox)).astype(np.float32)
    ref = solve.forward(p, steps=steps, state0=N0.astype(np.float64))
    got = _run(p, steps, N0)
    assert got["fused"] == 1
    assert np.abs(got["state"] - ref.state).max() <= 1e-5 * np.abs(ref.state).max()
    assert np.allclose(got["energy"].ravel(), ref.state.sum(axis=0), rtol=1e-5, atol=1e-6)
    b = got["budget"]
    assert np.allclose(b[:, 3:], ref.escaped, rtol=1e-5, atol=1e-7 * ref.escaped.max())
    assert np.allclose(b[:, 2], ref.in_domain, rtol=1e-5)


def test_moves_fused_only_where_they_apply():
    """Split advance, the implicit source, two-level angles and the sweep
    option keep the separate sweep kernel."""
    import torch
    base = W.small_problem(nside=2, nx=10, ny=9, nz=8, steps=3, seed=2, advance="phase")
    cases = [(base, 1), (base.copy(transport="sweep"), 0), (base.copy(advance="split"), 0),
             (base.copy(source="implicit"), 0),
             (W.small_problem(nside=4, nx=10, ny=9, nz=8, steps=3, seed=2,
                              advance="phase").copy(nside_scatter=2), 0)]
    with torch.cuda.stream(torch.cuda.Stream()):
        for prob, want in cases:
            m = T.Medium.from_problem(prob)
            assert m.info().moves_fused == want, (prob.advance, prob.transport, prob.source)
            m.close()


def test_moves_in_collision_bf16_many_tiles_match_oracle():
    """BF16-split with the moves in the collision on a grid of 360 tiles (so
    workgroups run several tiles each, prefetching the next one's rows): the
    per-step detector records against the FP64 oracle's (relative L2 below
    1e-4 on bins above 1e-6 of the peak, all together and each detector)."""
    p = W.small_problem(nside=4, nx=48, ny=48, nz=40, mua=0.02, mus=2.0, g=0.8, steps=60,
                        seed=29, advance="phase", precision="bf16split", det_cone_deg=0.0)
    assert p.nvox // 256 > 256
    ref = solve.forward(p, steps=60)
    got = _run(p, 60)
    assert got["fused"] == 1
    det, want = got["det"], ref.det
    mask = want > 1e-6 * want.max()
    assert want.max() > 0 and mask.sum() > 20
    e = np.linalg.norm(det[mask] - want[mask]) / np.linalg.norm(want[mask])
    assert e < 1e-4, e
    for k in range(want.shape[0]):
        mk = want[k] > 1e-6 * want.max()
        if mk.any():
            assert np.linalg.norm(det[k][mk] - want[k][mk]) / np.linalg.norm(want[k][mk]) < 1e-4
