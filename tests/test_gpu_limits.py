"""The largest grids the C-ABI takes: 2560 x 2560 x 16 (104 857 600 voxels)
and 4096 x 4096 x 6 (100 663 296 voxels, the longest rows), below the limit of
107 374 080 voxels that the collision kernels' 32-bit offsets over five rows
set, and 4096, the largest extent.  One step from a state that is non-zero in
small cubes (corners, edges, the interior) with 12 directions, compared at
every direction of the voxels around them with the single-output FP64 oracle
(oracle/pointwise.py) to 2e-6 of the largest sampled value."""
import numpy as np
import pytest

from paper_2105_01028_amd import trinity as T
from paper_2105_01028_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("shape", [(2560, 2560, 16), (4096, 4096, 6)])
def test_largest_grids_single_step(shape):
    import torch

    from oracle import pointwise
    nx, ny, nz = shape
    p = W.small_problem(nside=1, nx=nx, ny=ny, nz=nz, mua=0.05, mus=2.0, g=0.8, steps=1,
                        advance="phase", total_photons=0.0)
    rng = np.random.default_rng(nx + nz)
    p.mua[...] *= rng.uniform(0.7, 1.3, (1, ny, nx)).astype(np.float32)
    assert p.nvox <= 107374080 and max(shape) <= 4096
    centres = [(0, 0, 0), (nx - 1, ny - 1, nz - 1), (nx - 1, 0, nz // 2), (0, ny - 1, 1),
               (nx // 2, ny // 2, nz // 2), (int(rng.integers(2, nx - 2)),
                                              int(rng.integers(2, ny - 2)), nz - 2)]
    ndir = 12

    def cube(r):
        out = set()
        for cx, cy, cz in centres:
            for dz in range(-r, r + 1):
                for dy in range(-r, r + 1):
                    for dx in range(-r, r + 1):
                        x, y, z = cx + dx, cy + dy, cz + dz
                        if 0 <= x < nx and 0 <= y < ny and 0 <= z < nz:
                            out.add((z * ny + y) * nx + x)
        return np.array(sorted(out))
    vox, out_vox = cube(2), cube(1)
    cols = rng.uniform(0.0, 1.0, (ndir, len(vox))).astype(np.float32)
    where = {int(v): i for i, v in enumerate(vox)}
    print(f"[{nx}x{ny}x{nz}] {p.nvox} voxels", flush=True)
    with torch.cuda.stream(torch.cuda.Stream()):
        m = T.Medium.from_problem(p)
        state = torch.zeros((ndir, p.nvox), dtype=torch.float32, device="cuda")
        state[:, torch.as_tensor(vox, device="cuda")] = torch.as_tensor(cols, device="cuda")
        m.set_state(state)
        m.step(1)
        m.synchronize()
        m.get_state(state)
        torch.cuda.synchronize()
        got = state[:, torch.as_tensor(out_vox, device="cuda")].cpu().numpy()
        b = m.read_budget()
        m.close()
        del state
    L = pointwise.build(p)
    zero = np.zeros(ndir)

    def column(w):
        i = where.get(int(w))
        return zero if i is None else cols[:, i].astype(np.float64)
    ref = np.stack([pointwise.step_outputs(L, column, int(v)) for v in out_vox], axis=1)
    scale = np.abs(ref).max()
    assert scale > 0
    assert np.abs(got - ref).max() <= 2e-6 * scale
    # the budget of the step: what was in the box is absorbed, escaped or still in it
    total = float(cols.astype(np.float64).sum())
    assert abs(b[0, 1] + b[0, 2] + b[0, 3:].sum() - total) <= 2e-6 * total


def test_mfma_probe_reports_a_rate_within_the_peak():
    """tr_probe_mfma runs both shapes and reports a positive rate no higher
    than the datasheet dense peak (157.3 TFLOP/s FP32, 2500 bf16) plus 2 %."""
    for kind, peak in ((T.TR_PROBE_MFMA_F32, 157.3), (T.TR_PROBE_MFMA_BF16, 2500.0)):
        tf, ms = T.probe_mfma(kind, iters=2000, blocks=512)
        print(f"probe kind {kind}: {tf:.1f} TFLOP/s in {ms:.3f} ms", flush=True)
        assert ms > 0.0 and 0.0 < tf <= 1.02 * peak
