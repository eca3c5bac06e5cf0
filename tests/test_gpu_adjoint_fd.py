"""The full-size adjoint (64^3 medium, 192 directions, 500 steps, checkpoints
every 50, in the launch configuration the benchmark times) against central
finite differences of the FP64 oracle's loss, L = sum over detectors and
bins of (y - y_target)^2 with the target of the perturbed medium (each
sphere's mu_a x 1.2).  tests/golden/make_golden.py adjoint64_fd wrote the
differences, calling only the oracle: step 1e-4 of each coefficient, along a
+-1 pattern over 20 voxels (for mu_a and mu_s) and at 4 of them one by one,
for 20 voxels drawn over the whole medium and 20 drawn between the source
and the nearer detectors.

The target differs from the medium's own signals by little more than an FP32
solve's rounding of them (L is 1e-22 against signals of 1e-6), so the
adjoint is seeded with the oracle's dL/dy = 2 (y0 - target): the GPU then
computes J^T g for the FP64 g, which is what the differences measure."""
import os

import numpy as np
import pytest

from paper_2105_01028_amd import trinity as T
from paper_2105_01028_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fd(golden_dir):
    return np.load(os.path.join(golden_dir, "adjoint64_fd_oracle.npz"))


@pytest.fixture(scope="module")
def gradient(fd):
    import torch
    p = W.config5()
    with torch.cuda.stream(torch.cuda.Stream()):
        m = T.Medium.from_problem(p)
        m.solve_checkpointed(p.steps, 50)
        y = m.read_detectors()
        gmua, gmus = m.backward(2.0 * (fd["y0"] - fd["target"]))
        m.close()
    # the GPU's signals are the oracle's to the FP32 solve's rounding
    y0 = fd["y0"]
    mask = y0 > 1e-6 * y0.max()
    assert np.linalg.norm(y[mask] - y0[mask]) / np.linalg.norm(y0[mask]) < 1e-4
    return {"mua": gmua.astype(np.float64).ravel() * p.mua.astype(np.float64).ravel(),
            "mus": gmus.astype(np.float64).ravel() * p.mus.astype(np.float64).ravel()}


@pytest.mark.parametrize("draw", ["box", "near"])
@pytest.mark.parametrize("which", ["mua", "mus"])
def test_adjoint_matches_fp64_oracle_finite_differences(fd, gradient, draw, which):
    """dL/d eps (mu_v -> mu_v (1 + eps s_v)) from the adjoint against the FP64
    central differences: along the pattern to 1e-3 of the sum of the terms'
    magnitudes, at each single voxel to 1e-3 of itself."""
    gm = gradient[which]
    vox, sgn = fd[f"vox_{draw}"], fd[f"sgn_{draw}"]
    terms = gm[vox] * sgn
    pred, want = float(terms.sum()), float(fd[f"dir_{draw}_{which}"])
    scale = float(np.abs(terms).sum())
    print(f"[{draw} {which}] along the pattern: adjoint {pred:.6e}, FP64 differences {want:.6e} "
          f"(terms {scale:.3e})", flush=True)
    assert scale > 0 and abs(pred - want) <= 1e-3 * scale
    for i, v in enumerate(vox[:len(fd[f"single_{draw}_{which}"])]):
        w = float(fd[f"single_{draw}_{which}"][i])
        print(f"[{draw} {which}] voxel {int(v)}: adjoint {gm[v]:.6e}, FP64 differences {w:.6e}",
              flush=True)
        assert w != 0 and abs(gm[v] - w) <= 1e-3 * abs(w), (draw, which, int(v))
