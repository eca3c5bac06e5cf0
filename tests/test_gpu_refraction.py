"""Multi-step parity of the 768-direction refraction path against stored FP64
oracle records: the heterogeneous medium of the air-hole study (Sec. 3.3: an
air cylinder with Fresnel reflection and refraction at its wall, Eq. 13-14,
and absorbing spheres) scaled to 32^3, at nside 8 (768 directions: the
collision kernels that stream P through LDS), split advance, 200 steps, in
FP32 and in BF16-split.  tests/golden/make_golden.py refraction32 wrote the
records, calling only the oracle."""
import os

import numpy as np
import pytest

from oracle import solve
from paper_2105_01028_amd import workloads as W

from test_gpu_parity import (assert_elementwise, budget_closure, closure_bound,
                             elementwise_bound, fresnel_ulps, rel_l2_above, run_gpu)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def golden(golden_dir):
    return np.load(os.path.join(golden_dir, "refraction32_oracle.npz"))


@pytest.fixture(scope="module")
def icpt_ulps():
    p = W.config3(nx=32)
    return fresnel_ulps(solve.build(p, steps=1).icpt)


@pytest.mark.parametrize("precision", ["fp32", "bf16split"])
def test_refraction32_768_directions_200_steps(precision, golden, icpt_ulps):
    """Per-step detector records (relative L2 < 1e-4 on bins above 1e-6 of the
    peak, all detectors together and each on its own), every budget row, the
    energy density of every voxel and every direction of the sampled voxels
    element by element (forward error bound of non-negative sums; BF16-split
    adds 2^-16 per step for the split of the scattered values)."""
    steps = int(golden["steps"])
    p = W.config3(nx=32).copy(precision=precision)
    assert p.ndir == 768
    got = run_gpu(p, steps=steps)
    print(f"[{precision}] refraction 32^3 x 768, {steps} steps", flush=True)
    assert got["info"].ninterceptions == int(golden["ninterceptions"]) > 0
    assert abs(got["info"].dt_ps - float(golden["dt"])) < 1e-12
    det, ref = got["steps"], golden["det"]
    assert det.shape == ref.shape
    e_all = rel_l2_above(det.ravel(), ref.ravel())
    assert e_all < 1e-4, e_all
    for k in range(ref.shape[0]):
        if ref[k].max() > 1e-6 * ref.max():
            assert rel_l2_above(det[k], ref[k]) < 1e-4, k
    # budget: oracle rows are (injected, absorbed, in the box, escaped per face)
    b, ob = got["budget"], golden["budget"]
    assert np.allclose(b[:, 0], ob[:, 0], rtol=1e-6, atol=1e-15)
    for q_gpu, q_ref in ((1, 1), (2, 2)):
        assert np.allclose(b[:, q_gpu], ob[:, q_ref], rtol=1e-4, atol=1e-9 * ob[:, q_ref].max())
    for f in range(6):
        assert np.allclose(b[:, 3 + f], ob[:, 3 + f], rtol=1e-4, atol=1e-9 * ob[:, 3:].max()), f
    ulps = 129.0 if precision == "bf16split" else 1.0
    assert budget_closure(b) < closure_bound(b, ulps=ulps)
    # the field element by element
    per_step = 2.0 ** -16 if precision == "bf16split" else 0.0
    bound = elementwise_bound(steps, p.ndir, icpt_ulps, per_step)
    st = got["state"]
    cols, vox = golden["cols"], golden["vox"]
    pk = np.abs(cols).max()
    r1 = assert_elementwise(st[:, vox], cols, bound, 1e-12 * pk)
    E, Eref = st.astype(np.float64).sum(axis=0), golden["energy"]
    r2 = assert_elementwise(E, Eref, bound, 1e-12 * Eref.max())
    print(f"[{precision}] detectors rel L2 {e_all:.2e}; max rel error: sampled columns {r1:.2e}, "
          f"energy {r2:.2e}; bound {bound:.2e}", flush=True)
