"""The single-output step of oracle/pointwise.py against the whole-field
oracle: the lattice neighbours one voxel at a time against the whole-grid
downwind maps, and every output of one step (collide and transport, with and
without index jumps, phase and split advance) against solve.forward."""
import numpy as np
import pytest

from oracle import pointwise, solve
from paper_2105_01028_amd import workloads as W


def test_neighbours_match_downwind_maps():
    p = W.small_problem(nside=2, nx=9, ny=7, nz=6, steps=1)
    L = pointwise.build(p)
    for d in range(len(L.dirs)):
        dest, _ = L.lat.downwind(d)
        for v in range(p.nvox):
            assert pointwise.downwind_of(L, d, v) == dest[v]
        up = np.full(p.nvox, -1)
        ok = dest >= 0
        up[dest[ok]] = np.nonzero(ok)[0]
        for v in range(p.nvox):
            assert pointwise.upwind_of(L, d, v) == up[v]


def _interface_problem(shape, seed):
    nx, ny, nz = shape
    p = W.small_problem(nside=2, nx=nx, ny=ny, nz=nz, mua=0.05, mus=3.0, g=0.8, steps=1,
                        seed=seed, advance="split", total_photons=0.0)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    n = np.full((nz, ny, nx), 1.4, np.float32)
    n[(x - nx / 2) ** 2 + (y - ny / 2) ** 2 + (z - nz / 2) ** 2 < (min(shape) / 3) ** 2] = 1.0
    n[:, :, : max(1, nx // 5)] = 1.33
    p.n = n
    return p


@pytest.mark.parametrize("case", ["phase", "split", "interfaces", "twolevel", "implicit"])
def test_outputs_match_whole_field_step(case):
    if case == "interfaces":
        p = _interface_problem((10, 9, 8), 3)
    elif case == "twolevel":
        p = W.small_problem(nside=4, nx=7, ny=6, nz=5, mua=0.05, mus=3.0, g=0.8, steps=1,
                            seed=4, advance="phase", total_photons=0.0).copy(nside_scatter=2)
    elif case == "implicit":
        p = W.small_problem(nside=2, nx=9, ny=8, nz=7, mua=0.05, mus=3.0, g=0.8, steps=1,
                            seed=4, advance="split", total_photons=0.0).copy(source="implicit")
    else:
        p = W.small_problem(nside=2, nx=9, ny=8, nz=7, mua=0.05, mus=3.0, g=0.8, steps=1,
                            seed=4, advance=case, total_photons=0.0)
    rng = np.random.default_rng(5)
    N0 = rng.uniform(0, 1, (p.ndir, p.nvox))
    m = 3 if case in ("phase", "twolevel") else 0
    ref = solve.forward(p, steps=1, state0=N0, start_step=m).state
    L = pointwise.build(p)
    if case == "interfaces":
        assert len(solve.build(p).icpt) > 0
    for v in range(p.nvox):
        got = pointwise.step_outputs(L, lambda w: N0[:, w], v, m)
        assert np.allclose(got, ref[:, v], rtol=1e-12, atol=1e-14), v
