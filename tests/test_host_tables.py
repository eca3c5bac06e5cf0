"""The C++ host set-up, called through the C-ABI without a GPU, reproduces the
oracle's independently computed tables: exactly for integers, to FP64
rounding for reals.  Also checks that the library exports every symbol the
header declares."""
import os
import re

import numpy as np
import pytest

from oracle import angles, lattice, medium, optics, setup
from paper_2105_01028_amd import trinity as T
from paper_2105_01028_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    hdr = open(os.path.join(ROOT, "include", "trinity.h")).read()
    declared = set(re.findall(r"\b(tr_[a-z_]+)\s*\(", hdr))
    assert len(declared) >= 20
    L = T.lib()
    for name in sorted(declared):
        assert hasattr(L, name), name
    assert declared == set(T.EXPORTED)


@pytest.mark.parametrize("nside", [1, 2, 4, 8])
def test_directions(nside):
    assert np.abs(T.host_directions(nside) - angles.healpix_ring(nside)).max() < 2e-16


@pytest.mark.parametrize("nside,g,norm", [(2, 0.9, "sinkhorn"), (4, 0.85, "sinkhorn"),
                                          (2, 0.0, "sinkhorn"), (2, 0.9, "row"),
                                          (8, 0.9, "sinkhorn")])
def test_phase_matrix(nside, g, norm):
    ref = angles.phase_matrix(angles.healpix_ring(nside), g, norm)
    got = T.host_phase_matrix(nside, g, norm)
    # both stop the scaling once row sums are within 1e-14 of one
    assert np.abs(got - ref).max() < 1e-14 * np.abs(ref).max()


@pytest.mark.parametrize("nside,shape", [(2, (16, 16, 16)), (4, (9, 13, 7)), (8, (5, 6, 40))])
def test_lattice(nside, shape):
    nz, ny, nx = shape
    lat = lattice.RayLattice(angles.healpix_ring(nside), shape)
    axis, sign, off = T.host_lattice(nside, nx, ny, nz)
    assert np.array_equal(axis, lat.axis)
    assert np.array_equal(sign, lat.sign)
    for d in range(len(lat.dirs)):
        na = lat.ext[lat.axis[d]]
        assert np.array_equal(off[d, :, : na + 1], lat.offset[d])


@pytest.mark.parametrize("coef", ["paper", "abs_exact"])
def test_coefficients(coef):
    p = W.small_problem(nx=7, ny=5, nz=6, mua=0.03, mus=4.0, n=1.4, seed=4, coef=coef)
    n = p.n.copy()
    n[2:4] = 1.0
    mua = p.mua.copy()
    mua[2:4] = 0.0
    mus = p.mus.copy()
    mus[2:4] = 0.0
    p = p.copy(n=n, mua=mua, mus=mus)
    a, b, r, dt = T.host_coefficients(p)
    dt_ref = medium.time_step(p.dx_mm, np.asarray(p.n, np.float64))
    ar, br, _, _ = medium.collision_coefficients(p.mua, p.mus, np.asarray(p.n, np.float64),
                                                 dt_ref, coef)
    assert abs(dt - dt_ref) < 1e-15 * dt_ref
    assert np.abs(a - ar.ravel()).max() < 1e-15
    assert np.abs(b - br.ravel()).max() < 1e-15
    nref = medium.reference_index(p.n)
    assert np.array_equal(r, (nref / np.asarray(p.n, np.float64)).ravel())


@pytest.mark.parametrize("nside", [2, 4, 8])
def test_cone_sets(nside):
    d = angles.healpix_ring(nside)
    for face, normal in setup.FACE_NORMALS.items():
        for cone in (15.0, 30.0):
            assert T.host_cone_set(nside, normal, cone) == setup.cone_set(d, normal, cone)


def test_pulse():
    got = T.host_pulse(4.6699, 20.0, 10.0, 1.0, 0, 200)
    ref = setup.pulse_weights(200, 4.6699, 20.0, 10.0, 1.0)
    assert np.abs(got - ref).max() < 1e-16


def test_interceptions_match_oracle():
    p = W.config3(nx=24)
    p = p.copy(nside=2)
    got = T.host_interceptions(p)
    lat = lattice.RayLattice(angles.healpix_ring(2), p.shape)
    ref = optics.interceptions(lat, np.asarray(p.n, np.float64))
    assert len(got) == len(ref) > 100
    for g, r in zip(got, ref):
        assert g[0] == r[0] and g[1] == r[1] and g[2] == r[2]
        assert abs(g[3] - r[3]) < 1e-14
        assert g[4] == r[4] and g[5] == r[5]


def test_invalid_descriptor_is_rejected():
    p = W.small_problem()
    assert T.bytes_required(T.grid_desc(p)) > 0
    assert T.bytes_required(T.grid_desc(p.copy(transport="sweep"))) > 0
    bad = T.grid_desc(p)
    bad.transport = 2
    assert T.bytes_required(bad) == 0
    bad = T.grid_desc(p)
    bad.nside = 0
    assert T.bytes_required(bad) == 0
    with pytest.raises(T.TrinityError) as e:
        T.lib()  # loaded
        import ctypes
        h = ctypes.c_void_p()
        mua = np.zeros(p.nvox, np.float32)
        T._check(T.lib().tr_create_medium(ctypes.byref(bad), mua.ctypes.data, mua.ctypes.data,
                                          mua.ctypes.data, 0, 0, ctypes.byref(h)))
    assert e.value.status == T.TR_EINVAL
    assert "nside" in str(e.value)


def test_grid_voxel_limit():
    """The collision kernels address five rows of the field with 32-bit byte
    offsets: 107374080 voxels (after padding to 256) is the largest grid."""
    p = W.small_problem(nside=1)
    d = T.grid_desc(p)
    d.nx, d.ny, d.nz = 4096, 4096, 6          # 100663296 voxels
    assert T.bytes_required(d) > 0
    d.nx, d.ny, d.nz = 4096, 4096, 7          # 117440512 voxels
    assert T.bytes_required(d) == 0
    d.nx, d.ny, d.nz = 2560, 2560, 16         # 104857600 voxels
    assert T.bytes_required(d) > 0
    d.nx, d.ny, d.nz = 2560, 2560, 17         # 111411200 voxels
    assert T.bytes_required(d) == 0


@pytest.mark.parametrize("nf,nc", [(2, 1), (4, 1), (8, 2), (16, 4), (16, 16)])
def test_host_parents_match_oracle(nf, nc):
    from oracle import angles
    assert np.array_equal(T.host_parents(nf, nc), angles.parents(nf, nc))


def test_bytes_required_with_index():
    """tr_bytes_required_n adds what n decides.  A uniform n in phase advance
    adds nothing; the retarded advance adds its history of H fields, H the
    oracle's floor(max D) + 1 (so two time steps, or two uniform indices,
    differ by exactly the difference of their H fields); an index jump adds
    the interface tables; an invalid n, or
    phase advance with a varying n, gives 0."""
    from oracle import medium, retarded
    p = W.small_problem(nside=2, nx=13, ny=10, nz=9)
    d = T.grid_desc(p)
    assert T.bytes_required_n(d, p.n) == T.bytes_required(d) > 0
    C0 = medium.C0_MM_PER_PS
    n0 = float(p.n.flat[0])
    # one field: 48 directions padded to 64 rows (a multiple of 32) of the
    # voxels padded to a multiple of 256, float32
    row = 4 * 64 * (-(-p.nvox // 256) * 256)
    sizes = {}
    for courant in (1.0, 0.5, 0.2):
        q = p.copy(advance="retarded", dt_ps=courant * p.dx_mm * n0 / C0)
        H = retarded.build(q).H
        b = T.bytes_required_n(T.grid_desc(q), q.n)
        assert T.bytes_required(T.grid_desc(q)) == 0
        sizes[courant] = (H, b)
    (h1, b1), (h5, b5), (h2, b2) = sizes[1.0], sizes[0.5], sizes[0.2]
    assert h1 < h5 < h2
    assert b5 - b1 == (h5 - h1) * row and b2 - b5 == (h2 - h5) * row
    # a slab of air at a fifth of the crossing time of the fastest light
    n = p.n.copy()
    n[3:5] = 1.0
    q = p.copy(n=n, advance="retarded", dt_ps=0.2 * p.dx_mm / C0)
    H = retarded.build(q).H
    bq = T.bytes_required_n(T.grid_desc(q), n)
    # the longest hop is in the tissue: the same history as all tissue, plus
    # the interface and class tables; all air has the shortest history
    qu = p.copy(advance="retarded", dt_ps=0.2 * p.dx_mm / C0)
    qa = qu.copy(n=np.ones_like(p.n))
    Ha = retarded.build(qa).H
    assert retarded.build(qu).H == H > Ha
    bu = T.bytes_required_n(T.grid_desc(qu), qu.n)
    assert bq > bu
    assert bu - T.bytes_required_n(T.grid_desc(qa), qa.n) == (H - Ha) * row
    # split advance: the index jump adds interface tables
    s = p.copy(n=n, advance="split")
    assert T.bytes_required_n(T.grid_desc(s), n) > T.bytes_required(T.grid_desc(s))
    assert T.bytes_required_n(T.grid_desc(p.copy(advance="phase")), n) == 0
    bad = p.n.copy()
    bad[0, 0, 0] = 0.5
    assert T.bytes_required_n(d, bad) == 0
    with pytest.raises(ValueError):
        T.bytes_required_n(d, p.n[:-1])


@pytest.mark.parametrize("nside,shape", [(2, (7, 5, 6)), (4, (9, 8, 5)), (4, (6, 11, 7)),
                                         (1, (3, 4, 9))])
def test_move_tables_against_oracle_lattice(nside, shape):
    """The move tables of the fused collision and of its adjoint, checked
    against the oracle's lattice (Sec. 2.1, Fig. 1): a forward entry moves each
    voxel to its downwind voxel or flags its exit; a reversed entry moves each
    voxel back to its upwind voxel (the one whose photons moved into it) or
    flags that none is in the box.  The exits, sent around the box by the
    wrap offsets of the faces they leave through, land one to one on the
    voxels the other way has nothing for: forward exits on the voxels with no
    upwind voxel, reversed exits on the voxels whose photons leave."""
    from oracle import angles, lattice
    nx, ny, nz = shape
    tab, dr = T.host_move_tables(nside, nx, ny, nz)
    rtab, rdr = T.host_move_tables(nside, nx, ny, nz, reverse=True)
    assert np.array_equal(dr, rdr)
    dirs = angles.healpix_ring(nside)
    lat = lattice.RayLattice(dirs, (nz, ny, nx))
    p = lat.coords()
    v = np.arange(nx * ny * nz)
    ext = (nx, ny, nz)
    stride = (1, nx, nx * ny)
    LF = np.zeros(v.size, np.int64)
    for ax in range(3):
        LF |= (p[ax] == 0).astype(np.int64) << (2 * ax)
        LF |= (p[ax] == ext[ax] - 1).astype(np.int64) << (2 * ax + 1)
    wrap = [(1 if f & 1 else -1) * ext[f >> 1] * stride[f >> 1] for f in range(6)]

    def around(src, w, hits):
        t = src + (w >> 6)
        for f in range(6):
            t = t - np.where((hits >> f) & 1, wrap[f], 0)
        return t

    for d in range(len(dirs)):
        a = lat.axis[d]
        assert dr[d] & 0xFF == 10 * a
        dest, _ = lat.downwind(d)
        inside = dest >= 0
        up = np.full(v.size, -1)
        up[dest[inside]] = v[inside]
        has_up = up >= 0
        w = tab[d, p[a]].astype(np.int64)
        hits = w & 63 & LF
        assert np.all(hits[inside] == 0) and np.all(hits[~inside] != 0)
        assert np.array_equal(v[inside] + (w[inside] >> 6), dest[inside])
        assert np.array_equal(np.sort(around(v[~inside], w[~inside], hits[~inside])),
                              v[~has_up])
        rw = rtab[d, p[a]].astype(np.int64)
        rhits = rw & 63 & LF
        assert np.all(rhits[has_up] == 0) and np.all(rhits[~has_up] != 0)
        assert np.array_equal(v[has_up] + (rw[has_up] >> 6), up[has_up])
        assert np.array_equal(np.sort(around(v[~has_up], rw[~has_up], rhits[~has_up])),
                              v[~inside])
    assert not tab[len(dirs):].any() and not rtab[len(dirs):].any()


def test_mfma_probe_rejects_bad_arguments_before_touching_the_device():
    """tr_probe_mfma checks its arguments on the host (no GPU here)."""
    import ctypes
    tf, ms = ctypes.c_double(), ctypes.c_double()
    lib = T.lib()
    for kind, iters, blocks in ((2, 10, 10), (-1, 10, 10), (0, 0, 10), (0, (1 << 20) + 1, 10),
                                (1, 10, 0), (1, 10, (1 << 16) + 1)):
        assert lib.tr_probe_mfma(kind, iters, blocks, ctypes.byref(tf),
                                 ctypes.byref(ms)) == T.TR_EINVAL
    assert lib.tr_probe_mfma(0, 10, 10, None, ctypes.byref(ms)) == T.TR_EINVAL
