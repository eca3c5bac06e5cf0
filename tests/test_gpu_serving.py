"""Continuous-batching server on the GPU: a request's result is the same bits
alone and in a mix (also when it joins a running batch), requests queue on
the device-memory budget, invalid requests are refused without disturbing the
others, and results match the single-medium path and the FP64 oracle."""
import numpy as np
import pytest

from oracle import solve
from paper_2105_01028_amd import trinity as T
from paper_2105_01028_amd import workloads as W

pytestmark = pytest.mark.gpu


def _ctx():
    import torch
    assert torch.cuda.is_available()
    return torch.cuda.stream(torch.cuda.Stream())


def req(side=12, steps=40, seed=0, src=None, nside=2):
    rng = np.random.default_rng(seed)
    p = W.small_problem(nside=nside, nx=side, ny=side + 2, nz=side - 1, mua=0.02, mus=2.5,
                        g=0.7, n=1.4, steps=steps, seed=seed, det_cone_deg=0.0)
    if src is not None:
        p.src_ix, p.src_iy = src
    else:
        p.src_ix, p.src_iy = (int(v) for v in rng.integers(1, side - 3, 2))
    return p


def drain(srv, ids, max_rounds=10000):
    for _ in range(max_rounds):
        srv.advance(24)
        if all(srv.info(i).status in (T.REQ_DONE, T.REQ_FAILED, T.REQ_CANCELLED) for i in ids):
            return
    raise AssertionError("server did not finish")


def test_alone_equals_mix_bitwise():
    a = req(12, 50, 1)
    others = [req(16, 30, 2), req(9, 70, 3), req(20, 45, 4)]
    with _ctx():
        s1 = T.Server(nside=2, g=0.7, max_slots=8)
        ia = s1.submit(a)
        drain(s1, [ia])
        alone, bud_alone = s1.result(ia)
        s1.close()
        s2 = T.Server(nside=2, g=0.7, max_slots=8)
        ids = [s2.submit(p) for p in others[:2]] + [s2.submit(a)] + [s2.submit(others[2])]
        drain(s2, ids)
        mixed, bud_mixed = s2.result(ids[2])
        s2.close()
    assert np.array_equal(alone, mixed)
    assert np.array_equal(bud_alone[:, 0], bud_mixed[:, 0])


def test_late_joiner_equals_alone():
    """B arrives while A is half done and joins the running batch."""
    a, b = req(14, 60, 5), req(11, 50, 6)
    with _ctx():
        s = T.Server(nside=2, g=0.7, max_slots=4)
        ia = s.submit(a)
        s.advance(25)
        assert s.info(ia).status == T.REQ_RUNNING
        ib = s.submit(b)
        s.advance(8)
        assert s.info(ib).status == T.REQ_RUNNING and s.info(ia).status == T.REQ_RUNNING
        drain(s, [ia, ib])
        ra, rb = s.result(ia)[0], s.result(ib)[0]
        s.close()
        ref = {}
        for p, key in ((a, "a"), (b, "b")):
            s1 = T.Server(nside=2, g=0.7, max_slots=4)
            i = s1.submit(p)
            drain(s1, [i])
            ref[key] = s1.result(i)[0]
            s1.close()
    assert np.array_equal(ra, ref["a"])
    assert np.array_equal(rb, ref["b"])


def test_server_matches_medium_and_oracle():
    p = req(12, 60, 7)
    with _ctx():
        s = T.Server(nside=2, g=0.7, max_slots=2)
        i = s.submit(p)
        drain(s, [i])
        det, bud = s.result(i)
        s.close()
        m = T.Medium.from_problem(p)
        m.solve(p.steps)
        det_m = m.read_detectors()
        m.close()
    assert np.array_equal(det, det_m)
    ref = solve.forward(p).binned(p.bin_ps, p.nbins)
    mask = ref > 1e-6 * ref.max()
    assert np.linalg.norm(det[mask] - ref[mask]) / np.linalg.norm(ref[mask]) < 1e-4


def test_admission_by_budget():
    a, b, c = req(16, 40, 8), req(16, 40, 9), req(16, 40, 10)
    with _ctx():
        probe = T.Server(nside=2, g=0.7)
        need = probe.request_bytes(a)
        probe.close()
        s = T.Server(nside=2, g=0.7, budget_bytes=int(need * 1.5), max_slots=8)
        ids = [s.submit(x) for x in (a, b, c)]
        running, queued = s.advance(10)
        assert (running, queued) == (1, 2)
        assert [s.info(i).status for i in ids] == [T.REQ_RUNNING, T.REQ_QUEUED, T.REQ_QUEUED]
        drain(s, ids)
        assert all(s.info(i).status == T.REQ_DONE for i in ids)
        # queued time of the last one covers the two before it
        assert s.info(ids[2]).queued_ms >= s.info(ids[1]).queued_ms
        s.close()
        big = T.Server(nside=2, g=0.7, budget_bytes=need // 2)
        with pytest.raises(T.TrinityError) as e:
            big.submit(a)
        assert e.value.status == T.TR_ENOMEM
        big.close()


def test_bad_requests_refused_others_unaffected():
    good = req(12, 30, 11)
    bad = req(12, 30, 12)
    bad.mua = bad.mua.copy()
    bad.mua[2, 3, 4] = np.nan
    het = req(12, 30, 13)
    het.n = het.n.copy()
    het.n[0, 0, 0] = 1.0
    with _ctx():
        s = T.Server(nside=2, g=0.7)
        ig = s.submit(good)
        for p in (bad, het):
            with pytest.raises(T.TrinityError) as e:
                s.submit(p)
            assert e.value.status == T.TR_EINVAL
        drain(s, [ig])
        det, _ = s.result(ig)
        s.close()
        s1 = T.Server(nside=2, g=0.7)
        i1 = s1.submit(good)
        drain(s1, [i1])
        assert np.array_equal(det, s1.result(i1)[0])
        s1.close()


def test_cancel():
    a, b, c = req(12, 200, 14), req(12, 40, 15), req(12, 40, 16)
    with _ctx():
        s = T.Server(nside=2, g=0.7, max_slots=2)
        ia, ib, ic = s.submit(a), s.submit(b), s.submit(c)
        s.advance(10)
        s.cancel(ia)          # running
        s.cancel(ic)          # queued
        drain(s, [ia, ib, ic])
        assert s.info(ia).status == T.REQ_CANCELLED
        assert s.info(ic).status == T.REQ_CANCELLED
        assert s.info(ib).status == T.REQ_DONE
        with pytest.raises(T.TrinityError):
            s.result(ia)
        det_b = s.result(ib)[0]
        s.close()
        s1 = T.Server(nside=2, g=0.7)
        i1 = s1.submit(b)
        drain(s1, [i1])
        assert np.array_equal(det_b, s1.result(i1)[0])
        s1.close()


def test_destroy_with_requests_in_flight():
    """Destroying a server with requests running and queued waits for the
    work already queued on its stream and frees everything; a new server
    then serves as before."""
    with _ctx():
        s = T.Server(nside=2, g=0.7, max_slots=2)
        ids = [s.submit(req(12, 300, 17 + k)) for k in range(4)]
        running, queued = s.advance(8)
        assert running == 2 and queued == 2
        assert s.info(ids[0]).status == T.REQ_RUNNING
        s.close()
        s2 = T.Server(nside=2, g=0.7)
        i = s2.submit(req(12, 30, 11))
        drain(s2, [i])
        assert s2.info(i).status == T.REQ_DONE
        s2.close()


def test_phantom_scale_stream_smoke():
    """A few requests of the serving workload (192 directions, 32^3 .. 48^3)
    with shortened step counts complete and conserve light."""
    reqs = W.serving_stream(4, seed=4, sides=(32, 48), steps_range=(60, 90))
    from paper_2105_01028_amd import serve
    with _ctx():
        s = T.Server(nside=4, g=0.85, max_slots=4)
        out = serve.run_stream(s, reqs, chunk_steps=32, keep_results=True)
        s.close()
    assert out["completed"] == 4 and len(out["results"]) == 4
    for det, bud in out["results"].values():
        assert np.isfinite(det).all() and det.sum() > 0
        inj = bud[:, 0].sum()
        closure = abs(inj - bud[:, 1].sum() - bud[:, 3:].sum() - bud[-1, 2]) / inj
        assert closure < 2.0 ** -23 * bud[:, 2].sum() / inj + 1e-12
