"""GPU adjoint against the FP64 oracle's gradient (itself pinned to finite
differences), through the torch.autograd.Function, and against finite
differences of GPU solves."""
import numpy as np
import pytest

from oracle import adjoint, solve
from paper_2105_01028_amd import trinity as T
from paper_2105_01028_amd import workloads as W

pytestmark = pytest.mark.gpu


def _problem(nside=2, steps=40, seed=21):
    return W.small_problem(nside=nside, nx=11, ny=9, nz=8, mua=0.05, mus=1.5, g=0.7, n=1.4,
                           steps=steps, seed=seed, det_cone_deg=0.0)


def _target(p):
    ref = p.copy(mua=(p.mua * 1.3).astype(np.float32))
    return solve.forward(ref).binned(p.bin_ps, p.nbins)


def _gpu_grad(p, target, ckpt):
    import torch
    with torch.cuda.stream(torch.cuda.Stream()):
        m = T.Medium.from_problem(p)
        m.solve_checkpointed(p.steps, ckpt)
        y = m.read_detectors()
        before = m.read_detector_steps()
        gmua, gmus = m.backward(2.0 * (y - target))
        after = m.read_detector_steps()
        state = m.get_state()
        m.step(3)
        cont = m.read_detector_steps()
        m.close()
        m2 = T.Medium.from_problem(p)
        m2.solve(p.steps)
        state2 = m2.get_state()
        m2.step(3)
        cont2 = m2.read_detector_steps()
        m2.close()
    return gmua, gmus, (before, after, state, cont, state2, cont2)


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("nside,ckpt,coef,transport", [
    (2, 7, "paper", "auto"), (2, 40, "paper", "auto"), (4, 13, "abs_exact", "auto"),
    # media stepped with the separate sweep: the adjoint's separate transposed sweep
    (2, 7, "paper", "sweep"), (4, 13, "abs_exact", "sweep")])
def test_gradient_matches_oracle(nside, ckpt, coef, transport):
    """Media stepped with the moves in the collision (transport auto) take the
    adjoint whose transposed collision does the transposed moves in its
    epilogue; media stepped with the sweep take the separate transposed
    sweep.  Both against the oracle's gradient."""
    p = _problem(nside).copy(coef=coef, transport=transport)
    target = _target(p)
    gmua_ref, gmus_ref, _ = adjoint.gradient(p, target)
    gmua, gmus, _ = _gpu_grad(p, target, ckpt)
    assert rel_l2(gmua, gmua_ref) < 1e-4
    assert rel_l2(gmus, gmus_ref) < 1e-4


@pytest.mark.parametrize("transport", ["auto", "sweep"])
def test_backward_leaves_medium_unchanged(transport):
    p = _problem().copy(transport=transport)
    _, _, (before, after, state, cont, state2, cont2) = _gpu_grad(p, _target(p), 9)
    assert np.array_equal(before, after)
    assert np.array_equal(state, state2)
    assert np.array_equal(cont, cont2)


def test_autograd_function():
    import torch
    from paper_2105_01028_amd.autograd import detector_signals
    p = _problem(steps=30)
    target = _target(p)
    mua = torch.tensor(p.mua, device="cuda", requires_grad=True)
    mus = torch.tensor(p.mus, device="cuda", requires_grad=True)
    y = detector_signals(mua, mus, p, ckpt_every=10)
    loss = ((y - torch.as_tensor(target, device="cuda")) ** 2).sum()
    loss.backward()
    gmua_ref, gmus_ref, L_ref = adjoint.gradient(p, target)
    assert abs(loss.item() - L_ref) < 1e-4 * L_ref
    assert rel_l2(mua.grad.cpu().numpy(), gmua_ref) < 1e-4
    assert rel_l2(mus.grad.cpu().numpy(), gmus_ref) < 1e-4


def test_gradient_against_gpu_finite_differences():
    """Central differences of the GPU loss at voxels near the source, step
    1e-2 relative (large enough for fp32 solves)."""
    import torch
    p = _problem(steps=40)
    target = _target(p)
    gmua, gmus, _ = _gpu_grad(p, target, 10)

    def loss(pp):
        with torch.cuda.stream(torch.cuda.Stream()):
            m = T.Medium.from_problem(pp)
            m.solve(pp.steps)
            y = m.read_detectors()
            m.close()
        return float(np.sum((y - target) ** 2))
    vox = np.argsort(-np.abs(gmua.ravel()))[:5]
    for which, g in (("mua", gmua), ("mus", gmus)):
        for v in vox:
            base = getattr(p, which)
            h = 1e-2 * float(base.flat[v])
            vals = []
            for sgn in (1, -1):
                arr = base.copy()
                arr.flat[v] += np.float32(sgn * h)
                dh = float(arr.flat[v]) - float(base.flat[v])
                vals.append((loss(p.copy(**{which: arr})), dh))
            fd = (vals[0][0] - vals[1][0]) / (vals[0][1] - vals[1][1])
            assert abs(fd - g.flat[v]) <= 2e-3 * abs(g.flat[v]) + 1e-6 * np.abs(g).max(), (which, v)


def test_adjoint_full_size_directional_derivatives():
    """The 64^3 / 192-direction / 500-step adjoint medium with checkpoints every
    50 steps: for a fixed linear read-out L = sum w * y of the binned detector
    signals, the adjoint gradient's directional derivatives along a global
    scaling and a block pattern of mu_a and mu_s match central differences of
    GPU solves (step 1 %, where fp32 rounding of the solves is negligible)."""
    import torch
    p = W.config5()
    rng = np.random.default_rng(7)
    with torch.cuda.stream(torch.cuda.Stream()):
        m = T.Medium.from_problem(p)
        m.solve_checkpointed(p.steps, 50)
        y = m.read_detectors()
        w = rng.uniform(0.5, 1.5, y.shape) / np.maximum(y.max(axis=1, keepdims=True), 1e-300)
        gmua, gmus = m.backward(w)
        m.close()

        def lin(pp):
            mm = T.Medium.from_problem(pp)
            mm.solve(pp.steps)
            yy = mm.read_detectors()
            mm.close()
            return float(np.sum(w * yy))
        pat = np.kron(rng.choice([-1.0, 1.0], size=(8, 8, 8)), np.ones((8, 8, 8)))
        for which, g in (("mua", gmua), ("mus", gmus)):
            base = getattr(p, which).astype(np.float64)
            for dirn in (base, base * pat):
                plus = (base + 1e-2 * dirn).astype(np.float32)
                minus = (base - 1e-2 * dirn).astype(np.float32)
                fd = lin(p.copy(**{which: plus})) - lin(p.copy(**{which: minus}))
                pred = float(np.sum(g.astype(np.float64) * (plus.astype(np.float64) - minus)))
                assert abs(fd - pred) <= 2e-3 * abs(pred), (which, fd, pred)
