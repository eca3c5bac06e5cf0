"""torch.autograd.Function around the library's forward solve and adjoint.

detector_signals(mua, mus, prob) returns the binned detector signals of the
forward solve as a tensor; backpropagating through it runs the library's
hand-written adjoint (tr_backward), which differentiates the solve with
respect to the per-voxel absorption and scattering coefficients.  Both
directions run in the library's HIP kernels."""
import numpy as np
import torch

from . import trinity as T


class TrinityFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, mua, mus, prob, ckpt_every):
        dev = mua.device
        n = torch.as_tensor(np.ascontiguousarray(prob.n, np.float32)).to(dev)
        m = T.Medium(T.grid_desc(prob), mua.detach().float().contiguous(),
                     mus.detach().float().contiguous(), n)
        m.set_source(prob.src_ix, prob.src_iy, prob.src_w, prob.src_cone_deg, prob.t0_ps,
                     prob.fwhm_ps, prob.total_photons)
        m.set_detectors(prob.det_face, prob.det_i, prob.det_j, prob.det_cone_deg, prob.bin_ps,
                        prob.nbins)
        m.solve_checkpointed(prob.steps, ckpt_every)
        ctx.medium = m
        ctx.shape = mua.shape
        return torch.from_numpy(m.read_detectors()).to(dev)

    @staticmethod
    def backward(ctx, grad):
        m = ctx.medium
        dmua, dmus = m.backward(grad.detach().double().cpu().numpy())
        m.close()
        ctx.medium = None
        dev = grad.device
        return (torch.from_numpy(dmua).to(dev).view(ctx.shape),
                torch.from_numpy(dmus).to(dev).view(ctx.shape), None, None)


def detector_signals(mua, mus, prob, ckpt_every=50):
    """Binned detector signals [ndet, nbins] (float64) of the solve of `prob`
    with the given mu_a, mu_s tensors (float32, shape [nz, ny, nx], on the GPU)."""
    return TrinityFn.apply(mua, mus, prob, ckpt_every)
