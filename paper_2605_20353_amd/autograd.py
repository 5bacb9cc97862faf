"""The sampled GCP objective as a differentiable torch function.

F~(A) = sum_s w_s f(x_s, m_s(A)) over a sampled set of tensor entries (Sec.
3.1.1), with m_s = sum_r prod_k A_k[i_k(s), r] (eq. cp).  Its gradient is the
sampled MTTKRP of eq. gcp-gradient with y_s = w_s f'(x_s, m_s), so the
backward pass is one gcp_loss_grad call scaled by the incoming gradient.

Two ways to keep the samples between forward and backward:
  * recompute (default): the forward keeps only (seed, step, client); the
    backward draws the very same samples again inside the kernel (the RNG is
    counter-based) and recomputes every model value -- nothing per sample is
    stored, whatever the sample count;
  * materialised: the forward stores the sample list (coordinates, values,
    weights: 8d + 2w bytes per sample) and the backward reads it.
Both give the same gradient up to the order of floating-point additions.
"""
from __future__ import annotations

import torch

from . import _lib as G


class GCPLoss(torch.autograd.Function):
    """F~ = GCPLoss.apply(A, tensor, R, loss, sample_params, recompute, tile).

    A: the model as ONE contiguous [sum_k I_k, R] (or flat) device tensor of
    the tensor's dtype.  Returns a float64 scalar on A's device."""

    @staticmethod
    def forward(ctx, A, tensor, R, loss, sp, recompute=True, tile=None):
        A = A.contiguous()
        samples = None
        if not recompute:
            samples = G.gcp_sample(tensor, sp)
            _, L = G.gcp_loss_grad(tensor, sp, A, R, loss, loss_only=True, samples=samples, tile=tile)
        else:
            _, L = G.gcp_loss_grad(tensor, sp, A, R, loss, loss_only=True, tile=tile)
        ctx.save_for_backward(A)
        ctx.tensor, ctx.R, ctx.loss, ctx.sp, ctx.tile = tensor, R, loss, sp, tile
        ctx.samples = samples
        ctx.A_shape = A.shape
        return L.reshape(())

    @staticmethod
    def backward(ctx, grad_out):
        (A,) = ctx.saved_tensors
        scale = grad_out.detach().to(A.dtype).reshape(1).contiguous()
        Gr, _ = G.gcp_loss_grad(ctx.tensor, ctx.sp, A, ctx.R, ctx.loss, scale=scale, want_loss=False,
                                samples=ctx.samples, tile=ctx.tile)
        ctx.samples = None
        return Gr.reshape(ctx.A_shape), None, None, None, None, None, None


def gcp_loss(A: torch.Tensor, tensor, R: int, loss: str, sp: G.SampleParams, recompute: bool = True,
             tile: G.Tile | None = None) -> torch.Tensor:
    """Differentiable sampled GCP objective of the model A (see GCPLoss)."""
    return GCPLoss.apply(A, tensor, R, loss, sp, recompute, tile)


class KruskalModel(torch.nn.Module):
    """A Kruskal model stored as ONE contiguous parameter [sum_k I_k, R] with
    a [I_k, R] view per mode (the single factor array of Sec. 3.1.3)."""

    def __init__(self, dims, R: int, init: torch.Tensor | None = None, dtype=torch.float32, device="cuda"):
        super().__init__()
        self.dims = [int(n) for n in dims]
        self.R = int(R)
        if init is None:
            init = torch.zeros(sum(self.dims), R, dtype=dtype, device=device)
        self.A = torch.nn.Parameter(init.detach().to(device=device, dtype=dtype).reshape(sum(self.dims), R)
                                    .contiguous().clone())

    def factors(self):
        out, off = [], 0
        for n in self.dims:
            out.append(self.A[off:off + n])
            off += n
        return out

    def forward(self, tensor, loss: str, sp: G.SampleParams, recompute: bool = True, tile=None):
        return gcp_loss(self.A, tensor, self.R, loss, sp, recompute, tile)
