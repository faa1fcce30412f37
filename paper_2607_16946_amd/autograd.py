"""PyTorch autograd over the C ABI: phi(x) differentiable in the queries and the coefficients.

Forward runs pts_eval with statistics; backward runs pts_grad_x (queries) and
pts_backward_params (coefficients), both hand-written HIP sweeps.  PyTorch is
used for tensors, streams and the autograd graph only.
"""

from __future__ import annotations

import torch

from . import binding


class _SDFFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x: torch.Tensor, a: torch.Tensor, cloud: binding.Cloud):
        x = x.contiguous()
        sdf, stats = binding.eval(cloud.rec, cloud.N, x, cloud.params, stats=True)
        ctx.save_for_backward(x, stats)
        ctx.cloud = cloud
        return sdf

    @staticmethod
    def backward(ctx, gout: torch.Tensor):
        x, stats = ctx.saved_tensors
        cl = ctx.cloud
        gout = gout.contiguous().to(torch.float32)
        gx = ga = None
        if ctx.needs_input_grad[0]:
            gx = binding.grad_x(cl.rec, cl.N, x, stats, gout, cl.params)
        if ctx.needs_input_grad[1]:
            ga = binding.backward_params(cl.rec, cl.p, cl.n, cl.a, x, stats, gout, cl.params)
        return gx, ga, None


def sdf(x: torch.Tensor, cloud: binding.Cloud) -> torch.Tensor:
    """phi at x [Q,3]; gradients flow to x and to cloud.a (if it requires grad)."""
    return _SDFFn.apply(x, cloud.a, cloud)


class TorusSDF(torch.nn.Module):
    """A point cloud as a differentiable signed distance field (Algorithm 1).

    p, n are fixed buffers; the coefficients a (N x 6, order a00, a01, a10,
    a11, a02, a20) are a Parameter.  The tori are refitted on the device
    whenever a has changed since the last forward.
    """

    def __init__(self, p: torch.Tensor, n: torch.Tensor, a: torch.Tensor, C: float = 64.0,
                 kfloor_rel: float = 1e-6):
        super().__init__()
        self.register_buffer("p", p.detach().contiguous())
        self.register_buffer("n", n.detach().contiguous())
        self.a = torch.nn.Parameter(a.detach().clone().contiguous())
        self.C, self.kfloor_rel = C, kfloor_rel
        self._cloud = None
        self._version = None

    def cloud(self) -> binding.Cloud:
        v = self.a._version
        if self._cloud is None or self._version != v:
            self._cloud = binding.Cloud(self.p, self.n, self.a.detach(), self.C, self.kfloor_rel)
            self._version = v
        return self._cloud

    def forward(self, x: torch.Tensor) -> torch.Tensor:
        cl = self.cloud()
        return _SDFFn.apply(x, self.a, cl)
