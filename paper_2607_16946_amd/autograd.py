"""PyTorch autograd over the C ABI: phi(x) differentiable in the queries, the
coefficients, the points and the normals (Sec. 6).

Forward runs pts_eval with statistics; backward runs pts_grad_x (queries) and
pts_backward_params (coefficients only) or pts_backward_points (any of
coefficients, points, normals), all hand-written HIP sweeps.  PyTorch is used
for tensors, streams and the autograd graph only.
"""

from __future__ import annotations

import torch

from . import binding


class _SDFFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x: torch.Tensor, a: torch.Tensor, p: torch.Tensor, n: torch.Tensor, cloud: binding.Cloud):
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
        gx = ga = gp = gn = None
        if ctx.needs_input_grad[0]:
            gx = binding.grad_x(cl.rec, cl.N, x, stats, gout, cl.params)
        want = "".join(c for c, need in zip("apn", ctx.needs_input_grad[1:4]) if need)
        if want == "a":
            ga = binding.backward_params(cl.rec, cl.p, cl.n, cl.a, x, stats, gout, cl.params)
        elif want:
            ga, gp, gn = binding.backward_points(cl.rec, cl.p, cl.n, cl.a, x, stats, gout, cl.params, want=want)
        return gx, ga, gp, gn, None


def sdf(x: torch.Tensor, cloud: binding.Cloud) -> torch.Tensor:
    """phi at x [Q,3]; gradients flow to x and to cloud.a, cloud.p, cloud.n (those that require grad)."""
    return _SDFFn.apply(x, cloud.a, cloud.p, cloud.n, cloud)


class TorusSDF(torch.nn.Module):
    """A point cloud as a differentiable signed distance field (Algorithm 1).

    The coefficients a (N x 6, order a00, a01, a10, a11, a02, a20) are a
    Parameter; the points p and normals n are Parameters too when
    learn_points / learn_normals is set, else fixed buffers.  The tori are
    refitted on the device whenever any of them has changed since the last
    forward.
    """

    def __init__(self, p: torch.Tensor, n: torch.Tensor, a: torch.Tensor, C: float = 64.0,
                 kfloor_rel: float = 1e-6, learn_points: bool = False, learn_normals: bool = False):
        super().__init__()
        p = p.detach().clone().contiguous()
        n = n.detach().clone().contiguous()
        if learn_points:
            self.p = torch.nn.Parameter(p)
        else:
            self.register_buffer("p", p)
        if learn_normals:
            self.n = torch.nn.Parameter(n)
        else:
            self.register_buffer("n", n)
        self.a = torch.nn.Parameter(a.detach().clone().contiguous())
        self.C, self.kfloor_rel = C, kfloor_rel
        self._cloud = None
        self._version = None

    def cloud(self) -> binding.Cloud:
        v = (self.a._version, self.p._version, self.n._version)
        if self._cloud is None or self._version != v:
            self._cloud = binding.Cloud(self.p.detach(), self.n.detach(), self.a.detach(), self.C, self.kfloor_rel)
            self._version = v
        return self._cloud

    def forward(self, x: torch.Tensor) -> torch.Tensor:
        cl = self.cloud()
        return _SDFFn.apply(x, self.a, self.p, self.n, cl)
