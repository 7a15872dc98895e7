"""Poisson negative log-likelihood of the ptychographic forward model as a
``torch.autograd.Function`` over the HIP adjoint (``pty_nll_forward`` /
``pty_nll_backward``).

L = sum_j sum_q [I_jq - d_jq log(I_jq + 1e-6)],  I_j = sum_k |F(P_k S_j O)|^2,
for the counts d and positions loaded into the :class:`~.plan.Plan`.  The
forward call stores no exit waves; the backward call recomputes them
(checkpointing).  Gradients follow PyTorch's convention for complex tensors.
"""
from __future__ import annotations

import torch


class NLL(torch.autograd.Function):
    """loss = NLL.apply(obj, probe, positions, plan).

    obj: (H, W) complex64 CUDA tensor; probe: (K, N, N) complex64 CUDA tensor;
    positions: (J, 2) float tensor of top-left corners, handed to the library
    as a float32 device tensor (no host round trip when it already is one);
    plan: a Plan with the counts loaded.  Returns a float64 scalar tensor on
    obj's device.
    """

    @staticmethod
    def forward(ctx, obj, probe, positions, plan):
        pos = positions.detach().to(device=obj.device, dtype=torch.float32).contiguous()
        obj_c = obj.detach().contiguous()
        probe_c = probe.detach().contiguous()
        loss = plan.nll_forward(obj_c, probe_c, pos)
        ctx.save_for_backward(obj_c, probe_c, pos)
        ctx.plan = plan
        ctx.pos_dtype = positions.dtype
        ctx.pos_device = positions.device
        return torch.tensor(loss, dtype=torch.float64, device=obj.device)

    @staticmethod
    def backward(ctx, grad_out):
        obj, probe, pos = ctx.saved_tensors
        plan = ctx.plan
        need_o, need_p, need_r = ctx.needs_input_grad[0], ctx.needs_input_grad[1], ctx.needs_input_grad[2]
        g_obj = torch.empty_like(obj) if need_o else None
        g_probe = torch.empty_like(probe) if need_p else None
        g_pos = torch.empty((plan.n_pos, 2), dtype=torch.float32, device=obj.device) if need_r else None
        plan.nll_backward(obj, probe, float(grad_out), g_obj, g_probe, g_pos, positions=pos)
        if g_pos is not None:
            g_pos = g_pos.to(device=ctx.pos_device, dtype=ctx.pos_dtype)
        return g_obj, g_probe, g_pos, None


def nll(obj, probe, positions, plan):
    return NLL.apply(obj, probe, positions, plan)
