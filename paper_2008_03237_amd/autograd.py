"""torch.autograd.Function over the C ABI residual and its adjoint kernels.

    R = DLPNOResidual.apply(T, B, plan)

forward runs dlpno_residual; backward runs dlpno_residual_vjp, which returns
dL/dT (the transpose of the residual's linear part applied to dL/dR) and
dL/dB^Q (general, unsymmetrised B; the B^Q T intermediates are recomputed in
the kernel, not stored).  B must be the device tensor the plan was created
with: the plan reads it in place.  Differentiating a Lagrangian
L = E(T) + <Lambda, R(T, B)> this way gives the Lambda-equation gradients.
"""
import torch


class DLPNOResidual(torch.autograd.Function):
    @staticmethod
    def forward(ctx, T, B, plan):
        if B.data_ptr() != plan._dev[0].data_ptr():
            raise ValueError("B must be the tensor the plan was created with")
        R = plan.residual(T.detach())
        ctx.save_for_backward(T.detach())
        ctx.plan = plan
        return R

    @staticmethod
    def backward(ctx, G):
        (T,) = ctx.saved_tensors
        want_dB = ctx.needs_input_grad[1]
        dT, dB = ctx.plan.vjp(T, G.contiguous(), want_dB=want_dB)
        return (dT if ctx.needs_input_grad[0] else None), (dB if want_dB else None), None


def residual(T, B, plan):
    return DLPNOResidual.apply(T, B, plan)
