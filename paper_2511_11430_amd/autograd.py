"""Differentiation of the particle sums and of multi-step wake programs.

``VPMFunction`` wraps one self evaluation (u, dGamma/dt) = F(x, Gamma) of Eqs. 2-5 as a
torch.autograd.Function whose backward is the hand-written adjoint kernel
(``vpm_backward``).  ``ControlPointVelocity`` does the same for the velocity at blade
control points (Sec. II.A collocation points).

``RK3Program`` differentiates a whole program: n_steps of the low-storage third-order
Runge-Kutta scheme of Sec. II.B on (x, Gamma), then the loss L = sum_c (u_c . z)^2 on
control points.  The forward pass keeps every stage's input state in device memory
(checkpoints: 3 n_steps states of 6 N values), so the backward pass replays the stages in
reverse without recomputing the trajectory: at each stage it applies the RK3 register
adjoint (``vpm_rk3_stage_backward``) and adds J_F^T seed with ``vpm_backward`` at the
stage's checkpointed input.

All arithmetic runs in libvpm kernels; this module only orders the calls and allocates
tensors.
"""
import torch

from . import (SIGMA_SOURCE, vpm_axial_loss, vpm_backward, vpm_eval_velocity_stretching, vpm_rk3_stage,
               vpm_rk3_stage_backward)


class VPMFunction(torch.autograd.Function):
    """(u, dgamma) = F(x, gamma; sigma), self evaluation, transposed scheme."""

    @staticmethod
    def forward(ctx, x, gamma, sigma, sigma_rule=SIGMA_SOURCE):
        x, gamma, sigma = x.contiguous(), gamma.contiguous(), sigma.contiguous()
        u, dg = vpm_eval_velocity_stretching(x, gamma, sigma, sigma_rule=sigma_rule)
        ctx.save_for_backward(x, gamma, sigma)
        ctx.sigma_rule = sigma_rule
        return u, dg

    @staticmethod
    def backward(ctx, u_bar, dg_bar):
        x, gamma, sigma = ctx.saved_tensors
        if u_bar is None:
            u_bar = torch.zeros_like(x)
        if dg_bar is None:
            dg_bar = torch.zeros_like(x)
        xb, gb, _, _ = vpm_backward(x, gamma, sigma, u_bar.contiguous(), dg_bar.contiguous(),
                                    sigma_rule=ctx.sigma_rule)
        return xb, gb, None, None


class ControlPointVelocity(torch.autograd.Function):
    """u_c = velocity induced by the particles at fixed points y (source-core rule)."""

    @staticmethod
    def forward(ctx, x, gamma, sigma, y):
        x, gamma, sigma, y = x.contiguous(), gamma.contiguous(), sigma.contiguous(), y.contiguous()
        u, _ = vpm_eval_velocity_stretching(x, gamma, sigma, y)
        ctx.save_for_backward(x, gamma, sigma, y)
        return u

    @staticmethod
    def backward(ctx, u_bar):
        x, gamma, sigma, y = ctx.saved_tensors
        xb, gb, _, _ = vpm_backward(x, gamma, sigma, u_bar.contiguous(), None, y, None, None)
        return xb, gb, None, None


def rk3_forward(x0, gamma0, sigma, n_steps, dt, y_ctrl, checkpoints=None):
    """Run the program; optionally append each stage's input (x, gamma) to ``checkpoints``.
    Returns (x, gamma, u_ctrl, loss) with loss a 0-d tensor."""
    x, g = x0.clone(), gamma0.clone()
    qx, qg = torch.zeros_like(x), torch.zeros_like(x)
    u, dg = torch.empty_like(x), torch.empty_like(x)
    for _ in range(n_steps):
        for k in range(3):
            if checkpoints is not None:
                checkpoints.append((x.clone(), g.clone()))
            vpm_eval_velocity_stretching(x, g, sigma, u_out=u, dgamma_out=dg)
            vpm_rk3_stage(k, dt, x, g, qx, qg, u, dg)
    uc, _ = vpm_eval_velocity_stretching(x, g, sigma, y_ctrl)
    loss, _ = vpm_axial_loss(uc, want_seed=False)
    return x, g, uc, loss


def rk3_backward(checkpoints, x, g, sigma, uc, y_ctrl, dt, loss_bar=None):
    """Gradient of the loss with respect to the program's initial (x, gamma).  loss_bar:
    float64 CUDA scalar (None = 1)."""
    xb, gb = torch.zeros_like(x), torch.zeros_like(x)
    # seed on the control-point velocity: dL/du_c = 2 loss_bar u_z z
    _, ucb = vpm_axial_loss(uc, loss_bar=loss_bar)
    vpm_backward(x, g, sigma, ucb, None, y_ctrl, None, None, x_src_bar=xb, gamma_src_bar=gb)
    qxb, qgb = torch.zeros_like(x), torch.zeros_like(x)
    us, ds = torch.empty_like(x), torch.empty_like(x)
    n_stages = len(checkpoints)
    for i in reversed(range(n_stages)):
        k = i % 3
        xk, gk = checkpoints[i]
        vpm_rk3_stage_backward(k, dt, xb, gb, qxb, qgb, us, ds)
        vpm_backward(xk, gk, sigma, us, ds, x_src_bar=xb, gamma_src_bar=gb)
    return xb, gb


class RK3Program(torch.autograd.Function):
    """loss = program(x0, gamma0) with stage checkpoints kept in device memory."""

    @staticmethod
    def forward(ctx, x0, gamma0, sigma, n_steps, dt, y_ctrl):
        ckpt = []
        x, g, uc, loss = rk3_forward(x0.contiguous(), gamma0.contiguous(), sigma.contiguous(), int(n_steps),
                                     float(dt), y_ctrl.contiguous(), ckpt)
        ctx.ckpt = ckpt
        ctx.dt = float(dt)
        ctx.save_for_backward(x, g, sigma, uc, y_ctrl)
        return loss

    @staticmethod
    def backward(ctx, loss_bar):
        x, g, sigma, uc, y_ctrl = ctx.saved_tensors
        lb = loss_bar.detach().to(torch.float64).reshape(()).contiguous()
        xb, gb = rk3_backward(ctx.ckpt, x, g, sigma, uc, y_ctrl.contiguous(), ctx.dt, lb)
        ctx.ckpt = None
        return xb, gb, None, None, None, None


def rk3_program_loss(x0, gamma0, sigma, n_steps, dt, y_ctrl):
    """Differentiable loss of the RK3 wake program (see RK3Program)."""
    return RK3Program.apply(x0, gamma0, sigma, n_steps, dt, y_ctrl)
