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
stage's checkpointed input.  ``rk3_gradient_recompute`` gives the same gradient keeping no
stage inputs (each is recomputed from the initial state), for programs whose checkpoints
would not fit.

An optional fixed lattice of straight segments (blade rings, frozen wake lines: a, b, strength,
core radius, Vatistas exponent) acts on the particles in every stage: its velocity and its
share of the stretching join F (``vpm_eval_segments_gradient``), its velocity adds at the
control points, and the backward pass adds the segments' vector-Jacobian product
(``vpm_segments_backward``).  The lattice itself is not differentiated.

All arithmetic runs in libvpm kernels; this module only orders the calls and allocates
tensors.
"""
import torch

from . import (SIGMA_SOURCE, vpm_axial_loss, vpm_backward, vpm_convert, vpm_eval_segments,
               vpm_eval_segments_gradient, vpm_eval_velocity_stretching, vpm_rk3_stage, vpm_rk3_stage_backward,
               vpm_segments_backward)


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


def rk3_forward(x0, gamma0, sigma, n_steps, dt, y_ctrl, checkpoints=None, segments=None):
    """Run the program.  The state (x0, gamma0) may be float64 while sigma and y_ctrl are
    float32: then the RK3 registers stay in FP64 and each evaluation reads an FP32 copy of the
    state (mixed program).  Optionally appends each stage's evaluation input to
    ``checkpoints``.  Returns (x, gamma, u_ctrl, loss, (x_eval, gamma_eval)) with loss a
    float64 0-d tensor."""
    edt = sigma.dtype
    mixed = x0.dtype != edt
    x, g = x0.clone(), gamma0.clone()
    qx, qg = torch.zeros_like(x), torch.zeros_like(x)
    if mixed:
        xe, ge = torch.empty(x.shape, dtype=edt, device=x.device), torch.empty(x.shape, dtype=edt, device=x.device)
        vpm_convert(x, xe)
        vpm_convert(g, ge)
    else:
        xe, ge = x, g
    u, dg = torch.empty_like(xe), torch.empty_like(xe)
    for _ in range(n_steps):
        for k in range(3):
            if checkpoints is not None:
                checkpoints.append((xe.clone(), ge.clone()))
            vpm_eval_velocity_stretching(xe, ge, sigma, u_out=u, dgamma_out=dg)
            if segments is not None:
                sa, sb, sg, rc, vn = segments
                vpm_eval_segments_gradient(sa, sb, sg, xe, rc, vn, gamma_tgt=ge, want_grad=False, u_out=u,
                                           dgamma_out=dg, accumulate=True)
            if mixed:
                vpm_rk3_stage(k, dt, x, g, qx, qg, u, dg, x_eval=xe, gamma_eval=ge)
            else:
                vpm_rk3_stage(k, dt, x, g, qx, qg, u, dg)
    uc, _ = vpm_eval_velocity_stretching(xe, ge, sigma, y_ctrl)
    if segments is not None:
        sa, sb, sg, rc, vn = segments
        vpm_eval_segments(sa, sb, sg, y_ctrl, rc, vn, u_out=uc, accumulate=True)
    loss, _ = vpm_axial_loss(uc, want_seed=False)
    return x, g, uc, loss, (xe, ge)


def rk3_backward(checkpoints, final_eval, sigma, uc, y_ctrl, dt, state_dtype, loss_bar=None, segments=None):
    """Gradient of the loss with respect to the program's initial (x, gamma), in state_dtype.
    loss_bar: float64 CUDA scalar (None = 1)."""
    xe, ge = final_eval
    mixed = state_dtype != xe.dtype
    xb = torch.zeros(xe.shape, dtype=state_dtype, device=xe.device)
    gb = torch.zeros_like(xb)
    # FP32 gradient contributions are collected in (ix, ig) and added into the FP64 adjoint
    # state before each stage adjoint reads it.
    ix, ig = (torch.zeros_like(xe), torch.zeros_like(xe)) if mixed else (xb, gb)
    # seed on the control-point velocity: dL/du_c = 2 loss_bar u_z z
    _, ucb = vpm_axial_loss(uc, loss_bar=loss_bar)
    vpm_backward(xe, ge, sigma, ucb, None, y_ctrl, None, None, x_src_bar=ix, gamma_src_bar=ig)
    qxb, qgb = torch.zeros_like(xb), torch.zeros_like(xb)
    us, ds = torch.empty_like(xe), torch.empty_like(xe)

    def fold():
        if mixed:
            vpm_convert(ix, xb, accumulate=True)
            vpm_convert(ig, gb, accumulate=True)
            ix.zero_()
            ig.zero_()

    for i in reversed(range(len(checkpoints))):
        k = i % 3
        xk, gk = checkpoints[i]
        fold()
        vpm_rk3_stage_backward(k, dt, xb, gb, qxb, qgb, us, ds)
        vpm_backward(xk, gk, sigma, us, ds, x_src_bar=ix, gamma_src_bar=ig)
        if segments is not None:
            sa, sb, sg, rc, vn = segments
            vpm_segments_backward(sa, sb, sg, xk, rc, vn, us, ds, gamma_tgt=gk, x_bar=ix, gamma_bar=ig)
    fold()
    return xb, gb


def rk3_gradient_recompute(x0, gamma0, sigma, n_steps, dt, y_ctrl, segments=None):
    """Gradient of the program's loss with respect to (x0, gamma0) keeping no stage inputs:
    the backward pass re-runs the forward program from the initial state up to each stage it
    needs (quadratic in the number of stages, memory of one state).  Returns (loss, x_bar,
    gamma_bar); the same calls in the same order as with checkpoints, so the same bits."""
    n_stages = 3 * int(n_steps)
    x, g, uc, loss, final_eval = rk3_forward(x0, gamma0, sigma, n_steps, dt, y_ctrl, None, segments)
    del x, g
    xe, ge = final_eval
    state_dtype = x0.dtype
    mixed = state_dtype != xe.dtype
    xb = torch.zeros(xe.shape, dtype=state_dtype, device=xe.device)
    gb = torch.zeros_like(xb)
    ix, ig = (torch.zeros_like(xe), torch.zeros_like(xe)) if mixed else (xb, gb)
    _, ucb = vpm_axial_loss(uc, loss_bar=None)
    vpm_backward(xe, ge, sigma, ucb, None, y_ctrl, None, None, x_src_bar=ix, gamma_src_bar=ig)
    qxb, qgb = torch.zeros_like(xb), torch.zeros_like(xb)
    us, ds = torch.empty_like(xe), torch.empty_like(xe)

    def fold():
        if mixed:
            vpm_convert(ix, xb, accumulate=True)
            vpm_convert(ig, gb, accumulate=True)
            ix.zero_()
            ig.zero_()

    for i in reversed(range(n_stages)):
        # the input of stage i: re-run the program's first i stages
        xk, gk = _stage_input(x0, gamma0, sigma, dt, i, segments)
        fold()
        vpm_rk3_stage_backward(i % 3, dt, xb, gb, qxb, qgb, us, ds)
        vpm_backward(xk, gk, sigma, us, ds, x_src_bar=ix, gamma_src_bar=ig)
        if segments is not None:
            sa, sb, sg, rc, vn = segments
            vpm_segments_backward(sa, sb, sg, xk, rc, vn, us, ds, gamma_tgt=gk, x_bar=ix, gamma_bar=ig)
        del xk, gk
    fold()
    return loss, xb, gb


def _stage_input(x0, gamma0, sigma, dt, i, segments):
    """The evaluation input of stage i (0-based) of the program, by re-running stages 0..i-1."""
    edt = sigma.dtype
    mixed = x0.dtype != edt
    x, g = x0.clone(), gamma0.clone()
    qx, qg = torch.zeros_like(x), torch.zeros_like(x)
    if mixed:
        xe, ge = torch.empty(x.shape, dtype=edt, device=x.device), torch.empty(x.shape, dtype=edt, device=x.device)
        vpm_convert(x, xe)
        vpm_convert(g, ge)
    else:
        xe, ge = x, g
    u, dg = torch.empty_like(xe), torch.empty_like(xe)
    for k in range(i):  # as in rk3_forward
        vpm_eval_velocity_stretching(xe, ge, sigma, u_out=u, dgamma_out=dg)
        if segments is not None:
            sa, sb, sg, rc, vn = segments
            vpm_eval_segments_gradient(sa, sb, sg, xe, rc, vn, gamma_tgt=ge, want_grad=False, u_out=u,
                                       dgamma_out=dg, accumulate=True)
        if mixed:
            vpm_rk3_stage(k % 3, dt, x, g, qx, qg, u, dg, x_eval=xe, gamma_eval=ge)
        else:
            vpm_rk3_stage(k % 3, dt, x, g, qx, qg, u, dg)
    return xe.clone(), ge.clone()


class RK3Program(torch.autograd.Function):
    """loss = program(x0, gamma0) with stage checkpoints kept in device memory."""

    @staticmethod
    def forward(ctx, x0, gamma0, sigma, n_steps, dt, y_ctrl, segments=None):
        ckpt = []
        _, _, uc, loss, final_eval = rk3_forward(x0.contiguous(), gamma0.contiguous(), sigma.contiguous(),
                                                 int(n_steps), float(dt), y_ctrl.contiguous(), ckpt, segments)
        ctx.segments = segments
        ctx.ckpt = ckpt
        ctx.final_eval = final_eval
        ctx.dt = float(dt)
        ctx.state_dtype = x0.dtype
        ctx.save_for_backward(sigma, uc, y_ctrl)
        return loss

    @staticmethod
    def backward(ctx, loss_bar):
        sigma, uc, y_ctrl = ctx.saved_tensors
        lb = loss_bar.detach().to(torch.float64).reshape(()).contiguous()
        xb, gb = rk3_backward(ctx.ckpt, ctx.final_eval, sigma, uc, y_ctrl.contiguous(), ctx.dt, ctx.state_dtype,
                              lb, ctx.segments)
        ctx.ckpt = None
        ctx.final_eval = None
        ctx.segments = None
        return xb, gb, None, None, None, None, None


def rk3_program_loss(x0, gamma0, sigma, n_steps, dt, y_ctrl, segments=None):
    """Differentiable loss of the RK3 wake program (see RK3Program).  float64 (x0, gamma0)
    with float32 (sigma, y_ctrl) runs the mixed program.  ``segments`` = (a, b, strength,
    core_radius, vatistas_n), device arrays in sigma's dtype: a fixed lattice acting on the
    particles."""
    if segments is not None:
        sa, sb, sg, rc, vn = segments
        segments = (sa.contiguous(), sb.contiguous(), sg.contiguous(), float(rc), int(vn))
    return RK3Program.apply(x0, gamma0, sigma, n_steps, dt, y_ctrl, segments)
