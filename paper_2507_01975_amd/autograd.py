"""torch.autograd.Function wrappers of the library's forward and adjoint calls.

Every forward and every backward runs in libldsv: the backward of each
Function is the hand-written vector-Jacobian product of the corresponding
entry point (App. B.2-B.5 discretisation, Eq. 2 recursion; the gradient of
the unrolled loss of Sec. 4.1), never torch's own differentiation of the
forward.  These classes only connect the calls to torch's autograd graph so
that the solver composes with other torch code:

    fv_step(solver, prm, u, v, coef=None)        one RK step, grads to u, v, coef
    project(solver, u, v)                        the pressure projection
    learned_step(solver, prm, net, u, v, k)      one learned step, grads to
                                                 u, v and net's parameters
    rollout(solver, prm, net, u0, v0, n, ...)    n learned steps with
                                                 checkpointing, grads to u0,
                                                 v0 and net's parameters
    fluxblock_step(solver, prm, fnet, u, v)      one step of the paper's
                                                 flux-block model (uniform
                                                 kernels + FNOs), grads to
                                                 u, v and every parameter
                                                 tensor of the FluxNetParams

The network parameters are the FP32 master tensors of a
``ldsv.NetParams`` (``net.master_w`` [Cout][3][3][Cin] and ``net.b``); give
them ``requires_grad`` to receive gradients.  The forward refreshes the bf16
copies from the masters, so parameters updated in place by an optimiser are
picked up.  Gradients of the learned calls assume that no guard fallback
happened (differentiate with ``fallback_enable = 0``).
"""
import torch

from . import ldsv


def _zeros_if_none(g, like):
    return torch.zeros_like(like) if g is None else g.contiguous()


class _FVStep(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u, v, coef, solver, prm):
        u, v = u.contiguous(), v.contiguous()
        c = coef.contiguous() if coef is not None else None
        uo, vo = solver.fv_step(prm, u, v, coef=c)
        ctx.solver, ctx.prm = solver, prm
        ctx.save_for_backward(u, v, c)
        ctx.has_coef = c is not None
        return uo, vo

    @staticmethod
    def backward(ctx, gu, gv):
        u, v, c = ctx.saved_tensors
        gu = _zeros_if_none(gu, u)
        gv = _zeros_if_none(gv, v)
        gc = torch.zeros_like(c) if (ctx.has_coef and ctx.needs_input_grad[2]) else None
        gui, gvi = ctx.solver.fv_step_bwd(ctx.prm, u, v, gu, gv, coef=c if ctx.has_coef else None,
                                          gcoef=gc)
        return gui, gvi, gc, None, None


class _Project(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u, v, solver):
        uo, vo = u.clone(memory_format=torch.contiguous_format), \
            v.clone(memory_format=torch.contiguous_format)
        solver.project(uo, vo)
        ctx.solver = solver
        return uo, vo

    @staticmethod
    def backward(ctx, gu, gv):
        # the projection is symmetric: its adjoint is itself
        gu = gu.clone(memory_format=torch.contiguous_format)
        gv = gv.clone(memory_format=torch.contiguous_format)
        ctx.solver.project(gu, gv)
        return gu, gv, None


def _net_params(net):
    return list(net.master_w) + list(net.b)


def _net_grads(dW):
    return list(dW.w) + list(dW.b)


class _LearnedStep(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u, v, solver, prm, net, step_index, *params):
        u, v = u.contiguous(), v.contiguous()
        net.refresh()
        uo, vo = solver.learned_fv_step(prm, net, u, v, step_index)
        ctx.solver, ctx.prm, ctx.net, ctx.k = solver, prm, net, step_index
        ctx.save_for_backward(u, v)
        return uo, vo

    @staticmethod
    def backward(ctx, gu, gv):
        u, v = ctx.saved_tensors
        gu = _zeros_if_none(gu, u)
        gv = _zeros_if_none(gv, v)
        dW = ldsv.NetGradBuffers(ctx.net)
        gui, gvi = ctx.solver.learned_fv_step_bwd(ctx.prm, ctx.net, u, v, ctx.k, gu, gv, dW)
        return (gui, gvi, None, None, None, None) + tuple(_net_grads(dW))


class _LearnedDStep(torch.autograd.Function):
    """The learned step with the derivative-stencil network beside the
    coefficient network; parameters: net's, then dnet's."""

    @staticmethod
    def forward(ctx, u, v, solver, prm, net, dnet, step_index, *params):
        u, v = u.contiguous(), v.contiguous()
        net.refresh()
        dnet.refresh()
        uo, vo = solver.learned_d_fv_step(prm, net, dnet, u, v, step_index)
        ctx.solver, ctx.prm, ctx.net, ctx.dnet, ctx.k = solver, prm, net, dnet, step_index
        ctx.save_for_backward(u, v)
        return uo, vo

    @staticmethod
    def backward(ctx, gu, gv):
        u, v = ctx.saved_tensors
        gu = _zeros_if_none(gu, u)
        gv = _zeros_if_none(gv, v)
        dW = ldsv.NetGradBuffers(ctx.net)
        dWd = ldsv.NetGradBuffers(ctx.dnet)
        gui, gvi = ctx.solver.learned_d_fv_step_bwd(ctx.prm, ctx.net, ctx.dnet, u, v, ctx.k, gu,
                                                    gv, dW, dWd)
        return (gui, gvi, None, None, None, None, None) + tuple(_net_grads(dW)) + \
            tuple(_net_grads(dWd))


class _Rollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u0, v0, solver, prm, net, nsteps, first_index, checkpoint_every, *params):
        u0, v0 = u0.contiguous(), v0.contiguous()
        net.refresh()
        tu, tv = solver.rollout(prm, u0, v0, nsteps, save_every=1, net=net,
                                first_index=first_index)
        ctx.solver, ctx.prm, ctx.net = solver, prm, net
        ctx.nsteps, ctx.first, ctx.ce = nsteps, first_index, checkpoint_every
        ctx.save_for_backward(u0, v0)
        return tu, tv

    @staticmethod
    def backward(ctx, gtu, gtv):
        u0, v0 = ctx.saved_tensors
        shape = (ctx.nsteps,) + tuple(u0.shape)
        gtu = torch.zeros(shape, dtype=u0.dtype, device=u0.device) if gtu is None \
            else gtu.contiguous()
        gtv = torch.zeros(shape, dtype=v0.dtype, device=v0.device) if gtv is None \
            else gtv.contiguous()
        dW = ldsv.NetGradBuffers(ctx.net)
        gu0, gv0 = ctx.solver.rollout_bwd(ctx.prm, ctx.net, u0, v0, ctx.nsteps, dW,
                                          checkpoint_every=ctx.ce, first_index=ctx.first,
                                          g_traj=(gtu, gtv), want_input_grad=True)
        return (gu0, gv0, None, None, None, None, None, None) + tuple(_net_grads(dW))


def _fluxblock_params(fnet):
    out = [fnet.stencil_w]
    for f in fnet.fno:
        if f is not None:
            out += [f.lift_w, f.lift_b, f.spec_w, f.point_w, f.point_b, f.proj_w, f.proj_b]
    return out


class _FluxBlockStep(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u, v, solver, prm, fnet, *params):
        u, v = u.contiguous(), v.contiguous()
        uo, vo = solver.fluxblock_step(prm, fnet, u, v)
        ctx.solver, ctx.prm, ctx.fnet = solver, prm, fnet
        ctx.save_for_backward(u, v)
        return uo, vo

    @staticmethod
    def backward(ctx, gu, gv):
        u, v = ctx.saved_tensors
        gu = _zeros_if_none(gu, u)
        gv = _zeros_if_none(gv, v)
        gb = ldsv.FluxNetGradBuffers(ctx.fnet)
        gui, gvi = ctx.solver.fluxblock_step_bwd(ctx.prm, ctx.fnet, u, v, gu, gv, gb)
        grads = [gb.stencil_w]
        for f in gb.fno:
            if f is not None:
                grads += f.tensors()
        return (gui, gvi, None, None, None) + tuple(grads)


def fluxblock_step(solver, prm, fnet, u, v):
    """One step of the flux-block model; differentiable in u, v and the
    FluxNetParams tensors (give them requires_grad)."""
    return _FluxBlockStep.apply(u, v, solver, prm, fnet, *_fluxblock_params(fnet))


def fv_step(solver, prm, u, v, coef=None):
    """One plain (or fixed-coefficient) FV time step; differentiable in u, v
    and coef."""
    return _FVStep.apply(u, v, coef, solver, prm)


def project(solver, u, v):
    """The pressure projection P(u, v); differentiable (P^T = P)."""
    return _Project.apply(u, v, solver)


def learned_step(solver, prm, net, u, v, step_index):
    """One learned step producing u_{step_index}; differentiable in u, v and
    the network's master parameters."""
    return _LearnedStep.apply(u, v, solver, prm, net, step_index, *_net_params(net))


def learned_d_step(solver, prm, net, dnet, u, v, step_index):
    """One learned step with per-cell learned derivative stencils (dnet beside
    net); differentiable in u, v and both networks' master parameters."""
    return _LearnedDStep.apply(u, v, solver, prm, net, dnet, step_index, *_net_params(net),
                               *_net_params(dnet))


def rollout(solver, prm, net, u0, v0, nsteps, first_index=1, checkpoint_every=8):
    """States u_{first_index} .. u_{first_index + nsteps - 1} ([T, B, Ny, Nx])
    of the learned recursion; the backward recomputes segments of
    checkpoint_every steps from stored checkpoints."""
    return _Rollout.apply(u0, v0, solver, prm, net, nsteps, first_index, checkpoint_every,
                          *_net_params(net))
