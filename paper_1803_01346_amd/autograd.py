"""torch.autograd bindings of the library's reverse mode (argument marshalling
only: the forward and reverse passes run in libscfft).

Both functions need a context with a fixed exterior iteration count
(fixed_iter > 0), which makes the discrete map smooth.

    RhsEval.apply(h, sim, t_s)                       -> hdot
    Integrate.apply(h0, sim, t0_s, t1_s, steps, every) -> h(t1)

RhsEval clears the warm start before every call, so each call starts the
exterior iteration from Ohm's law and is a pure function of h.  Integrate
runs the fixed-step mode of the integrator from a cleared warm start; its
backward runs the checkpointed adjoint (scfft_integrate_adjoint), which
repeats the forward pass to lay down checkpoints every `every` steps.
"""
import torch

from . import scfft


class RhsEval(torch.autograd.Function):
    @staticmethod
    def forward(ctx, h, sim, t_s):
        h = h.contiguous()
        scfft.scfft_reset_warm(sim.ctx)
        hdot, _ = sim.rhs_eval(t_s, h)
        ctx.sim = sim
        ctx.save_for_backward(h)
        return hdot

    @staticmethod
    def backward(ctx, g):
        (h,) = ctx.saved_tensors
        sim = ctx.sim
        hbar = sim.empty_field()
        scfft.scfft_rhs_vjp(sim.ctx, h, False, g.contiguous(), None, hbar)
        return hbar, None, None


def adjoint_workspace(sim, steps, every):
    """A device buffer for scfft_integrate_adjoint, 256-byte aligned."""
    nbytes = scfft.scfft_adjoint_workspace_size(sim.ctx, steps, every)
    raw = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
    off = (-raw.data_ptr()) % 256
    return raw[off:off + nbytes]


class Integrate(torch.autograd.Function):
    @staticmethod
    def forward(ctx, h0, sim, t0_s, t1_s, steps, every):
        h0 = h0.contiguous()
        hT = h0.detach().clone()
        scfft.scfft_reset_warm(sim.ctx)
        scfft.scfft_integrate(sim.ctx, t0_s, t1_s, hT, scfft.default_ode_opts(fixed_steps=steps))
        ctx.sim = sim
        ctx.args = (t0_s, t1_s, steps, every)
        ctx.save_for_backward(h0)
        return hT

    @staticmethod
    def backward(ctx, g):
        (h0,) = ctx.saved_tensors
        sim = ctx.sim
        t0_s, t1_s, steps, every = ctx.args
        ws = adjoint_workspace(sim, steps, every)
        h0_bar = sim.empty_field()
        scfft.scfft_integrate_adjoint(sim.ctx, t0_s, t1_s, steps, every, ws, h0, g.contiguous(), None,
                                      h0_bar, want_p_bar=False)
        return h0_bar, None, None, None, None, None
