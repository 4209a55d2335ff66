"""torch.autograd bindings of the library's reverse mode (argument marshalling
only: the forward and reverse passes run in libscfft).

Both functions need a context with a fixed exterior iteration count
(fixed_iter > 0), which makes the discrete map smooth.

    RhsEval.apply(h, sim, t_s)                       -> hdot
    Integrate.apply(h0, sim, t0_s, t1_s, steps, every) -> h(t1)
    IntegrateParams.apply(h0, kappa, n_power, p, sim, t0_s, t1_s, steps, every) -> h(t1)

RhsEval clears the warm start before every call, so each call starts the
exterior iteration from Ohm's law and is a pure function of h.  Integrate
runs the fixed-step mode of the integrator from a cleared warm start; its
backward runs the checkpointed adjoint (scfft_integrate_adjoint), which
repeats the forward pass to lay down checkpoints every `every` steps.
"""
import math

import torch

from . import scfft

MU0 = 4e-7 * math.pi


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


def drive_vector(sim):
    """The dimensionless applied-field vector p of the context's drive
    (h_e(t) = p f(t), Eq. 8 units): direction times amplitude / (mu0 jc l)."""
    d = sim.cfg["drive"]
    dv = torch.tensor(d["direction"], dtype=torch.float64)
    dv = dv / torch.linalg.norm(dv)
    return dv * (d["amp_T"] / (MU0 * sim.h_scale))


def _set_drive_vector(sim, p):
    d = dict(sim.cfg["drive"])
    kind = d.pop("kind")
    a = float(torch.linalg.norm(p))
    d["direction"] = tuple(float(v) / a for v in p) if a > 0 else (0.0, 0.0, 1.0)
    d["amp_T"] = a * MU0 * sim.h_scale
    sim.drive = scfft.make_drive(kind, **d)
    scfft.scfft_set_drive(sim.ctx, sim.drive)


class IntegrateParams(torch.autograd.Function):
    """h(t1) of the fixed-step integration as a function of the initial state
    h0, the critical-density map kappa = jc(x)/jc (Eq. 1 with a local jc), the
    power n and the applied-field vector p (any drive h_e = p f(t)); one
    checkpointed adjoint run gives all four gradients.  The gradient in a
    global jc at fixed units is that of a uniform scaling of kappa,
    sum(kappa_bar * kappa) / jc; the gradient in a field angle follows from
    p_bar by the chain rule.  kappa (context precision, [Nz][Ny][Nx]) and p
    are set on the context; n must equal the context's power (the material
    is fixed when the context is created)."""

    @staticmethod
    def forward(ctx, h0, kappa, n_power, p, sim, t0_s, t1_s, steps, every):
        if abs(float(n_power) - float(sim.cfg["n_power"])) > 1e-12 * abs(float(sim.cfg["n_power"])):
            raise ValueError("n_power must equal the context's power (create a context per n)")
        scfft.scfft_set_jc_map(sim.ctx, kappa.detach().to(sim.dtype).contiguous())
        _set_drive_vector(sim, p.detach().double().cpu())
        h0 = h0.contiguous()
        hT = h0.detach().clone()
        scfft.scfft_reset_warm(sim.ctx)
        scfft.scfft_integrate(sim.ctx, t0_s, t1_s, hT, scfft.default_ode_opts(fixed_steps=steps))
        ctx.sim = sim
        ctx.args = (t0_s, t1_s, steps, every)
        ctx.save_for_backward(h0, kappa, p)
        return hT

    @staticmethod
    def backward(ctx, g):
        h0, kappa, p = ctx.saved_tensors
        sim = ctx.sim
        t0_s, t1_s, steps, every = ctx.args
        scfft.scfft_set_jc_map(sim.ctx, kappa.detach().to(sim.dtype).contiguous())
        _set_drive_vector(sim, p.detach().double().cpu())
        ws = adjoint_workspace(sim, steps, every)
        h0_bar = sim.empty_field()
        hT = sim.empty_field()
        kbar = torch.zeros(kappa.shape, dtype=sim.dtype, device="cuda")
        n_bar, p_bar = scfft.scfft_integrate_adjoint(sim.ctx, t0_s, t1_s, steps, every, ws, h0,
                                                     g.contiguous(), hT, h0_bar, kbar)
        return (h0_bar, kbar.to(kappa.dtype), torch.tensor(n_bar, dtype=torch.float64),
                torch.tensor(p_bar, dtype=p.dtype, device=p.device), None, None, None, None, None)
