"""Gradients of a phase-field run through the library's discrete adjoint.

run_phase_field(phi0, sigma, M, W, params, u0, nsteps) returns phi after
nsteps time steps as a differentiable function of the initial phase field and
of sigma, M and W (0-d float64 tensors). The forward pass keeps a native
checkpoint every k = ceil(sqrt(nsteps)) steps; the backward pass walks the
segments in reverse, recomputes each segment's k states from its checkpoint
(with the float64 and float32 forms the recomputing step writes the state it
starts from, so no separate read-out runs) and applies the adjoint step
kernel to each, so memory is O(sqrt(nsteps)) states. Every forward and adjoint step runs in libpflbm's kernels; this module
only schedules them.
"""
import math

import torch

from .solver import Solver


class PhaseFieldRun(torch.autograd.Function):
    @staticmethod
    def forward(ctx, phi0, sigma, M, W, params, u0, nsteps, precision, k, adjoint):
        d = dict(params)
        d["sigma"], d["M"], d["W"] = float(sigma), float(M), float(W)
        if d.get("model", "AC") not in ("AC", "CH", "NL", "L18", "L14"):
            raise ValueError("unknown phase-field model %r" % d.get("model"))
        if adjoint not in ("fp64", "fp32"):
            raise ValueError("adjoint precision must be 'fp64' or 'fp32', not %r" % (adjoint,))
        if adjoint == "fp32" and d.get("model", "AC") not in ("AC", "CH"):
            raise ValueError("the float32 adjoint covers the AC and CH models")
        if adjoint == "fp32" and d.get("model", "AC") == "CH" and precision not in ("fp64", "fp32"):
            raise ValueError("the float32 CH adjoint needs a float64 or float32 forward pass")
        s = Solver(d, precision=precision, device=phi0.device)
        s.init(phi0, u0)
        nsteps = int(nsteps)
        if k is None or k <= 0:
            k = max(1, int(math.ceil(math.sqrt(max(nsteps, 1)))))
        cks = []
        start = 0
        while start < nsteps:
            cks.append((start, s.save_state()))
            n = min(k, nsteps - start)
            s.step(n)
            start += n
        phiN, _, _, _ = s.fields()
        ctx.solver = s
        ctx.cks = cks
        ctx.k = k
        ctx.nsteps = nsteps
        ctx.u0 = u0
        ctx.adjoint = adjoint
        ctx.save_for_backward(phi0)
        return phiN.to(phi0.dtype)

    @staticmethod
    def backward(ctx, grad_phi):
        s = ctx.solver
        (phi0,) = ctx.saved_tensors
        if ctx.adjoint == "fp32":
            return PhaseFieldRun._backward_f32(ctx, s, phi0, grad_phi)
        dev = s.device
        shape = s.shape
        # the CH and Liang states also hold (phi u) of the previous step; L
        # depends on phi alone, so its adjoint starts at zero
        ch = s.d.get("model", "AC") in ("CH", "L18", "L14")
        lam_pu = torch.zeros((3,) + shape, dtype=torch.float64, device=dev) if ch else None
        out_pu = torch.empty_like(lam_pu) if ch else None
        dparams = torch.zeros(3, dtype=torch.float64, device=dev)
        work = s.adjoint_workspace()
        # the nonlocal model's phase field is a corrected sum h, so its seed
        # reads h of the final state, which the solver still holds
        h_final = s.get_distributions()[1] if s.d.get("model", "AC") == "NL" else None
        lam_g, lam_h = s.adjoint_seed(h_final, grad_phi.to(device=dev, dtype=torch.float64).reshape(shape),
                                      dparams, work)
        del h_final
        out_g = torch.empty_like(lam_g)
        out_h = torch.empty_like(lam_h)
        record = s.precision in ("fp64", "fp32")
        for start, buf in reversed(ctx.cks):
            n = min(ctx.k, ctx.nsteps - start)
            s.load_state(buf)
            states = []
            for _ in range(n):
                if record:
                    states.append(s.step_record())
                else:
                    g, h = s.get_distributions()
                    states.append((g, h, s.get_phiu() if ch else None))
                    s.step(1)
            for g, h, pu in reversed(states):
                if ch:
                    s.adjoint_step_pu(g, h, pu, lam_g, lam_h, lam_pu, out_g, out_h, out_pu, dparams, work)
                    lam_pu, out_pu = out_pu, lam_pu
                else:
                    s.adjoint_step(g, h, lam_g, lam_h, out_g, out_h, dparams, work)
                lam_g, out_g = out_g, lam_g
                lam_h, out_h = out_h, lam_h
            del states
        if ch:
            dphi0 = s.adjoint_init_pu(phi0, ctx.u0, None, lam_g, lam_h, lam_pu, dparams, work)
        else:
            dphi0 = s.adjoint_init(phi0, ctx.u0, None, lam_g, lam_h)
        return (dphi0.to(phi0.dtype).reshape(phi0.shape), dparams[0], dparams[1], dparams[2],
                None, None, None, None, None, None)

    @staticmethod
    def _backward_f32(ctx, s, phi0, grad_phi):
        """The same schedule with the float32 adjoint (AC and CH): states in
        float32, lambda float32, parameter sums float64."""
        dev = s.device
        ch = s.d.get("model", "AC") == "CH"
        dparams = torch.zeros(3, dtype=torch.float64, device=dev)
        work = s.adjoint_workspace()
        lam_g, lam_h = s.adjoint_seed_phi_f32(grad_phi.to(device=dev).reshape(s.shape))
        lam_pu = torch.zeros((3,) + s.shape, dtype=torch.float32, device=dev) if ch else None
        out_pu = torch.empty_like(lam_pu) if ch else None
        out_g = torch.empty_like(lam_g)
        out_h = torch.empty_like(lam_h)
        record = s.precision in ("fp64", "fp32")
        if ch and not record:
            raise ValueError("the float32 CH adjoint needs a float64 or float32 forward pass")
        for start, buf in reversed(ctx.cks):
            n = min(ctx.k, ctx.nsteps - start)
            s.load_state(buf)
            states = []
            for _ in range(n):
                if record:
                    states.append(s.step_record(f32=True))
                else:
                    states.append(s.get_distributions_f32() + (None,))
                    s.step(1)
            for g, h, pu in reversed(states):
                if ch:
                    s.adjoint_step_pu_f32(g, h, pu, lam_g, lam_h, lam_pu, out_g, out_h, out_pu, dparams, work)
                    lam_pu, out_pu = out_pu, lam_pu
                else:
                    s.adjoint_step_f32(g, h, lam_g, lam_h, out_g, out_h, dparams, work)
                lam_g, out_g = out_g, lam_g
                lam_h, out_h = out_h, lam_h
            del states
        if ch:
            dphi0 = s.adjoint_init_pu_f32(phi0, ctx.u0, None, lam_g, lam_h, lam_pu, dparams, work)
        else:
            dphi0 = s.adjoint_init_f32(phi0, ctx.u0, None, lam_g, lam_h)
        return (dphi0.to(phi0.dtype).reshape(phi0.shape), dparams[0], dparams[1], dparams[2],
                None, None, None, None, None, None)


def run_phase_field(phi0, sigma, M, W, params, u0=None, nsteps=1, precision="fp64", k=None, adjoint="fp64"):
    """phi after nsteps steps; differentiable in phi0, sigma, M, W. adjoint
    picks the arithmetic of the backward pass: "fp64", or "fp32" (AC and CH
    models: half the bytes per adjoint step, float32 rounding in the
    gradient)."""
    return PhaseFieldRun.apply(phi0, sigma, M, W, params, u0, nsteps, precision, k, adjoint)
