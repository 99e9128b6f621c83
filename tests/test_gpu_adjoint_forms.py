"""The checkpointed backward pass of every model over a forward pass in each
storage form: with the float64 and float32 forms the recomputing step records
the state, with the 16-bit forms each recomputed state is read out (and, for
the models with a (phi u) state, its (phi u)). The gradients are those of the
form's own trajectory; they must be finite and agree with the float64 run's
within what the form's storage rounding (2^-24, 2^-11, 2^-8 relative for
float32, fp16, bf16) makes of them: the M term weighs the non-equilibrium
h - h_eq, a small difference that magnifies the rounding of h and g by up to
about ten times over these 12 steps of the 2-D droplet in shear, so 1e-3,
1e-2 and 5e-2 relative are asserted."""
TOL = {"fp32": 1e-3, "mixed_fp16": 1e-2, "mixed_bf16": 5e-2}
import sys

import numpy as np
import pytest

from paper_2511_11360_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _case(model):
    d, phi, u = wl.static_droplet_2d(n=32, R=9.0)
    d.update(W=3.0, model=model, rho_H=3.0, visc_interp="mu", nu_L=d["nu_H"] * 1.5)
    if model in ("CH", "L14"):
        d.update(eta=1.0, M=0.04)
    if model == "NL":
        d["lam"] = 0.5
    phi = wl.droplet_phi(d, (16.0, 16.0), 9.0)
    x, y, z = wl.grid(d)
    u = wl.zero_velocity(d)
    u[0] = 0.01 * np.sin(2 * np.pi * (y + 0.5) / 32)
    return d, phi, u


def _grad(d, phi, u, steps, target, precision):
    import torch
    from paper_2511_11360_amd.autograd import run_phase_field
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")  # noqa: E731
    phi0 = dev(phi).requires_grad_(True)
    ps = [torch.tensor(d[k], dtype=torch.float64, requires_grad=True) for k in ("sigma", "M", "W")]
    phiN = run_phase_field(phi0, *ps, d, dev(u), steps, precision=precision)
    L = 0.5 * ((phiN - dev(target)) ** 2).sum()
    L.backward()
    return phi0.grad.cpu().numpy(), np.array([float(t.grad.detach().cpu()) for t in ps])


@pytest.mark.parametrize("precision", ["fp32", "mixed_fp16", "mixed_bf16"])
@pytest.mark.parametrize("model", ["AC", "CH", "NL", "L18", "L14"])
def test_backward_over_every_storage_form(model, precision):
    d, phi, u = _case(model)
    target = wl.droplet_phi(d, (16.5, 15.5), 9.4)
    g64, p64 = _grad(d, phi, u, 12, target, "fp64")
    g, p = _grad(d, phi, u, 12, target, precision)
    assert np.isfinite(g).all() and np.isfinite(p).all()
    rel = np.abs(p - p64) / np.abs(p64)
    eg = np.max(np.abs(g - g64)) / np.max(np.abs(g64))
    _say("  %s %s: params rel %s, dL/dphi0 %.2e" % (model, precision, np.array2string(rel, precision=2), eg))
    assert np.all(rel <= TOL[precision]) and eg <= TOL[precision]
