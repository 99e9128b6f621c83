"""The adjoint workload at its stated size: a 3-D droplet in simple shear,
D3Q19 + D3Q7, 128^3, walls normal to y moving at -+0.02 in x, periodic x
and z, R = 24, Ca = 0.2, 2000 steps with ceil(sqrt(2000)) = 45 native
checkpoints, loss L = 1/2 sum (phi_N - phi*)^2 against a seeded tanh-ellipsoid
target phi*.

- float64 forward pass: the adjoint's dL/d(sigma, M, W) and <dL/dphi0, v>
  (v a seeded direction on the interface) match central differences of the
  HIP float64 run within 1e-6 relative;
- float32 forward pass (the workload's stated precision): the same gradients
  from the float64 adjoint applied to the recomputed float32 states, against
  the float64 ones; their relative differences are printed and bounded;
- float32 forward and float32 adjoint: against the float64 adjoint of the
  same float32 states, within sqrt(2000) x 1.2e-5 = 5.4e-4 (float32 roundings
  of each adjoint step, n u = 1.2e-5, adding as independent errors), rounded
  up to 1e-3, and against the float64 run within the float32 forward bound.
"""
import sys

import numpy as np
import pytest

from paper_2511_11360_amd import workloads as wl

pytestmark = pytest.mark.gpu

STEPS = 2000


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _dev(a):
    import torch
    return torch.as_tensor(a, dtype=torch.float64, device="cuda")


def _grad(d, phi, u, target, v, precision, adjoint="fp64"):
    import torch
    from paper_2511_11360_amd.autograd import run_phase_field
    phi0 = _dev(phi).requires_grad_(True)
    sig = torch.tensor(d["sigma"], dtype=torch.float64, requires_grad=True)
    M = torch.tensor(d["M"], dtype=torch.float64, requires_grad=True)
    W = torch.tensor(d["W"], dtype=torch.float64, requires_grad=True)
    phiN = run_phase_field(phi0, sig, M, W, d, _dev(u), STEPS, precision=precision, adjoint=adjoint)
    L = 0.5 * ((phiN - _dev(target)) ** 2).sum()
    L.backward()
    gv = float((phi0.grad * _dev(v)).sum())
    return float(L), {"sigma": float(sig.grad), "M": float(M.grad), "W": float(W.grad), "phi0.v": gv}


def _loss(d, phi, u, target):
    from paper_2511_11360_amd.solver import Solver
    s = Solver(d, precision="fp64")
    s.init(phi, u)
    s.step(STEPS)
    ph = s.fields()[0]
    return float(0.5 * ((ph - _dev(target)) ** 2).sum())


def test_sheared_droplet_128_full_run_gradients():
    d, phi, u, target = wl.sheared_droplet_3d()
    assert (d["nx"], d["ny"], d["nz"]) == (128, 128, 128)
    v = wl.seeded_field(phi.shape, 41, -1.0, 1.0) * 4.0 * phi * (1.0 - phi)
    _say("case adjoint config 128^3, %d steps, float64 forward" % STEPS)
    L64, g64 = _grad(d, phi, u, target, v, "fp64")
    _say("  L %.12e" % L64)
    for name in ("sigma", "M", "W"):
        h = 1e-5 * d[name]
        fd = (_loss(dict(d, **{name: d[name] + h}), phi, u, target)
              - _loss(dict(d, **{name: d[name] - h}), phi, u, target)) / (2 * h)
        _say("  dL/d%s adjoint %.10e  central FD %.10e  rel %.2e"
             % (name, g64[name], fd, abs(g64[name] - fd) / abs(fd)))
        assert abs(g64[name] - fd) <= 1e-6 * abs(fd)
    eps = 1e-5
    fd = (_loss(d, phi + eps * v, u, target) - _loss(d, phi - eps * v, u, target)) / (2 * eps)
    _say("  <dL/dphi0, v> adjoint %.10e  central FD %.10e  rel %.2e"
         % (g64["phi0.v"], fd, abs(g64["phi0.v"] - fd) / abs(fd)))
    assert abs(g64["phi0.v"] - fd) <= 1e-6 * abs(fd)

    _say("case adjoint config 128^3, %d steps, float32 forward" % STEPS)
    L32, g32 = _grad(d, phi, u, target, v, "fp32")
    _say("  L float32 %.12e (float64 %.12e, rel %.2e)" % (L32, L64, abs(L32 - L64) / abs(L64)))
    for name in ("sigma", "M", "W", "phi0.v"):
        rel = abs(g32[name] - g64[name]) / abs(g64[name])
        _say("  dL/d%s float32 forward %.10e  float64 forward %.10e  rel %.2e"
             % (name, g32[name], g64[name], rel))
        assert rel < 1e-2

    _say("case adjoint config 128^3, %d steps, float32 forward, float32 adjoint" % STEPS)
    _, g3232 = _grad(d, phi, u, target, v, "fp32", adjoint="fp32")
    for name in ("sigma", "M", "W", "phi0.v"):
        rel = abs(g3232[name] - g32[name]) / abs(g32[name])
        rel64 = abs(g3232[name] - g64[name]) / abs(g64[name])
        _say("  dL/d%s float32 adjoint %.10e  rel to float64 adjoint (same states) %.2e, to float64 run %.2e"
             % (name, g3232[name], rel, rel64))
        assert rel < 1e-3
        assert rel64 < 1e-2
