"""Discrete adjoint of the nonlocal (Chai2018) and hybrid (Hu2019) phase
field, Secs. II.C.3-4: the step uses phi* = sum h + (1 - lam) R / 2 with the
source R of Eq. nonlocalAC and the multiplier gamma of Eq.
lagrange_multiplier, a sum over every node, so its adjoint carries two global
sums. Against complex-step tangents of the oracle:

- one step: <J v, w> = <v, J^T w> and the parameter terms (lam 0 and 0.9;
  2-D, 3-D between moving walls on D3Q19 and D3Q27, a degenerate box);
- the seed (transpose of the corrected phi* that pflbm_fields reports) and
  its M and W terms;
- the initialisation h = h_eq(phi0, u0) of Eq. Chai_geq;
- whole trajectories through the checkpointed autograd function.
"""
import sys

import numpy as np
import pytest

from oracle import derivatives as dv
from oracle import model as om
from paper_2511_11360_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _dev(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _cases(lam):
    d1, phi1, u1 = wl.static_droplet_2d(n=32, R=9.0)
    d1.update(W=3.0, model="NL", lam=lam, rho_H=3.0, visc_interp="mu", nu_L=d1["nu_H"] * 1.5)
    phi1 = wl.droplet_phi(d1, (16.0, 16.0), 9.0)
    x, y, z = wl.grid(d1)
    u1 = wl.zero_velocity(d1)
    u1[0] = 0.01 * np.sin(2 * np.pi * (y + 0.5) / 32)
    d2, phi2, u2, _ = wl.sheared_droplet_3d(n=24, R=7.0, uw=0.02, W=2.5)
    d2.update(ny=22, rho_H=3.0, model="NL", lam=lam)
    phi2 = wl.droplet_phi(d2, (12.0, 10.5, 12.0), 7.0, periodic=False)
    x, y, z = wl.grid(d2)
    u2 = wl.zero_velocity(d2)
    u2[0] = -0.02 + 0.04 * (y + 0.5) / 22
    d3 = dict(d2, lattice="D3Q27_D3Q7")
    return {"droplet2d": (d1, phi1, u1), "sheared3d": (d2, phi2, u2), "sheared3d_q27": (d3, phi2, u2)}


def _transpose(d, phi, u, steps=12):
    import torch
    from paper_2511_11360_amd.solver import Solver
    p = om.Params(**d)
    st = om.run(p, om.init(p, phi, u), steps)
    rng = np.random.default_rng(3)
    vg = rng.standard_normal(st.g.shape) * 1e-3
    vh = rng.standard_normal(st.h.shape) * 1e-3
    wg = rng.standard_normal(st.g.shape)
    wh = rng.standard_normal(st.h.shape)
    Jg, Jh = dv.step_jvp(p, st, vg, vh)
    lhs_terms = np.concatenate([(Jg * wg).ravel(), (Jh * wh).ravel()])
    s = Solver(d, precision="fp64")
    work = s.adjoint_workspace()
    dparams = torch.zeros(3, dtype=torch.float64, device="cuda")
    og = torch.empty(st.g.shape, dtype=torch.float64, device="cuda")
    oh = torch.empty(st.h.shape, dtype=torch.float64, device="cuda")
    s.adjoint_step(_dev(st.g), _dev(st.h), _dev(wg), _dev(wh), og, oh, dparams, work)
    og, oh, dp = og.cpu().numpy(), oh.cpu().numpy(), dparams.cpu().numpy()
    rhs_terms = np.concatenate([(vg * og).ravel(), (vh * oh).ravel()])
    lhs, rhs = lhs_terms.sum(), rhs_terms.sum()
    scale = np.abs(lhs_terms).sum() + np.abs(rhs_terms).sum()
    _say("  <Jv,w> %.15e  <v,J^T w> %.15e" % (lhs, rhs))
    assert abs(lhs - rhs) <= 1e-12 * scale
    for k, name in enumerate(("sigma", "M", "W")):
        tg, th = dv.step_param_tangent(p, st, name)
        terms = np.concatenate([(tg * wg).ravel(), (th * wh).ravel()])
        ref = terms.sum()
        _say("  d/d%s: oracle %.12e  hip %.12e" % (name, ref, dp[k]))
        assert abs(ref - dp[k]) <= 1e-12 * np.abs(terms).sum() + 1e-300


@pytest.mark.parametrize("lam", [0.0, 0.9])
@pytest.mark.parametrize("case", ["droplet2d", "sheared3d", "sheared3d_q27"])
def test_nl_adjoint_step_is_transpose_of_oracle_tangent(case, lam):
    d, phi, u = _cases(lam)[case]
    _say("case NL", case, "lam", lam)
    _transpose(d, phi, u)


def test_nl_adjoint_step_transpose_degenerate_box():
    d = wl.base_params(lattice="D3Q19_D3Q7", model="NL", lam=0.5, nx=4, ny=2, nz=3,
                       bc=("periodic", "wall", "periodic"), rho_H=3.0, rho_L=1.0, nu_H=0.05, nu_L=0.08,
                       M=0.05, W=2.5, sigma=0.01, visc_interp="mu")
    x, y, z = wl.grid(d)
    phi = 0.5 + 0.3 * (np.sin(2 * np.pi * (x + 0.3) / 4) * np.cos(2 * np.pi * (y + 0.2) / 2)
                       * np.cos(2 * np.pi * (z + 0.1) / 3))
    u = wl.zero_velocity(d)
    u[0] = 0.01 * np.cos(2 * np.pi * y / 2)
    _say("case NL degenerate 4 x 2 x 3, walls")
    _transpose(d, phi, u, steps=4)


@pytest.mark.parametrize("lam", [0.0, 0.9])
def test_nl_seed_is_transpose_of_corrected_phi(lam):
    import torch
    from paper_2511_11360_amd.solver import Solver
    d, phi, u = _cases(lam)["sheared3d"]
    _say("case NL seed lam", lam)
    p = om.Params(**d)
    st = om.run(p, om.init(p, phi, u), 6)
    rng = np.random.default_rng(7)
    vh = rng.standard_normal(st.h.shape)
    w = rng.standard_normal(phi.shape)
    t = dv.fields_phi_tangent(p, st, vh)
    s = Solver(d, precision="fp64")
    work = s.adjoint_workspace()
    dparams = torch.zeros(3, dtype=torch.float64, device="cuda")
    lg, lh = s.adjoint_seed(_dev(st.h), _dev(w), dparams, work)
    lg, lh, dp = lg.cpu().numpy(), lh.cpu().numpy(), dparams.cpu().numpy()
    assert np.all(lg == 0.0)
    lhs, rhs = (t * w).sum(), (vh * lh).sum()
    _say("  <J v, w> %.15e  <v, J^T w> %.15e" % (lhs, rhs))
    assert abs(lhs - rhs) <= 1e-12 * (np.abs(t * w).sum() + np.abs(vh * lh).sum())
    for k, name in enumerate(("sigma", "M", "W")):
        terms = dv.fields_phi_tangent(p, st, name=name) * w
        _say("  d/d%s: oracle %.12e  hip %.12e" % (name, terms.sum(), dp[k]))
        assert abs(terms.sum() - dp[k]) <= 1e-12 * np.abs(terms).sum() + 1e-300


def test_nl_adjoint_init_is_transpose_of_oracle_tangent():
    from paper_2511_11360_amd.solver import Solver
    d, phi, u = _cases(0.0)["sheared3d"]
    p = om.Params(**d)
    p0 = 1e-3 * wl.seeded_field(phi.shape, 10, -1.0, 1.0)
    v = wl.seeded_field(phi.shape, 9, -1.0, 1.0)
    Jg, Jh = dv.init_jvp(p, phi, v, u, p0)
    rng = np.random.default_rng(4)
    wg = rng.standard_normal(Jg.shape)
    wh = rng.standard_normal(Jh.shape)
    s = Solver(d, precision="fp64")
    dphi0 = s.adjoint_init(phi, u, p0, _dev(wg), _dev(wh)).cpu().numpy()
    lhs_terms = np.concatenate([(Jg * wg).ravel(), (Jh * wh).ravel()])
    lhs, rhs = lhs_terms.sum(), (v * dphi0).sum()
    _say("case NL init  <J v, w> %.15e  <v, J^T w> %.15e" % (lhs, rhs))
    assert abs(lhs - rhs) <= 1e-12 * (np.abs(lhs_terms).sum() + np.abs(v * dphi0).sum())


def _grad_hip(d, phi, u, steps, target, k=None):
    import torch
    from paper_2511_11360_amd.autograd import run_phase_field
    phi0 = _dev(phi).requires_grad_(True)
    sig = torch.tensor(d["sigma"], dtype=torch.float64, requires_grad=True)
    M = torch.tensor(d["M"], dtype=torch.float64, requires_grad=True)
    W = torch.tensor(d["W"], dtype=torch.float64, requires_grad=True)
    phiN = run_phase_field(phi0, sig, M, W, d, _dev(u), steps, k=k)
    L = 0.5 * ((phiN - _dev(target)) ** 2).sum()
    L.backward()
    return (float(L), phi0.grad.cpu().numpy(), float(sig.grad.detach().cpu()),
            float(M.grad.detach().cpu()), float(W.grad.detach().cpu()))


@pytest.mark.parametrize("case,lam,steps", [("droplet2d", 0.0, 40), ("sheared3d", 0.9, 24)])
def test_nl_trajectory_gradient_vs_oracle_complex_step(case, lam, steps):
    d, phi, u = _cases(lam)[case]
    _say("case NL trajectory", case, "lam", lam, "steps", steps)
    p = om.Params(**d)
    if case == "droplet2d":
        target = wl.droplet_phi(d, (16.5, 15.5), 9.4)
    else:
        target = wl.droplet_phi(d, (12.4, 10.5, 11.8), 7.3, periodic=False)
    L, gphi0, gs, gM, gW = _grad_hip(d, phi, u, steps, target)
    for name, g in (("sigma", gs), ("M", gM), ("W", gW)):
        ref = dv.cs_param(p, name, phi, u, steps, target)
        _say("  dL/d%s hip %.12e oracle-cs %.12e" % (name, g, ref))
        assert abs(g - ref) <= 1e-9 * abs(ref)
    v = wl.seeded_field(phi.shape, 11, -1.0, 1.0)
    ref = dv.cs_phi0(p, v, phi, u, steps, target)
    got = float(np.sum(gphi0 * v))
    _say("  <dL/dphi0, v> hip %.12e oracle-cs %.12e" % (got, ref))
    assert abs(got - ref) <= 1e-9 * abs(ref)
