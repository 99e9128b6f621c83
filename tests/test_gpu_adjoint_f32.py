"""The float32 adjoint of the AC step (Sec. II.C.1) and of the CH step (Sec.
II.D.1, with its (phi u) state) through the C ABI.

It runs the passes of the float64 adjoint in float32 arithmetic on float32
arrays; the parameter terms are summed in float64. Checks:

- one step at a float32 forward state: the result against the float64
  adjoint of the same (float32-valued) inputs, element by element, and the
  transpose identity <J v, w> = <v, J^T w> with the oracle's complex-step
  tangent, both at float32 tolerance (2-D, 3-D between moving walls, D3Q27);
- the seed and the initialisation adjoint against their float64 forms;
- whole trajectories: float64 forward states, adjoint sweeps in float64,
  in float64 on the states rounded to float32, and in float32; the float32
  sweep against the second (what the float32 arithmetic adds), the first
  reported beside it (what rounding the states to float32 costs), and the
  checkpointed autograd path (adjoint="fp32", "fp64") against the sweeps;
- the same for the CH model through the _pu forms;
- error paths: other models, aliasing, null pointers.

Tolerances. The phase field, its stencils, phi (1 - phi), the cubic term of
mu and the non-equilibrium h_eq - h (CH: of the rest population, which holds
nearly all of phi) are formed in float64 from the float32 state, so no
float32 difference cancels; every other output is a sum of a few
dozen products at the end of a chain of at most a few hundred float32
operations, each with relative error u = 2^-24 = 6.0e-8: n u = 1.2e-5 of the
largest term for n = 200. One step takes 2e-5 of max|lambda_out| and, for the
inner-product identity and the parameter terms, of the sum of |terms|. Along
N steps the per-step errors add, as independent roundings as sqrt(N): with
N <= 40 the trajectory tests take 1e-4 (sqrt(40) x 1.2e-5 = 7.6e-5) of the
largest gradient entry and of each parameter gradient.
"""
import sys

import numpy as np
import pytest

from oracle import derivatives as dv
from oracle import model as om
from paper_2511_11360_amd import pflbm as P
from paper_2511_11360_amd import workloads as wl

pytestmark = pytest.mark.gpu

STEP_TOL = 2e-5
TRAJ_TOL = 1e-4


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _dev(a, dtype=None):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype or torch.float64, device="cuda")


def _cases():
    d1, phi1, u1 = wl.static_droplet_2d(n=32, R=9.0)
    d1.update(W=3.0, rho_H=3.0, visc_interp="mu", nu_L=d1["nu_H"] * 1.5)
    phi1 = wl.droplet_phi(d1, (16.0, 16.0), 9.0)
    x, y, z = wl.grid(d1)
    u1 = wl.zero_velocity(d1)
    u1[0] = 0.01 * np.sin(2 * np.pi * (y + 0.5) / 32)
    d2, phi2, u2, _ = wl.sheared_droplet_3d(n=24, R=7.0, uw=0.02, W=2.5)
    d2.update(ny=22, rho_H=3.0)
    phi2 = wl.droplet_phi(d2, (12.0, 10.5, 12.0), 7.0, periodic=False)
    x, y, z = wl.grid(d2)
    u2 = wl.zero_velocity(d2)
    u2[0] = -0.02 + 0.04 * (y + 0.5) / 22
    d3 = dict(d2, lattice="D3Q27_D3Q7")
    out = {"droplet2d": (d1, phi1, u1), "sheared3d": (d2, phi2, u2), "sheared3d_q27": (d3, phi2, u2)}
    for k, (d, phi, u) in list(out.items()):
        out["ch_" + k] = (dict(d, model="CH", eta=1.0, M=0.04), phi, u)
    return out


ALL = ["droplet2d", "sheared3d", "sheared3d_q27", "ch_droplet2d", "ch_sheared3d", "ch_sheared3d_q27"]


@pytest.mark.parametrize("case", ALL)
def test_f32_adjoint_step_against_f64_and_oracle_tangent(case):
    import torch
    from paper_2511_11360_amd.solver import Solver
    d, phi, u = _cases()[case]
    ch = d["model"] == "CH"
    _say("case f32 adjoint step", case)
    p = om.Params(**d)
    st = om.run(p, om.init(p, phi, u), 12)
    # the forward state and lambda as float32 values, used by both adjoints
    g32, h32 = st.g.astype(np.float32), st.h.astype(np.float32)
    pu32 = st.phiu_prev.astype(np.float32) if ch else None
    rng = np.random.default_rng(3)
    wg = rng.standard_normal(st.g.shape).astype(np.float32)
    wh = rng.standard_normal(st.h.shape).astype(np.float32)
    wpu = rng.standard_normal((3,) + phi.shape).astype(np.float32) if ch else None
    s = Solver(d, precision="fp64")
    work = s.adjoint_workspace()
    f32, f64 = torch.float32, torch.float64
    outs = {}
    for dt in (f32, f64):
        og = torch.empty(st.g.shape, dtype=dt, device="cuda")
        oh = torch.empty(st.h.shape, dtype=dt, device="cuda")
        dp = torch.zeros(3, dtype=f64, device="cuda")
        if ch:
            opu = torch.empty((3,) + phi.shape, dtype=dt, device="cuda")
            fn = s.adjoint_step_pu_f32 if dt == f32 else s.adjoint_step_pu
            fn(_dev(g32, dt), _dev(h32, dt), _dev(pu32, dt), _dev(wg, dt), _dev(wh, dt), _dev(wpu, dt),
               og, oh, opu, dp, work)
            outs[dt] = (og.double().cpu().numpy(), oh.double().cpu().numpy(), opu.double().cpu().numpy(),
                        dp.cpu().numpy())
        else:
            fn = s.adjoint_step_f32 if dt == f32 else s.adjoint_step
            fn(_dev(g32, dt), _dev(h32, dt), _dev(wg, dt), _dev(wh, dt), og, oh, dp, work)
            outs[dt] = (og.double().cpu().numpy(), oh.double().cpu().numpy(), None, dp.cpu().numpy())
    og, oh, opu, dp = outs[f32]
    og64, oh64, opu64, dp64 = outs[f64]
    assert np.isfinite(og).all() and np.isfinite(oh).all()
    eg = np.max(np.abs(og - og64)) / np.max(np.abs(og64))
    eh = np.max(np.abs(oh - oh64)) / np.max(np.abs(oh64))
    _say("  max|dg|/max|g| %.3e  max|dh|/max|h| %.3e" % (eg, eh))
    assert eg <= STEP_TOL and eh <= STEP_TOL
    if ch:
        epu = np.max(np.abs(opu - opu64)) / np.max(np.abs(opu64))
        _say("  max|dpu|/max|pu| %.3e" % epu)
        assert epu <= STEP_TOL
    # each parameter term is a float64 sum of float32 per-node products: its
    # error bound scales with the sum of |terms| of the oracle's tangent
    st32 = om.State(g32.astype(np.float64), h32.astype(np.float64),
                    pu32.astype(np.float64) if ch else None)
    for k, name in enumerate(("sigma", "M", "W")):
        t = dv.step_param_tangent(p, st32, name)
        terms = np.concatenate([(t[0] * wg).ravel(), (t[1] * wh).ravel()]
                               + ([(t[2] * wpu).ravel()] if ch else []))
        _say("  d/d%s: oracle %.10e f64 %.10e f32 %.10e" % (name, terms.sum(), dp64[k], dp[k]))
        assert abs(dp[k] - terms.sum()) <= STEP_TOL * np.abs(terms).sum()
        assert abs(dp[k] - dp64[k]) <= STEP_TOL * np.abs(terms).sum()

    # transpose identity with the oracle's tangent at the float32 state
    vg = rng.standard_normal(st.g.shape) * 1e-3
    vh = rng.standard_normal(st.h.shape) * 1e-3
    if ch:
        vpu = rng.standard_normal((3,) + phi.shape) * 1e-3
        Jg, Jh, Jpu = dv.step_jvp(p, st32, vg, vh, vpu)
        lhs_terms = np.concatenate([(Jg * wg).ravel(), (Jh * wh).ravel(), (Jpu * wpu).ravel()])
        rhs_terms = np.concatenate([(vg * og).ravel(), (vh * oh).ravel(), (vpu * opu).ravel()])
    else:
        Jg, Jh = dv.step_jvp(p, st32, vg, vh)
        lhs_terms = np.concatenate([(Jg * wg).ravel(), (Jh * wh).ravel()])
        rhs_terms = np.concatenate([(vg * og).ravel(), (vh * oh).ravel()])
    lhs, rhs = lhs_terms.sum(), rhs_terms.sum()
    sc = np.abs(lhs_terms).sum() + np.abs(rhs_terms).sum()
    _say("  <Jv,w> %.12e  <v,J^T w> %.12e  rel %.2e" % (lhs, rhs, abs(lhs - rhs) / sc))
    assert abs(lhs - rhs) <= STEP_TOL * sc


def test_f32_seed_and_init_against_f64():
    import torch
    from paper_2511_11360_amd.solver import Solver
    d, phi, u = _cases()["sheared3d"]
    _say("case f32 seed and init, sheared3d")
    s = Solver(d, precision="fp64")
    w = wl.seeded_field(phi.shape, 5, -1.0, 1.0)
    lg, lh = s.adjoint_seed_phi_f32(_dev(w))
    lg64, lh64 = s.adjoint_seed_phi(_dev(w))
    assert lg.dtype == torch.float32
    assert torch.equal(lg.double(), lg64.to(torch.float32).double())
    assert torch.equal(lh.double(), lh64.to(torch.float32).double())

    p0 = 1e-3 * wl.seeded_field(phi.shape, 10, -1.0, 1.0)
    rng = np.random.default_rng(4)
    Qg, Qh = s.Qg, s.Qh
    wg = rng.standard_normal((Qg,) + phi.shape).astype(np.float32)
    wh = rng.standard_normal((Qh,) + phi.shape).astype(np.float32)
    d32 = s.adjoint_init_f32(phi, u, p0, _dev(wg, torch.float32), _dev(wh, torch.float32))
    d64 = s.adjoint_init(phi, u, p0, _dev(wg), _dev(wh))
    assert d32.dtype == torch.float32
    d32, d64 = d32.double().cpu().numpy(), d64.cpu().numpy()
    e = np.max(np.abs(d32 - d64)) / np.max(np.abs(d64))
    _say("  init: max|d|/max %.3e" % e)
    assert e <= STEP_TOL


def test_f32_ch_seed_and_init_against_f64():
    import torch
    from paper_2511_11360_amd.solver import Solver
    d, phi, u = _cases()["ch_sheared3d"]
    _say("case f32 CH seed and init, sheared3d")
    s = Solver(d, precision="fp64")
    w = wl.seeded_field(phi.shape, 5, -1.0, 1.0)
    lg, lh = s.adjoint_seed_phi_f32(_dev(w))
    lg64, lh64 = s.adjoint_seed_phi(_dev(w))
    assert torch.equal(lh.double(), lh64.to(torch.float32).double()) and torch.all(lg == 0)
    p0 = 1e-3 * wl.seeded_field(phi.shape, 10, -1.0, 1.0)
    rng = np.random.default_rng(4)
    wg = rng.standard_normal((s.Qg,) + phi.shape).astype(np.float32)
    wh = rng.standard_normal((s.Qh,) + phi.shape).astype(np.float32)
    wpu = rng.standard_normal((3,) + phi.shape).astype(np.float32)
    work = s.adjoint_workspace()
    f32 = torch.float32
    dp32 = torch.zeros(3, dtype=torch.float64, device="cuda")
    dp64 = torch.zeros(3, dtype=torch.float64, device="cuda")
    d32 = s.adjoint_init_pu_f32(phi, u, p0, _dev(wg, f32), _dev(wh, f32), _dev(wpu, f32), dp32, work)
    d64 = s.adjoint_init_pu(phi, u, p0, _dev(wg), _dev(wh), _dev(wpu), dp64, work)
    assert d32.dtype == f32
    d32, d64 = d32.double().cpu().numpy(), d64.cpu().numpy()
    e = np.max(np.abs(d32 - d64)) / np.max(np.abs(d64))
    dp32, dp64 = dp32.cpu().numpy(), dp64.cpu().numpy()
    _say("  init: max|d|/max %.3e; sigma %.10e / %.10e, W %.10e / %.10e"
         % (e, dp32[0], dp64[0], dp32[2], dp64[2]))
    assert e <= STEP_TOL
    # the sigma and W terms are float64 sums of per-node terms formed in float64
    # from float32 lambda: equal to the float64 form's up to summation order
    assert np.all(np.abs(dp32 - dp64) <= 1e-12 * np.abs(dp64).max())


def _manual(d, phi, u, steps, target):
    """dL/dphi0 and dL/d(sigma, M, W) of L = 1/2 sum (phi_N - phi*)^2 by
    three adjoint sweeps over the stored states of a float64 forward run:
    "64" the float64 adjoint, "64r" the float64 adjoint on the states rounded
    to float32, "32" the float32 adjoint on the float32 states."""
    import torch
    from paper_2511_11360_amd.solver import Solver
    ch = d["model"] == "CH"
    s = Solver(d, precision="fp64")
    s.init(phi, u)
    states = [s.step_record() for _ in range(steps)]
    dphi = s.fields()[0] - _dev(target)
    work = s.adjoint_workspace()
    out = {}
    for mode in ("64", "64r", "32"):
        dt = torch.float32 if mode == "32" else torch.float64
        dp = torch.zeros(3, dtype=torch.float64, device="cuda")
        if mode == "32":
            lg, lh = s.adjoint_seed_phi_f32(dphi)
        else:
            lg, lh = s.adjoint_seed_phi(dphi)
        og, oh = torch.empty_like(lg), torch.empty_like(lh)
        lpu = torch.zeros((3,) + s.shape, dtype=dt, device="cuda") if ch else None
        opu = torch.empty_like(lpu) if ch else None
        for g, h, pu in reversed(states):
            if mode == "64r":
                g, h = g.float().double(), h.float().double()
                pu = pu.float().double() if ch else None
            elif mode == "32":
                g, h = g.float(), h.float()
                pu = pu.float() if ch else None
            if ch:
                fn = s.adjoint_step_pu_f32 if mode == "32" else s.adjoint_step_pu
                fn(g, h, pu, lg, lh, lpu, og, oh, opu, dp, work)
                lpu, opu = opu, lpu
            else:
                fn = s.adjoint_step_f32 if mode == "32" else s.adjoint_step
                fn(g, h, lg, lh, og, oh, dp, work)
            lg, og = og, lg
            lh, oh = oh, lh
        if ch:
            fn = s.adjoint_init_pu_f32 if mode == "32" else s.adjoint_init_pu
            d0 = fn(phi, u, None, lg, lh, lpu, dp, work)
        else:
            fn = s.adjoint_init_f32 if mode == "32" else s.adjoint_init
            d0 = fn(phi, u, None, lg, lh)
        out[mode] = (d0.double().cpu().numpy(), dp.cpu().numpy())
    return out


def _grad(d, phi, u, steps, target, adjoint, precision="fp64"):
    import torch
    from paper_2511_11360_amd.autograd import run_phase_field
    phi0 = _dev(phi).requires_grad_(True)
    sig = torch.tensor(d["sigma"], dtype=torch.float64, requires_grad=True)
    M = torch.tensor(d["M"], dtype=torch.float64, requires_grad=True)
    W = torch.tensor(d["W"], dtype=torch.float64, requires_grad=True)
    phiN = run_phase_field(phi0, sig, M, W, d, _dev(u), steps, precision=precision, adjoint=adjoint)
    L = 0.5 * ((phiN - _dev(target)) ** 2).sum()
    L.backward()
    return (phi0.grad.cpu().numpy(), np.array([float(t.grad.detach().cpu()) for t in (sig, M, W)]))


@pytest.mark.parametrize("case,steps", [("droplet2d", 40), ("sheared3d", 24), ("sheared3d_q27", 24),
                                        ("ch_droplet2d", 40), ("ch_sheared3d", 24)])
def test_f32_trajectory_gradient(case, steps):
    d, phi, u = _cases()[case]
    _say("case f32 trajectory", case, "steps", steps)
    if case.endswith("droplet2d"):
        target = wl.droplet_phi(d, (16.5, 15.5), 9.4)
    else:
        target = wl.droplet_phi(d, (12.4, 10.5, 11.8), 7.3, periodic=False)
    r = _manual(d, phi, u, steps, target)
    (g64, p64), (g64r, p64r), (g32, p32) = r["64"], r["64r"], r["32"]
    # the float32 arithmetic, against the float64 adjoint of the same states
    for k, name in enumerate(("sigma", "M", "W")):
        _say("  dL/d%s f64 %.10e f64(rounded states) %.10e f32 %.10e | arith %.2e states %.2e"
             % (name, p64[k], p64r[k], p32[k], abs(p32[k] - p64r[k]) / abs(p64r[k]),
                abs(p64r[k] - p64[k]) / abs(p64[k])))
        assert abs(p32[k] - p64r[k]) <= TRAJ_TOL * abs(p64r[k])
    e_ar = np.max(np.abs(g32 - g64r)) / np.max(np.abs(g64r))
    e_st = np.max(np.abs(g64r - g64)) / np.max(np.abs(g64))
    _say("  dL/dphi0: arith %.3e states %.3e" % (e_ar, e_st))
    assert e_ar <= TRAJ_TOL
    # the checkpointed autograd path runs the same kernels on the same states
    ga, pa = _grad(d, phi, u, steps, target, "fp32")
    assert np.max(np.abs(ga - g32)) <= 1e-12 * np.max(np.abs(g32))
    assert np.all(np.abs(pa - p32) <= 1e-12 * np.abs(p32))
    gb, pb = _grad(d, phi, u, steps, target, "fp64")
    assert np.max(np.abs(gb - g64)) <= 1e-12 * np.max(np.abs(g64))


def test_f32_adjoint_error_paths():
    import torch
    from paper_2511_11360_amd.solver import Solver
    d = wl.base_params(lattice="D3Q19_D3Q7", model="L18", nx=8, ny=6, nz=5, rho_H=3.0, rho_L=1.0,
                       nu_H=0.05, nu_L=0.08, M=0.05, W=2.5, sigma=0.01)
    s = Solver(d, precision="fp64")
    s.init(np.full(s.shape, 0.5), wl.zero_velocity(d))
    g, h = s.get_distributions_f32()
    assert g.dtype == torch.float32
    work = s.adjoint_workspace()
    pu = torch.zeros((3,) + s.shape, dtype=torch.float32, device="cuda")
    with pytest.raises(P.PflbmError, match="AC and CH models") as e:
        s.adjoint_step_pu_f32(g, h, pu, g.clone(), h.clone(), pu.clone(), torch.empty_like(g),
                              torch.empty_like(h), torch.empty_like(pu), None, work)
    assert e.value.status == P.PFLBM_EUNSUPPORTED
    with pytest.raises(P.PflbmError, match="AC and CH models"):
        s.adjoint_seed_phi_f32(torch.zeros(s.shape, device="cuda"))
    # CH needs the (phi u) form, and the form checks its pu pointers
    s = Solver(dict(d, model="CH"), precision="fp64")
    s.init(np.full(s.shape, 0.5), wl.zero_velocity(d))
    with pytest.raises(P.PflbmError, match="_pu entry points") as e:
        s.adjoint_step_f32(g, h, g.clone(), h.clone(), torch.empty_like(g), torch.empty_like(h), None, work)
    assert e.value.status == P.PFLBM_EUNSUPPORTED
    lpu = pu.clone()
    with pytest.raises(P.PflbmError, match="alias") as e:
        s.adjoint_step_pu_f32(g, h, pu, g.clone(), h.clone(), lpu, torch.empty_like(g), torch.empty_like(h),
                              lpu, None, s.adjoint_workspace())
    assert e.value.status == P.PFLBM_EINVAL
    s.adjoint_step_pu_f32(g, h, pu, g.clone(), h.clone(), lpu, torch.empty_like(g), torch.empty_like(h),
                          torch.empty_like(pu), None, s.adjoint_workspace())

    d = dict(d, model="AC")
    s = Solver(d, precision="fp64")
    s.init(np.full(s.shape, 0.5), wl.zero_velocity(d))
    work = s.adjoint_workspace()
    with pytest.raises(P.PflbmError, match="no \\(phi u\\) state") as e:
        s.adjoint_step_pu_f32(g, h, pu, g.clone(), h.clone(), pu.clone(), torch.empty_like(g),
                              torch.empty_like(h), torch.empty_like(pu), None, work)
    assert e.value.status == P.PFLBM_EUNSUPPORTED
    g, h = s.get_distributions_f32()
    g64, h64 = s.get_distributions()
    assert torch.equal(g.double(), g64.to(torch.float32).double())
    assert torch.equal(h.double(), h64.to(torch.float32).double())
    lg = g.clone()
    with pytest.raises(P.PflbmError, match="alias") as e:
        s.adjoint_step_f32(g, h, lg, h.clone(), lg, torch.empty_like(h), None, work)
    assert e.value.status == P.PFLBM_EINVAL
    with pytest.raises(P.PflbmError, match="null pointer"):
        s.adjoint_step_f32(g, h, lg, h.clone(), torch.empty_like(g), torch.empty_like(h), None, None)
    # the handle still works
    s.adjoint_step_f32(g, h, lg, h.clone(), torch.empty_like(g), torch.empty_like(h), None, work)
    s.step(1)


@pytest.mark.parametrize("precision", ["mixed_fp16", "mixed_bf16"])
def test_16_bit_forward_with_both_adjoints(precision):
    """A 16-bit forward pass has no recording step: the backward pass reads
    each recomputed state out (float64, or float32 for the float32 adjoint).
    Both adjoints then differentiate the same 16-bit trajectory and agree to
    the float32 trajectory tolerance; the CH model's float32 adjoint needs a
    recording step and refuses such a forward pass."""
    d, phi, u = _cases()["droplet2d"]
    target = wl.droplet_phi(d, (16.5, 15.5), 9.4)
    _say("case 16-bit forward", precision)
    g64, p64 = _grad(d, phi, u, 24, target, "fp64", precision)
    g32, p32 = _grad(d, phi, u, 24, target, "fp32", precision)
    assert np.isfinite(g64).all() and np.isfinite(p64).all()
    for k, name in enumerate(("sigma", "M", "W")):
        _say("  dL/d%s f64 %.10e f32 %.10e" % (name, p64[k], p32[k]))
        assert abs(p32[k] - p64[k]) <= TRAJ_TOL * abs(p64[k])
    assert np.max(np.abs(g32 - g64)) <= TRAJ_TOL * np.max(np.abs(g64))
    dc, phic, uc = _cases()["ch_droplet2d"]
    with pytest.raises(ValueError, match="float64 or float32 forward"):
        _grad(dc, phic, uc, 4, target, "fp32", precision)

