"""Full-size checks of the other configured workloads, each in the launch
configuration the library picks for it (automatic tile and z block):

- 2-D Rayleigh-Taylor, 256 x 1024, walls top and bottom, AC and CH, float64
  and float32: the oracle steps the whole box once from the HIP state after
  2000 steps and every node is compared;
- 3-D sheared droplet, 128^3, walls moving at -+0.02, float64 and float32:
  the oracle steps blocks 5 wide in x and z (periodic) and spanning the whole
  walled axis, cut around sampled columns;
- droplet-laden turbulence, 512^3 (grid of 256 workgroups, each marching all
  512 planes; element offsets past 2^31), fp16-stored g and float32: 5^3
  blocks around sampled nodes;
- the discrete adjoint step at 128^3 on the sheared droplet: with lambda
  supported on a block and a perturbation v on a block next to it,
  <J v, lambda> from oracle complex-step tangents on a cut-out block equals
  <v, J^T lambda> from the HIP adjoint of the whole box, and so do the
  parameter derivatives.

The next state at a node depends on the state within two nodes, so a block
reproduces the whole box at its centre (pinned for the nonlocal model in
test_oracle_nonlocal.py; the argument is the same for every model)."""
import functools
import sys

import numpy as np
import pytest

from gpu_helpers import hydrostatic_p0
from oracle import derivatives as dv
from oracle import model as om
from paper_2511_11360_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _float_fraction(got_g, ref_g, got_h, ref_h, w, rel_g, floor_g):
    """Worst error as a fraction of the tolerance of a float32-arithmetic form:
    g relative rel_g of |g / w| plus floor_g (units of g / w); h 2e-6 relative
    plus 2e-6 absolute: h is float32 and the collision closes each node's
    phase-field balance on its last population (phi* minus the sum of the
    others), whose absolute error is then several float32 ulps of phi (phi <= 1,
    2^-24 each), up to about 1e-6."""
    eg = np.max(np.abs(got_g - ref_g) / w[:, None] / (rel_g * np.abs(ref_g / w[:, None]) + floor_g))
    eh = np.max(np.abs(got_h - ref_h) / (2e-6 * np.abs(ref_h) + 2e-6))
    return eg, eh


def _cut(t, zs, ys, xs):
    """t[:, zs][:, :, ys][:, :, :, xs] of a device tensor, as numpy."""
    import torch
    iz = torch.as_tensor(zs, device=t.device)
    iy = torch.as_tensor(ys, device=t.device)
    ix = torch.as_tensor(xs, device=t.device)
    return t[:, iz][:, :, iy][:, :, :, ix].cpu().numpy()


@pytest.mark.parametrize("model", ["AC", "CH"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_rayleigh_taylor_full_box_step(model, precision):
    from paper_2511_11360_amd.solver import Solver
    d, phi, u = wl.rayleigh_taylor_2d(model=model)
    assert (d["nx"], d["ny"]) == (256, 1024)
    s = Solver(d, precision=precision)
    s.init(phi, u, hydrostatic_p0(d, phi))
    s.step(1999)
    pu = None
    if model == "CH":
        f_phi, f_u, _, _ = s.fields()
        pu = (f_phi[None] * f_u).cpu().numpy()
    s.step(1)
    g0, h0 = [t.cpu().numpy() for t in s.get_distributions()]
    s.step(1)
    g1, h1 = [t.cpu().numpy() for t in s.get_distributions()]
    p = om.Params(**d)
    if pu is not None:
        pu = np.concatenate([pu, np.zeros_like(pu[:1])])   # (phi u) with u_z = 0 in 2-D
    out = om.step(p, om.State(g0, h0, pu))
    w = p.lattices[0].w
    if precision == "fp64":
        eg = np.abs(g1 - out.g).max()
        eh = np.abs(h1 - out.h).max()
        _say("  RT %s fp64, 262144 nodes: max|dg| %.3e max|dh| %.3e" % (model, eg, eh))
        assert eg <= 1e-14 and eh <= 1e-14
    else:
        eg, eh = _float_fraction(g1.reshape(9, -1), out.g.reshape(9, -1), h1, out.h, w, 2e-6, 2e-6)
        _say("  RT %s fp32, 262144 nodes: worst g %.3e, h %.3e of tolerance" % (model, eg, eh))
        assert eg <= 1.0 and eh <= 1.0


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_sheared_droplet_128_sampled_columns(precision):
    from paper_2511_11360_amd.solver import Solver
    d, phi, u, _ = wl.sheared_droplet_3d()
    n = d["nx"]
    assert (d["nx"], d["ny"], d["nz"]) == (128, 128, 128)
    s = Solver(d, precision=precision)
    s.init(phi, u)
    s.step(199)
    g0, h0 = s.get_distributions()
    s.step(1)
    g1, h1 = s.get_distributions()
    p = om.Params(**dict(d, nx=5, nz=5))
    w = p.lattices[0].w
    rng = np.random.default_rng(128)
    cols = [tuple(rng.integers(0, n, 2)) for _ in range(12)] + [(0, 0), (n - 1, n - 1), (64, 0)]
    ys = np.arange(n)
    worst = 0.0
    for (x, z) in cols:
        xs, zs = np.arange(x - 2, x + 3) % n, np.arange(z - 2, z + 3) % n
        out = om.step(p, om.State(_cut(g0, zs, ys, xs), _cut(h0, zs, ys, xs)))
        ref_g, ref_h = out.g[:, 2, :, 2], out.h[:, 2, :, 2]
        got_g = g1[:, z, :, x].cpu().numpy()
        got_h = h1[:, z, :, x].cpu().numpy()
        if precision == "fp64":
            e = max(np.abs(got_g - ref_g).max(), np.abs(got_h - ref_h).max())
            assert e <= 1e-14, ((x, z), e)
        else:
            eg, eh = _float_fraction(got_g, ref_g, got_h, ref_h, w, 2e-6, 2e-6)
            e = max(eg, eh)
            assert e <= 1.0, ((x, z), eg, eh)
        worst = max(worst, e)
    _say("  sheared 128^3 %s, %d columns of 128 nodes: worst %.3e (%s)"
         % (precision, len(cols), worst, "abs" if precision == "fp64" else "fraction of tolerance"))


@functools.lru_cache(maxsize=1)
def _turbulence_512():
    _say("  generating the 512^3 droplet-laden turbulence")
    d, phi, u, _ = wl.droplet_turbulence_3d(n=512)
    return d, phi, u


@pytest.mark.parametrize("precision", ["mixed_fp16", "mixed_bf16", "fp32", "fp64"])
def test_turbulence_512_sampled_nodes(precision):
    import torch
    from paper_2511_11360_amd.solver import Solver
    d, phi, u = _turbulence_512()
    n = d["nx"]
    s = Solver(d, precision=precision)
    s.init(phi, u)
    s.step(19)
    g0, h0 = s.get_distributions()
    s.step(1)
    g1, h1 = s.get_distributions()
    p = om.Params(**dict(d, nx=5, ny=5, nz=5))
    w = p.lattices[0].w
    rng = np.random.default_rng(512)
    pts = [tuple(rng.integers(0, n, 3)) for _ in range(24)]
    pts += [(0, 0, 0), (n - 1, n - 1, n - 1), (255, 256, 511), (256, 0, 255), (511, 3, 0)]
    worst = 0.0
    for (x, y, z) in pts:
        zs, ys, xs = [np.arange(c - 2, c + 3) % n for c in (z, y, x)]
        out = om.step(p, om.State(_cut(g0, zs, ys, xs), _cut(h0, zs, ys, xs)))
        ref_g, ref_h = out.g[:, 2, 2, 2], out.h[:, 2, 2, 2]
        got_g = g1[:, z, y, x].cpu().numpy()
        got_h = h1[:, z, y, x].cpu().numpy()
        if precision == "fp64":
            e = max(np.max(np.abs(got_g - ref_g)), np.max(np.abs(got_h - ref_h)))
            assert e <= 1e-14, ((x, y, z), e)
            worst = max(worst, e)
            continue
        if precision == "fp32":
            eg, eh = _float_fraction(got_g[:, None], ref_g[:, None], got_h, ref_h, w, 2e-6, 2e-6)
        elif precision == "mixed_bf16":
            # bf16 of g / w, stochastically rounded: below one ulp (2^-7)
            eg, eh = _float_fraction(got_g[:, None], ref_g[:, None], got_h, ref_h, w, 2.0 ** -6, 1e-6)
        else:
            # fp16 of 4096 g / w, stochastically rounded: below one ulp (2^-10
            # relative), tolerance twice that; float32 arithmetic
            eg, eh = _float_fraction(got_g[:, None], ref_g[:, None], got_h, ref_h, w, 2.0 ** -9, 1e-6)
        e = max(eg, eh)
        assert e <= 1.0, ((x, y, z), eg, eh)
        worst = max(worst, e)
    _say("  turbulence 512^3 %s, %d nodes: worst %.3e %s"
         % (precision, len(pts), worst, "abs" if precision == "fp64" else "of tolerance"))
    del g0, h0, g1, h1, s
    torch.cuda.empty_cache()


@pytest.mark.parametrize("arith", ["fp64", "fp32"])
def test_adjoint_128_block_supported(arith):
    """AC adjoint at full size; "fp32" runs the float32 adjoint on the state
    rounded to float32 (the oracle's tangent taken at that state), to the
    float32 tolerance of the one-step tests (2e-5 of the sum of |terms|)."""
    import torch
    from paper_2511_11360_amd.solver import Solver
    f32 = arith == "fp32"
    tol = 2e-5 if f32 else 1e-12
    d, phi, u, _ = wl.sheared_droplet_3d()
    n = d["nx"]
    s = Solver(d, precision="fp64")
    s.init(phi, u)
    s.step(50)
    fg, fh = s.get_distributions_f32() if f32 else s.get_distributions()
    Qg, Qh = fg.shape[0], fh.shape[0]
    rng = np.random.default_rng(7)
    # lambda on two 4^3 blocks (by the low wall; on the droplet interface,
    # R = 24 around the centre, where the parameter terms live) and v on a 3^3
    # block next to each; (z, y, x) corners
    lam_blocks = [(40, 1, 70), (62, 62, 86)]
    v_blocks = [(42, 3, 68), (63, 63, 88)]
    lam_g = torch.zeros_like(fg)
    lam_h = torch.zeros_like(fh)
    wvals, vvals = [], []
    for (z, y, x) in lam_blocks:
        wg = rng.standard_normal((Qg, 4, 4, 4))
        wh = rng.standard_normal((Qh, 4, 4, 4))
        if f32:   # lambda as the float32 values both sides use
            wg, wh = wg.astype(np.float32).astype(np.float64), wh.astype(np.float32).astype(np.float64)
        lam_g[:, z:z + 4, y:y + 4, x:x + 4] = torch.as_tensor(wg, device="cuda")
        lam_h[:, z:z + 4, y:y + 4, x:x + 4] = torch.as_tensor(wh, device="cuda")
        wvals.append((wg, wh))
    for _ in v_blocks:
        vvals.append((rng.standard_normal((Qg, 3, 3, 3)) * 1e-3, rng.standard_normal((Qh, 3, 3, 3)) * 1e-3))
    work = s.adjoint_workspace()
    dparams = torch.zeros(3, dtype=torch.float64, device="cuda")
    og = torch.empty_like(fg)
    oh = torch.empty_like(fh)
    (s.adjoint_step_f32 if f32 else s.adjoint_step)(fg, fh, lam_g, lam_h, og, oh, dparams, work)
    rhs_terms = []
    for (z, y, x), (vg, vh) in zip(v_blocks, vvals):
        og_v = og[:, z:z + 3, y:y + 3, x:x + 3].double().cpu().numpy()
        oh_v = oh[:, z:z + 3, y:y + 3, x:x + 3].double().cpu().numpy()
        rhs_terms += [(vg * og_v).ravel(), (vh * oh_v).ravel()]
    rhs_terms = np.concatenate(rhs_terms)
    # J^T lambda vanishes beyond two nodes of lambda's support
    assert og[:, 80:100].abs().max().item() == 0.0 and oh[:, 80:100].abs().max().item() == 0.0
    # oracle block: x 60..99, z 32..71 (periodic cut, at least 6 nodes beyond
    # every support), y whole (walls)
    x0, z0, B = 60, 32, 40
    xs, zs, ys = np.arange(x0, x0 + B), np.arange(z0, z0 + B), np.arange(n)
    st = om.State(_cut(fg.double(), zs, ys, xs), _cut(fh.double(), zs, ys, xs))
    p = om.Params(**dict(d, nx=B, nz=B))
    Wg, Wh = np.zeros_like(st.g), np.zeros_like(st.h)
    for (z, y, x), (wg, wh) in zip(lam_blocks, wvals):
        Wg[:, z - z0:z - z0 + 4, y:y + 4, x - x0:x - x0 + 4] = wg
        Wh[:, z - z0:z - z0 + 4, y:y + 4, x - x0:x - x0 + 4] = wh
    Vg, Vh = np.zeros_like(st.g), np.zeros_like(st.h)
    for (z, y, x), (vg, vh) in zip(v_blocks, vvals):
        Vg[:, z - z0:z - z0 + 3, y:y + 3, x - x0:x - x0 + 3] = vg
        Vh[:, z - z0:z - z0 + 3, y:y + 3, x - x0:x - x0 + 3] = vh
    Jg, Jh = dv.step_jvp(p, st, Vg, Vh)
    lhs_terms = np.concatenate([(Jg * Wg).ravel(), (Jh * Wh).ravel()])
    lhs, rhs = lhs_terms.sum(), rhs_terms.sum()
    scale = np.abs(lhs_terms).sum() + np.abs(rhs_terms).sum()
    _say("  128^3 adjoint (%s): <Jv,w> %.15e  <v,J^T w> %.15e" % (arith, lhs, rhs))
    assert abs(lhs) > 1e-3 * scale          # the blocks interact
    assert abs(lhs - rhs) <= tol * scale
    dp = dparams.cpu().numpy()
    for k, name in enumerate(("sigma", "M", "W")):
        tg, th = dv.step_param_tangent(p, st, name)
        terms = np.concatenate([(tg * Wg).ravel(), (th * Wh).ravel()])
        ref = terms.sum()
        _say("  d/d%s: oracle %.12e  hip %.12e" % (name, ref, dp[k]))
        assert abs(ref) > 1e-6 * np.abs(terms).sum()   # the interface block contributes
        assert abs(ref - dp[k]) <= tol * np.abs(terms).sum() + 1e-300


@pytest.mark.parametrize("model", ["CH", "L18"])
def test_adjoint_128_block_supported_pu(model):
    """The same full-size check for the CH and Liang2018 models, whose state
    and adjoint also carry (phi u) of the previous step: lambda (with
    lambda_pu) on the two 4^3 blocks, the perturbation (with v_pu) on the two
    3^3 blocks. Liang2018 takes stationary walls (its linear shear stays in
    u0)."""
    import torch
    from paper_2511_11360_amd.solver import Solver
    d, phi, u, _ = wl.sheared_droplet_3d()
    d = dict(d, model=model, eta=1.0)
    if model == "L18":
        d["wall_u"] = ((0.0, 0.0, 0.0), (0.0, 0.0, 0.0))
    n = d["nx"]
    s = Solver(d, precision="fp64")
    s.init(phi, u)
    s.step(50)
    fg, fh, fpu = s.step_record()
    Qg, Qh = fg.shape[0], fh.shape[0]
    rng = np.random.default_rng(8)
    lam_blocks = [(40, 1, 70), (62, 62, 86)]
    v_blocks = [(42, 3, 68), (63, 63, 88)]
    lam = [torch.zeros_like(fg), torch.zeros_like(fh), torch.zeros_like(fpu)]
    wvals, vvals = [], []
    for (z, y, x) in lam_blocks:
        ws = [rng.standard_normal((q, 4, 4, 4)) for q in (Qg, Qh, 3)]
        for t, w_ in zip(lam, ws):
            t[:, z:z + 4, y:y + 4, x:x + 4] = torch.as_tensor(w_, device="cuda")
        wvals.append(ws)
    for _ in v_blocks:
        vvals.append([rng.standard_normal((q, 3, 3, 3)) * 1e-3 for q in (Qg, Qh, 3)])
    work = s.adjoint_workspace()
    dparams = torch.zeros(3, dtype=torch.float64, device="cuda")
    out = [torch.empty_like(fg), torch.empty_like(fh), torch.empty_like(fpu)]
    s.adjoint_step_pu(fg, fh, fpu, lam[0], lam[1], lam[2], out[0], out[1], out[2], dparams, work)
    rhs_terms = []
    for (z, y, x), vs in zip(v_blocks, vvals):
        for t, v_ in zip(out, vs):
            rhs_terms.append((v_ * t[:, z:z + 3, y:y + 3, x:x + 3].cpu().numpy()).ravel())
    rhs_terms = np.concatenate(rhs_terms)
    for t in out:
        assert t[:, 80:100].abs().max().item() == 0.0
    x0, z0, B = 60, 32, 40
    xs, zs, ys = np.arange(x0, x0 + B), np.arange(z0, z0 + B), np.arange(n)
    st = om.State(_cut(fg, zs, ys, xs), _cut(fh, zs, ys, xs), _cut(fpu, zs, ys, xs))
    p = om.Params(**dict(d, nx=B, nz=B))
    W = [np.zeros_like(st.g), np.zeros_like(st.h), np.zeros_like(st.phiu_prev)]
    V = [np.zeros_like(st.g), np.zeros_like(st.h), np.zeros_like(st.phiu_prev)]
    for (z, y, x), ws in zip(lam_blocks, wvals):
        for A, w_ in zip(W, ws):
            A[:, z - z0:z - z0 + 4, y:y + 4, x - x0:x - x0 + 4] = w_
    for (z, y, x), vs in zip(v_blocks, vvals):
        for A, v_ in zip(V, vs):
            A[:, z - z0:z - z0 + 3, y:y + 3, x - x0:x - x0 + 3] = v_
    J = dv.step_jvp(p, st, V[0], V[1], V[2])
    lhs_terms = np.concatenate([(Jk * Wk).ravel() for Jk, Wk in zip(J, W)])
    lhs, rhs = lhs_terms.sum(), rhs_terms.sum()
    scale = np.abs(lhs_terms).sum() + np.abs(rhs_terms).sum()
    _say("  128^3 %s adjoint: <Jv,w> %.15e  <v,J^T w> %.15e" % (model, lhs, rhs))
    assert abs(lhs) > 1e-3 * scale
    assert abs(lhs - rhs) <= 1e-12 * scale
    dp = dparams.cpu().numpy()
    for k, name in enumerate(("sigma", "M", "W")):
        t = dv.step_param_tangent(p, st, name)
        terms = np.concatenate([(tk * Wk).ravel() for tk, Wk in zip(t, W)])
        ref = terms.sum()
        _say("  d/d%s: oracle %.12e  hip %.12e" % (name, ref, dp[k]))
        assert abs(ref) > 1e-6 * np.abs(terms).sum()
        assert abs(ref - dp[k]) <= 1e-12 * np.abs(terms).sum() + 1e-300
