"""Discrete adjoint of the HIP step against derivatives of the oracle.

One step: <J v, w> (tangent by complex step of the oracle) equals <v, J^T w>
(the HIP adjoint kernel), and the parameter terms equal the oracle's complex
step tangents. Whole trajectories: gradients of L = 1/2 sum (phi_N - phi*)^2
through the checkpointed autograd function against complex steps of the oracle
and central differences of the HIP forward path."""
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


def _cases():
    d1, phi1, u1 = wl.static_droplet_2d(n=32, R=9.0)
    d1.update(W=3.0)
    phi1 = wl.droplet_phi(d1, (16.0, 16.0), 9.0)
    d2, phi2, u2, _ = wl.sheared_droplet_3d(n=24, R=7.0, uw=0.02, W=2.5)
    d2["ny"] = 22
    d2["rho_H"] = 3.0
    phi2 = wl.droplet_phi(d2, (12.0, 10.5, 12.0), 7.0, periodic=False)
    x, y, z = wl.grid(d2)
    u2 = wl.zero_velocity(d2)
    u2[0] = -0.02 + 0.04 * (y + 0.5) / 22
    d3 = dict(d2, lattice="D3Q27_D3Q7")
    return {"droplet2d": (d1, phi1, u1), "sheared3d": (d2, phi2, u2), "sheared3d_q27": (d3, phi2, u2)}


def _dev(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


@pytest.mark.parametrize("case", ["droplet2d", "sheared3d", "sheared3d_q27"])
def test_adjoint_step_is_transpose_of_oracle_tangent(case):
    d, phi, u = _cases()[case]
    d = dict(d, rho_H=3.0, visc_interp="mu", nu_L=d["nu_H"] * 1.5)
    _say("case", case)
    _check_transpose(d, phi, u)


# boxes one or two nodes wide along some axes: the wrapped (or wall-clamped)
# neighbours of a node coincide with the node itself or its one partner, and
# with walls two nodes apart both layers are wall layers
DEGENERATE = [
    ("D3Q19_D3Q7", (3, 2, 4), ("periodic", "periodic", "periodic")),
    ("D3Q19_D3Q7", (1, 3, 2), ("periodic", "periodic", "periodic")),
    ("D3Q19_D3Q7", (4, 2, 3), ("periodic", "wall", "periodic")),
    ("D3Q19_D3Q7", (2, 5, 1), ("periodic", "wall", "periodic")),
    ("D3Q27_D3Q7", (3, 2, 4), ("periodic", "periodic", "periodic")),
    ("D3Q27_D3Q7", (4, 2, 3), ("periodic", "wall", "periodic")),
    ("D2Q9_D2Q5", (1, 6, 1), ("periodic", "wall", "periodic")),
    ("D2Q9_D2Q5", (3, 1, 1), ("periodic", "periodic", "periodic")),
]


@pytest.mark.parametrize("lattice,n,bc", DEGENERATE)
def test_adjoint_step_transpose_degenerate_boxes(lattice, n, bc):
    nx, ny, nz = n
    d = wl.base_params(lattice=lattice, model="AC", nx=nx, ny=ny, nz=nz, bc=bc, rho_H=3.0, rho_L=1.0,
                       nu_H=0.05, nu_L=0.08, M=0.05, W=2.5, sigma=0.01, visc_interp="mu")
    x, y, z = wl.grid(d)
    phi = 0.5 + 0.3 * (np.sin(2 * np.pi * (x + 0.3) / nx) * np.cos(2 * np.pi * (y + 0.2) / ny)
                       * np.cos(2 * np.pi * (z + 0.1) / nz))
    u = wl.zero_velocity(d)
    u[0] = 0.01 * np.cos(2 * np.pi * y / ny)
    _say("case", lattice, n, bc[1])
    _check_transpose(d, phi, u)


def _check_transpose(d, phi, u):
    import torch
    from paper_2511_11360_amd.solver import Solver
    p = om.Params(**d)
    st = om.run(p, om.init(p, phi, u), 12)
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
    return (float(L), phi0.grad.cpu().numpy(), float(sig.grad.cpu()), float(M.grad.cpu()),
            float(W.grad.cpu()))


@pytest.mark.parametrize("case,steps", [("droplet2d", 40), ("sheared3d", 24), ("sheared3d_q27", 16)])
def test_trajectory_gradient_vs_oracle_complex_step(case, steps):
    d, phi, u = _cases()[case]
    _say("case", case, "steps", steps)
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


def test_checkpointing_does_not_change_gradients():
    d, phi, u = _cases()["droplet2d"]
    target = wl.droplet_phi(d, (16.5, 15.5), 9.4)
    a = _grad_hip(d, phi, u, 30, target, k=30)     # all states of one segment
    b = _grad_hip(d, phi, u, 30, target, k=4)      # 8 segments
    c = _grad_hip(d, phi, u, 30, target)           # ceil(sqrt(30)) = 6
    assert np.array_equal(a[1], b[1]) and np.array_equal(a[1], c[1])
    assert a[2:] == b[2:] == c[2:]


def test_gradient_vs_hip_central_differences_sheared_droplet():
    """Reduced shear workload (moving walls, tanh-ellipsoid target): adjoint
    gradient against central differences of the HIP float64 forward run."""
    import torch
    from paper_2511_11360_amd.solver import Solver
    d, phi, u, target = wl.sheared_droplet_3d(n=40, R=10.0, uw=0.02, W=3.0)
    d["ny"] = 38
    phi = wl.droplet_phi(d, (20.0, 18.5, 20.0), 10.0, periodic=False)
    x, y, z = wl.grid(d)
    u = wl.zero_velocity(d)
    u[0] = -0.02 + 0.04 * (y + 0.5) / 38
    target = target[:, :38, :]
    steps = 120
    L, gphi0, gs, gM, gW = _grad_hip(d, phi, u, steps, target)

    def loss(dd):
        s = Solver(dd, precision="fp64")
        s.init(phi, u)
        s.step(steps)
        ph = s.fields()[0]
        return float(0.5 * ((ph - _dev(target)) ** 2).sum())

    for name, g in (("sigma", gs), ("M", gM), ("W", gW)):
        h = 1e-4 * d[name]
        fd = (loss(dict(d, **{name: d[name] + h})) - loss(dict(d, **{name: d[name] - h}))) / (2 * h)
        _say("  dL/d%s adjoint %.10e  central FD %.10e" % (name, g, fd))
        assert abs(g - fd) <= 1e-6 * abs(fd)
