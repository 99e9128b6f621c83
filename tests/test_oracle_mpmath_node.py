"""Brute-force pin of one node of the oracle's step: the whole collision
(phi moment, stencils, local coefficients, forces, both collisions) evaluated
at 50 significant digits with mpmath, written independently from the paper's
equations, against the oracle's float64 post-collision populations.

Steps (Sec. II.C.1 and Sec. III stencils): phi = sum h (Eq.
fakhari_phi_update); grad phi = 3 sum w c phi(x + c), lap phi =
6 sum w (phi(x + c) - phi(x)); rho, mu linear in phi, nu = mu / rho,
tau = 3 nu + 1/2 (Eqs. fakhari_rho_update, mu_linear, fakhari_tau_model);
mu_phi = 4 beta phi (phi - 1)(phi - 1/2) - kappa lap phi with beta =
12 sigma / W, kappa = 3 sigma W / 2 (Eqs. chemical_potential, coefficients);
p* = sum g, p = rho p* / 3 (Eq. fakhari_p_update); F_s = mu_phi grad phi,
F_b = rho g, F_p = -(p / rho) grad rho; the viscous force from the
non-equilibrium stress at u* (the reading of F_mu's strain rate); u = j +
F / (2 rho) (Eq. fakhari_velocity_update); h: BGK with Eqs. fakhari_geq and
fakhari_G_modified; g: MRT with the viscous stress moments at 1/tau and every
other moment at s_o (orthogonal moment basis), which for an unweighted
orthogonal basis is g* = g - s_o (g - g_eq) - (1/tau - s_o) P (g - g_eq)
+ (1 - s_o / 2) F_i with P the orthogonal projector onto the traceless
quadratic forms of the velocities (Eq. fakhari_F for F_i).
"""
import itertools

import numpy as np
import pytest

mp = pytest.importorskip("mpmath")

from oracle import model as om  # noqa: E402
from paper_2511_11360_amd import workloads as wl  # noqa: E402


def _velocities(dim, max_sq):
    """Velocity set with components in {-1, 0, 1} and |c|^2 <= max_sq, with the
    weights of the standard D2Q9 / D2Q5 / D3Q19 / D3Q7 lattices at
    c_s^2 = 1/3 (D3Q7: rest weight 0)."""
    weights = {
        (2, 2): {0: mp.mpf(4) / 9, 1: mp.mpf(1) / 9, 2: mp.mpf(1) / 36},
        (2, 1): {0: mp.mpf(1) / 3, 1: mp.mpf(1) / 6},
        (3, 2): {0: mp.mpf(1) / 3, 1: mp.mpf(1) / 18, 2: mp.mpf(1) / 36},
        (3, 1): {0: mp.mpf(0), 1: mp.mpf(1) / 6},
    }[(dim, max_sq)]
    out = []
    for c in itertools.product((-1, 0, 1), repeat=dim):
        s = sum(v * v for v in c)
        if s <= max_sq:
            c3 = tuple(c) + (0,) * (3 - dim)
            out.append((c3, weights[s]))
    return out


def _node(d, g, h, node):
    """Post-collision g and h at `node` (x, y, z) of a periodic box, in mpmath."""
    dim = 2 if d["lattice"].startswith("D2") else 3
    G = _velocities(dim, 2)
    H = _velocities(dim, 1)
    nz, ny, nx = g.shape[1:]
    gidx = {c: i for i, c in enumerate(map(tuple, om.Params(**d).lattices[0].c.tolist()))}
    hidx = {c: i for i, c in enumerate(map(tuple, om.Params(**d).lattices[1].c.tolist()))}
    f = mp.mpf

    def at(arr, idx, pos):
        x, y, z = pos
        return f(float(arr[idx, z % nz, y % ny, x % nx]))

    def phi_at(pos):
        return mp.fsum(at(h, hidx[c], pos) for c, _ in H)

    x0 = tuple(node)
    phi = phi_at(x0)
    grad = [mp.mpf(0)] * 3
    lap = mp.mpf(0)
    for c, w in G:
        pn = phi_at(tuple(x0[k] + c[k] for k in range(3)))
        for k in range(3):
            grad[k] += 3 * w * c[k] * pn
        lap += 6 * w * (pn - phi)
    rH, rL = f(d["rho_H"]), f(d["rho_L"])
    rho = rL + phi * (rH - rL)
    mu_visc = rL * f(d["nu_L"]) + phi * (rH * f(d["nu_H"]) - rL * f(d["nu_L"]))
    nu = mu_visc / rho
    tau = 3 * nu + f(1) / 2
    sigma, W, M = f(d["sigma"]), f(d["W"]), f(d["M"])
    beta, kappa = 12 * sigma / W, 3 * sigma * W / 2
    mu_phi = 4 * beta * phi * (phi - 1) * (phi - f(1) / 2) - kappa * lap
    gv = {c: at(g, gidx[c], x0) for c, _ in G}
    hv = {c: at(h, hidx[c], x0) for c, _ in H}
    ps = mp.fsum(gv.values())
    pres = rho * ps / 3
    grho = [(rH - rL) * grad[k] for k in range(3)]
    body = [f(v) for v in d["gravity"]]
    F0 = [mu_phi * grad[k] + rho * body[k] - pres / rho * grho[k] for k in range(3)]
    j = [mp.fsum(c[k] * gv[c] for c, _ in G) for k in range(3)]
    us = [j[k] + F0[k] / (2 * rho) for k in range(3)]

    def geq(c, w, u):
        cu = sum(c[k] * u[k] for k in range(3))
        uu = sum(u[k] * u[k] for k in range(3))
        return w * (ps + 3 * cu + f(9) / 2 * cu * cu - f(3) / 2 * uu)

    Pi = [[mp.fsum(c[a] * c[b] * (gv[c] - geq(c, w, us)) for c, w in G) for b in range(3)]
          for a in range(3)]
    S = [[-3 * Pi[a][b] / tau for b in range(3)] for a in range(3)]
    Fmu = [nu * sum(S[a][b] * grho[b] for b in range(3)) for a in range(3)]
    F = [F0[k] + Fmu[k] for k in range(3)]
    u = [j[k] + F[k] / (2 * rho) for k in range(3)]
    uu = sum(u[k] * u[k] for k in range(3))
    # phase field
    tp = 3 * M + f(1) / 2
    eps = f(d["normal_eps"])
    norm = mp.sqrt(sum(grad[k] * grad[k] for k in range(3)) + eps * eps)
    hout = {}
    for c, w in H:
        eu = sum(c[k] * u[k] for k in range(3))
        heq = w * phi * (1 + 3 * eu + f(9) / 2 * eu * eu - f(3) / 2 * uu)
        Ga = w * (4 / W) * phi * (1 - phi) * sum(c[k] * grad[k] for k in range(3)) / norm
        hout[c] = hv[c] - (hv[c] - heq) / tp + (1 - 1 / (2 * tp)) * Ga
    # hydrodynamics: two-rate MRT as a projector on the traceless quadratic forms
    cs = [c for c, _ in G]
    forms = [lambda c: c[0] * c[0] - c[1] * c[1], lambda c: c[0] * c[1]]
    if dim == 3:
        forms = [lambda c: 3 * c[0] * c[0] - (c[0] ** 2 + c[1] ** 2 + c[2] ** 2),
                 lambda c: c[1] * c[1] - c[2] * c[2],
                 lambda c: c[0] * c[1], lambda c: c[1] * c[2], lambda c: c[0] * c[2]]
    Qm = mp.matrix([[fm(c) for fm in forms] for c in cs])
    P = Qm * mp.inverse(Qm.T * Qm) * Qm.T
    neq = mp.matrix([gv[c] - geq(c, w, u) for c, w in G])
    Pn = P * neq
    so = f(d["s_other"])
    gout = {}
    for i, (c, w) in enumerate(G):
        Fi = 3 * w * sum(c[k] * F[k] for k in range(3)) / rho
        gout[c] = gv[c] - so * neq[i] - (1 / tau - so) * Pn[i] + (1 - so / 2) * Fi
    return ({gidx[c]: v for c, v in gout.items()}, {hidx[c]: v for c, v in hout.items()})


@pytest.mark.parametrize("lattice,shape,node", [
    ("D2Q9_D2Q5", (1, 5, 5), (2, 2, 0)),
    ("D3Q19_D3Q7", (3, 3, 3), (1, 1, 1)),
])
def test_one_node_matches_fifty_digit_evaluation(lattice, shape, node):
    """Random populations around an interface (rho ratio 3, unequal
    viscosities, s_o = 1.3, gravity): the oracle's post-collision g and h at
    one node equal the 50-digit evaluation to 1e-15 relative to the node's
    sum of |populations| (the scale of the moment sums; measured up to 2e-16:
    a few float64 roundings of the moment-space inverse)."""
    mp.mp.dps = 50
    nz, ny, nx = shape
    d = wl.base_params(lattice=lattice, nx=nx, ny=ny, nz=nz, rho_H=3.0, rho_L=1.0,
                       nu_H=0.05, nu_L=0.12, M=0.05, W=3.0, sigma=0.02, s_other=1.3,
                       gravity=(1e-4, -2e-4, 0.0 if nz == 1 else 5e-5))
    p = om.Params(**d)
    rng = np.random.default_rng(23)
    gl, hl = p.lattices
    phi = rng.uniform(0.2, 0.8, size=p.shape)
    h = np.array([hl.w[a] * phi for a in range(hl.Q)]) + rng.uniform(-0.01, 0.01, (hl.Q,) + p.shape)
    if hl.w[0] == 0:
        h[0] = 0.0
    g = np.array([gl.w[i] * (0.02 + 0.0 * phi) for i in range(gl.Q)]) \
        + rng.uniform(-0.002, 0.002, (gl.Q,) + p.shape)
    st = om.State(g, h)
    m = om.macroscopic(p, st)
    go = om.collide_g(p, st, m)
    ho = om.collide_h(p, st, m)
    gm, hm = _node(d, g, h, node)
    x, y, z = node
    gscale = np.sum(np.abs(go[:, z, y, x]))
    hscale = np.sum(np.abs(ho[:, z, y, x]))
    for i, v in gm.items():
        assert abs(float(v) - go[i, z, y, x]) <= 1e-15 * gscale, (i, float(v), go[i, z, y, x])
    for a, v in hm.items():
        assert abs(float(v) - ho[a, z, y, x]) <= 1e-15 * hscale, (a, float(v), ho[a, z, y, x])
