"""Pins of the oracle's Liang2018 model (Sec. II.C: Eqs. liang_geq, liang_feq,
liang_G_final, liang_F_final, liang_velocity_update, liang_p_update) and of
Liang2014 with its own hydrodynamics (Sec. II.D.1: Eqs. liang2_feq, liang2_F,
Gamma_beta, liang2014_velocity_update).

What the lattice moments and the model's definition fix, independent of the
oracle's code: the zeroth to second moments of f_eq (0, rho u,
p I + rho u u) and of the force populations (u.grad rho, F,
c_s^2 [(u.grad rho) I + u grad rho + grad rho u]); the velocity and pressure
updates return u and p exactly from an equilibrium state; fixed points at rest
and in uniform flow; the shear-wave decay rate nu k^2 with the non-stress
moments at a different rate; exact momentum growth under a uniform force;
conservation of sum phi; Young-Laplace for a static droplet within 8 %.
"""
import numpy as np
import pytest

from oracle import model as om
from oracle.lattice import CS2


def _p(**kw):
    d = dict(lattice="D2Q9_D2Q5", model="L18", nx=32, ny=32, rho_H=10.0, rho_L=1.0,
             nu_H=0.1, nu_L=0.1, M=0.02, W=4.0, sigma=0.01)
    d.update(kw)
    return om.Params(**d)


def _moments(lat, f):
    m0 = f.sum(axis=0)
    m1 = np.array([sum(lat.c[i][a] * f[i] for i in range(lat.Q)) for a in range(3)])
    m2 = np.array([[sum(lat.c[i][a] * lat.c[i][b] * f[i] for i in range(lat.Q)) for b in range(3)]
                   for a in range(3)])
    return m0, m1, m2


@pytest.mark.parametrize("lat", ["D2Q9_D2Q5", "D3Q19_D3Q7", "D3Q27_D3Q7"])
def test_equilibrium_and_force_moments(lat):
    d3 = lat != "D2Q9_D2Q5"
    p = _p(lattice=lat, nx=5, ny=4, nz=3 if d3 else 1)
    rng = np.random.default_rng(11)
    sh = p.shape
    rho = rng.uniform(1, 10, sh)
    pres = rng.standard_normal(sh) * 1e-3
    u = rng.standard_normal((3,) + sh) * 0.05
    gr = rng.standard_normal((3,) + sh) * 0.3
    F = rng.standard_normal((3,) + sh) * 1e-4
    if not d3:
        u[2] = gr[2] = F[2] = 0
    lat_g = p.lattices[0]
    m0, m1, m2 = _moments(lat_g, om.f_eq_liang(p, rho, pres, u))
    assert np.abs(m0).max() < 1e-14
    assert np.abs(m1 - rho * u).max() < 1e-14
    dim = 3 if d3 else 2
    for a in range(dim):
        for b in range(dim):
            assert np.abs(m2[a, b] - (pres * (a == b) + rho * u[a] * u[b])).max() < 1e-14
    udr = sum(u[a] * gr[a] for a in range(3))
    m0, m1, m2 = _moments(lat_g, om.force_liang(p, F, u, gr))
    assert np.abs(m0 - udr).max() < 1e-15
    assert np.abs(m1 - F).max() < 1e-15
    for a in range(dim):
        for b in range(dim):
            ref = CS2 * (udr * (a == b) + u[a] * gr[b] + gr[a] * u[b])
            assert np.abs(m2[a, b] - ref).max() < 1e-15


def test_velocity_and_pressure_recovered_from_equilibrium():
    p = _p(nx=6, ny=5, sigma=0.0)
    rng = np.random.default_rng(2)
    phi = np.full(p.shape, 0.7)
    rho = np.full(p.shape, 0.7 * 10 + 0.3)
    pres = rng.standard_normal(p.shape) * 1e-3
    u = np.zeros((3,) + p.shape)
    u[:2] = rng.standard_normal((2,) + p.shape) * 0.05
    st = om.State(om.f_eq_liang(p, rho, pres, u), om.h_eq_nl(p, phi, u), phi * u)
    m = om.macroscopic(p, st)
    assert np.abs(m["u"] - u).max() < 1e-15
    assert np.abs(m["p"] - pres).max() < 1e-16


@pytest.mark.parametrize("lat", ["D2Q9_D2Q5", "D3Q19_D3Q7"])
def test_fixed_points(lat):
    d3 = lat != "D2Q9_D2Q5"
    p = _p(lattice=lat, nx=5, ny=4, nz=3 if d3 else 1)
    st = om.init(p, np.full(p.shape, 0.4))
    st2 = om.run(p, st, 5)
    assert np.abs(st2.g - st.g).max() < 1e-16 and np.abs(st2.h - st.h).max() < 1e-15
    u = np.zeros((3,) + p.shape)
    u[0], u[1] = 0.03, -0.02
    st = om.init(p, np.full(p.shape, 1.0), u)
    st2 = om.run(p, st, 5)
    f = om.fields(p, st2)
    assert np.abs(f[1][0] - 0.03).max() < 1e-15 and np.abs(f[1][1] + 0.02).max() < 1e-15


@pytest.mark.parametrize("lat,s_o", [("D2Q9_D2Q5", None), ("D3Q19_D3Q7", 1.0)])
def test_shear_wave_viscosity(lat, s_o):
    L_ = 32
    nu = 0.04
    d3 = lat != "D2Q9_D2Q5"
    p = _p(lattice=lat, nx=4, ny=L_, nz=4 if d3 else 1, rho_H=1.0, rho_L=1.0, nu_H=nu, nu_L=nu,
           s_other=s_o if s_o else 1.0 / (3 * nu + 0.5))
    k = 2 * np.pi / L_
    u = np.zeros((3,) + p.shape)
    u[0] = 1e-3 * np.sin(k * np.arange(L_))[None, :, None]
    st = om.run(p, om.init(p, np.full(p.shape, 1.0), u), 300)
    uu = om.fields(p, st)[1]
    amp = np.sum(uu[0][0, :, 0] * np.sin(k * np.arange(L_))) / (L_ / 2)
    rate = -np.log(amp / 1e-3) / 300
    assert abs(rate / (nu * k * k) - 1) < 0.01


def test_uniform_force_momentum_growth():
    """Uniform phase (rho = 3.7): sum e f grows by N F each step and rho u
    adds the half step F / 2 (Eq. liang_velocity_update): (n + 1/2) N F."""
    p = _p(nx=10, ny=8, force=(2e-6, -1e-6, 0.0))
    st = om.run(p, om.init(p, np.full(p.shape, 0.3)), 40)
    m = om.macroscopic(p, st)
    N = 80
    assert abs((m["rho"] * m["u"][0]).sum() - 40.5 * N * 2e-6) < 1e-15
    assert abs((m["rho"] * m["u"][1]).sum() + 40.5 * N * 1e-6) < 1e-15


def test_phase_conservation_droplet():
    p = _p(nx=20, ny=16)
    x, y = np.meshgrid(np.arange(20), np.arange(16))
    phi = (0.5 + 0.5 * np.tanh(2 * (5 - np.sqrt((x - 9.6) ** 2 + (y - 7.8) ** 2)) / 4.0))[None]
    st = om.run(p, om.init(p, phi), 200)
    assert abs(st.h.sum() - phi.sum()) < 1e-12 * phi.sum()


# ---------------------------------------------------------------- Liang2014 with its hydrodynamics
@pytest.mark.parametrize("lat", ["D2Q9_D2Q5", "D3Q19_D3Q7", "D3Q27_D3Q7"])
def test_liang14_force_moments(lat):
    """Eq. liang2_F with Gamma, s of Eq. Gamma_beta: sum F = u.grad rho,
    sum e F = F', sum e e F = (u.A) I + B u + u B - 3 (u.B) u u with
    A = grad(rho c_s^2), B = A + F' (lattice isotropy to fourth order)."""
    d3 = lat != "D2Q9_D2Q5"
    p = _p(lattice=lat, model="L14", nx=5, ny=4, nz=3 if d3 else 1)
    rng = np.random.default_rng(5)
    sh = p.shape
    rho = rng.uniform(1, 10, sh)
    u = rng.standard_normal((3,) + sh) * 0.05
    gr = rng.standard_normal((3,) + sh) * 0.3
    Fp = rng.standard_normal((3,) + sh) * 1e-3
    if not d3:
        u[2] = gr[2] = Fp[2] = 0
    m0, m1, m2 = _moments(p.lattices[0], om.force_liang14(p, Fp, u, rho, gr))
    A = CS2 * gr
    B = A + Fp
    uA = sum(u[a] * A[a] for a in range(3))
    uB = sum(u[a] * B[a] for a in range(3))
    assert np.abs(m0 - sum(u[a] * gr[a] for a in range(3))).max() < 1e-15
    assert np.abs(m1 - Fp).max() < 1e-15
    dim = 3 if d3 else 2
    for a in range(dim):
        for b in range(dim):
            ref = uA * (a == b) + B[a] * u[b] + B[b] * u[a] - 3 * uB * u[a] * u[b]
            assert np.abs(m2[a, b] - ref).max() < 1e-15


def test_liang14_velocity_solves_its_implicit_update():
    """rho u = sum e f + F'/2 with F' = F_s + F_a + F_b and F_a proportional to
    u (Eq. liang2014_velocity_update solved in closed form), on a droplet with
    a perturbed off-equilibrium state."""
    p = _p(model="L14", nx=24, ny=20, eta=1.0)
    x, y = np.meshgrid(np.arange(24), np.arange(20))
    phi = (0.5 + 0.5 * np.tanh(2 * (6 - np.sqrt((x - 11.3) ** 2 + (y - 9.6) ** 2)) / 4.0))[None]
    rng = np.random.default_rng(9)
    u0 = np.zeros((3,) + p.shape)
    u0[:2] = 0.02 * rng.standard_normal((2,) + p.shape)
    st = om.init(p, phi, u0)
    st.g = st.g + 1e-4 * rng.standard_normal(st.g.shape)
    m = om.macroscopic(p, st)
    gl = p.lattices[0]
    j = np.array([sum(gl.c[i][a] * st.g[i] for i in range(gl.Q)) for a in range(3)])
    assert np.abs(m["rho"] * m["u"] - j - 0.5 * m["F"]).max() < 1e-16
    assert np.abs(m["lap_mu"]).max() > 1e-6          # the F_a term is active


@pytest.mark.parametrize("lat", ["D2Q9_D2Q5", "D3Q19_D3Q7"])
def test_liang14_fixed_point_and_shear_wave(lat):
    d3 = lat != "D2Q9_D2Q5"
    p = _p(lattice=lat, model="L14", nx=5, ny=4, nz=3 if d3 else 1)
    st = om.init(p, np.full(p.shape, 0.4))
    st2 = om.run(p, st, 5)
    assert np.abs(st2.g - st.g).max() < 1e-16 and np.abs(st2.h - st.h).max() < 4e-15
    L_ = 32
    nu = 0.04
    p = _p(lattice=lat, model="L14", nx=4, ny=L_, nz=4 if d3 else 1, rho_H=1.0, rho_L=1.0,
           nu_H=nu, nu_L=nu, s_other=1.0 if d3 else 1.0 / (3 * nu + 0.5))
    k = 2 * np.pi / L_
    u = np.zeros((3,) + p.shape)
    u[0] = 1e-3 * np.sin(k * np.arange(L_))[None, :, None]
    st = om.run(p, om.init(p, np.full(p.shape, 1.0), u), 300)
    uu = om.fields(p, st)[1]
    amp = np.sum(uu[0][0, :, 0] * np.sin(k * np.arange(L_))) / (L_ / 2)
    assert abs(-np.log(amp / 1e-3) / 300 / (nu * k * k) - 1) < 0.01


@pytest.mark.parametrize("model", ["L18", "L14"])
def test_laplace_law_and_conservation(model):
    """Static droplet R = 10 (rho ratio 10), 2500 steps: Young-Laplace
    dp R / sigma = 1 within 8 % (measured 0.945 for Liang2018 and 0.992 for
    Liang2014, converging to 0.946 and 0.996); a surface force off by a factor
    moves it by that factor. sum phi kept."""
    p = _p(model=model, nx=64, ny=64)
    x, y = np.meshgrid(np.arange(64), np.arange(64))
    phi = (0.5 + 0.5 * np.tanh(2 * (10 - np.sqrt((x - 32) ** 2 + (y - 32) ** 2)) / p.W))[None]
    st = om.run(p, om.init(p, phi), 2500)
    assert abs(st.h.sum() - phi.sum()) < 1e-11 * phi.sum()
    d = om.diagnostics(p, st, centre=(32.0, 32.0), R=10.0)
    v = (d["p_in"] - d["p_out"]) * 10.0 / p.sigma
    assert abs(v - 1) < 0.08, v
