"""Pins of the oracle's nonlocal / hybrid Allen-Cahn phase-field side (Sec.
II.C, Chai2018 and Hu2019; Eqs. nonlocalAC, lagrange_multiplier, Chai_geq,
chai_G, Hu_G, chai2018_phi_update).

What the mathematics fixes, independent of the oracle's code:
  - a uniform field is stationary (gamma cancels the bulk term exactly, so a
    wrong sign or scale of gamma moves it);
  - sum_x R = 0 for any field (definition of gamma) and, with it, sum_x phi is
    conserved by the scheme;
  - a planar slab with tanh profiles is a stationary solution of the nonlocal
    AC equation (gamma = 0 by symmetry; the bulk term balances the Laplacian for
    the tanh of width W), so the discrete profile stays within the scheme's
    discretisation error of it (a bulk term off by 2 leaves it by 5x more);
  - the nonlocal multiplier coarsens: of two droplets the smaller loses volume
    to the larger, the total kept (Sec. IV results on volume transfer between
    droplets), while the conservative AC model leaves both nearly unchanged;
  - moments of the hybrid source: sum_a G_a = (1 - lam) R and
    sum_a e_a G_a = lam x the conservative flux.
"""
import numpy as np
import pytest

from oracle import model as om


def _p(**kw):
    d = dict(lattice="D2Q9_D2Q5", model="NL", nx=64, ny=64, rho_H=1.0, rho_L=1.0,
             nu_H=0.1, nu_L=0.1, M=0.02, W=4.0, sigma=0.01)
    d.update(kw)
    return om.Params(**d)


@pytest.mark.parametrize("lattice", ["D2Q9_D2Q5", "D3Q19_D3Q7"])
def test_uniform_field_is_stationary(lattice):
    p = _p(lattice=lattice, nx=6, ny=5, nz=4 if lattice.startswith("D3") else 1, lam=0.3)
    st = om.init(p, np.full(p.shape, 0.3))
    m = om.macroscopic(p, st)
    # gamma = (32 / W^2)(phi - 1) phi (phi - 1/2) / ((1 - phi) phi) = -(32 / W^2)(phi - 1/2)
    assert abs(m["gamma"] - (-(32.0 / 16.0) * (0.3 - 0.5))) < 1e-15
    assert np.abs(m["R"]).max() < 1e-17
    st2 = om.run(p, st, 4)
    assert np.abs(st2.h - st.h).max() < 1e-16 and np.abs(st2.g - st.g).max() < 1e-16


def test_source_sums_to_zero_and_phi_is_conserved():
    p = _p(nx=40, ny=36, lam=0.0)
    rng = np.random.default_rng(7)
    phi = rng.uniform(0.0, 1.0, size=p.shape)
    R, gamma = om.nonlocal_source(p, phi)
    assert abs(R.sum()) < 1e-15 * np.abs(R).sum() * 10
    # droplet, 300 steps: sum of phi (= sum of the corrected phi) is invariant
    x, y = np.meshgrid(np.arange(40), np.arange(36))
    phi0 = (0.5 + 0.5 * np.tanh(2 * (9 - np.sqrt((x - 17.3) ** 2 + (y - 18.1) ** 2)) / p.W))[None]
    for lam in (0.0, 0.9):
        q = _p(nx=40, ny=36, lam=lam)
        st = om.run(q, om.init(q, phi0), 300)
        assert abs(st.h.sum() - phi0.sum()) < 1e-12 * phi0.sum()
        assert abs(om.fields(q, st)[0].sum() - phi0.sum()) < 1e-12 * phi0.sum()


@pytest.mark.parametrize("lam", [0.0, 0.9])
def test_planar_slab_stays_near_the_tanh_profile(lam):
    p = _p(nx=64, ny=4, lam=lam)
    x = np.arange(64)[None, None, :] * np.ones(p.shape)
    phi0 = 0.5 + 0.5 * np.tanh(2 * (16 - np.abs(x - 31.5)) / p.W)
    st = om.init(p, phi0)
    assert abs(om.macroscopic(p, st)["gamma"]) < 1e-13
    st = om.run(p, st, 500)
    dev = np.abs(om.fields(p, st)[0] - phi0).max()
    # measured 0.012 (lam 0) / 0.007 (lam 0.9); a bulk term twice too large: 0.058
    assert dev < 0.02


def test_nonlocal_multiplier_coarsens_two_droplets():
    x, y = np.meshgrid(np.arange(100), np.arange(64))
    drop = lambda cx, r: 0.5 + 0.5 * np.tanh(2 * (r - np.sqrt((x - cx) ** 2 + (y - 32) ** 2)) / 4.0)
    phi0 = np.maximum(drop(20, 8.0), drop(70, 14.0))[None]
    out = {}
    for model in ("NL", "AC"):
        p = _p(nx=100, ny=64, model=model)
        f = om.fields(p, om.run(p, om.init(p, phi0), 1000))[0][0]
        out[model] = (f[:, :45].sum() - phi0[0][:, :45].sum(), f[:, 45:].sum() - phi0[0][:, 45:].sum())
    small, large = out["NL"]
    v_small = phi0[0][:, :45].sum()
    assert small < -0.15 * v_small and large > 0      # volume moves to the larger droplet
    assert abs(small + large) < 1e-9 * phi0.sum()      # total kept
    assert max(abs(v) for v in out["AC"]) < 0.01 * v_small


@pytest.mark.parametrize("lam", [0.0, 0.35, 1.0])
def test_hybrid_source_moments(lam):
    """sum_a G_a = (1 - lam) R and sum_a e_a G_a = lam (flux of the conservative
    model), through the collision: G = (h* - h + (h - h_eq)/tau_phi) / (1 - 1/(2 tau_phi))."""
    p = _p(nx=24, ny=20, lam=lam)
    x, y = np.meshgrid(np.arange(24), np.arange(20))
    phi0 = (0.5 + 0.5 * np.tanh(2 * (6 - np.sqrt((x - 11.2) ** 2 + (y - 9.7) ** 2)) / p.W))[None]
    rng = np.random.default_rng(3)
    u0 = np.zeros((3,) + p.shape)
    u0[:2] = 0.01 * rng.standard_normal((2,) + p.shape)
    st = om.init(p, phi0, u0)
    st.h = st.h * (1 + 1e-3 * rng.standard_normal(st.h.shape))   # off equilibrium
    m = om.macroscopic(p, st)
    tp = om.tau_phi(p)
    G = (om.collide_h(p, st, m) - st.h + (st.h - om.h_eq_nl(p, m["phi"], m["u"])) / tp) / (1 - 1 / (2 * tp))
    hl = p.lattices[1]
    # G is recovered from h* - h (h ~ 0.2): rounding ~1e-15; R itself is ~1e-5
    assert np.abs(G.sum(axis=0) - (1 - lam) * m["R"]).max() < 2e-14
    Gac = om.G_ac(p, m["phi"], m["grad"])
    for a in range(2):
        first = sum(hl.c[k][a] * G[k] for k in range(hl.Q))
        ref = lam * sum(hl.c[k][a] * Gac[k] for k in range(hl.Q))
        assert np.abs(first - ref).max() < 2e-14
    # h_eq of Eq. Chai_geq: zeroth moment phi, first moment phi u
    heq = om.h_eq_nl(p, m["phi"], m["u"])
    assert np.abs(heq.sum(axis=0) - m["phi"]).max() < 1e-15
    for a in range(2):
        assert np.abs(sum(hl.c[k][a] * heq[k] for k in range(hl.Q)) - m["phi"] * m["u"][a]).max() < 1e-16


def test_block_step_with_the_box_multiplier_matches_the_box():
    """Locality with the multiplier supplied: apart from gamma, the next state
    at a node depends on the state within two nodes (streaming one, the phi
    stencil one more). A periodic 5^3 block cut around a node of a 3-D box and
    stepped with the box's gamma must reproduce the box's step at its centre;
    with the block's own sums in place of gamma it must not (the sums of Eq.
    lagrange_multiplier span the whole box)."""
    n = 12
    p = om.Params(lattice="D3Q19_D3Q7", model="NL", nx=n, ny=n, nz=n, rho_H=5.0, rho_L=1.0,
                  nu_H=0.05, nu_L=0.05, M=0.05, W=3.0, sigma=0.01, lam=0.5)
    z, y, x = np.meshgrid(*(np.arange(n),) * 3, indexing="ij")
    r = np.sqrt((x - 5.3) ** 2 + (y - 6.1) ** 2 + (z - 5.7) ** 2)
    st = om.run(p, om.init(p, 0.5 + 0.5 * np.tanh(2 * (3.5 - r) / p.W)), 3)
    gamma = om.macroscopic(p, st)["gamma"]
    full = om.step(p, st)
    pb = om.Params(**dict(p.__dict__, nx=5, ny=5, nz=5, gamma_given=gamma))
    pb_own = om.Params(**dict(p.__dict__, nx=5, ny=5, nz=5))
    own_err = 0.0
    for (cz, cy, cx) in [(5, 6, 6), (0, 11, 3), (8, 2, 9)]:
        idx = np.ix_(*(np.arange(c - 2, c + 3) % n for c in (cz, cy, cx)))
        blk = om.State(st.g[(slice(None),) + idx], st.h[(slice(None),) + idx])
        out = om.step(pb, blk)
        assert np.abs(out.g[:, 2, 2, 2] - full.g[:, cz, cy, cx]).max() < 1e-15
        assert np.abs(out.h[:, 2, 2, 2] - full.h[:, cz, cy, cx]).max() < 1e-15
        own = om.step(pb_own, blk)
        own_err = max(own_err, np.abs(own.h[:, 2, 2, 2] - full.h[:, cz, cy, cx]).max())
    assert own_err > 1e-8
