"""FP64 parity of the HIP path with the oracle: every distribution, element by
element, on the same seeded inputs, max |difference| <= 1e-12.

The two sides share no arithmetic; both start from the inputs of
paper_2511_11360_amd.workloads. Sizes cover several 64 x 4 tiles, ragged
x/y tails and a ragged last z block, walls, moving walls, gravity, the frozen
phase field, both phase-field models, and odd and even step counts (the state
then sits in one or the other of the two buffers of each distribution).
"""
import sys

import numpy as np
import pytest

from gpu_helpers import (gpu_dists, gpu_run, hydrostatic_p0, max_abs_per_population,
                         oracle_envelope, oracle_run, small_3d)
from oracle import model as om
from paper_2511_11360_amd import workloads as wl

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _parity(d, phi, u, steps, tag, p0=None):
    _say("case", tag, "shape", (d["nx"], d["ny"], d["nz"]), "steps", steps)
    s = gpu_run(d, phi, u, steps, p0=p0)
    g, h = gpu_dists(s)
    p, st = oracle_run(d, phi, u, steps, p0=p0)
    eg = max_abs_per_population(g, st.g)
    eh = max_abs_per_population(h, st.h)
    _say("  max|dg| %.3e max|dh| %.3e" % (eg.max(), eh.max()))
    assert np.all(np.isfinite(g)) and np.all(np.isfinite(h))
    assert eg.max() <= TOL, eg
    assert eh.max() <= TOL, eh
    return s, p, st


def test_static_droplet_2d_ac_1000():
    d, phi, u = wl.static_droplet_2d()
    _parity(d, phi, u, 1000, "static droplet 2-D AC")


def test_static_droplet_2d_ch_1000():
    d, phi, u = wl.static_droplet_2d()
    d["model"] = "CH"
    _parity(d, phi, u, 1000, "static droplet 2-D CH")


def test_rayleigh_taylor_walls_ragged_ch():
    d, phi, u = wl.rayleigh_taylor_2d(model="CH", nx=70, ny=90)
    _parity(d, phi, u, 1001, "RT 2-D walls CH")


def test_rayleigh_taylor_walls_ragged_ac_hydrostatic():
    """AC with gravity from a hydrostatic start (pressure input path), 1001
    steps, every distribution within 1e-12. With normal_eps = 1e-3 the layout
    is well conditioned: two oracle runs whose initial populations differ by
    one ulp stay within 1e-15 of each other over the 1001 steps."""
    d, phi, u = wl.rayleigh_taylor_2d(model="AC", nx=70, ny=90)
    d["normal_eps"] = 1e-3
    _parity(d, phi, u, 1001, "RT 2-D walls AC hydrostatic, normal_eps 1e-3", p0=hydrostatic_p0(d, phi))


def test_rayleigh_taylor_walls_ragged_ac_rest_start():
    """The Rayleigh-Taylor layout's own start (zero velocity, zero pressure),
    AC, 1001 steps, every distribution within 1e-12. With normal_eps = 1e-2 the
    acoustic start-up no longer amplifies rounding (oracle one-ulp spread
    7.5e-16 after 1001 steps)."""
    d, phi, u = wl.rayleigh_taylor_2d(model="AC", nx=70, ny=90)
    d["normal_eps"] = 1e-2
    _parity(d, phi, u, 1001, "RT 2-D walls AC rest start, normal_eps 1e-2")


def test_rayleigh_taylor_ac_default_normal_within_twice_the_oracle_spread():
    """With the default normal_eps = 1e-4 the RT layout is ill conditioned even
    from a hydrostatic start: phi overshoots 1 by 2e-5 in the heavy bulk, where
    the gradient is far below eps, and the antidiffusion flux there amplifies
    rounding (two oracle runs one ulp apart: 7e-13 in h after 101 steps, 5e-12
    after 301, 1e-7 after 1001). After 101 steps g must match to 1e-12 and h
    within 1e-12 plus twice that oracle-vs-oracle spread."""
    d, phi, u = wl.rayleigh_taylor_2d(model="AC", nx=70, ny=90)
    p0 = hydrostatic_p0(d, phi)
    steps = 101
    s = gpu_run(d, phi, u, steps, p0=p0)
    g, h = gpu_dists(s)
    eg_env, eh_env, st = oracle_envelope(d, phi, u, steps, p0=p0)
    eg = max_abs_per_population(g, st.g)
    eh = max_abs_per_population(h, st.h)
    _say("  RT AC hydrostatic 101: max|dg| %.3e max|dh| %.3e (oracle spread %.3e)"
         % (eg.max(), eh.max(), eh_env.max()))
    assert np.all(np.isfinite(g)) and np.all(np.isfinite(h))
    assert eg.max() <= TOL
    assert eh.max() <= TOL + 2 * eh_env.max()


def test_layered_poiseuille_frozen_phi():
    d, phi, u = wl.layered_poiseuille()
    _parity(d, phi, u, 1000, "layered Poiseuille")


def test_droplet_vortex_3d_ragged_ac_1000():
    d, phi, u = small_3d(model="AC")
    _parity(d, phi, u, 1000, "3-D vortex droplet AC")


def test_droplet_vortex_3d_ragged_ch():
    d, phi, u = small_3d(model="CH")
    _parity(d, phi, u, 301, "3-D vortex droplet CH")


@pytest.mark.parametrize("model", ["AC", "CH"])
def test_sheared_droplet_3d_moving_walls(model):
    d, phi, u, _ = wl.sheared_droplet_3d(n=24, R=7.0, uw=0.02, W=2.5)
    d["model"] = model
    d["ny"] = 22
    phi = wl.droplet_phi(d, (12.0, 10.5, 12.0), 7.0, periodic=False)
    x, y, z = wl.grid(d)
    u = wl.zero_velocity(d)
    u[0] = -0.02 + 0.04 * (y + 0.5) / 22
    _parity(d, phi, u, 301, "3-D sheared droplet " + model)


_TILE_CASES = {}


def _tile_cases():
    """The two tile-test cases with their oracle results (computed once)."""
    if not _TILE_CASES:
        d, phi, u = small_3d(nx=150, ny=26, nz=25)
        _TILE_CASES["periodic"] = (d, phi, u, 60, oracle_run(d, phi, u, 60)[1])
        d, phi, u, _ = wl.sheared_droplet_3d(n=24, R=7.0, uw=0.02, W=2.5)
        d["nx"], d["ny"] = 70, 22
        phi = wl.droplet_phi(d, (35.0, 10.5, 12.0), 7.0, periodic=False)
        x, y, z = wl.grid(d)
        u = wl.zero_velocity(d)
        u[0] = -0.02 + 0.04 * (y + 0.5) / 22
        _TILE_CASES["walls"] = (d, phi, u, 40, oracle_run(d, phi, u, 40)[1])
    return _TILE_CASES


@pytest.mark.parametrize("tile", ["64x4", "128x2", "256x1", "256x4", "128x8"])
def test_step_tiles(tile):
    """Every step-kernel tile shape against the oracle, in float64: a ragged
    periodic box (150 x 26 x 25: x and y tails in every shape, ragged last z
    block) and moving walls (70 x 22 x 24)."""
    # 256x4 and 128x8 are 1024 threads: float64 there runs with spilled
    # registers (slow, still exact); the automatic choice uses 256x4 for float32
    # and 16-bit g, 128x8 for Liang2014 with 16-bit g
    for name, (d, phi, u, steps, st) in _tile_cases().items():
        s = gpu_run(d, phi, u, steps, tile=tile, zblock=7)
        g, h = gpu_dists(s)
        eg = max_abs_per_population(g, st.g).max()
        eh = max_abs_per_population(h, st.h).max()
        _say("  tile %s %s: max|dg| %.3e max|dh| %.3e" % (tile, name, eg, eh))
        assert eg <= TOL and eh <= TOL


def test_zblock_and_s_other_variants():
    d, phi, u = small_3d(nx=30, ny=27, nz=23, s_other=1.2, visc_interp="nu", nu_H=0.03)
    for zb in (1, 5, 23):
        _say("zblock", zb)
        s = gpu_run(d, phi, u, 120, zblock=zb)
        g, h = gpu_dists(s)
        p, st = oracle_run(d, phi, u, 120)
        assert max_abs_per_population(g, st.g).max() <= TOL
        assert max_abs_per_population(h, st.h).max() <= TOL


@pytest.mark.parametrize("model", ["AC", "NL", "L18", "L14"])
@pytest.mark.parametrize("precision", ["fp64", "fp32", "mixed_fp16"])
def test_automatic_zblock_matches_fixed_depth(model, precision):
    """The automatic z-block depth changes only the launch grid. On the
    1024-thread 256 x 4 tile (one resident workgroup per compute unit) a
    40 x 128 x 50 box gets z blocks sized to one round over the compute units
    (7 planes on 256 units, the last block 1 plane); every population must
    equal the run with 5-plane blocks bit for bit, since each node takes the
    same arithmetic whatever block it falls in (Liang2014 included: its
    kernel forms mu_phi on each block's own halo). So must a single 50-plane
    block, whose march starts at a different plane in every workgroup and
    wraps around the periodic z axis."""
    d, phi, u = small_3d(nx=40, ny=128, nz=50, R=9.0, model=model)
    out = []
    for zb in (0, 5, 50):
        _say("  %s %s zblock %d" % (model, precision, zb))
        out.append(gpu_dists(gpu_run(d, phi, u, 60, precision=precision, tile="256x4", zblock=zb)))
    g0, h0 = out[0]
    for g1, h1 in out[1:]:
        assert np.array_equal(g0, g1) and np.array_equal(h0, h1)


def test_fields_and_diagnostics_match_oracle():
    d, phi, u = wl.static_droplet_2d()
    s = gpu_run(d, phi, u, 401)
    p, st = oracle_run(d, phi, u, 401)
    f_phi, f_u, f_p, f_rho = [t.cpu().numpy() for t in s.fields()]
    o_phi, o_u, o_p, o_rho = om.fields(p, st)
    assert np.max(np.abs(f_phi - o_phi)) < 1e-12
    assert np.max(np.abs(f_u - o_u)) < 1e-13
    assert np.max(np.abs(f_p - o_p)) < 1e-13
    assert np.max(np.abs(f_rho - o_rho)) < 1e-11
    dg = s.volume(centre=(32.0, 32.0), R=16.0)
    do = om.diagnostics(p, st, centre=(32.0, 32.0), R=16.0)
    for k in ("V_phi", "sum_phi"):
        assert abs(dg[k] - do[k]) < 1e-10 * abs(do[k])
    assert dg["V_count"] == do["V_count"]
    assert abs(dg["phi_min"] - do["phi_min"]) < 1e-12
    assert abs(dg["phi_max"] - do["phi_max"]) < 1e-12
    assert abs(dg["umax"] - do["umax"]) < 1e-13
    assert dg["n_in"] == do["n_in"] and dg["n_out"] == do["n_out"]
    assert abs(dg["p_in"] - do["p_in"]) < 1e-12 and abs(dg["p_out"] - do["p_out"]) < 1e-12
    assert dg["unstable"] == 0


def test_checkpoint_and_set_distributions_roundtrip():
    d, phi, u = small_3d(model="CH", nx=18, ny=9, nz=7)
    s = gpu_run(d, phi, u, 7)          # state in the second buffers
    ck = s.save_state()
    s.step(5)
    g1, h1 = gpu_dists(s)
    s.load_state(ck)
    assert s.step_count() == 7
    s.step(5)
    g2, h2 = gpu_dists(s)
    assert np.array_equal(g1, g2) and np.array_equal(h1, h2)
    # canonical read-out and write-back are inverse
    s.load_state(ck)
    g, h = gpu_dists(s)
    s.set_distributions(g, h)
    g3, h3 = gpu_dists(s)
    assert np.array_equal(g, g3) and np.array_equal(h, h3)


def test_set_distributions_at_moving_walls_continues_in_parity():
    """Canonical write-back next to moving walls (the wall term is removed on
    the way in and added back by the pull): read-out, write-back, 40 more steps
    against the oracle continued from the same canonical state."""
    d, phi, u, _ = wl.sheared_droplet_3d(n=24, R=7.0, uw=0.02, W=2.5)
    d["ny"] = 22
    phi = wl.droplet_phi(d, (12.0, 10.5, 12.0), 7.0, periodic=False)
    x, y, z = wl.grid(d)
    u = wl.zero_velocity(d)
    u[0] = -0.02 + 0.04 * (y + 0.5) / 22
    s = gpu_run(d, phi, u, 9)
    g, h = gpu_dists(s)
    s.set_distributions(g, h)
    g2, h2 = gpu_dists(s)
    assert np.abs(g2 - g).max() <= 4e-16 * np.abs(g).max() and np.array_equal(h, h2)
    p = om.Params(**d)
    st = om.State(g.copy(), h.copy())
    s.step(40)
    g3, h3 = gpu_dists(s)
    st = om.run(p, st, 40)
    assert max_abs_per_population(g3, st.g).max() <= TOL
    assert max_abs_per_population(h3, st.h).max() <= TOL


def test_oracle_state_injected_continues_in_parity():
    """Load the oracle's state at step 50 through the canonical ABI and continue
    (AC: the canonical distributions are the whole state)."""
    d, phi, u = wl.static_droplet_2d(n=48, R=12.0)
    p, st = oracle_run(d, phi, u, 51)
    s = gpu_run(d, phi, u, 0)
    s.set_distributions(st.g, st.h)
    s.step(100)
    g, h = gpu_dists(s)
    st2 = om.run(p, st, 100)
    assert max_abs_per_population(g, st2.g).max() <= TOL
    assert max_abs_per_population(h, st2.h).max() <= TOL


@pytest.mark.parametrize("model", ["AC", "CH", "NL"])
@pytest.mark.parametrize("precision", ["fp32", "mixed_fp16"])
def test_float_forms_conserve_phase_field_mass(model, precision):
    """Every model conserves sum phi exactly in exact arithmetic; the float32
    phase-field collision closes each node's balance on its last population, so
    the sum only takes unbiased rounding (without it the rounded weights add
    about 3e-8 / tau_phi of the mass per step: 5e-5 after 1000 steps here)."""
    d, phi, u = wl.static_droplet_2d()
    d["model"] = model
    s = gpu_run(d, phi, u, 1000, precision=precision)
    v = s.fields()[0].cpu().numpy().sum()
    drift = abs(v - phi.sum()) / phi.sum()
    _say("  %s %s: sum phi drift %.2e after 1000 steps" % (model, precision, drift))
    assert drift < 2e-6
