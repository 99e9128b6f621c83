"""Liang2018 (Sec. II.C: conservative AC with its conservative-form
hydrodynamics) on the HIP path against the oracle: float64 distributions
element by element (<= 1e-12) on D2Q9 and both 3-D lattices, every tile,
stationary walls with gravity (hydrostatic start), the frozen phase field
with a force density, two MRT rates, fields and diagnostics, checkpoints;
conservation and error bounds of the reduced forms. Cases are well
conditioned (two oracle runs one ulp apart stay within 2e-15)."""
import sys

import numpy as np
import pytest

from gpu_helpers import (gpu_dists, gpu_run, hydrostatic_p0, max_abs_per_population,
                         oracle_run, small_3d)
from oracle import model as om
from paper_2511_11360_amd import workloads as wl

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _check(d, phi, u, steps, tag, p0=None, **kw):
    _say("case", tag, "shape", (d["nx"], d["ny"], d["nz"]), "steps", steps, kw)
    s = gpu_run(d, phi, u, steps, p0=p0, **kw)
    g, h = gpu_dists(s)
    p, st = oracle_run(d, phi, u, steps, p0=p0)
    eg = max_abs_per_population(g, st.g).max()
    eh = max_abs_per_population(h, st.h).max()
    _say("  max|dg| %.3e max|dh| %.3e" % (eg, eh))
    assert np.all(np.isfinite(g)) and np.all(np.isfinite(h))
    assert eg <= TOL and eh <= TOL
    return s, p, st


def test_liang_static_droplet_2d_1000_fields_and_diagnostics():
    d, phi, u = wl.static_droplet_2d()
    d["model"] = "L18"
    s, p, st = _check(d, phi, u, 1000, "static droplet 2-D Liang2018")
    f_phi, f_u, f_p, f_rho = [a.cpu().numpy() for a in s.fields()]
    o_phi, o_u, o_p, o_rho = om.fields(p, st)
    assert np.abs(f_phi - o_phi).max() <= TOL and np.abs(f_u - o_u).max() <= TOL
    # rho = rho_L + (rho_H - rho_L) phi carries phi's difference times 9: relative bound
    assert np.abs(f_p - o_p).max() <= TOL and np.abs(f_rho - o_rho).max() <= TOL * d["rho_H"]
    dg, do = s.volume(centre=(32.0, 32.0), R=16.0), om.diagnostics(p, st, centre=(32.0, 32.0), R=16.0)
    assert abs(dg["p_in"] - do["p_in"]) <= TOL and abs(dg["p_out"] - do["p_out"]) <= TOL


def test_liang_rayleigh_taylor_walls_hydrostatic():
    d, phi, u = wl.rayleigh_taylor_2d(model="L18", nx=70, ny=90)
    _check(d, phi, u, 301, "RT 2-D walls Liang2018 hydrostatic", p0=hydrostatic_p0(d, phi))


def test_liang_layered_poiseuille_frozen_phi():
    d, phi, u = wl.layered_poiseuille()
    d["model"] = "L18"
    _check(d, phi, u, 1000, "layered Poiseuille Liang2018")


@pytest.mark.parametrize("lattice,tile", [("D3Q19_D3Q7", "auto"), ("D3Q19_D3Q7", "256x1"),
                                          ("D3Q27_D3Q7", "128x2")])
def test_liang_3d_vortex_droplet(lattice, tile):
    d, phi, u = small_3d(model="L18", lattice=lattice, s_other=1.3)
    _check(d, phi, u, 300, "3-D vortex droplet Liang2018 " + lattice, tile=tile, zblock=5)


def test_liang_3d_stationary_walls_checkpoint():
    d, phi, u, _ = wl.sheared_droplet_3d(n=24, R=7.0, uw=0.02, W=2.5)
    d["model"], d["ny"], d["rho_H"] = "L18", 22, 5.0
    d["wall_u"] = ((0.0, 0.0, 0.0), (0.0, 0.0, 0.0))
    phi = wl.droplet_phi(d, (12.0, 10.5, 12.0), 7.0, periodic=False)
    x, y, z = wl.grid(d)
    u = wl.zero_velocity(d)
    u[0] = 0.02 * np.sin(np.pi * (y + 0.5) / 22)
    s, p, st = _check(d, phi, u, 201, "3-D walled droplet Liang2018")
    ck = s.save_state()
    s.step(10)
    g1, h1 = gpu_dists(s)
    s.load_state(ck)
    s.step(10)
    g2, h2 = gpu_dists(s)
    assert np.array_equal(g1, g2) and np.array_equal(h1, h2)


@pytest.mark.parametrize("precision", ["fp32", "mixed_fp16", "mixed_bf16"])
def test_liang_reduced_forms(precision):
    d, phi, u = small_3d(model="L18")
    ref = gpu_run(d, phi, u, 400)
    s = gpu_run(d, phi, u, 400, precision=precision)
    fr = [a.cpu().numpy() for a in ref.fields()]
    fs = [a.cpu().numpy() for a in s.fields()]
    e_phi = np.linalg.norm(fs[0] - fr[0]) / np.linalg.norm(fr[0])
    e_u = np.linalg.norm(fs[1] - fr[1]) / np.linalg.norm(fr[1])
    drift = abs(fs[0].sum() - phi.sum()) / phi.sum()
    _say("  Liang2018 %s: rel L2 phi %.2e u %.2e, sum phi drift %.2e" % (precision, e_phi, e_u, drift))
    assert drift < 2e-6
    bound = {"fp32": (1e-4, 1e-4), "mixed_fp16": (1e-4, 2e-3), "mixed_bf16": (1e-2, 3e-2)}[precision]
    assert e_phi < bound[0] and e_u < bound[1]


def test_liang_rejects_moving_walls_and_fp16_range():
    from paper_2511_11360_amd import pflbm as P
    import ctypes
    d, phi, u, _ = wl.sheared_droplet_3d(n=24, R=7.0, uw=0.02, W=2.5)
    d["model"] = "L18"
    n = ctypes.c_size_t()
    assert P.lib().pflbm_state_bytes(ctypes.byref(P.make_params(d)), ctypes.byref(n)) == P.PFLBM_EINVAL
    d2 = wl.base_params(model="L18", rho_H=100.0)
    assert P.lib().pflbm_state_bytes(ctypes.byref(P.make_params(d2, "mixed_fp16")), ctypes.byref(n)) == P.PFLBM_EINVAL
    assert P.lib().pflbm_state_bytes(ctypes.byref(P.make_params(d2, "mixed_bf16")), ctypes.byref(n)) == 0


# ---------------------------------------------------------------- Liang2014 with its hydrodynamics
def test_liang14_static_droplet_2d_1000_fields():
    d, phi, u = wl.static_droplet_2d()
    d["model"] = "L14"
    s, p, st = _check(d, phi, u, 1000, "static droplet 2-D Liang2014")
    f_phi, f_u, f_p, f_rho = [a.cpu().numpy() for a in s.fields()]
    o_phi, o_u, o_p, o_rho = om.fields(p, st)
    assert np.abs(f_phi - o_phi).max() <= TOL and np.abs(f_u - o_u).max() <= TOL
    assert np.abs(f_p - o_p).max() <= TOL
    dg, do = s.volume(centre=(32.0, 32.0), R=16.0), om.diagnostics(p, st, centre=(32.0, 32.0), R=16.0)
    assert abs(dg["p_in"] - do["p_in"]) <= TOL and abs(dg["p_out"] - do["p_out"]) <= TOL


def test_liang14_rayleigh_taylor_walls():
    d, phi, u = wl.rayleigh_taylor_2d(model="L14", nx=70, ny=90)
    _check(d, phi, u, 501, "RT 2-D walls Liang2014")


@pytest.mark.parametrize("lattice,tile,steps", [("D3Q19_D3Q7", "auto", 300), ("D3Q19_D3Q7", "256x1", 300),
                                                ("D3Q19_D3Q7", "256x4", 300), ("D3Q19_D3Q7", "128x8", 300),
                                                ("D3Q27_D3Q7", "128x2", 200)])
def test_liang14_3d_vortex_droplet(lattice, tile, steps):
    d, phi, u = small_3d(model="L14", lattice=lattice, s_other=1.3)
    _check(d, phi, u, steps, "3-D vortex droplet Liang2014 " + lattice, tile=tile, zblock=5)


@pytest.mark.parametrize("precision", ["fp32", "mixed_fp16"])
def test_liang14_reduced_forms(precision):
    d, phi, u = small_3d(model="L14")
    ref = gpu_run(d, phi, u, 400)
    s = gpu_run(d, phi, u, 400, precision=precision)
    fr = [a.cpu().numpy() for a in ref.fields()]
    fs = [a.cpu().numpy() for a in s.fields()]
    e_phi = np.linalg.norm(fs[0] - fr[0]) / np.linalg.norm(fr[0])
    e_u = np.linalg.norm(fs[1] - fr[1]) / np.linalg.norm(fr[1])
    drift = abs(fs[0].sum() - phi.sum()) / phi.sum()
    _say("  Liang2014 %s: rel L2 phi %.2e u %.2e, sum phi drift %.2e" % (precision, e_phi, e_u, drift))
    assert drift < 2e-6
    assert e_phi < 1e-4 and e_u < (1e-4 if precision == "fp32" else 2e-3)
