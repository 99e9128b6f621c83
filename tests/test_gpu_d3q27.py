"""D3Q27 hydrodynamics (the paper's own 3-D lattice, Sec. IV) with the D3Q7
phase field on the HIP path against the oracle: float64 distributions element
by element (<= 1e-12) for the three phase-field models, every step tile,
moving walls, fields and diagnostics, canonical I/O; conservation and error
bounds of the reduced forms. Cases are well conditioned (two oracle runs one
ulp apart stay within 2e-15 over the steps used)."""
import sys

import numpy as np
import pytest

from gpu_helpers import gpu_dists, gpu_run, max_abs_per_population, oracle_run, small_3d
from oracle import model as om
from paper_2511_11360_amd import workloads as wl

pytestmark = pytest.mark.gpu

TOL = 1e-12
LAT = "D3Q27_D3Q7"


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _check(d, phi, u, steps, tag, **kw):
    _say("case", tag, "shape", (d["nx"], d["ny"], d["nz"]), "steps", steps, kw)
    s = gpu_run(d, phi, u, steps, **kw)
    g, h = gpu_dists(s)
    assert g.shape[0] == 27
    p, st = oracle_run(d, phi, u, steps)
    eg = max_abs_per_population(g, st.g).max()
    eh = max_abs_per_population(h, st.h).max()
    _say("  max|dg| %.3e max|dh| %.3e" % (eg, eh))
    assert np.all(np.isfinite(g)) and np.all(np.isfinite(h))
    assert eg <= TOL and eh <= TOL
    return s, p, st


def _sheared(model):
    d, phi, u, _ = wl.sheared_droplet_3d(n=24, R=7.0, uw=0.02, W=2.5)
    d["lattice"], d["model"], d["ny"] = LAT, model, 22
    phi = wl.droplet_phi(d, (12.0, 10.5, 12.0), 7.0, periodic=False)
    x, y, z = wl.grid(d)
    u = wl.zero_velocity(d)
    u[0] = -0.02 + 0.04 * (y + 0.5) / 22
    return d, phi, u


@pytest.mark.parametrize("model,tile", [("AC", "auto"), ("CH", "128x2"), ("NL", "256x1")])
def test_d3q27_vortex_droplet_ragged(model, tile):
    d, phi, u = small_3d(model=model, lattice=LAT, s_other=1.3)
    s, p, st = _check(d, phi, u, 300, "D3Q27 vortex droplet " + model, tile=tile, zblock=5)
    if model == "AC":
        f_phi, f_u, f_p, f_rho = [a.cpu().numpy() for a in s.fields()]
        o_phi, o_u, o_p, o_rho = om.fields(p, st)
        assert np.abs(f_phi - o_phi).max() <= TOL and np.abs(f_u - o_u).max() <= TOL
        assert np.abs(f_p - o_p).max() <= TOL
        dg, do = s.volume(), om.diagnostics(p, st)
        assert abs(dg["sum_phi"] - do["sum_phi"]) <= 1e-12 * do["sum_phi"]
        assert dg["V_count"] == do["V_count"]


@pytest.mark.parametrize("model", ["AC", "CH"])
def test_d3q27_sheared_droplet_moving_walls(model):
    d, phi, u = _sheared(model)
    _check(d, phi, u, 301, "D3Q27 sheared droplet " + model)


def test_d3q27_canonical_write_back_and_checkpoint():
    d, phi, u = _sheared("AC")
    s = gpu_run(d, phi, u, 7)
    ck = s.save_state()
    g, h = gpu_dists(s)
    s.set_distributions(g, h)
    g2, h2 = gpu_dists(s)
    assert np.abs(g2 - g).max() <= 4e-16 * np.abs(g).max() and np.array_equal(h, h2)
    s.step(20)
    g3, h3 = gpu_dists(s)
    s.load_state(ck)
    s.step(20)
    g4, h4 = gpu_dists(s)
    assert np.array_equal(g3, g4) and np.array_equal(h3, h4)
    st = om.run(om.Params(**d), om.State(g.copy(), h.copy()), 20)
    assert max_abs_per_population(g3, st.g).max() <= TOL
    assert max_abs_per_population(h3, st.h).max() <= TOL


@pytest.mark.parametrize("precision", ["fp32", "mixed_fp16"])
def test_d3q27_reduced_forms(precision):
    d, phi, u = small_3d(lattice=LAT)
    ref = gpu_run(d, phi, u, 400)
    s = gpu_run(d, phi, u, 400, precision=precision)
    fr = [a.cpu().numpy() for a in ref.fields()]
    fs = [a.cpu().numpy() for a in s.fields()]
    e_phi = np.linalg.norm(fs[0] - fr[0]) / np.linalg.norm(fr[0])
    e_u = np.linalg.norm(fs[1] - fr[1]) / np.linalg.norm(fr[1])
    drift = abs(fs[0].sum() - phi.sum()) / phi.sum()
    _say("  D3Q27 %s: rel L2 phi %.2e u %.2e, sum phi drift %.2e" % (precision, e_phi, e_u, drift))
    assert drift < 2e-6
    assert e_phi < 1e-4 and e_u < (1e-4 if precision == "fp32" else 2e-3)
