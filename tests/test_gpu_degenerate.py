"""Degenerate boxes against the oracle, float64, every model: boxes one or two
nodes wide along some axes (every neighbour of a node along such an axis is
the node itself or its one partner), on the three lattice pairs, periodic or
with walls, in the automatic launch configuration and in the 1024-thread
tiles (a 256- or 128-wide tile over a 1-5 node wide box: all but a few lanes
idle, all halo positions wrapped or clamped). Oracle one-ulp spread on these
cases after 40 steps: at most 6e-16."""
import sys

import numpy as np
import pytest

from gpu_helpers import gpu_dists, gpu_run, max_abs_per_population, oracle_run
from paper_2511_11360_amd import workloads as wl

pytestmark = pytest.mark.gpu

TOL = 1e-12
STEPS = 40

CASES = [
    ("D3Q19_D3Q7", (1, 1, 1), ("periodic", "periodic", "periodic")),
    ("D3Q19_D3Q7", (1, 3, 2), ("periodic", "periodic", "periodic")),
    ("D3Q19_D3Q7", (3, 1, 4), ("periodic", "periodic", "periodic")),
    ("D3Q19_D3Q7", (5, 2, 3), ("periodic", "wall", "periodic")),
    ("D3Q27_D3Q7", (2, 3, 1), ("periodic", "periodic", "periodic")),
    ("D2Q9_D2Q5", (1, 1, 1), ("periodic", "periodic", "periodic")),
    ("D2Q9_D2Q5", (1, 6, 1), ("periodic", "wall", "periodic")),
]


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _case(lattice, n, bc, model):
    nx, ny, nz = n
    d = wl.base_params(lattice=lattice, model=model, nx=nx, ny=ny, nz=nz, bc=bc, rho_H=3.0, rho_L=1.0,
                       nu_H=0.05, nu_L=0.08, M=0.05, W=2.5, sigma=0.01, gravity=(0.0, -1e-5, 0.0))
    if model == "NL":
        d["lam"] = 0.5
    x, y, z = wl.grid(d)
    phi = 0.5 + 0.3 * (np.sin(2 * np.pi * (x + 0.3) / nx) * np.cos(2 * np.pi * (y + 0.2) / ny)
                       * np.cos(2 * np.pi * (z + 0.1) / nz))
    u = wl.zero_velocity(d)
    u[0] = 0.01 * np.cos(2 * np.pi * y / ny)
    return d, phi, u


@pytest.mark.parametrize("model", ["AC", "CH", "NL", "L18", "L14"])
@pytest.mark.parametrize("lattice,n,bc", CASES)
def test_degenerate_box_matches_oracle(lattice, n, bc, model):
    d, phi, u = _case(lattice, n, bc, model)
    _, st = oracle_run(d, phi, u, STEPS)
    tiles = ["auto"] if lattice == "D2Q9_D2Q5" else ["auto", "256x4", "128x8"]
    for tile in tiles:
        _say("  %s %s %s %s tile %s" % (lattice, n, bc[1], model, tile))
        s = gpu_run(d, phi, u, STEPS, tile=tile)
        g, h = gpu_dists(s)
        eg = max_abs_per_population(g, st.g).max()
        eh = max_abs_per_population(h, st.h).max()
        assert eg <= TOL and eh <= TOL, (tile, eg, eh)


def test_zero_steps_leave_the_initial_state():
    """step(0) is a no-op: the distributions stay those of the initialisation."""
    d, phi, u = _case("D3Q19_D3Q7", (3, 1, 4), ("periodic", "periodic", "periodic"), "CH")
    _, st = oracle_run(d, phi, u, 0)
    s = gpu_run(d, phi, u, 0)
    s.step(0)
    g, h = gpu_dists(s)
    assert max_abs_per_population(g, st.g).max() <= TOL
    assert max_abs_per_population(h, st.h).max() <= TOL
    assert s.step_count() == 0
