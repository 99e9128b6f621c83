"""The recording step (pflbm_step_record, _f32): one step that also writes the
state it starts from. The recorded state equals the canonical read-out
(pflbm_get_distributions, pflbm_get_phiu, pflbm_get_distributions_f32) taken
just before a plain step, bit for bit, and the state after it equals the
plain step's, for every model, on 2-D, D3Q19 and D3Q27 boxes with walls and
a ragged x extent over the 128 x 2 tile, in the float64 and float32 forms."""
import sys

import numpy as np
import pytest

from paper_2511_11360_amd import pflbm as P
from paper_2511_11360_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _params(lattice, model):
    d3 = lattice != "D2Q9_D2Q5"
    n = (131, 6, 5) if d3 else (70, 9, 1)
    moving = model in ("AC", "CH", "NL")
    d = wl.base_params(lattice=lattice, model=model, nx=n[0], ny=n[1], nz=n[2],
                       bc=("periodic", "wall", "periodic"), rho_H=3.0, rho_L=1.0, nu_H=0.05, nu_L=0.08,
                       M=0.05, W=2.5, sigma=0.01, visc_interp="mu")
    if moving:
        d["wall_u"] = ((-0.02, 0.0, 0.0), (0.02, 0.0, 0.0))
    if model == "NL":
        d["lam"] = 0.5
    x, y, z = wl.grid(d)
    phi = 0.5 + 0.4 * np.sin(2 * np.pi * (x + 0.3) / n[0]) * np.cos(2 * np.pi * (y + 0.2) / n[1])
    u = wl.zero_velocity(d)
    u[0] = 0.01 * np.cos(2 * np.pi * (y + 0.5) / n[1])
    return d, phi, u


CASES = [(lat, m) for lat in ("D2Q9_D2Q5", "D3Q19_D3Q7", "D3Q27_D3Q7") for m in ("AC", "CH", "NL", "L18", "L14")]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("lattice,model", CASES)
def test_recorded_state_is_the_read_out_and_the_step_is_the_plain_step(lattice, model, precision):
    import torch
    from paper_2511_11360_amd.solver import Solver
    _say("case record", lattice, model, precision)
    d, phi, u = _params(lattice, model)
    s1 = Solver(d, precision=precision)
    s2 = Solver(d, precision=precision)
    for s in (s1, s2):
        s.init(phi, u)
        s.step(3)
    ch = model in ("CH", "L18", "L14")
    for _ in range(2):
        g, h, pu = s1.step_record()
        g2, h2 = s2.get_distributions()
        assert torch.equal(g, g2) and torch.equal(h, h2)
        if ch:
            assert torch.equal(pu, s2.get_phiu())
        else:
            assert pu is None
        s2.step(1)
    a1, b1 = s1.get_distributions()
    a2, b2 = s2.get_distributions()
    assert torch.equal(a1, a2) and torch.equal(b1, b2)
    gf, hf, pf = s1.step_record(f32=True)
    g3, h3 = s2.get_distributions_f32()
    assert gf.dtype == torch.float32
    assert torch.equal(gf, g3) and torch.equal(hf, h3)
    if ch:
        assert torch.equal(pf, s2.get_phiu().float())
    else:
        assert pf is None


def test_record_refuses_the_16_bit_forms_and_null_outputs():
    import torch
    from paper_2511_11360_amd.solver import Solver
    d, phi, u = _params("D3Q19_D3Q7", "AC")
    s = Solver(d, precision="mixed_fp16")
    s.init(phi, u)
    with pytest.raises(P.PflbmError, match="float64 and float32 forms") as e:
        s.step_record()
    assert e.value.status == P.PFLBM_EUNSUPPORTED
    s.step(1)
    s = Solver(d, precision="fp64")
    s.init(phi, u)
    g = torch.empty((19,) + s.shape, dtype=torch.float64, device="cuda")
    with pytest.raises(P.PflbmError, match="null output") as e:
        s._check(s.L.pflbm_step_record(s.h, g.data_ptr(), None, None), s.h)
    assert e.value.status == P.PFLBM_EINVAL
    s.step(1)
