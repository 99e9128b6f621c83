"""Two solvers on two side streams (default priority), their steps and
adjoint steps launched interleaved without synchronisation in between, give
bit for bit the results of the same calls run one after the other on the
default stream: the library keeps no state across handles (the no-alloc
scratch aside), and the wrapper allocates on each solver's own stream."""
import numpy as np
import pytest

from paper_2511_11360_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _case(model, shift):
    d = wl.base_params(lattice="D3Q19_D3Q7", model=model, nx=70, ny=12, nz=10,
                       bc=("periodic", "wall", "periodic"), rho_H=3.0, rho_L=1.0, nu_H=0.05, nu_L=0.08,
                       M=0.05, W=2.5, sigma=0.01, visc_interp="mu")
    x, y, z = wl.grid(d)
    phi = 0.5 + 0.4 * np.sin(2 * np.pi * (x + shift) / 70) * np.cos(2 * np.pi * (y + 0.2) / 12)
    u = wl.zero_velocity(d)
    u[0] = 0.01 * np.cos(2 * np.pi * (y + 0.5) / 12)
    return d, phi, u


def _drive(solvers, rounds):
    """Steps and one adjoint step per solver and round, launched in turn; the
    test's own tensor work for a solver runs on that solver's stream."""
    import torch
    outs = []
    for s in solvers:
        with torch.cuda.stream(s.stream):
            outs.append({"work": s.adjoint_workspace(), "dp": torch.zeros(3, dtype=torch.float64, device="cuda")})
    for _ in range(rounds):
        for s, o in zip(solvers, outs):
            with torch.cuda.stream(s.stream):
                s.step(7)
                g, h, _ = s.step_record()
                lam = o.get("lam") or (torch.ones_like(g), torch.ones_like(h))
                og, oh = torch.empty_like(g), torch.empty_like(h)
                s.adjoint_step(g, h, lam[0], lam[1], og, oh, o["dp"], o["work"])
                o["lam"] = (og, oh)
    res = []
    for s, o in zip(solvers, outs):
        with torch.cuda.stream(s.stream):
            g, h = s.get_distributions()
            phi = s.fields()[0]
        res.append((g, h, phi, o["lam"][0], o["lam"][1], o["dp"]))
    return res


def test_side_streams_match_the_default_stream():
    import torch
    from paper_2511_11360_amd.solver import Solver
    cases = [_case("AC", 0.3), _case("AC", 0.7)]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    side = []
    for (d, phi, u), st in zip(cases, streams):
        s = Solver(d, precision="fp64", stream=st)
        s.init(phi, u)
        side.append(s)
    got = _drive(side, 5)
    for st in streams:
        st.synchronize()
    ref = []
    for d, phi, u in cases:
        s = Solver(d, precision="fp64")
        s.init(phi, u)
        ref.append(_drive([s], 5)[0])
    torch.cuda.synchronize()
    for a, b in zip(got, ref):
        for x, y in zip(a, b):
            assert torch.equal(x, y)
