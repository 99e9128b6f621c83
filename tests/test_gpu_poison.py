"""Unwritten memory stays unread: every buffer the library writes before it
reads (the caller-owned state, the adjoint workspace, the adjoint and
recording outputs) is filled with 0xFF bytes (a NaN in float64, float32,
fp16 and bf16) before use, and the results must equal, bit for bit, those of
the same calls on zero-filled buffers. A kernel that read a slot nobody wrote
(padding of a population plane, a partial-sum slot, a halo cell, an output
element it does not cover) would carry the NaN into the result.

Boxes: 2-D 70 x 9, 3-D 131 x 6 x 5 with walls on y (ragged against every
tile), D3Q19 and D3Q27; every model and storage form."""
import sys

import numpy as np
import pytest

from paper_2511_11360_amd import workloads as wl

pytestmark = pytest.mark.gpu

MODELS = ["AC", "CH", "NL", "L18", "L14"]


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _params(lattice, model):
    d3 = lattice != "D2Q9_D2Q5"
    n = (131, 6, 5) if d3 else (70, 9, 1)
    d = wl.base_params(lattice=lattice, model=model, nx=n[0], ny=n[1], nz=n[2],
                       bc=("periodic", "wall", "periodic"), rho_H=3.0, rho_L=1.0, nu_H=0.05, nu_L=0.08,
                       M=0.05, W=2.5, sigma=0.01, visc_interp="mu")
    if model in ("AC", "CH", "NL"):
        d["wall_u"] = ((-0.02, 0.0, 0.0), (0.02, 0.0, 0.0))
    if model == "NL":
        d["lam"] = 0.5
    x, y, z = wl.grid(d)
    phi = 0.5 + 0.4 * np.sin(2 * np.pi * (x + 0.3) / n[0]) * np.cos(2 * np.pi * (y + 0.2) / n[1])
    u = wl.zero_velocity(d)
    u[0] = 0.01 * np.cos(2 * np.pi * (y + 0.5) / n[1])
    return d, phi, u


def _state_bytes(d, precision):
    import ctypes
    from paper_2511_11360_amd import pflbm as P
    p = P.make_params(dict(d), precision, 0, 0, "auto")
    nb = ctypes.c_size_t()
    assert P.lib().pflbm_state_bytes(ctypes.byref(p), ctypes.byref(nb)) == 0
    return nb.value


def _run(d, phi, u, precision, fill):
    import torch
    from paper_2511_11360_amd.solver import Solver
    buf = torch.full((_state_bytes(d, precision),), fill, dtype=torch.uint8, device="cuda")
    s = Solver(d, precision=precision, state=buf)
    s.init(phi, u)
    s.step(5)
    g, h = s.get_distributions()
    f = s.fields()
    v = s.volume()
    return s, g, h, f, v


@pytest.mark.parametrize("precision", ["fp64", "fp32", "mixed_fp16", "mixed_bf16"])
@pytest.mark.parametrize("lattice", ["D2Q9_D2Q5", "D3Q19_D3Q7", "D3Q27_D3Q7"])
def test_poisoned_state_buffer_changes_nothing(lattice, precision):
    import torch
    for model in MODELS:
        _say("case poison state", lattice, model, precision)
        d, phi, u = _params(lattice, model)
        _, g0, h0, f0, v0 = _run(d, phi, u, precision, 0)
        _, g1, h1, f1, v1 = _run(d, phi, u, precision, 255)
        assert torch.isfinite(g1).all() and torch.isfinite(h1).all()
        assert torch.equal(g0, g1) and torch.equal(h0, h1)
        for a, b in zip(f0, f1):
            assert torch.equal(a, b)
        # diagnostics: equal, NaN where both are NaN (no pressure regions asked)
        for k in v0:
            assert v0[k] == v1[k] or (np.isnan(v0[k]) and np.isnan(v1[k])), k


@pytest.mark.parametrize("lattice", ["D2Q9_D2Q5", "D3Q19_D3Q7", "D3Q27_D3Q7"])
@pytest.mark.parametrize("model", MODELS)
def test_poisoned_adjoint_workspace_and_outputs_change_nothing(lattice, model):
    import torch
    from paper_2511_11360_amd.solver import Solver
    _say("case poison adjoint", lattice, model)
    d, phi, u = _params(lattice, model)
    s = Solver(d, precision="fp64")
    s.init(phi, u)
    s.step(3)
    ch = model in ("CH", "L18", "L14")
    g, h, pu = s.step_record()
    gen = torch.Generator(device="cuda").manual_seed(2)
    lg = torch.randn(g.shape, dtype=torch.float64, device="cuda", generator=gen)
    lh = torch.randn(h.shape, dtype=torch.float64, device="cuda", generator=gen)
    lpu = torch.randn((3,) + s.shape, dtype=torch.float64, device="cuda", generator=gen) if ch else None
    res = []
    for fill in (0, 255):
        work = s.adjoint_workspace().fill_(fill)
        og = torch.empty_like(g).view(torch.uint8).fill_(fill).view(torch.float64)
        oh = torch.empty_like(h).view(torch.uint8).fill_(fill).view(torch.float64)
        dp = torch.zeros(3, dtype=torch.float64, device="cuda")
        if ch:
            opu = torch.empty_like(lpu).view(torch.uint8).fill_(fill).view(torch.float64)
            s.adjoint_step_pu(g, h, pu, lg, lh, lpu, og, oh, opu, dp, work)
            d0 = s.adjoint_init_pu(phi, u, None, og, oh, opu, dp, work)
            res.append((og, oh, opu, dp, d0))
        else:
            s.adjoint_step(g, h, lg, lh, og, oh, dp, work)
            if model == "NL":
                seed = s.adjoint_seed(h, torch.ones(s.shape, dtype=torch.float64, device="cuda"), dp, work)
                d0 = s.adjoint_init(phi, u, None, og, oh)
                res.append((og, oh, dp, d0) + seed)
            else:
                d0 = s.adjoint_init(phi, u, None, og, oh)
                res.append((og, oh, dp, d0))
    for a, b in zip(*res):
        assert torch.isfinite(b).all()
        assert torch.equal(a, b)
    if model == "AC":
        out = []
        g32, h32, _ = s.step_record(f32=True)
        for fill in (0, 255):
            work = s.adjoint_workspace().fill_(fill)
            og = torch.empty_like(g32).view(torch.uint8).fill_(fill).view(torch.float32)
            oh = torch.empty_like(h32).view(torch.uint8).fill_(fill).view(torch.float32)
            dp = torch.zeros(3, dtype=torch.float64, device="cuda")
            s.adjoint_step_f32(g32, h32, lg.float(), lh.float(), og, oh, dp, work)
            out.append((og, oh, dp))
        for a, b in zip(*out):
            assert torch.isfinite(b).all()
            assert torch.equal(a, b)


@pytest.mark.parametrize("lattice", ["D2Q9_D2Q5", "D3Q19_D3Q7"])
def test_poisoned_recording_outputs_are_written_everywhere(lattice):
    import torch
    from paper_2511_11360_amd.solver import Solver
    d, phi, u = _params(lattice, "CH")
    s = Solver(d, precision="fp32")
    s.init(phi, u)
    s.step(2)
    ref_g, ref_h = s.get_distributions()
    ref_pu = s.get_phiu()
    from paper_2511_11360_amd.solver import _ptr
    # the raw entry point, outputs preset to NaN
    g = torch.full_like(ref_g, float("nan"))
    h = torch.full_like(ref_h, float("nan"))
    pu = torch.full_like(ref_pu, float("nan"))
    s._check(s.L.pflbm_step_record(s.h, _ptr(g), _ptr(h), _ptr(pu)), s.h)
    assert torch.equal(g, ref_g) and torch.equal(h, ref_h) and torch.equal(pu, ref_pu)
