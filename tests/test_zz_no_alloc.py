"""pflbm_adjoint_step_noalloc (the adjoint step on the library's own device
scratch, for callers that cannot allocate) against pflbm_adjoint_step with a
caller workspace, through the C ABI: equal bit for bit on two calls in a row,
the second on a smaller box, and a box beyond the scratch rejected."""
import sys

import pytest

from gpu_helpers import small_3d

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _pair(d, phi, u, seed):
    import torch
    from paper_2511_11360_amd.solver import Solver
    s = Solver(d, precision="fp64")
    s.init(phi, u)
    s.step(5)
    fg, fh = s.get_distributions()
    gen = torch.Generator(device=fg.device).manual_seed(seed)
    lg = torch.randn(fg.shape, dtype=torch.float64, device=fg.device, generator=gen)
    lh = torch.randn(fh.shape, dtype=torch.float64, device=fg.device, generator=gen)
    out = []
    for noalloc in (False, True):
        og, oh = torch.full_like(fg, float("nan")), torch.full_like(fh, float("nan"))
        dp = torch.zeros(3, dtype=torch.float64, device=fg.device)
        if noalloc:
            s.adjoint_step_noalloc(fg, fh, lg, lh, og, oh, dp)
        else:
            s.adjoint_step(fg, fh, lg, lh, og, oh, dp, s.adjoint_workspace())
        torch.cuda.synchronize()
        out.append((og, oh, dp))
    return out


def test_noalloc_adjoint_equals_workspace_adjoint():
    import torch
    for nx, ny, nz, bc in ((36, 34, 30, "wall"), (14, 12, 11, "periodic")):
        _say("case no-alloc adjoint %dx%dx%d %s" % (nx, ny, nz, bc))
        d, phi, u = small_3d(nx=nx, ny=ny, nz=nz, R=min(nx, ny, nz) / 4.0)
        if bc == "wall":
            d["bc"] = ("periodic", "wall", "periodic")
            d["wall_u"] = ((-0.01, 0.0, 0.0), (0.01, 0.0, 0.0))
        (g1, h1, p1), (g2, h2, p2) = _pair(d, phi, u, nx)
        assert bool(torch.isfinite(g2).all()) and bool(torch.isfinite(h2).all())
        assert torch.equal(g1, g2) and torch.equal(h1, h2) and torch.equal(p1, p2)


def test_noalloc_adjoint_rejects_boxes_beyond_its_scratch():
    import torch
    from paper_2511_11360_amd import pflbm as P
    from paper_2511_11360_amd import workloads as wl
    from paper_2511_11360_amd.solver import Solver
    d = wl.base_params(lattice="D3Q19_D3Q7", nx=130, ny=130, nz=130)
    s = Solver(d, precision="fp64")
    z = torch.zeros((19, 130, 130, 130), dtype=torch.float64, device="cuda")
    zh = torch.zeros((7, 130, 130, 130), dtype=torch.float64, device="cuda")
    dp = torch.zeros(3, dtype=torch.float64, device="cuda")
    with pytest.raises(P.PflbmError) as e:
        s.adjoint_step_noalloc(z, zh, z, zh, z.clone(), zh.clone(), dp)
    assert e.value.status == P.PFLBM_EINVAL
    # the handle stays usable
    s.init(torch.zeros((130, 130, 130), dtype=torch.float64, device="cuda"))
    s.step(1)
