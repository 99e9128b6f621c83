"""Shared helpers of the GPU tests: run the HIP path and the oracle on the
same seeded inputs."""
import numpy as np

from oracle import model as om


def oracle_run(d, phi, u, steps, p0=None):
    p = om.Params(**d)
    st = om.init(p, phi, u, p0)
    return p, om.run(p, st, steps)


def gpu_run(d, phi, u, steps, precision="fp64", p0=None, **kw):
    from paper_2511_11360_amd.solver import Solver
    s = Solver(d, precision=precision, **kw)
    s.init(phi, u, p0)
    s.step(steps)
    return s


def gpu_dists(s):
    g, h = s.get_distributions()
    return g.cpu().numpy(), h.cpu().numpy()


def max_abs_per_population(a, b):
    return np.max(np.abs(a - b).reshape(a.shape[0], -1), axis=1)


def small_3d(nx=28, ny=26, nz=24, R=7.0, u0=0.02, **kw):
    """Droplet in a Taylor-Green-like vortex on a ragged periodic box. The
    droplet is resolved (R / W = 2.8) and its tails vanish before the box edge,
    so the run is well conditioned: a 1e-15 perturbation of the initial state
    stays at round-off level (an under-resolved droplet is not, since the
    conservative AC flux has no defined normal where grad phi vanishes)."""
    from paper_2511_11360_amd import workloads as wl
    d = wl.base_params(lattice="D3Q19_D3Q7", nx=nx, ny=ny, nz=nz, rho_H=10.0, rho_L=1.0,
                       nu_H=0.05, nu_L=0.05, M=0.05, W=2.5, sigma=0.01)
    d.update(kw)
    phi = wl.droplet_phi(d, (nx / 2, ny / 2, nz / 2), R)
    x, y, z = wl.grid(d)
    kx, ky, kz = 2 * np.pi / nx, 2 * np.pi / ny, 2 * np.pi / nz
    # divergence-free (a compressive start moves phi off 1 inside the droplet,
    # where the antidiffusion flux then amplifies rounding)
    u = np.stack([u0 * ky * np.sin(kx * x) * np.cos(ky * y) * np.cos(kz * z) / kx,
                  -u0 * np.cos(kx * x) * np.sin(ky * y) * np.cos(kz * z),
                  np.zeros_like(x)])
    return d, phi, u


def oracle_envelope(d, phi, u, steps, seed=0, p0=None):
    """Spread of the oracle itself under rounding: two oracle runs whose initial
    populations differ by one relative ulp (random sign) everywhere. Returns
    the max |difference| per population of g and h after `steps` steps."""
    p = om.Params(**d)
    a = om.init(p, phi, u, p0)
    b = a.copy()
    rng = np.random.default_rng(seed)
    b.g = b.g * (1 + 2.0 ** -52 * rng.choice([-1.0, 1.0], size=b.g.shape))
    b.h = b.h * (1 + 2.0 ** -52 * rng.choice([-1.0, 1.0], size=b.h.shape))
    a = om.run(p, a, steps)
    b = om.run(p, b, steps)
    return max_abs_per_population(a.g, b.g), max_abs_per_population(a.h, b.h), a


def hydrostatic_p0(d, phi):
    """Initial pressure in hydrostatic balance with F_b = rho g along y
    (trapezoidal sum from the first row), so no acoustic start-up transient."""
    rho = d["rho_L"] + phi * (d["rho_H"] - d["rho_L"])
    gy = d["gravity"][1]
    p0 = np.zeros_like(rho)
    for j in range(1, d["ny"]):
        p0[:, j, :] = p0[:, j - 1, :] + 0.5 * (rho[:, j, :] + rho[:, j - 1, :]) * gy
    return p0 - p0.mean()
