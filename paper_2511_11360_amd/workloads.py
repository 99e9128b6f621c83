"""Seeded synthetic inputs: initial phase field, initial velocity and the
parameter set of each workload.

This module holds no step arithmetic of the method. It only builds the initial
conditions the paper prescribes (tanh interface profiles of Secs. III and IV)
and derives the physical parameters of each workload from its dimensionless
groups. Both the HIP path's tests and the oracle's tests take their inputs from
here; parameters come back as a plain dict whose keys name the physical
quantities (lattice, model, nx, ny, nz, bc, wall_u, rho_H, rho_L, nu_H, nu_L,
visc_interp, M, W, sigma, eta, gravity, force, s_other, freeze_phi,
normal_eps, lam).

Arrays are float64, scalars (nz, ny, nx), vectors (dim, nz, ny, nx), x fastest;
node (i, j, k) sits at (x, y, z) = (i, j, k).
"""
import math

import numpy as np


def base_params(**kw):
    p = dict(lattice="D2Q9_D2Q5", model="AC", nx=64, ny=64, nz=1,
             bc=("periodic", "periodic", "periodic"),
             wall_u=((0.0, 0.0, 0.0), (0.0, 0.0, 0.0)),
             rho_H=1.0, rho_L=1.0, nu_H=0.1, nu_L=0.1, visc_interp="mu",
             M=0.02, W=4.0, sigma=0.01, eta=1.0,
             gravity=(0.0, 0.0, 0.0), force=(0.0, 0.0, 0.0),
             s_other=1.0, freeze_phi=False, normal_eps=1e-4, lam=0.0)
    p.update(kw)
    return p


def grid(p):
    nz, ny, nx = p["nz"], p["ny"], p["nx"]
    z, y, x = np.meshgrid(np.arange(nz, dtype=float), np.arange(ny, dtype=float),
                          np.arange(nx, dtype=float), indexing="ij")
    return x, y, z


def _periodic_delta(d, n, periodic):
    return d - n * np.round(d / n) if periodic else d


def droplet_phi(p, centre, R, periodic=True):
    """Heavy droplet: phi = 1/2 + 1/2 tanh(2 (R - r) / W) (Eq. init-phi-circle and
    its 3-D form), r the (minimum-image) distance to the centre."""
    x, y, z = grid(p)
    dim = 2 if p["lattice"].startswith("D2") else 3
    r2 = np.zeros_like(x)
    for coord, c, n in zip((x, y, z)[:dim], centre, (p["nx"], p["ny"], p["nz"])):
        d = _periodic_delta(coord - c, n, periodic)
        r2 += d * d
    return 0.5 + 0.5 * np.tanh(2.0 * (R - np.sqrt(r2)) / p["W"])


def zero_velocity(p):
    dim = 2 if p["lattice"].startswith("D2") else 3
    return np.zeros((dim, p["nz"], p["ny"], p["nx"]))


# ---------------------------------------------------------------------------
# workloads

def static_droplet_2d(n=64, R=16.0):
    """2-D static droplet, 64 x 64 periodic, R = 16 centred, W = 4, sigma = 0.01,
    M = 0.02, rho_H/rho_L = 10, tau_g = 0.8 (nu = 0.1), zero initial velocity."""
    p = base_params(nx=n, ny=n, rho_H=10.0, rho_L=1.0, nu_H=0.1, nu_L=0.1,
                    M=0.02, W=4.0, sigma=0.01)
    phi = droplet_phi(p, (n / 2, n / 2), R)
    return p, phi, zero_velocity(p)


def rayleigh_taylor_2d(model="AC", nx=256, ny=1024, At=0.5, Re=3000.0, Ug=0.04,
                       M=0.1, W=4.0, sigma=5e-5):
    """2-D Rayleigh-Taylor (Sec. III.C layout): L0 x 4 L0, walls top and bottom,
    periodic in x, heavy fluid on top of the interface
    y_t = 2 L0 + 0.05 L0 cos(2 pi x / L0). Gravity from U_g = sqrt(g L0);
    viscosity from Re = (L0/nu) sqrt(At g L0 / (1 + At))."""
    L0 = nx
    g = Ug * Ug / L0
    nu = L0 * math.sqrt(At * g * L0 / (1 + At)) / Re
    rho_L = 1.0
    rho_H = rho_L * (1 + At) / (1 - At)
    p = base_params(model=model, nx=nx, ny=ny, nz=1,
                    bc=("periodic", "wall", "periodic"),
                    rho_H=rho_H, rho_L=rho_L, nu_H=nu, nu_L=nu, M=M, W=W, sigma=sigma,
                    gravity=(0.0, -g, 0.0))
    x, y, _ = grid(p)
    yt = ny / 2 + 0.05 * L0 * np.cos(2 * math.pi * x / L0)
    phi = 0.5 + 0.5 * np.tanh(2.0 * (y - yt) / W)
    return p, phi, zero_velocity(p)


def layered_poiseuille(nx=10, ny=100, uc=1e-3, ratio=1000.0, nu=1.0 / 3.0, W=4.0,
                       M=0.1, sigma=1e-3):
    """Layered two-phase Poiseuille flow (Sec. III.D): heavy fluid below y = H,
    light above, walls at y = 0 and y = Ny (half a spacing outside the nodes at
    j + 1/2 in the channel coordinate), phi frozen, driven by the uniform force
    density G_x = u_c (mu_H + mu_L) / H^2. Density and viscosity ratios 1000."""
    H = ny / 2.0
    rho_H, rho_L = 1.0, 1.0 / ratio
    mu_H, mu_L = rho_H * nu, rho_L * nu
    Gx = uc * (mu_H + mu_L) / H ** 2
    p = base_params(nx=nx, ny=ny, bc=("periodic", "wall", "periodic"),
                    rho_H=rho_H, rho_L=rho_L, nu_H=nu, nu_L=nu, M=M, W=W, sigma=sigma,
                    force=(Gx, 0.0, 0.0), freeze_phi=True)
    _, y, _ = grid(p)
    yc = y + 0.5                    # channel coordinate, walls at 0 and ny
    phi = 0.5 + 0.5 * np.tanh(2.0 * (H - yc) / W)
    return p, phi, zero_velocity(p)


def taylor_green_droplet_3d(n=256, u0=0.05, Re=1000.0, R=40.0, We=10.0, W=4.0,
                            M=0.05, ratio=10.0):
    """3-D droplet in a Taylor-Green vortex: n^3 periodic, droplet (heavy,
    rho_H/rho_L = 10) of radius R centred; u = u0 sin kx cos ky cos kz,
    v = -u0 cos kx sin ky cos kz, w = 0, k = 2 pi / n; Re = u0 (n / 2 pi) / nu;
    We = rho_H u_rms^2 (2R) / sigma with u_rms = u0 / sqrt(12) per component."""
    k = 2 * math.pi / n
    nu = u0 * (n / (2 * math.pi)) / Re
    rho_L = 1.0
    rho_H = ratio * rho_L
    urms = u0 / math.sqrt(12.0)
    sigma = rho_H * urms * urms * 2 * R / We
    p = base_params(lattice="D3Q19_D3Q7", nx=n, ny=n, nz=n, rho_H=rho_H, rho_L=rho_L,
                    nu_H=nu, nu_L=nu, M=M, W=W, sigma=sigma)
    c = n / 2.0
    phi = droplet_phi(p, (c, c, c), R * n / 256.0 if n != 256 else R)
    x, y, z = grid(p)
    u = np.stack([u0 * np.sin(k * x) * np.cos(k * y) * np.cos(k * z),
                  -u0 * np.cos(k * x) * np.sin(k * y) * np.cos(k * z),
                  np.zeros_like(x)])
    return p, phi, u


def sheared_droplet_3d(n=128, R=24.0, uw=0.02, Ca=0.2, W=4.0, M=0.05, nu=1.0 / 6.0,
                       seed=4):
    """3-D droplet in simple shear: walls normal to y moving at -uw (low) and +uw
    (high) in x, periodic in x and z, droplet of radius R centred, density ratio
    1; Ca = mu gamma R / sigma with gamma = 2 uw / n. Also returns a seeded
    target field: a tanh ellipsoid with semi-axes R (1 + e_i), e_i ~ U(-0.1, 0.1)."""
    gamma = 2 * uw / n
    mu = 1.0 * nu
    sigma = mu * gamma * R / Ca
    p = base_params(lattice="D3Q19_D3Q7", nx=n, ny=n, nz=n,
                    bc=("periodic", "wall", "periodic"),
                    wall_u=((-uw, 0.0, 0.0), (uw, 0.0, 0.0)),
                    rho_H=1.0, rho_L=1.0, nu_H=nu, nu_L=nu, M=M, W=W, sigma=sigma)
    c = n / 2.0
    phi = droplet_phi(p, (c, c - 0.5, c), R, periodic=False)
    rng = np.random.default_rng(seed)
    e = rng.uniform(-0.1, 0.1, size=3)
    x, y, z = grid(p)
    s = np.sqrt(((x - c) / (R * (1 + e[0]))) ** 2 + ((y - c + 0.5) / (R * (1 + e[1]))) ** 2
                + ((z - c) / (R * (1 + e[2]))) ** 2)
    target = 0.5 + 0.5 * np.tanh(2.0 * R * (1 - s) / W)
    u = zero_velocity(p)
    u[0] = -uw + 2 * uw * (y + 0.5) / n     # linear shear profile between the walls
    return p, phi, u, target


def random_spectrum_velocity(n, k0=4.0, urms=0.04, seed=5):
    """Random-phase solenoidal field with E(k) ~ k^4 exp(-2 (k/k0)^2), scaled to
    a per-component rms of urms (seeded). Phases are drawn on the modes with
    |k_x|, |k_y|, |k_z| <= kmax = min(n/2 - 1, ceil(8 k0)) only (beyond 8 k0,
    E(k) is below 1e-40 of its peak), then each component is the real part of
    its zero-padded inverse FFT (multi-threaded)."""
    import os
    import scipy.fft as sfft
    rng = np.random.default_rng(seed)
    km = int(min(n // 2 - 1, math.ceil(8 * k0)))
    kb = np.arange(-km, km + 1, dtype=float)
    KX, KY, KZ = kb[:, None, None], kb[None, :, None], kb[None, None, :]
    K2 = KX ** 2 + KY ** 2 + KZ ** 2
    nz_ = K2 > 0
    amp = np.zeros_like(K2)
    # shell energy E(k) spread over 4 pi k^2 modes -> |u_k| ~ sqrt(E / k^2)
    amp[nz_] = np.sqrt(K2[nz_] ** 2 * np.exp(-2 * K2[nz_] / (k0 * k0)) / K2[nz_])
    comps = np.array([amp * np.exp(1j * rng.uniform(0, 2 * np.pi, size=K2.shape)) for _ in range(3)])
    # project out the compressive part: u_k <- u_k - k (k . u_k) / k^2
    kd = (KX * comps[0] + KY * comps[1] + KZ * comps[2]) / np.where(nz_, K2, 1.0)
    comps = comps - np.array([KX * kd, KY * kd, KZ * kd])
    idx = np.arange(-km, km + 1) % n
    u = np.empty((3, n, n, n))
    full = np.zeros((n, n, n), dtype=np.complex128)
    for c in range(3):
        full[np.ix_(idx, idx, idx)] = comps[c]
        u[c] = sfft.ifftn(full, workers=os.cpu_count() or 1).real
    u *= urms / np.sqrt((u * u).mean(axis=(1, 2, 3)).mean())
    # arrays are (k_x, k_y, k_z) -> (z, y, x)
    return np.ascontiguousarray(np.transpose(u, (0, 3, 2, 1)))


def droplet_turbulence_3d(n=512, ndrop=64, R=16.0, We=5.0, W=4.0, M=0.05, ratio=10.0,
                          urms=0.04, k0=4.0, nu=None, seed_u=5, seed_pos=55):
    """Droplet-laden decaying isotropic turbulence: n^3 periodic, ndrop heavy
    droplets of radius R at seeded non-overlapping positions (minimum centre
    distance 2R + 2W), We = rho_H urms^2 (2R) / sigma. Each droplet's tanh
    profile is evaluated in a periodic box of half-width R + 6W around it
    (beyond it the profile is below 1e-10); overlapping tails combine by max."""
    rho_L = 1.0
    rho_H = ratio
    sigma = rho_H * urms * urms * 2 * R / We
    if nu is None:
        nu = 0.0128 * n / 256.0
    p = base_params(lattice="D3Q19_D3Q7", nx=n, ny=n, nz=n, rho_H=rho_H, rho_L=rho_L,
                    nu_H=nu, nu_L=nu, M=M, W=W, sigma=sigma)
    rng = np.random.default_rng(seed_pos)
    centres = []
    dmin = 2 * R + 2 * W
    while len(centres) < ndrop:
        c = rng.uniform(0, n, size=3)
        ok = True
        for q in centres:
            d = c - q
            d -= n * np.round(d / n)
            if np.dot(d, d) < dmin * dmin:
                ok = False
                break
        if ok:
            centres.append(c)
    phi = np.zeros((n, n, n))
    h = int(np.ceil(R + 6 * W))
    for c in centres:
        idx = [np.arange(int(np.floor(ci)) - h, int(np.floor(ci)) + h + 2) for ci in c]
        dx = [(ix - ci) for ix, ci in zip(idx, c)]
        r = np.sqrt(dx[2][:, None, None] ** 2 + dx[1][None, :, None] ** 2 + dx[0][None, None, :] ** 2)
        local = 0.5 + 0.5 * np.tanh(2.0 * (R - r) / W)
        sl = np.ix_(idx[2] % n, idx[1] % n, idx[0] % n)
        phi[sl] = np.maximum(phi[sl], local)
    u = random_spectrum_velocity(n, k0=k0, urms=urms, seed=seed_u)
    return p, phi, u, np.array(centres)


def seeded_field(shape, seed, lo=0.0, hi=1.0):
    """Uniform random field, for perturbation and direction vectors in tests."""
    return np.random.default_rng(seed).uniform(lo, hi, size=shape)
