"""Oracle of one time step of the coupled phase-field lattice Boltzmann solver.

Model (Sec. II.C.1, Fakhari2017 conservative Allen-Cahn) with the CH variant
of Sec. II.D.1 (Liang2014 phase-field equation) as the second model and the
nonlocal / hybrid Allen-Cahn phase-field side of Sec. II.C (Chai2018, Hu2019
with weight lam) as the third, Liang2018 (Sec. II.C, conservative AC with
its own conservative-form hydrodynamics) as the fourth, and Liang2014 with its
full hydrodynamic coupling (Sec. II.D.1: CH phase field, Eqs. liang2_feq,
liang2_F, the F_a force and the modified velocity update) as the fifth. Notation
(see the package docstring): g = hydrodynamic distribution (paper's f_beta),
h = phase-field distribution (paper's g_alpha), W = interface width xi,
M = mobility M_phi.

Arrays are (Q, nz, ny, nx) for distributions, (3, nz, ny, nx) for vectors and
(nz, ny, nx) for scalars, x fastest; 2-D runs have nz = 1 and zero z
components. Node (i, j, k) sits at position (x, y, z) = (i, j, k); walls sit
half a spacing outside the first and last node of a walled axis.

Every function accepts float64 or complex128 arrays and parameters, so that a
complex-step derivative runs through the same code: square roots are taken of
x.x (no conjugation) and branches test real parts only.

Order within one step, all node-local except the stencils and the streaming:
  O1  phi = sum_a h_a                               Eq. fakhari_phi_update
      (nonlocal: phi = phi* + (1 - lam) R / 2 with phi* = sum_a h_a and the
      source R of Eq. chai_G at phi*, gamma of Eq. lagrange_multiplier;
      Eq. chai2018_phi_update)
  O2  ghost phi: periodic wrap, mirror at walls     (n . grad phi = 0, Sec. II.A)
  O3  grad phi, lap phi, isotropic central stencils  Sec. III, stencil equations
  O4  rho, nu, tau                                  Eqs. fakhari_rho_update,
                                                    mu_linear / fakhari_mu_update,
                                                    fakhari_tau_model
  O5  chemical potential mu_phi                     Eq. chemical_potential
  O6  p* = sum g, p = rho c_s^2 p*                  Eq. fakhari_p_update
  O7  F_s, F_b, F_p                                 total-force paragraph, Sec. II.C.1
  O8  F_mu = nu (grad u + grad u^T) . grad rho, with the strain rate taken
      from the non-equilibrium second moment of g at the velocity without F_mu
  O9  u = sum c g + F / (2 rho)                     Eq. fakhari_velocity_update
  O10 h collision (BGK)                             Eqs. fakhari_g_simplified,
                                                    fakhari_geq, fakhari_G_modified
                                                    (CH: liang2_geq, liang2_G;
                                                    nonlocal: Chai_geq, Hu_G)
  O11 g collision (MRT form of Eq. fakhari_f_simplified with Eqs. fakhari_feq,
      fakhari_F)
  O12 push streaming, halfway bounce-back at walls
"""
from dataclasses import dataclass, field, replace

import numpy as np

from .lattice import CS2, PAIRS
from . import mrt

PHI_H = 1.0   # heavy-phase label, Sec. II
PHI_L = 0.0   # light-phase label
PHI_0 = 0.5 * (PHI_H + PHI_L)   # interface value

PERIODIC = "periodic"
WALL = "wall"


@dataclass
class Params:
    lattice: str = "D2Q9_D2Q5"       # or "D3Q19_D3Q7"
    model: str = "AC"                 # "AC" (Fakhari2017), "CH" (Liang2014 h-equation)
                                      # "NL" (Chai2018 nonlocal AC, blended with the
                                      # conservative flux by lam as in Hu2019), "L18"
                                      # (Liang2018: phase field and hydrodynamics) or
                                      # "L14" (Liang2014 CH with its own hydrodynamics)
    nx: int = 64
    ny: int = 64
    nz: int = 1
    bc: tuple = (PERIODIC, PERIODIC, PERIODIC)   # per axis x, y, z
    wall_u: tuple = ((0.0, 0.0, 0.0), (0.0, 0.0, 0.0))  # low / high wall velocity
    rho_H: float = 1.0
    rho_L: float = 1.0
    nu_H: float = 0.1
    nu_L: float = 0.1
    visc_interp: str = "mu"           # "mu": Eq. mu_linear; "nu": Eq. fakhari_mu_update
    M: float = 0.02
    W: float = 4.0
    sigma: float = 0.01
    eta: float = 1.0                  # CH mobility parameter of Eq. liang2_geq
    gravity: tuple = (0.0, 0.0, 0.0)  # F_b = rho * gravity
    force: tuple = (0.0, 0.0, 0.0)    # uniform force density added to F_b
    s_other: float = 1.0              # MRT rate of every non-stress moment
    freeze_phi: bool = False          # keep h (hence phi) fixed, Sec. III.D
    normal_eps: float = 1e-4          # regularisation of |grad phi| in the normal
    lam: float = 0.0                  # NL: weight of the conservative flux (0: Chai2018)
    gamma_given: float = None         # NL: multiplier to use instead of the sums over
                                      # this box (for stepping a block cut out of a
                                      # larger box, whose sums span the whole box)

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def lattices(self):
        return PAIRS[self.lattice]

    @property
    def dim(self):
        return self.lattices[0].dim

    def walled_axis(self):
        """Index (0=x, 1=y, 2=z) of the single walled axis, or None."""
        ax = [a for a in range(3) if self.bc[a] == WALL]
        if len(ax) > 1:
            raise ValueError("walls on more than one axis are not supported")
        return ax[0] if ax else None


@dataclass
class State:
    g: np.ndarray              # (Qg, nz, ny, nx) post-streaming hydrodynamic populations
    h: np.ndarray              # (Qh, nz, ny, nx) post-streaming phase-field populations
    phiu_prev: np.ndarray = None   # (3, nz, ny, nx) (phi u) of the previous step, CH only

    def copy(self):
        return State(self.g.copy(), self.h.copy(),
                     None if self.phiu_prev is None else self.phiu_prev.copy())


# --------------------------------------------------------------------------
# stencils (O2, O3)

_ARRAY_AXIS = {0: 2, 1: 1, 2: 0}   # physical axis -> array axis of (nz, ny, nx)


def pad_ghost(p, a):
    """One ghost layer on every side: periodic wrap, or the mirror image of the
    first node at a wall (a halfway wall makes the ghost equal to that node)."""
    for ax in range(3):
        width = [(0, 0)] * a.ndim
        width[a.ndim - 3 + _ARRAY_AXIS[ax]] = (1, 1)
        a = np.pad(a, width, mode="wrap" if p.bc[ax] == PERIODIC else "edge")
    return a


def neighbour(p, padded, c):
    """Value at x + c read from a ghost-padded scalar field."""
    nz, ny, nx = p.shape
    return padded[1 + c[2]:1 + c[2] + nz, 1 + c[1]:1 + c[1] + ny, 1 + c[0]:1 + c[0] + nx]


def gradient(p, phi):
    """grad phi = (1/c_s^2) sum_i w_i c_i phi(x + c_i) on the hydrodynamic lattice."""
    lat = p.lattices[0]
    P = pad_ghost(p, phi)
    out = np.zeros((3,) + phi.shape, dtype=phi.dtype)
    for i in range(lat.Q):
        nb = neighbour(p, P, lat.c[i])
        for a in range(3):
            if lat.c[i][a] != 0:
                out[a] = out[a] + lat.w[i] * lat.c[i][a] * nb
    return out / CS2


def laplacian(p, phi):
    """lap phi = (2/c_s^2) sum_i w_i [phi(x + c_i) - phi(x)]."""
    lat = p.lattices[0]
    P = pad_ghost(p, phi)
    out = np.zeros_like(phi)
    for i in range(lat.Q):
        out = out + lat.w[i] * (neighbour(p, P, lat.c[i]) - phi)
    return 2.0 * out / CS2


# --------------------------------------------------------------------------
# equilibria and sources

def _cdot(c, v):
    """c . v for one integer velocity c and a (3, ...) vector field."""
    out = 0.0
    for a in range(3):
        if c[a] != 0:
            out = out + c[a] * v[a]
    return out


def _vdot(u, v):
    return u[0] * v[0] + u[1] * v[1] + u[2] * v[2]


def g_eq(p, pstar, u):
    """Eq. fakhari_feq with p/(rho c_s^2) = p*: w [p* + c.u/c_s^2 + (c.u)^2/(2c_s^4) - u.u/(2c_s^2)]."""
    lat = p.lattices[0]
    uu = _vdot(u, u)
    out = np.empty((lat.Q,) + pstar.shape, dtype=np.result_type(pstar, u))
    for i in range(lat.Q):
        cu = _cdot(lat.c[i], u)
        out[i] = lat.w[i] * (pstar + cu / CS2 + cu * cu / (2 * CS2 * CS2) - uu / (2 * CS2))
    return out


def f_eq_liang(p, rho, pres, u):
    """Eq. liang_feq (also Eq. liang2_feq): rest (p/c_s^2)(w_0 - 1) + rho w_0 [...],
    others (p/c_s^2) w + rho w [e.u/c_s^2 + (e.u)^2/(2 c_s^4) - u.u/(2 c_s^2)]."""
    lat = p.lattices[0]
    uu = _vdot(u, u)
    out = np.empty((lat.Q,) + rho.shape, dtype=np.result_type(rho, pres, u))
    for i in range(lat.Q):
        cu = _cdot(lat.c[i], u)
        kin = rho * lat.w[i] * (cu / CS2 + cu * cu / (2 * CS2 * CS2) - uu / (2 * CS2))
        out[i] = pres / CS2 * (lat.w[i] - 1 if i == 0 else lat.w[i]) + kin
    return out


def force_liang(p, F, u, grad_rho):
    """Eq. liang_F_final: w [u.grad rho + e.F/c_s^2 + u grad rho : (e e - c_s^2 I)/c_s^2]."""
    lat = p.lattices[0]
    udr = _vdot(u, grad_rho)
    out = np.empty((lat.Q,) + udr.shape, dtype=np.result_type(F, u, grad_rho))
    for i in range(lat.Q):
        c = lat.c[i]
        tens = 0.0 * udr
        for a in range(3):
            for b in range(3):
                tens = tens + u[a] * grad_rho[b] * (c[a] * c[b] - CS2 * (a == b))
        out[i] = lat.w[i] * (udr + _cdot(c, F) / CS2 + tens / CS2)
    return out


def force_liang14(p, Fp, u, rho, grad_rho):
    """Eq. liang2_F: (e - u)/c_s^2 . [Gamma(u) grad(rho c_s^2) + F' s(u)] with
    Gamma, s of Eq. Gamma_beta and F' = F_s + F_a + F_b."""
    lat = p.lattices[0]
    uu = _vdot(u, u)
    A = CS2 * grad_rho
    out = np.empty((lat.Q,) + rho.shape, dtype=np.result_type(Fp, u, grad_rho))
    for i in range(lat.Q):
        c = lat.c[i]
        cu = _cdot(c, u)
        gam = lat.w[i] * (cu / CS2 + cu * cu / (2 * CS2 * CS2) - uu / (2 * CS2))
        s_ = lat.w[i] + gam
        emu = [c[a] - u[a] for a in range(3)]
        out[i] = (sum(emu[a] * (gam * A[a] + Fp[a] * s_) for a in range(3))) / CS2
    return out


def h_eq_ac(p, phi, u):
    """Eq. fakhari_geq: w phi [1 + e.u/c_s^2 + (e.u)^2/(2c_s^4) - u.u/(2c_s^2)]."""
    lat = p.lattices[1]
    uu = _vdot(u, u)
    out = np.empty((lat.Q,) + phi.shape, dtype=np.result_type(phi, u))
    for a in range(lat.Q):
        eu = _cdot(lat.c[a], u)
        out[a] = lat.w[a] * phi * (1 + eu / CS2 + eu * eu / (2 * CS2 * CS2) - uu / (2 * CS2))
    return out


def h_eq_ch(p, phi, mu_phi, u):
    """Eq. liang2_geq: rest phi + (w_0 - 1) eta mu; others w eta mu + w e.(phi u)/c_s^2."""
    lat = p.lattices[1]
    out = np.empty((lat.Q,) + phi.shape, dtype=np.result_type(phi, mu_phi, u))
    phiu = phi * u
    for a in range(lat.Q):
        if a == 0:
            out[a] = phi + (lat.w[0] - 1) * p.eta * mu_phi
        else:
            out[a] = lat.w[a] * p.eta * mu_phi + lat.w[a] * _cdot(lat.c[a], phiu) / CS2
    return out


def h_eq_nl(p, phi, u):
    """Eq. Chai_geq: w phi (1 + e.u / c_s^2)."""
    lat = p.lattices[1]
    out = np.empty((lat.Q,) + phi.shape, dtype=np.result_type(phi, u))
    for a in range(lat.Q):
        out[a] = lat.w[a] * phi * (1 + _cdot(lat.c[a], u) / CS2)
    return out


def nonlocal_source(p, phi):
    """Source of the nonlocal AC equation (Eqs. nonlocalAC, chai_G without the
    weight w_a) at the field phi, and the Lagrange multiplier gamma of Eq.
    lagrange_multiplier with the integrals taken as sums over all nodes:
        R = M [ -(4 beta / kappa) (phi - phi_H)(phi - phi_L)(phi - phi_0)
                + gamma (phi_H - phi)(phi - phi_L) ],
        gamma = sum (4 beta / kappa)(phi - phi_H)(phi - phi_L)(phi - phi_0)
                / sum (phi_H - phi)(phi - phi_L),
    so that sum R = 0. 4 beta / kappa = 32 / (W^2 (phi_H - phi_L)^2): sigma
    cancels (defined at sigma = 0). gamma = 0 when the denominator vanishes
    (phi is phi_H or phi_L everywhere, where the gamma term is zero anyway)."""
    c = 32.0 / (p.W * p.W * (PHI_H - PHI_L) ** 2)
    bulk = c * (phi - PHI_H) * (phi - PHI_L) * (phi - PHI_0)
    well = (PHI_H - phi) * (phi - PHI_L)
    if p.gamma_given is not None:
        gamma = p.gamma_given
    else:
        num = np.sum(bulk)
        den = np.sum(well)
        gamma = num / den if np.real(den) != 0 else 0.0 * num
    return p.M * (-bulk + gamma * well), gamma


def coefficients(p):
    """beta and kappa of Eqs. coefficient1 and coefficients."""
    dphi = PHI_H - PHI_L
    beta = 12 * p.sigma / (p.W * dphi ** 4)
    kappa = 3 * p.sigma * p.W / (2 * dphi ** 2)
    return beta, kappa


def chemical_potential(p, phi, lap):
    """Eq. chemical_potential."""
    beta, kappa = coefficients(p)
    return 4 * beta * (phi - PHI_H) * (phi - PHI_L) * (phi - PHI_0) - kappa * lap


def G_ac(p, phi, grad):
    """Eq. fakhari_G_modified: w e . [sqrt(2 beta/kappa) (phi_H-phi)(phi-phi_L) n].

    sqrt(2 beta / kappa) = 4 / (W (phi_H - phi_L)) once the sigma of
    Eqs. coefficient1 and coefficients cancels (also defined at sigma = 0).
    The normal grad phi / |grad phi| is regularised as
    grad phi / sqrt(grad phi . grad phi + eps^2) (eps = p.normal_eps). The paper
    leaves n undefined where the gradient vanishes; there, with 0 < phi < 1, the
    antidiffusion flux is anti-diffusive for gradients below (4/W) phi (1 - phi),
    so an unregularised normal amplifies round-off inside a droplet (two exact
    implementations drift apart). With eps = 1e-4 the flux differs from the
    paper's by (eps/|grad phi|)^2/2 < 2e-7 relative at the interface centre.
    eps = 0 is the paper's normal with the guard n = 0 where
    grad phi . grad phi = 0 (there the flux vanishes with the gradient)."""
    lat = p.lattices[1]
    gg = _vdot(grad, grad)
    s = gg + p.normal_eps * p.normal_eps
    pos = np.real(s) > 0
    inv = np.where(pos, 1.0 / np.sqrt(np.where(pos, s, 1.0)), 0.0)
    coef = 4.0 / (p.W * (PHI_H - PHI_L)) * (PHI_H - phi) * (phi - PHI_L) * inv
    out = np.empty((lat.Q,) + phi.shape, dtype=np.result_type(coef, grad))
    for a in range(lat.Q):
        out[a] = lat.w[a] * coef * _cdot(lat.c[a], grad)
    return out


def G_ch(p, dphiu_dt):
    """Eq. liang2_G: w e . d(phi u)/dt / c_s^2 (time derivative supplied by the caller)."""
    lat = p.lattices[1]
    out = np.empty((lat.Q,) + dphiu_dt.shape[1:], dtype=dphiu_dt.dtype)
    for a in range(lat.Q):
        out[a] = lat.w[a] * _cdot(lat.c[a], dphiu_dt) / CS2
    return out


def force_populations(p, F, rho):
    """Eq. fakhari_F: w c . F / (rho c_s^2)."""
    lat = p.lattices[0]
    out = np.empty((lat.Q,) + rho.shape, dtype=np.result_type(F, rho))
    for i in range(lat.Q):
        out[i] = lat.w[i] * _cdot(lat.c[i], F) / (rho * CS2)
    return out


# --------------------------------------------------------------------------
# macroscopic step (O1 - O9)

def _lin(vH, vL, phi):
    """Linear interpolation between phase values, as in Eq. fakhari_rho_update."""
    return vH * (phi - PHI_L) / (PHI_H - PHI_L) + vL * (phi - PHI_H) / (PHI_L - PHI_H)


def macroscopic(p, st):
    """O1-O9 at every node; returns a dict of the fields used by the collisions."""
    gl, hl = p.lattices
    # O1
    phi = st.h[0].copy()
    for a in range(1, hl.Q):
        phi = phi + st.h[a]
    R = gamma = None
    if p.model == "NL":
        R, gamma = nonlocal_source(p, phi)
        phi = phi + 0.5 * (1 - p.lam) * R
    # O2, O3
    grad = gradient(p, phi)
    lap = laplacian(p, phi)
    # O4
    rho = _lin(p.rho_H, p.rho_L, phi)
    grad_rho = (p.rho_H - p.rho_L) / (PHI_H - PHI_L) * grad
    if p.visc_interp == "mu":
        mu = _lin(p.rho_H * p.nu_H, p.rho_L * p.nu_L, phi)
        nu = mu / rho
    else:
        nu = _lin(p.nu_H, p.nu_L, phi)
    tau = nu / CS2 + 0.5
    # O5
    mu_phi = chemical_potential(p, phi, lap)
    if p.model == "L18":
        return _macroscopic_liang(p, st, phi, grad, lap, rho, grad_rho, nu, tau, mu_phi)
    if p.model == "L14":
        return _macroscopic_liang14(p, st, phi, grad, lap, rho, grad_rho, nu, tau, mu_phi)
    # O6
    pstar = st.g[0].copy()
    for i in range(1, gl.Q):
        pstar = pstar + st.g[i]
    pres = rho * CS2 * pstar
    # O7
    Fs = mu_phi * grad
    Fb = np.array([rho * p.gravity[a] + p.force[a] for a in range(3)])
    Fp = -(pres / rho) * grad_rho
    # O8
    j = np.zeros((3,) + phi.shape, dtype=st.g.dtype)
    for i in range(gl.Q):
        for a in range(3):
            if gl.c[i][a] != 0:
                j[a] = j[a] + gl.c[i][a] * st.g[i]
    u_star = j + (Fs + Fb + Fp) / (2 * rho)
    neq = st.g - g_eq(p, pstar, u_star)
    Pi = np.zeros((3, 3) + phi.shape, dtype=neq.dtype)
    for i in range(gl.Q):
        for a in range(3):
            for b in range(3):
                if gl.c[i][a] * gl.c[i][b] != 0:
                    Pi[a, b] = Pi[a, b] + gl.c[i][a] * gl.c[i][b] * neq[i]
    strain = -Pi / (tau * CS2)          # estimate of grad u + (grad u)^T
    Fmu = np.array([nu * (strain[a, 0] * grad_rho[0] + strain[a, 1] * grad_rho[1]
                          + strain[a, 2] * grad_rho[2]) for a in range(3)])
    # O9
    F = Fs + Fb + Fp + Fmu
    u = j + F / (2 * rho)
    return dict(phi=phi, grad=grad, lap=lap, rho=rho, nu=nu, tau=tau, mu_phi=mu_phi,
                pstar=pstar, p=pres, F=F, u=u, R=R, gamma=gamma)


def _macroscopic_liang(p, st, phi, grad, lap, rho, grad_rho, nu, tau, mu_phi):
    """Liang2018 hydrodynamics (Sec. II.C): F = F_s + F_b (no pressure or viscous
    force term), rho u = sum e f + F/2 (Eq. liang_velocity_update) and
    p = c_s^2 / (1 - w_0) [sum_{beta != 0} f + u.grad rho / 2
    + rho w_0 (-u.u / (2 c_s^2))] (Eq. liang_p_update)."""
    gl = p.lattices[0]
    Fs = mu_phi * grad
    Fb = np.array([rho * p.gravity[a] + p.force[a] for a in range(3)])
    F = Fs + Fb
    j = np.zeros((3,) + phi.shape, dtype=st.g.dtype)
    for i in range(gl.Q):
        for a in range(3):
            if gl.c[i][a] != 0:
                j[a] = j[a] + gl.c[i][a] * st.g[i]
    u = (j + 0.5 * F) / rho
    moving = st.g[1].copy()
    for i in range(2, gl.Q):
        moving = moving + st.g[i]
    w0 = gl.w[0]
    pres = CS2 / (1 - w0) * (moving + 0.5 * _vdot(u, grad_rho) + rho * w0 * (-_vdot(u, u) / (2 * CS2)))
    return dict(phi=phi, grad=grad, lap=lap, rho=rho, nu=nu, tau=tau, mu_phi=mu_phi,
                pstar=pres / (rho * CS2), p=pres, F=F, u=u, grad_rho=grad_rho, R=None, gamma=None)


def _macroscopic_liang14(p, st, phi, grad, lap, rho, grad_rho, nu, tau, mu_phi):
    """Liang2014 hydrodynamics (Sec. II.D.1): lap mu_phi with the same stencil
    and ghost rules as phi (so div(M grad mu_phi) = M lap mu_phi, M constant),
    u = (sum e f + (F_s + F_b)/2) / (rho - (rho_H - rho_L) M lap mu_phi / 2)
    (Eq. liang2014_velocity_update), F_a = (rho_H - rho_L) M lap mu_phi u, and
    p as in Eq. liang_p_update."""
    gl = p.lattices[0]
    lap_mu = laplacian(p, mu_phi)
    drho = (p.rho_H - p.rho_L) / (PHI_H - PHI_L)
    Fs = mu_phi * grad
    Fb = np.array([rho * p.gravity[a] + p.force[a] for a in range(3)])
    j = np.zeros((3,) + phi.shape, dtype=st.g.dtype)
    for i in range(gl.Q):
        for a in range(3):
            if gl.c[i][a] != 0:
                j[a] = j[a] + gl.c[i][a] * st.g[i]
    u = (j + 0.5 * (Fs + Fb)) / (rho - 0.5 * drho * p.M * lap_mu)
    Fa = drho * p.M * lap_mu * u
    moving = st.g[1].copy()
    for i in range(2, gl.Q):
        moving = moving + st.g[i]
    w0 = gl.w[0]
    pres = CS2 / (1 - w0) * (moving + 0.5 * _vdot(u, grad_rho) + rho * w0 * (-_vdot(u, u) / (2 * CS2)))
    return dict(phi=phi, grad=grad, lap=lap, rho=rho, nu=nu, tau=tau, mu_phi=mu_phi,
                pstar=pres / (rho * CS2), p=pres, F=Fs + Fa + Fb, u=u, grad_rho=grad_rho,
                lap_mu=lap_mu, R=None, gamma=None)


# --------------------------------------------------------------------------
# collisions (O10, O11)

def tau_phi(p):
    """Eq. fakhari_tau_model (AC) and its CH form of Sec. II.D.1."""
    if p.model in ("CH", "L14"):
        return p.M / (p.eta * CS2) + 0.5
    return p.M / CS2 + 0.5


def collide_h(p, st, m):
    """Eq. fakhari_g_simplified (BGK) for the phase-field populations."""
    tp = tau_phi(p)
    if p.model in ("CH", "L14"):
        heq = h_eq_ch(p, m["phi"], m["mu_phi"], m["u"])
        phiu = m["phi"] * m["u"]
        G = G_ch(p, phiu - st.phiu_prev)       # backward Euler, delta t = 1
    elif p.model == "L18":
        # Eqs. liang_geq and liang_G_final, d(phi u)/dt by backward Euler
        heq = h_eq_nl(p, m["phi"], m["u"])
        G = G_ch(p, m["phi"] * m["u"] - st.phiu_prev) + G_ac(p, m["phi"], m["grad"])
    elif p.model == "NL":
        # Eqs. Chai_geq and Hu_G (lam = 0: Eq. chai_G)
        heq = h_eq_nl(p, m["phi"], m["u"])
        w = p.lattices[1].w
        G = p.lam * G_ac(p, m["phi"], m["grad"])
        for a in range(p.lattices[1].Q):
            G[a] = G[a] + (1 - p.lam) * w[a] * m["R"]
    else:
        heq = h_eq_ac(p, m["phi"], m["u"])
        G = G_ac(p, m["phi"], m["grad"])
    return st.h - (st.h - heq) / tp + (1 - 1 / (2 * tp)) * G


def collide_g(p, st, m):
    """MRT form of Eq. fakhari_f_simplified: m* = m - S (m - m_eq) + (I - S/2) m_F."""
    gl = p.lattices[0]
    Mmat, stress = mrt.basis(gl)
    Minv = np.linalg.inv(Mmat)
    if p.model == "L18":
        geq = f_eq_liang(p, m["rho"], m["p"], m["u"])
        Fi = force_liang(p, m["F"], m["u"], m["grad_rho"])
    elif p.model == "L14":
        geq = f_eq_liang(p, m["rho"], m["p"], m["u"])
        Fi = force_liang14(p, m["F"], m["u"], m["rho"], m["grad_rho"])
    else:
        geq = g_eq(p, m["pstar"], m["u"])
        Fi = force_populations(p, m["F"], m["rho"])
    mom = np.tensordot(Mmat, st.g, axes=(1, 0))
    mom_eq = np.tensordot(Mmat, geq, axes=(1, 0))
    mom_F = np.tensordot(Mmat, Fi, axes=(1, 0))
    S = np.empty(mom.shape, dtype=np.result_type(m["tau"], p.s_other))
    for k in range(gl.Q):
        S[k] = 1.0 / m["tau"] if k in stress else p.s_other
    post = mom - S * (mom - mom_eq) + (1 - S / 2) * mom_F
    return np.tensordot(Minv, post, axes=(1, 0))


# --------------------------------------------------------------------------
# streaming (O12)

def stream(p, lat, post, kind):
    """Push streaming: f_i(x + c_i) <- f*_i(x), periodic wrap; halfway bounce-back
    at a wall: the population leaving through the wall returns to its node in the
    opposite direction, minus 2 w (c . u_w)/c_s^2 for g at a moving wall."""
    new = np.empty_like(post)
    for i in range(lat.Q):
        c = lat.c[i]
        new[i] = np.roll(post[i], shift=(c[2], c[1], c[0]), axis=(0, 1, 2))
    ax = p.walled_axis()
    if ax is None:
        return new
    arr_ax = _ARRAY_AXIS[ax]
    n = p.shape[arr_ax]
    opp = lat.opp
    for i in range(lat.Q):
        ci = lat.c[i][ax]
        if ci == 0:
            continue
        # nodes whose upstream neighbour x - c_i lies beyond the wall
        layer = 0 if ci > 0 else n - 1
        side = 0 if ci > 0 else 1
        sl = [slice(None)] * 3
        sl[arr_ax] = slice(layer, layer + 1)
        sl = tuple(sl)
        ib = opp[i]
        val = post[ib][sl]
        if kind == "g":
            uw = p.wall_u[side]
            cu = sum(lat.c[ib][a] * uw[a] for a in range(3))
            val = val - 2 * lat.w[ib] * cu / CS2
        # h: only face vectors cross a wall and u_w is tangential, so the
        # moving-wall term of h vanishes
        new[i][sl] = val
    return new


# --------------------------------------------------------------------------
# public API

def step(p, st):
    """One full time step; returns the new post-streaming state."""
    m = macroscopic(p, st)
    g_post = collide_g(p, st, m)
    g_new = stream(p, p.lattices[0], g_post, "g")
    if p.freeze_phi:
        h_new = st.h.copy()
    else:
        h_post = collide_h(p, st, m)
        h_new = stream(p, p.lattices[1], h_post, "h")
    phiu = m["phi"] * m["u"] if p.model in ("CH", "L18", "L14") else None
    return State(g_new, h_new, phiu)


def run(p, st, nsteps):
    for _ in range(nsteps):
        st = step(p, st)
    return st


def init(p, phi0, u0=None, p0=None):
    """h = h_eq(phi0, u0), g = g_eq(p0 / (rho0 c_s^2), u0); CH also stores phi0 u0.
    For NL this makes sum_a h_a = phi0 (the corrected phi of the first step then
    adds (1 - lam) R(phi0) / 2)."""
    phi0 = np.asarray(phi0)
    dt = np.result_type(phi0, 1.0)
    if u0 is None:
        u0 = np.zeros((3,) + p.shape, dtype=dt)
    else:
        u0 = np.asarray(u0)
        if u0.shape[0] == 2:
            u0 = np.concatenate([u0, np.zeros((1,) + p.shape, dtype=u0.dtype)])
    if p0 is None:
        p0 = np.zeros(p.shape, dtype=dt)
    rho0 = _lin(p.rho_H, p.rho_L, phi0)
    pstar0 = p0 / (rho0 * CS2)
    g = g_eq(p, pstar0, u0)
    if p.model == "CH":
        mu0 = chemical_potential(p, phi0, laplacian(p, phi0))
        h = h_eq_ch(p, phi0, mu0, u0)
        return State(g, h, phi0 * u0)
    if p.model == "NL":
        return State(g, h_eq_nl(p, phi0, u0), None)
    if p.model == "L18":
        return State(f_eq_liang(p, rho0, p0, u0), h_eq_nl(p, phi0, u0), phi0 * u0)
    if p.model == "L14":
        mu0 = chemical_potential(p, phi0, laplacian(p, phi0))
        return State(f_eq_liang(p, rho0, p0, u0), h_eq_ch(p, phi0, mu0, u0), phi0 * u0)
    return State(g, h_eq_ac(p, phi0, u0), None)


def fields(p, st):
    """(phi, u, p, rho) of the state; u has dim components."""
    m = macroscopic(p, st)
    return m["phi"], m["u"][:p.dim], m["p"], m["rho"]


def min_image(p, coord, centre, ax):
    d = coord - centre
    if p.bc[ax] == PERIODIC:
        n = (p.nx, p.ny, p.nz)[ax]
        d = d - n * np.round(d / n)
    return d


def diagnostics(p, st, centre=None, R=None):
    """FP64 diagnostics: volume (Eq. volume_continuous), volume by counting
    phi > phi_0 (Sec. IV.A), sum phi, phi extrema (delta phi_max, Sec. III.A),
    max |u|, and the mean pressure inside r < R - 2W and outside r > R + 2W."""
    m = macroscopic(p, st)
    phi = m["phi"].real
    u = m["u"].real
    pres = m["p"].real
    out = dict(
        V_phi=float(np.sum((phi - PHI_L) / (PHI_H - PHI_L))),
        V_count=float(np.count_nonzero(phi > PHI_0)),
        sum_phi=float(np.sum(phi)),
        phi_min=float(phi.min()),
        phi_max=float(phi.max()),
        umax=float(np.sqrt((u * u).sum(axis=0)).max()),
    )
    if centre is not None:
        z, y, x = np.meshgrid(np.arange(p.nz), np.arange(p.ny), np.arange(p.nx), indexing="ij")
        r2 = np.zeros(p.shape)
        for ax, coord in enumerate((x, y, z)):
            if ax < p.dim:
                d = min_image(p, coord.astype(float), centre[ax], ax)
                r2 = r2 + d * d
        r = np.sqrt(r2)
        W = float(np.real(p.W))
        inside = r < R - 2 * W
        outside = r > R + 2 * W
        out.update(p_in=float(pres[inside].mean()) if inside.any() else float("nan"),
                   p_out=float(pres[outside].mean()) if outside.any() else float("nan"),
                   n_in=int(inside.sum()), n_out=int(outside.sum()))
    return out
