"""Closed-form steady velocity of the layered two-phase Poiseuille flow
(Sec. III.D, Eq. analytical_solution), evaluated by adaptive quadrature on the
continuous diffuse-interface viscosity, and the L2 error of Eq. ux-error.

Channel coordinate Y in [-H, H], heavy fluid below Y = 0; the order parameter
is phi(Y) = 1/2 + 1/2 tanh(-2 Y / W) and the dynamic viscosity its linear
interpolation (Eq. mu_linear).
"""
import numpy as np
from scipy.integrate import quad


def mu_of_Y(Y, mu_H, mu_L, W):
    phi = 0.5 + 0.5 * np.tanh(-2.0 * Y / W)
    return mu_H * phi + mu_L * (1.0 - phi)


def analytic_ux(Ys, H, G, mu_H, mu_L, W):
    """u_x(Y) = G / I0 * [ I0 * int_Y^H Y'/mu dY' + I1 * int_H^Y 1/mu dY' ],
    I0 = int_{-H}^{H} 1/mu, I1 = int_{-H}^{H} Y/mu."""
    inv = lambda Y: 1.0 / mu_of_Y(Y, mu_H, mu_L, W)
    Yinv = lambda Y: Y / mu_of_Y(Y, mu_H, mu_L, W)
    opts = dict(limit=400, epsabs=0.0, epsrel=1e-12, points=[0.0])
    I0 = quad(inv, -H, H, **opts)[0]
    I1 = quad(Yinv, -H, H, **opts)[0]
    out = []
    for Y in Ys:
        pts = [0.0] if min(Y, H) < 0.0 < max(Y, H) else None
        o = dict(limit=400, epsabs=0.0, epsrel=1e-12, points=pts)
        a = quad(Yinv, Y, H, **o)[0]
        b = -quad(inv, Y, H, **o)[0]
        out.append(G / I0 * (I0 * a + I1 * b))
    return np.array(out)


def l2_error(u, ua):
    """Eq. ux-error."""
    u = np.asarray(u)
    ua = np.asarray(ua)
    return float(np.sqrt(np.sum((u - ua) ** 2) / np.sum(ua ** 2)))
