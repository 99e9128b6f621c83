"""Derivatives of the oracle by complex step and by central differences.

Test infrastructure only. The complex-step derivative of a real-analytic f is
Im f(x + i h v) / h, exact to rounding for tiny h (no subtractive
cancellation); every oracle routine accepts complex128 inputs for this.
"""
from dataclasses import replace

import numpy as np

from . import model as om


def _with(p, **kw):
    return replace(p, **kw)


def phi_after(p, phi0, u0, steps, p0=None):
    st = om.run(p, om.init(p, phi0, u0, p0), steps)
    return om.fields(p, st)[0]


def loss_l2(p, phi0, u0, steps, target):
    """L = 1/2 sum (phi_N - target)^2 (target real)."""
    d = phi_after(p, phi0, u0, steps) - target
    return 0.5 * np.sum(d * d)


def cs_param(p, name, phi0, u0, steps, target, h=1e-30):
    """dL/d(name) for name in sigma, M, W by complex step."""
    val = getattr(p, name)
    pc = _with(p, **{name: complex(val, h)})
    return float(np.imag(loss_l2(pc, phi0.astype(complex), u0, steps, target)) / h)


def cs_phi0(p, v, phi0, u0, steps, target, h=1e-30):
    """<dL/dphi0, v> by complex step along v."""
    return float(np.imag(loss_l2(p, phi0 + 1j * h * v, u0, steps, target)) / h)


def fd_param(p, name, phi0, u0, steps, target, rel=1e-5):
    """Central difference of L in one parameter."""
    val = getattr(p, name)
    dh = rel * abs(val)
    lp = loss_l2(_with(p, **{name: val + dh}), phi0, u0, steps, target)
    lm = loss_l2(_with(p, **{name: val - dh}), phi0, u0, steps, target)
    return float((lp - lm) / (2 * dh))


def step_jvp(p, st, vg, vh, h=1e-30):
    """Tangent of one step at state st along (vg, vh): (J v)_g, (J v)_h."""
    sc = om.State(st.g + 1j * h * vg, st.h + 1j * h * vh)
    out = om.step(p, sc)
    return np.imag(out.g) / h, np.imag(out.h) / h


def step_param_tangent(p, st, name, h=1e-30):
    """d(step output)/d(name) at state st."""
    pc = _with(p, **{name: complex(getattr(p, name), h)})
    sc = om.State(st.g.astype(complex), st.h.astype(complex))
    out = om.step(pc, sc)
    return np.imag(out.g) / h, np.imag(out.h) / h
