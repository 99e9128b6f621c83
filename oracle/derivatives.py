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


def step_jvp(p, st, vg, vh, vpu=None, h=1e-30):
    """Tangent of one step at state st along (vg, vh): (J v)_g, (J v)_h. A state
    that carries (phi u) of the previous step (the CH model) is perturbed along
    vpu too (zero if None) and its tangent (J v)_pu is returned third."""
    pu = None
    if st.phiu_prev is not None:
        pu = st.phiu_prev + (1j * h * vpu if vpu is not None else 0j)
    out = om.step(p, om.State(st.g + 1j * h * vg, st.h + 1j * h * vh, pu))
    if pu is None:
        return np.imag(out.g) / h, np.imag(out.h) / h
    return np.imag(out.g) / h, np.imag(out.h) / h, np.imag(out.phiu_prev) / h


def step_param_tangent(p, st, name, h=1e-30):
    """d(step output)/d(name) at state st (with the (phi u) part third when the
    state carries it)."""
    pc = _with(p, **{name: complex(getattr(p, name), h)})
    pu = None if st.phiu_prev is None else st.phiu_prev.astype(complex)
    out = om.step(pc, om.State(st.g.astype(complex), st.h.astype(complex), pu))
    if pu is None:
        return np.imag(out.g) / h, np.imag(out.h) / h
    return np.imag(out.g) / h, np.imag(out.h) / h, np.imag(out.phiu_prev) / h


def init_jvp(p, phi0, v, u0=None, p0=None, name=None, h=1e-30):
    """Tangent of the initial state (g, h[, phi u]) along v in phi0, or, with
    name given, with respect to that parameter (v unused)."""
    if name is None:
        st = om.init(p, phi0 + 1j * h * v, u0, p0)
    else:
        st = om.init(_with(p, **{name: complex(getattr(p, name), h)}), phi0.astype(complex), u0, p0)
    out = [np.imag(st.g) / h, np.imag(st.h) / h]
    if st.phiu_prev is not None:
        out.append(np.imag(st.phiu_prev) / h)
    return tuple(out)


def fields_phi_tangent(p, st, vh=None, name=None, h=1e-30):
    """Tangent of the phase field the state reports (om.fields: for the
    nonlocal model the corrected phi*) along vh in h, or, with name given,
    with respect to that parameter."""
    if name is None:
        sc = om.State(st.g.astype(complex), st.h + 1j * h * vh,
                      None if st.phiu_prev is None else st.phiu_prev.astype(complex))
        return np.imag(om.fields(p, sc)[0]) / h
    pc = _with(p, **{name: complex(getattr(p, name), h)})
    sc = om.State(st.g.astype(complex), st.h.astype(complex),
                  None if st.phiu_prev is None else st.phiu_prev.astype(complex))
    return np.imag(om.fields(pc, sc)[0]) / h
