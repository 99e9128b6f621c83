"""The derivative oracles agree with each other: complex step of the oracle
against central differences of the oracle (independent of the HIP path)."""
import numpy as np

from oracle import derivatives as dv
from oracle import model as om
from paper_2511_11360_amd import workloads as wl


def _small():
    """A resolved droplet (R / W = 3): its trajectory is well conditioned, so
    central differences are not swamped by amplified rounding."""
    d, phi, u = wl.static_droplet_2d(n=32, R=9.0)
    d.update(W=3.0)
    phi = wl.droplet_phi(d, (16.0, 16.0), 9.0)
    p = om.Params(**d)
    target = wl.droplet_phi(d, (16.5, 15.5), 9.4)
    return p, phi, u, target


def test_complex_step_matches_central_differences_params():
    p, phi, u, target = _small()
    for name in ("sigma", "M", "W"):
        cs = dv.cs_param(p, name, phi, u, 8, target)
        fd = dv.fd_param(p, name, phi, u, 8, target, rel=1e-5)
        assert abs(cs - fd) <= 1e-6 * abs(cs), (name, cs, fd)


def test_complex_step_matches_central_differences_phi0():
    p, phi, u, target = _small()
    v = wl.seeded_field(phi.shape, 7, -1.0, 1.0)
    cs = dv.cs_phi0(p, v, phi, u, 8, target)
    h = 1e-5
    fd = (dv.loss_l2(p, phi + h * v, u, 8, target) - dv.loss_l2(p, phi - h * v, u, 8, target)) / (2 * h)
    assert abs(cs - fd) <= 1e-6 * abs(cs)


def test_step_tangent_is_linear():
    p, phi, u, _ = _small()
    st = om.run(p, om.init(p, phi, u), 3)
    rng = np.random.default_rng(1)
    v1 = (rng.standard_normal(st.g.shape), rng.standard_normal(st.h.shape))
    v2 = (rng.standard_normal(st.g.shape), rng.standard_normal(st.h.shape))
    a = dv.step_jvp(p, st, *v1)
    b = dv.step_jvp(p, st, *v2)
    c = dv.step_jvp(p, st, v1[0] + 2 * v2[0], v1[1] + 2 * v2[1])
    for k in range(2):
        assert np.allclose(c[k], a[k] + 2 * b[k], rtol=1e-12, atol=1e-12)
