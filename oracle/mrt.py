"""Moment bases for the multiple-relaxation-time (MRT) collision of g.

The paper runs its 3-D hydrodynamics with an MRT operator (Sec. IV, lattice
paragraph) but prints neither basis nor rates. The reading taken here: the
orthogonal polynomial bases of Lallemand & Luo (2000) for D2Q9 and of
d'Humieres et al. (2002) for D3Q19, with the viscous-stress moments relaxed at
1/tau(x) (tau from Eq. fakhari_tau_model) and every other moment at one rate
s_o. Rows are written as polynomials of the velocity components and evaluated
on the oracle's own velocity table. For D3Q27 the rows up to second order are
written out and the seventeen higher monomials are orthogonalised against
them in exact rational arithmetic (Gram-Schmidt); with two rates the
collision depends only on the span of the stress rows, so any orthogonal
completion gives the same operator.
"""
from fractions import Fraction

import numpy as np

from .lattice import D2Q9, D3Q19, D3Q27


def _rows_d2q9(c):
    cx, cy = c[:, 0].astype(float), c[:, 1].astype(float)
    c2 = cx * cx + cy * cy
    rows = [
        np.ones_like(cx),                 # density
        -4 + 3 * c2,                      # energy
        4 - 10.5 * c2 + 4.5 * c2 * c2,    # energy squared
        cx,                               # j_x
        (-5 + 3 * c2) * cx,               # q_x
        cy,                               # j_y
        (-5 + 3 * c2) * cy,               # q_y
        cx * cx - cy * cy,                # p_xx  (stress)
        cx * cy,                          # p_xy  (stress)
    ]
    return np.array(rows), [7, 8]


def _rows_d3q19(c):
    cx, cy, cz = (c[:, k].astype(float) for k in range(3))
    c2 = cx * cx + cy * cy + cz * cz
    rows = [
        np.ones_like(cx),                          # density
        19 * c2 - 30,                              # energy
        (21 * c2 * c2 - 53 * c2 + 24) / 2,         # energy squared
        cx, (5 * c2 - 9) * cx,                     # j_x, q_x
        cy, (5 * c2 - 9) * cy,                     # j_y, q_y
        cz, (5 * c2 - 9) * cz,                     # j_z, q_z
        3 * cx * cx - c2,                          # 3 p_xx   (stress)
        (3 * c2 - 5) * (3 * cx * cx - c2),         # 3 pi_xx
        cy * cy - cz * cz,                         # p_ww     (stress)
        (3 * c2 - 5) * (cy * cy - cz * cz),        # pi_ww
        cx * cy, cy * cz, cx * cz,                 # p_xy, p_yz, p_xz (stress)
        (cy * cy - cz * cz) * cx,                  # m_x
        (cz * cz - cx * cx) * cy,                  # m_y
        (cx * cx - cy * cy) * cz,                  # m_z
    ]
    return np.array(rows), [9, 11, 13, 14, 15]


def _rows_d3q27(c):
    cx, cy, cz = ([int(v) for v in c[:, k]] for k in range(3))
    Q = len(cx)
    c2 = [cx[i] ** 2 + cy[i] ** 2 + cz[i] ** 2 for i in range(Q)]
    F = Fraction
    rows = [
        [F(1)] * Q,                                        # density
        [F(v) for v in cx], [F(v) for v in cy], [F(v) for v in cz],   # j
        [F(c2[i] - 2) for i in range(Q)],                  # energy (mean of c^2 is 2)
        [F(3 * cx[i] ** 2 - c2[i]) for i in range(Q)],     # 3 p_xx   (stress)
        [F(cy[i] ** 2 - cz[i] ** 2) for i in range(Q)],    # p_ww     (stress)
        [F(cx[i] * cy[i]) for i in range(Q)],              # p_xy     (stress)
        [F(cy[i] * cz[i]) for i in range(Q)],              # p_yz     (stress)
        [F(cx[i] * cz[i]) for i in range(Q)],              # p_xz     (stress)
    ]
    # the seventeen monomials cx^a cy^b cz^c (a, b, c <= 2) of degree >= 3
    expo = [(2, 1, 0), (2, 0, 1), (1, 2, 0), (0, 2, 1), (1, 0, 2), (0, 1, 2), (1, 1, 1),
            (2, 2, 0), (2, 0, 2), (0, 2, 2), (2, 1, 1), (1, 2, 1), (1, 1, 2),
            (2, 2, 1), (2, 1, 2), (1, 2, 2), (2, 2, 2)]
    for a, b, e in expo:
        v = [F(cx[i] ** a * cy[i] ** b * cz[i] ** e) for i in range(Q)]
        for r in rows:
            k = sum(x * y for x, y in zip(v, r)) / sum(y * y for y in r)
            v = [x - k * y for x, y in zip(v, r)]
        rows.append(v)
    return np.array([[float(x) for x in r] for r in rows]), [5, 6, 7, 8, 9]


_BUILDERS = {D2Q9.name: _rows_d2q9, D3Q19.name: _rows_d3q19, D3Q27.name: _rows_d3q27}
_CACHE = {}


def basis(lattice):
    """Return (M, stress_rows): M is Q x Q with M[k, i] = moment k of c_i
    (built once per lattice; callers must not modify M)."""
    if lattice.name not in _BUILDERS:
        raise ValueError("no MRT basis for " + lattice.name)
    if lattice.name not in _CACHE:
        _CACHE[lattice.name] = _BUILDERS[lattice.name](lattice.c)
    M, stress = _CACHE[lattice.name]
    return M, list(stress)
