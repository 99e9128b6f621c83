"""Moment bases for the multiple-relaxation-time (MRT) collision of g.

The paper runs its 3-D hydrodynamics with an MRT operator (Sec. IV, lattice
paragraph) but prints neither basis nor rates. The reading taken here: the
orthogonal polynomial bases of Lallemand & Luo (2000) for D2Q9 and of
d'Humieres et al. (2002) for D3Q19, with the viscous-stress moments relaxed at
1/tau(x) (tau from Eq. fakhari_tau_model) and every other moment at one rate
s_o. Rows are written as polynomials of the velocity components and evaluated
on the oracle's own velocity table.
"""
import numpy as np

from .lattice import D2Q9, D3Q19


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


def basis(lattice):
    """Return (M, stress_rows): M is Q x Q with M[k, i] = moment k of c_i."""
    if lattice.name == D2Q9.name:
        return _rows_d2q9(lattice.c)
    if lattice.name == D3Q19.name:
        return _rows_d3q19(lattice.c)
    raise ValueError("no MRT basis for " + lattice.name)
