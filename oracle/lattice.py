"""Velocity sets of the oracle (its own copy; the HIP path keeps its own).

Sec. III (2-D tests) uses D2Q9; Sec. IV uses a D3Q7 phase-field lattice with
c_s^2 = 1/3 for both lattices. The hydrodynamic 3-D lattice here is D3Q19 and
the 2-D phase-field lattice D2Q5 (readings listed in the design notes); the
paper's own 3-D hydrodynamic lattice, D3Q27 (Sec. IV), is the alternative.

Canonical population order (shared with the library's canonical I/O, since it
is an interface format):
  D2Q9 : 0 rest, 1 (+1,0), 2 (0,+1), 3 (-1,0), 4 (0,-1),
         5 (+1,+1), 6 (-1,+1), 7 (-1,-1), 8 (+1,-1)
  D2Q5 : the first five D2Q9 vectors
  D3Q19: 0 rest, 1 +x, 2 -x, 3 +y, 4 -y, 5 +z, 6 -z, then the twelve edge
         vectors in opposite pairs (+x+y,-x-y), (+x-y,-x+y), (+x+z,-x-z),
         (+x-z,-x+z), (+y+z,-y-z), (+y-z,-y+z)
  D3Q7 : the first seven D3Q19 vectors
  D3Q27: the nineteen D3Q19 vectors, then the eight corners in opposite pairs
         (+x+y+z,-x-y-z), (+x+y-z,-x-y+z), (+x-y+z,-x+y-z), (-x+y+z,+x-y-z)

Weights. D2Q9: 4/9, 1/9, 1/36. D2Q5 with c_s^2 = 1/3: 1/3, 1/6.
D3Q19: 1/3, 1/18, 1/36. D3Q27: 8/27, 2/27, 1/54, 1/216. D3Q7 with
c_s^2 = 1/3 (Sec. IV states c_s^2 = 1/3 for both lattices): the second-moment
condition sum w e e = c_s^2 I forces 1/6 on the six faces and therefore 0 on
the rest vector.
"""
from dataclasses import dataclass
from fractions import Fraction

import numpy as np

CS2 = 1.0 / 3.0  # lattice sound speed squared, every lattice here


@dataclass(frozen=True)
class Lattice:
    name: str
    dim: int
    c: np.ndarray        # (Q, 3) integer velocities; z component 0 in 2-D
    w_exact: tuple       # Fractions
    @property
    def Q(self):
        return self.c.shape[0]

    @property
    def w(self):
        return np.array([float(x) for x in self.w_exact])

    @property
    def opp(self):
        """Index of the opposite velocity -c_i."""
        out = []
        for ci in self.c:
            j = [k for k, ck in enumerate(self.c) if np.all(ck == -ci)]
            out.append(j[0])
        return np.array(out)


_F = Fraction
D2Q9 = Lattice(
    "D2Q9", 2,
    np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [-1, 0, 0], [0, -1, 0],
              [1, 1, 0], [-1, 1, 0], [-1, -1, 0], [1, -1, 0]]),
    (_F(4, 9),) + (_F(1, 9),) * 4 + (_F(1, 36),) * 4)

D2Q5 = Lattice(
    "D2Q5", 2,
    np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [-1, 0, 0], [0, -1, 0]]),
    (_F(1, 3),) + (_F(1, 6),) * 4)

D3Q19 = Lattice(
    "D3Q19", 3,
    np.array([[0, 0, 0],
              [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1],
              [1, 1, 0], [-1, -1, 0], [1, -1, 0], [-1, 1, 0],
              [1, 0, 1], [-1, 0, -1], [1, 0, -1], [-1, 0, 1],
              [0, 1, 1], [0, -1, -1], [0, 1, -1], [0, -1, 1]]),
    (_F(1, 3),) + (_F(1, 18),) * 6 + (_F(1, 36),) * 12)

D3Q7 = Lattice(
    "D3Q7", 3,
    np.array([[0, 0, 0], [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0],
              [0, 0, 1], [0, 0, -1]]),
    (_F(0),) + (_F(1, 6),) * 6)

D3Q27 = Lattice(
    "D3Q27", 3,
    np.concatenate([D3Q19.c, np.array([[1, 1, 1], [-1, -1, -1], [1, 1, -1], [-1, -1, 1],
                                       [1, -1, 1], [-1, 1, -1], [-1, 1, 1], [1, -1, -1]])]),
    (_F(8, 27),) + (_F(2, 27),) * 6 + (_F(1, 54),) * 12 + (_F(1, 216),) * 8)

# lattice pair id -> (hydrodynamic lattice of g, phase-field lattice of h)
PAIRS = {
    "D2Q9_D2Q5": (D2Q9, D2Q5),
    "D3Q19_D3Q7": (D3Q19, D3Q7),
    "D3Q27_D3Q7": (D3Q27, D3Q7),
}
