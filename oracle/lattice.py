"""Discrete velocity sets (oracle).

D2Q9 follows Sec. 2.1.1 of the paper: the velocity matrix and weight table
printed there, with c_s^2 = 1/3 and lattice units dx = dt = 1. The ordering
c_0..c_8 is the printed one (rest, east, north, west, south, NE, NW, SW, SE),
which the printed boundary rules (Eqs. wall, inlet, outlet) index into.

D3Q19 is not in the paper (it is 2D only and names 3D as future work); the
textbook set with weights 1/3, 1/18 (x6), 1/36 (x12) is used for the 3D
scale-up of the same operator.
"""

import numpy as np


class Lattice:
    """A velocity set: c (Q x d integer), w (Q,), opp (Q,), cs2."""

    def __init__(self, name, c, w):
        self.name = name
        self.c = np.asarray(c, dtype=np.int64)
        self.w = np.asarray(w, dtype=np.float64)
        self.Q, self.d = self.c.shape
        self.cs2 = 1.0 / 3.0
        # opposite direction: c_opp = -c
        opp = []
        for a in range(self.Q):
            match = [b for b in range(self.Q) if np.all(self.c[b] == -self.c[a])]
            assert len(match) == 1
            opp.append(match[0])
        self.opp = np.asarray(opp, dtype=np.int64)


# Sec. 2.1.1: c = [[0,1,0,-1,0,1,-1,-1,1],[0,0,1,0,-1,1,1,-1,-1]]
D2Q9 = Lattice(
    "D2Q9",
    c=[(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)],
    w=[4 / 9] + [1 / 9] * 4 + [1 / 36] * 4,
)


def _d3q19():
    c = [(0, 0, 0)]
    for ax in range(3):
        for sgn in (1, -1):
            v = [0, 0, 0]
            v[ax] = sgn
            c.append(tuple(v))
    for a, b in ((0, 1), (0, 2), (1, 2)):
        for sa in (1, -1):
            for sb in (1, -1):
                v = [0, 0, 0]
                v[a] = sa
                v[b] = sb
                c.append(tuple(v))
    w = [1 / 3] + [1 / 18] * 6 + [1 / 36] * 12
    return Lattice("D3Q19", c, w)


D3Q19 = _d3q19()
