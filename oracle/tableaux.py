"""Explicit Runge-Kutta tableaux (oracle; test infrastructure).

Paper: Sec. 3.4 describes an s-stage explicit RK method by coefficients
a_{r,j}, weights b_j and nodes c_r; the experiments use the classical
fourth-order method (``rk4``).  The sixth-order method is Butcher's
seven-stage scheme (J. C. Butcher, "On Runge-Kutta processes of high
order", J. Austral. Math. Soc. 4 (1964)); the paper's own high-order runs
use splitting methods whose coefficients are not reproduced here.

Pins: every order condition up to the claimed order is checked by
rooted-tree elementary weights in tests/test_oracle_basics.py, and the
observed convergence ratio under step halving in tests/test_oracle_solvers.py.
"""
from __future__ import annotations

from fractions import Fraction as F

import numpy as np


class Tableau:
    def __init__(self, name, a, b, c, order):
        self.name = name
        self.a_frac = a
        self.b_frac = b
        self.c_frac = c
        self.a = np.array([[float(x) for x in row] for row in a])
        self.b = np.array([float(x) for x in b])
        self.c = np.array([float(x) for x in c])
        self.order = order
        self.stages = len(b)
        # distinct node fractions inside a slice (c = 1 is the next slice's 0)
        self.cset = sorted({x for x in c if x < 1})

    def node_index(self, slice_i: int, r: int) -> int:
        c = self.c_frac[r]
        if c == 1:
            return (slice_i + 1) * len(self.cset)
        return slice_i * len(self.cset) + self.cset.index(c)

    def n_nodes(self, n_slices: int) -> int:
        return n_slices * len(self.cset) + 1


def _rk4():
    z = F(0)
    a = [[z, z, z, z],
         [F(1, 2), z, z, z],
         [z, F(1, 2), z, z],
         [z, z, F(1), z]]
    b = [F(1, 6), F(1, 3), F(1, 3), F(1, 6)]
    c = [z, F(1, 2), F(1, 2), F(1)]
    return Tableau("rk4", a, b, c, 4)


def _butcher6():
    z = F(0)
    a = [[z] * 7,
         [F(1, 3), z, z, z, z, z, z],
         [z, F(2, 3), z, z, z, z, z],
         [F(1, 12), F(1, 3), F(-1, 12), z, z, z, z],
         [F(-1, 16), F(9, 8), F(-3, 16), F(-3, 8), z, z, z],
         [z, F(9, 8), F(-3, 8), F(-3, 4), F(1, 2), z, z],
         [F(9, 44), F(-9, 11), F(63, 44), F(18, 11), z, F(-16, 11), z]]
    b = [F(11, 120), z, F(27, 40), F(27, 40), F(-4, 15), F(-4, 15), F(11, 120)]
    c = [z, F(1, 3), F(2, 3), F(1, 3), F(1, 2), F(1, 2), F(1)]
    return Tableau("rk6", a, b, c, 6)


RK4 = _rk4()
RK6 = _butcher6()
TABLEAUX = {"rk4": RK4, "rk6": RK6}

# the splitting steppers of Sec. 3.4 share the node-table interface
from .splitting import SP4, SP4_ABA, SP6, SP6_ABA, VERLET  # noqa: E402

TABLEAUX.update({"sp4": SP4, "sp6": SP6, "sp4a": SP4_ABA, "sp6a": SP6_ABA, "verlet": VERLET})
