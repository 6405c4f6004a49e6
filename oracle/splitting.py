"""Splitting ("BAB") steppers for the proposed method (oracle; test infrastructure).

Paper: Sec. 3.4, the splitting methods.  For y = (c, c'), c'' = -M(z) c with
M = U + Gamma^2, an s-step BAB method alternates kicks of c' and drifts of c:

    for r = 1 .. s:   c' <- c' - h b_r M(tau_{r-1}) c      (kick)
                      c  <- c  + h a_r c'                  (drift)
                      tau_r = tau_{r-1} + h a_r
    finally           c' <- c' - h b_{s+1} M(tau_s) c

with tau_0 = z_i.  Readings: the paper's P-hat / Q-hat
names are read as c / c' (as for the RK stages); kick r evaluates U at
tau_{r-1}, the position reached before that step's drift, and the final kick
uses its own weight b_{s+1} at tau_s (the printed formulas use tau_r before
it is defined and repeat b_s).  Each kick and drift keeps the current
Im(c^H c') when M is Hermitian, so without absorption the method conserves
reflected + transmitted flux exactly, at any step size.

The paper's sp4 and sp6 coefficients (from a reference it cites) are not
printed; the composition here is the fourth-order triple jump of the
Stormer-Verlet step (drift weights g1, g2, g1 with 2 g1 + g2 = 1 and
2 g1^3 + g2^3 = 0, i.e. g1 = 1 / (2 - 2^(1/3))), whose kick weights are the
half sums of neighbouring drift weights.  Pins: the observed order under
step halving and exact flux conservation (tests/test_oracle_splitting.py).
"""
from __future__ import annotations

import numpy as np


class Composition:
    """A BAB splitting method: drift weights a (s), kick weights b (s + 1).

    Kicks sit at tau_r / h - i = cumsum(a)[r - 1] (tau_0 = 0) inside slice i;
    ``cset`` lists the distinct kick positions of a slice other than 1 in
    the order the kicks use them (position 1 is the next slice's 0)."""

    def __init__(self, name, a, b, order):
        self.name = name
        self.a = np.asarray(a, dtype=np.float64)
        self.b = np.asarray(b, dtype=np.float64)
        assert self.b.size == self.a.size + 1
        self.order = order
        self.stages = self.b.size             # evaluations of M per slice (kicks)
        tau = np.concatenate([[0.0], np.cumsum(self.a)])
        self.tau = tau
        self.cset = []
        self._slot = []
        for t in tau:
            if abs(t - 1.0) < 1e-14:
                self._slot.append(None)
            else:
                if not any(abs(t - c) < 1e-14 for c in self.cset):
                    self.cset.append(float(t))
                self._slot.append(next(m for m, c in enumerate(self.cset) if abs(t - c) < 1e-14))

    def node_index(self, slice_i: int, r: int) -> int:
        m = self._slot[r]
        if m is None:
            return (slice_i + 1) * len(self.cset)
        return slice_i * len(self.cset) + m

    def n_nodes(self, n_slices: int) -> int:
        return n_slices * len(self.cset) + 1

    def step(self, Z: np.ndarray, Ms, h: float) -> np.ndarray:
        """One slice on every column of Z = [c; c']; Ms[r] = M(tau_r)."""
        n = Z.shape[0] // 2
        c = Z[:n].copy()
        q = Z[n:].copy()
        for r in range(self.a.size):
            q = q - h * self.b[r] * (Ms[r] @ c)
            c = c + h * self.a[r] * q
        q = q - h * self.b[-1] * (Ms[-1] @ c)
        return np.vstack([c, q])


def _verlet():
    return Composition("verlet", [1.0], [0.5, 0.5], 2)


def _triple_jump4():
    g1 = 1.0 / (2.0 - 2.0 ** (1.0 / 3.0))
    g2 = 1.0 - 2.0 * g1
    return Composition("sp4", [g1, g2, g1], [g1 / 2, (g1 + g2) / 2, (g1 + g2) / 2, g1 / 2], 4)


VERLET = _verlet()
SP4 = _triple_jump4()
