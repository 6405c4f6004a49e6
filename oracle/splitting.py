"""Splitting steppers (BAB and ABA forms) for the proposed method (oracle; test infrastructure).

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
half sums of neighbouring drift weights.  A sixth-order method follows by
the same construction one level up: the triple jump of that fourth-order
step, with weights w1, w0, w1, 2 w1 + w0 = 1 and 2 w1^5 + w0^5 = 0, i.e.
w1 = 1 / (2 - 2^(1/5)) (nine Stormer-Verlet steps of lengths w_i g_j).  The
ABA form exchanges the roles: a slice starts and ends with a drift and the
kicks sit in between (drift weights the half sums of neighbouring kick
weights); its kick r uses U at the position reached by the drifts before it.
Pins: the observed order under step halving and exact flux conservation
(tests/test_oracle_splitting.py).
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

    def step_tangent(self, Z, dZ, Ms, dMs, h):
        """The slice and its derivative along dZ and the tangents dMs of the
        M(tau_r) (each kick and drift is linear in (c, c'), so the tangent
        takes the same kicks and drifts plus -h b_r dM_r c in each kick)."""
        n = Z.shape[0] // 2
        c, q, dc, dq = Z[:n].copy(), Z[n:].copy(), dZ[:n].copy(), dZ[n:].copy()
        for r in range(self.a.size):
            dq = dq - h * self.b[r] * (dMs[r] @ c + Ms[r] @ dc)
            q = q - h * self.b[r] * (Ms[r] @ c)
            c = c + h * self.a[r] * q
            dc = dc + h * self.a[r] * dq
        dq = dq - h * self.b[-1] * (dMs[-1] @ c + Ms[-1] @ dc)
        q = q - h * self.b[-1] * (Ms[-1] @ c)
        return np.vstack([c, q]), np.vstack([dc, dq])


class CompositionABA:
    """An ABA splitting method: drift weights a (s + 1), kick weights b (s).

    A slice is c <- c + h a_0 c', then for r = 1 .. s: c' <- c' - h b_r
    M(tau_r) c, c <- c + h a_r c' with tau_r = z_i + h (a_0 + .. + a_{r-1}).
    ``cset`` lists the distinct kick positions in the order the kicks use
    them; none is at a slice boundary."""

    def __init__(self, name, a, b, order):
        self.name = name
        self.a = np.asarray(a, dtype=np.float64)
        self.b = np.asarray(b, dtype=np.float64)
        assert self.a.size == self.b.size + 1
        self.order = order
        self.stages = self.b.size
        self.tau = np.cumsum(self.a)[:-1]
        self.cset = []
        self._slot = []
        for t in self.tau:
            if not any(abs(t - c) < 1e-14 for c in self.cset):
                self.cset.append(float(t))
            self._slot.append(next(m for m, c in enumerate(self.cset) if abs(t - c) < 1e-14))

    def node_index(self, slice_i: int, r: int) -> int:
        return slice_i * len(self.cset) + self._slot[r]

    def n_nodes(self, n_slices: int) -> int:
        return n_slices * len(self.cset) + 1

    def step(self, Z: np.ndarray, Ms, h: float) -> np.ndarray:
        """One slice on every column of Z = [c; c']; Ms[r] = M(tau_r)."""
        n = Z.shape[0] // 2
        c = Z[:n].copy()
        q = Z[n:].copy()
        c = c + h * self.a[0] * q
        for r in range(self.b.size):
            q = q - h * self.b[r] * (Ms[r] @ c)
            c = c + h * self.a[r + 1] * q
        return np.vstack([c, q])

    def step_tangent(self, Z, dZ, Ms, dMs, h):
        """The slice and its derivative (as Composition.step_tangent)."""
        n = Z.shape[0] // 2
        c, q, dc, dq = Z[:n].copy(), Z[n:].copy(), dZ[:n].copy(), dZ[n:].copy()
        c = c + h * self.a[0] * q
        dc = dc + h * self.a[0] * dq
        for r in range(self.b.size):
            dq = dq - h * self.b[r] * (dMs[r] @ c + Ms[r] @ dc)
            q = q - h * self.b[r] * (Ms[r] @ c)
            c = c + h * self.a[r + 1] * q
            dc = dc + h * self.a[r + 1] * dq
        return np.vstack([c, q]), np.vstack([dc, dq])


def _half_sums(w):
    """Weights of the other kind in a composition of symmetric steps of
    lengths w: w_0 / 2, (w_0 + w_1) / 2, ..., w_last / 2."""
    w = list(w)
    return [w[0] / 2] + [(w[k] + w[k + 1]) / 2 for k in range(len(w) - 1)] + [w[-1] / 2]


def _triple_jump(p):
    """Outer weights w1, inner w0 of the triple jump raising order p to p + 2:
    2 w1 + w0 = 1 and 2 w1^(p+1) + w0^(p+1) = 0."""
    w1 = 1.0 / (2.0 - 2.0 ** (1.0 / (p + 1)))
    return w1, 1.0 - 2.0 * w1


def _steps4():
    g1, g2 = _triple_jump(2)
    return [g1, g2, g1]


def _steps6():
    w1, w0 = _triple_jump(4)
    return [w * g for w in (w1, w0, w1) for g in _steps4()]


def _verlet():
    return Composition("verlet", [1.0], [0.5, 0.5], 2)


def _triple_jump4():
    st = _steps4()
    return Composition("sp4", st, _half_sums(st), 4)


def _triple_jump6():
    st = _steps6()
    return Composition("sp6", st, _half_sums(st), 6)


def _aba(name, steps, order):
    return CompositionABA(name, _half_sums(steps), steps, order)


VERLET = _verlet()
SP4 = _triple_jump4()
SP6 = _triple_jump6()
SP4_ABA = _aba("sp4a", _steps4(), 4)
SP6_ABA = _aba("sp6a", _steps6(), 6)
