"""The conventional multi-slice method (oracle; test infrastructure).

Paper: Sec. 2.2.  The coefficient matrix is frozen at each slice midpoint
(Eq. ds0), the slice is propagated exactly by its matrix exponential
(Eq. ichimiya2), and the boundary value problem is solved either through
the whole product (Eq. ichimiya3-ichimiya4, ill-conditioned, only for thin
slabs) or by the recursive reflection technique (Eq. ri1-ri2).

Three independent formulations live here:

* ``eigen_multislice`` -- economical form Z (Sec. 3.1) with the exact
  slice map exp(h B_i), B_i = [[0, I], [-M_i, 0]], M_i = U(mid) + Gamma^2,
  evaluated from an eigendecomposition of the n x n matrix M_i:
  [[cos(hW), sin(hW) W^{-1}], [-W sin(hW), cos(hW)]] with W^2 = M_i (these
  are even functions of W, so no square-root branch is involved).  After
  each slice Z <- Z Q^{-1}; by Sec. 3.3 this is the recursive reflection
  technique.
* ``ichimiya_recursion`` -- the (tau, rho) form with A(z) of Eq. (tr1),
  exp(h A_i) by ``scipy.linalg.expm``, and the recursion of Eq. (ri1).
* ``global_product`` -- Eq. (ichimiya4) on the full product.

Pins: agreement of the three with each other and with the single-beam
closed form, L-independence for piecewise-constant potentials, flux
conservation (tests/test_oracle_solvers.py).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from .rk import initial_state, reflection


def _slice_map(M: np.ndarray, h: float) -> np.ndarray:
    lam, V = np.linalg.eig(M)
    w = np.sqrt(lam.astype(np.complex128))
    hw = h * w
    cos = np.cos(hw)
    small = np.abs(hw) < 1e-6
    sinc = np.where(small, h * (1 - hw * hw / 6.0), np.sin(hw) / np.where(small, 1.0, w))
    wsin = w * np.sin(hw)
    Vi = np.linalg.inv(V)
    C = (V * cos[None, :]) @ Vi
    S1 = (V * sinc[None, :]) @ Vi
    S2 = -(V * wsin[None, :]) @ Vi
    return np.block([[C, S1], [S2, C]])


def eigen_multislice(Mmid, gam, h, n_slices):
    """``Mmid(i)`` = U(z_i + h/2) + Gamma^2.  Returns rho(0)."""
    n = gam.size
    Z = initial_state(gam)
    for i in range(n_slices):
        Z = _slice_map(Mmid(i), h) @ Z
        Z = Z @ np.linalg.inv(Z[:n])
    return reflection(Z, gam)


def tau_rho_generator(U: np.ndarray, gam: np.ndarray) -> np.ndarray:
    """A(z) of Eq. (tr1)."""
    n = gam.size
    UG = 0.5j * U / gam[None, :]
    G = np.diag(1j * gam)
    return np.block([[UG + G, UG], [-UG, -UG - G]])


def ichimiya_recursion(Umid, gam, h, n_slices):
    """``Umid(i)`` = U(z_i + h/2) (without Gamma^2).  Returns rho(0)."""
    n = gam.size
    R = np.zeros((n, n), dtype=np.complex128)
    for i in range(n_slices):
        Ah = scipy.linalg.expm(h * tau_rho_generator(Umid(i), gam))
        X, Y, Zb, W = Ah[:n, :n], Ah[:n, n:], Ah[n:, :n], Ah[n:, n:]
        num = Zb + W @ R
        den = X + Y @ R
        R = np.linalg.solve(den.T, num.T).T
    e1 = np.zeros(n, dtype=np.complex128)
    e1[0] = 1.0
    return R @ e1


def global_product(Umid, gam, h, n_slices):
    """Eq. (ichimiya4): rho(0) = Z X^{-1} tau(0) from the whole product."""
    n = gam.size
    P = np.eye(2 * n, dtype=np.complex128)
    for i in range(n_slices):
        P = scipy.linalg.expm(h * tau_rho_generator(Umid(i), gam)) @ P
    X, Zb = P[:n, :n], P[n:, :n]
    e1 = np.zeros(n, dtype=np.complex128)
    e1[0] = 1.0
    return Zb @ np.linalg.solve(X, e1)
