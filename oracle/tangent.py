"""Tangent-linear (forward-mode) derivative of the RK and splitting methods (oracle; test infrastructure).

Differentiates ``rk.solve_ode_str`` along a direction dU of the potential
table.  Every step of Algorithm 1 (Sec. 3.2) is linear in Z, so the
tangent dZ is stepped by the same stages with the extra source
-(dU_r) Y_r^{(c)} in each stage (Sec. 3.4).  At a right-hand-side
transformation Z' = Z Q^{-1} (T = Q^{-1}, Q the upper block) the tangent
is the exact derivative dZ' = (dZ - Z' dQ) Q^{-1}, whose upper block is 0.
(By the invariance of Sec. 3.2, dropping the term Z' dQ Q^{-1} would not
change d rho(0) in exact arithmetic, but that term is what keeps the
tangent from growing along the dominant modes: without it the tangent's
norm grows like the unnormalised state and the final formula cancels
catastrophically on thick slabs.)  The final formula
rho = (Gamma Q + iP) x, (Gamma Q - iP) x = e_1 (Eq. vrhocomp, first
column) is differentiated by the product and inverse rules.

Pins: central finite differences of the oracle forward, and the
dot-product identity between this tangent and finite differences along
random directions (tests/test_oracle_solvers.py).
"""
from __future__ import annotations

import math

import numpy as np

from .rk import THRESHOLD, estcond_gershgorin, initial_state


def solve_ode_str_tangent(Mfun, dUfun, gam, h, n_slices, tab, threshold=THRESHOLD, y_bottom=None):
    """Returns (rho, drho).  ``dUfun(i, r)`` is the n x n tangent of U at the
    node of stage r of slice i (Gamma does not depend on U).  ``y_bottom``:
    the state [I; Y] of a bulk below the slab, held fixed (its tangent is 0)."""
    n = gam.size
    Z = initial_state(gam, y_bottom=y_bottom)
    dZ = np.zeros_like(Z)
    for i in range(n_slices):
        if hasattr(tab, "step_tangent"):
            # a splitting method (Sec. 3.4): kicks and drifts, each linear in Z
            Ms = [Mfun(i, r) for r in range(tab.stages)]
            dMs = [dUfun(i, r) for r in range(tab.stages)]
            Z, dZ = tab.step_tangent(Z, dZ, Ms, dMs, h)
            if estcond_gershgorin(Z[:n]) > threshold:
                T = np.linalg.inv(Z[:n])
                Z = Z @ T
                dZ = (dZ - Z @ dZ[:n]) @ T
            continue
        K, dK = [], []
        for r in range(tab.stages):
            Yr, dYr = Z.copy(), dZ.copy()
            for j in range(r):
                if tab.a[r, j] != 0.0:
                    Yr = Yr + h * tab.a[r, j] * K[j]
                    dYr = dYr + h * tab.a[r, j] * dK[j]
            M = Mfun(i, r)
            dU = dUfun(i, r)
            Kr = np.empty_like(Z)
            dKr = np.empty_like(Z)
            Kr[:n] = Yr[n:]
            dKr[:n] = dYr[n:]
            Kr[n:] = -(M @ Yr[:n])
            dKr[n:] = -(dU @ Yr[:n] + M @ dYr[:n])
            K.append(Kr)
            dK.append(dKr)
        for r in range(tab.stages):
            if tab.b[r] != 0.0:
                Z = Z + h * tab.b[r] * K[r]
                dZ = dZ + h * tab.b[r] * dK[r]
        if estcond_gershgorin(Z[:n]) > threshold:
            T = np.linalg.inv(Z[:n])
            Z = Z @ T
            dZ = (dZ - Z @ dZ[:n]) @ T
    Q, P, dQ, dP = Z[:n], Z[n:], dZ[:n], dZ[n:]
    top = gam[:, None] * Q - 1j * P
    bot = gam[:, None] * Q + 1j * P
    dtop = gam[:, None] * dQ - 1j * dP
    dbot = gam[:, None] * dQ + 1j * dP
    e1 = np.zeros(n, dtype=np.complex128)
    e1[0] = 1.0
    x = np.linalg.solve(top, e1)
    dx = -np.linalg.solve(top, dtop @ x)
    return bot @ x, dbot @ x + bot @ dx


def intensity_tangent(rho, drho, gam, open_mask, theta0, convention="flux"):
    """d eta_j = (Gamma_0/Gamma_j) 2 Re(conj(rho_j) d rho_j) on open beams."""
    d = np.zeros(rho.shape, dtype=np.float64)
    g0 = gam[0].real
    d[open_mask] = 2.0 * np.real(np.conj(rho[open_mask]) * drho[open_mask]) * g0 / gam[open_mask].real
    if convention == "paper":
        d *= math.sin(theta0)
    return d
