"""The proposed method: matrix ODE + explicit RK + RHST (oracle; test infrastructure).

Paper: Sec. 3.1 (Eq. ode2 and the economical form, Eq. mateq2 and
Eq. vrhocomp), Sec. 3.2 (right-hand-side transformation and Algorithm 1
"SolveODE_STR"), Sec. 3.4 (explicit Runge-Kutta stages).

What is computed for one (structure, angle) pair:

    y = (c, c'),  y' = B(z) y,  B = [[0, I], [-(U(z) + Gamma^2), 0]]
    Z(z_e) = Z0 (2n x n), stepped slice by slice from z_e = -D to 0;
    after each slice: xi = estimated condition number of the upper block Q;
    if xi > 1000: Z <- Z Q^{-1}  (RHST);
    finally Z <- S Z with S = [[Gamma, -iI], [Gamma, iI]],
    R = Z_lower Z_upper^{-1}, rho(0) = R[:, 0].

Readings where the paper is silent or ambiguous:
* Sec. 3.4 names the stage matrices p, q the other way round from Sec. 3.1;
  the stages here are the textbook explicit RK on y = (c, c'), and the RHST
  normalises the c-block (upper half), as Algorithm 1 does.
* Z0: the paper's S^{-1}[I; O] = (1/2)[Gamma^{-1}; iI] contains Gamma^{-1};
  [I; i Gamma] spans the same column space (it is S^{-1}[I;O] (2 Gamma)) and
  has no division, so it is the default.  Both are available.
* Bulk layer (Sec. 2.2, treatment of the bulk layer): below z_e the
  crystal may continue as the bulk.  Its bottom condition is given as the
  normalised state [I; Y] the bulk leaves at z_e (c' = Y c there, the form
  a right-hand-side transformation leaves); the vacuum is Y = i Gamma, and
  the reflection matrix at z_e is R = (Gamma + iY)(Gamma - iY)^{-1}.
* xi ("estcondGC"): the Gershgorin/Varah bound
  max_i(|q_ii| + r_i) / min_i(|q_ii| - r_i), r_i = sum_{j != i} |q_ij|,
  and +inf when some row is not strictly diagonally dominant.  It never
  underestimates cond_inf(Q) and equals 1 at Q = I.
* Threshold 1000 with a strict ">".
* Slab z in [-D, 0]; slice i spans [-D + i h, -D + (i+1) h]; stage r of
  slice i evaluates U at -D + (i + c_r) h.
* Intensity: ``flux`` |rho_j|^2 Gamma_0 / Gamma_j for open beams (current
  normalisation); ``paper`` multiplies by sin(theta0) as printed in Sec. 2.1.
"""
from __future__ import annotations

import math

import numpy as np

THRESHOLD = 1000.0


def boundary_matrix(gam: np.ndarray) -> np.ndarray:
    """S of Sec. 3.1: (tau, rho) = S (c, c')."""
    n = gam.size
    return np.block([[np.diag(gam), -1j * np.eye(n)], [np.diag(gam), 1j * np.eye(n)]])


def initial_state(gam: np.ndarray, literal: bool = False, y_bottom=None) -> np.ndarray:
    """Columns spanning the states at z_e allowed by the bottom condition.

    Default: rho(z_e) = 0.  With ``y_bottom`` = Y: c' = Y c at z_e, the
    state [I; Y] of a bulk below."""
    n = gam.size
    if y_bottom is not None:
        return np.vstack([np.eye(n, dtype=np.complex128), np.asarray(y_bottom, dtype=np.complex128)])
    if literal:
        return np.linalg.solve(boundary_matrix(gam), np.vstack([np.eye(n), np.zeros((n, n))]))
    return np.vstack([np.eye(n, dtype=np.complex128), 1j * np.diag(gam)])


def estcond_gershgorin(Q: np.ndarray) -> float:
    aq = np.abs(Q)
    d = np.diag(aq)
    r = aq.sum(axis=1) - d
    lo = d - r
    if np.any(lo <= 0):
        return math.inf
    return float(np.max(d + r) / np.min(lo))


def rk_slice(Z: np.ndarray, Ms, h: float, tab) -> np.ndarray:
    """One explicit RK step of y' = B y for every column of Z.

    ``Ms[r]`` is U(z_i + c_r h) + Gamma^2 for stage r.
    K_r = B_r Y_r,  Y_r = Y + h sum_{j<r} a_{rj} K_j,  Y <- Y + h sum b_r K_r.
    """
    n = Z.shape[0] // 2
    K = []
    for r in range(tab.stages):
        Yr = Z.copy()
        for j in range(r):
            if tab.a[r, j] != 0.0:
                Yr = Yr + h * tab.a[r, j] * K[j]
        Kr = np.empty_like(Z)
        Kr[:n] = Yr[n:]
        Kr[n:] = -(Ms[r] @ Yr[:n])
        K.append(Kr)
    out = Z.copy()
    for r in range(tab.stages):
        if tab.b[r] != 0.0:
            out = out + h * tab.b[r] * K[r]
    return out


def reflection_matrix(Z: np.ndarray, gam: np.ndarray) -> np.ndarray:
    """R with rho = R tau at the top of Z: R = Z_l Z_u^{-1} after S Z."""
    n = gam.size
    Q, P = Z[:n], Z[n:]
    top = gam[:, None] * Q - 1j * P
    bot = gam[:, None] * Q + 1j * P
    # R top = bot  ->  top^T R^T = bot^T
    return np.linalg.solve(top.T, bot.T).T


def normalised_lower(Z: np.ndarray) -> np.ndarray:
    """Y = P Q^{-1}: the lower block after Z <- Z Q^{-1} (Sec. 3.2)."""
    n = Z.shape[1]
    return Z[n:] @ np.linalg.inv(Z[:n])


def reflection(Z: np.ndarray, gam: np.ndarray) -> np.ndarray:
    """Final lines of Algorithm 1: rho(0) = first column of R (tau(0) = e_1)."""
    return reflection_matrix(Z, gam)[:, 0]


def solve_ode_str(Mfun, gam, h, n_slices, tab, threshold=THRESHOLD, literal_z0=False,
                  track_transform=False, y_bottom=None):
    """Algorithm 1 for one pair.

    ``Mfun(i, r)`` returns U(z_i + c_r h) + Gamma^2 (n x n); ``y_bottom``
    the state [I; Y] of a bulk below the slab (None: vacuum).
    Returns (rho0, info) with info = {"n_rhst", "decisions", "Z", "T"}.
    """
    Z = initial_state(gam, literal_z0, y_bottom)
    n = gam.size
    decisions = []
    T_acc = np.eye(n, dtype=np.complex128) if track_transform else None
    for i in range(n_slices):
        Ms = [Mfun(i, r) for r in range(tab.stages)]
        # an RK tableau, or a splitting composition (oracle/splitting.py) with its own step
        Z = tab.step(Z, Ms, h) if hasattr(tab, "step") else rk_slice(Z, Ms, h, tab)
        xi = estcond_gershgorin(Z[:n])
        do = xi > threshold
        decisions.append(bool(do))
        if do:
            T = np.linalg.inv(Z[:n])
            Z = Z @ T
            if track_transform:
                T_acc = T_acc @ T
    rho = reflection(Z, gam)
    return rho, {"n_rhst": int(sum(decisions)), "decisions": decisions, "Z": Z, "T": T_acc}


def transmission(Z, T_acc, gam):
    """tau(z_e) = 2 Gamma T^(L) x with (Gamma Q - i P) x = e_1 (Sec. 3.2: the
    accumulated transform T^(L) maps the normalised basis back to Z0)."""
    n = gam.size
    B = gam[:, None] * Z[:n] - 1j * Z[n:]
    e1 = np.zeros(n, dtype=np.complex128)
    e1[0] = 1.0
    x = np.linalg.solve(B, e1)
    return 2.0 * gam * (T_acc @ x)


def intensity(rho, gam, open_mask, theta0, convention="flux"):
    """Sec. 2.1: eta_j = |rho_j|^2 Gamma_0/Gamma_j for open beams, 0 otherwise
    (``paper`` convention: times sin(theta0))."""
    eta = np.zeros(rho.shape, dtype=np.float64)
    g0 = gam[0].real
    eta[open_mask] = np.abs(rho[open_mask]) ** 2 * g0 / gam[open_mask].real
    if convention == "paper":
        eta *= math.sin(theta0)
    return eta
