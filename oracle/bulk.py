"""The bulk layer below the surface region (oracle; test infrastructure).

Paper: Sec. 2.2, the treatment of the bulk layer, with the reflection-matrix
recursion of the same section (Eqs. ri1, ri2).  Below the surface region
whose atoms are fitted, the crystal continues as the ideal bulk, a stack of
identical unit layers.  The reflection matrix R_k at the top of k unit
layers (rho = R_k tau there) stops changing as k grows; that limit R_bulk
is computed once, before the structure search, and the surface region then
starts from the bottom condition rho(z_e) = R_bulk tau(z_e) instead of
rho(z_e) = 0.

In the proposed method one unit layer maps a bottom matrix R to a top
matrix F(R): Algorithm 1 over the layer's slices from the initial state
S^{-1}[I; R] (2 Gamma) (``rk.initial_state``), then R' = (Gamma Q + iP)
(Gamma Q - iP)^{-1} from the final Q, P (``rk.reflection_matrix``, whose
first column is rho(0)).

Readings (the paper gives no formulas for this step):
* R_0 is the caller's start (zero: vacuum below a finite bulk) and
  R_{k+1} = F(R_k).
* Convergence is tested per (structure, angle) pair on the absolute change,
  max_{j,k} |R_{k+1} - R_k| <= tol (entries of R are amplitude ratios of
  order one); the first R_{k+1} that passes is R_bulk, after k + 1 layers.
  A pair that does not pass within ``max_layers`` layers keeps its last R
  and reports -1.

Pins (tests/test_oracle_bulk.py): composition (a slab from R = 0 equals its
upper part started from the lower part's top matrix), the single-beam
closed form after k layers of a constant potential and its Fresnel limit,
decoupled beams, and the fixed point F(R_bulk) = R_bulk within tol.
"""
from __future__ import annotations

import numpy as np

from .rk import THRESHOLD, reflection_matrix, solve_ode_str


def layer_map(Mfun, gam, h, n_slices, tab, R, threshold=THRESHOLD):
    """F(R): the reflection matrix at the top of one unit layer whose bottom
    sees rho = R tau.  Returns (F(R), number of RHSTs)."""
    _, info = solve_ode_str(Mfun, gam, h, n_slices, tab, threshold=threshold, r_bottom=R)
    return reflection_matrix(info["Z"], gam), info["n_rhst"]


def bulk_reflection(Mfun, gam, h, n_slices, tab, tol, max_layers, R0=None, threshold=THRESHOLD):
    """Iterates R <- F(R) from R0 (zero if None).  Returns (R, layers) with
    layers the count of unit layers after which the change first stayed
    within tol, or -1 (and the last R) if max_layers did not reach it."""
    n = gam.size
    R = np.zeros((n, n), dtype=np.complex128) if R0 is None else np.asarray(R0, dtype=np.complex128)
    for k in range(1, max_layers + 1):
        Rn, _ = layer_map(Mfun, gam, h, n_slices, tab, R, threshold)
        if np.max(np.abs(Rn - R)) <= tol:
            return Rn, k
        R = Rn
    return R, -1
