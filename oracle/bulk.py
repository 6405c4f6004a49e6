"""The bulk layer below the surface region (oracle; test infrastructure).

Paper: Sec. 2.2, the treatment of the bulk layer, with the reflection-matrix
recursion of the same section (Eqs. ri1, ri2) and the right-hand-side
transformation of Sec. 3.2.  Below the surface region whose atoms are
fitted, the crystal continues as the ideal bulk, a stack of identical unit
layers.  The reflection matrix R_k at the top of k unit layers (rho = R_k tau
there) stops changing as k grows; the computation stops once it has
converged, and the result, computed once before the structure search,
replaces the vacuum below the surface region.

In the proposed method the stack is propagated upward layer by layer.  The
state carried from one layer to the next is the normalised [I; Y] that a
right-hand-side transformation leaves (Y = P Q^{-1}); the vacuum below the
stack is Y_0 = i Gamma.  One unit layer maps Y_k to Y_{k+1}: Algorithm 1
over the layer's slices from [I; Y_k], then the transformation at its top.
The reflection matrix of the stack is R_k = (Gamma + i Y_k)(Gamma - i Y_k)^{-1}
(the boundary matrix S applied to [I; Y_k]; R_0 = 0), and the surface region
then starts from [I; Y_bulk] (``rk.initial_state``).

Readings (the paper gives no formulas for this step):
* The state, not R, is what passes between layers: the stack is then
  Algorithm 1 over all its slices with a transformation at every layer
  boundary (which the invariance of Sec. 3.2 allows), and the initial state
  of the next layer, or of the surface, needs no division by Gamma (as
  S^{-1}[I; R] would).
* Step size: propagating up a long stack keeps the N modes that grow
  fastest upward, which are the physical ones (decaying into the bulk)
  only while the stepper's damping of fast oscillating beams per layer
  stays small against the separation that absorption gives the modes.
  Classical RK4 at h = 0.1 A damps beams with |K| h near 1.2 by about 0.6
  per 3.1 A layer; on the 21-beam test bulk a few hundred layers then
  drift to a wrong subspace (R grows without bound), while RK6 at
  h = 0.1 A or RK4 at h = 0.05 A converge steadily.  The same holds for a
  single solve through the stack; it is a limit of the discretisation,
  not of the iteration.
* Convergence is tested per (structure, angle) pair on the absolute change
  of R, max_{j,k} |R_k - R_{k-1}| <= tol (entries of R are amplitude ratios
  of order one); the first k that passes gives R_bulk and Y_bulk.  A pair
  that does not pass within ``max_layers`` layers keeps its last Y and R and
  reports -1.

Pins (tests/test_oracle_bulk.py): composition (a slab from the vacuum
equals its upper part started from the lower part's normalised top state),
the single-beam closed form after k unit layers of a constant potential and
its Fresnel limit, decoupled beams, the fixed point, and the relation of
[I; Y] to the bottom condition rho = R tau.
"""
from __future__ import annotations

import numpy as np

from .rk import THRESHOLD, normalised_lower, solve_ode_str


def reflection_of_state(Y, gam):
    """R with rho = R tau for the state [I; Y]: (Gamma + iY)(Gamma - iY)^{-1}."""
    G = np.diag(gam)
    top = G - 1j * Y
    bot = G + 1j * Y
    return np.linalg.solve(top.T, bot.T).T


def layer_map(Mfun, gam, h, n_slices, tab, Y, threshold=THRESHOLD):
    """Y' = P Q^{-1} at the top of one unit layer started from [I; Y]."""
    _, info = solve_ode_str(Mfun, gam, h, n_slices, tab, threshold=threshold, y_bottom=Y)
    return normalised_lower(info["Z"])


def bulk_reflection(Mfun, gam, h, n_slices, tab, tol, max_layers, threshold=THRESHOLD):
    """Propagates the stack from the vacuum (Y_0 = i Gamma, R_0 = 0).
    Returns (Y, R, layers): layers is the first k with
    max |R_k - R_{k-1}| <= tol, or -1 (with the last Y, R) if max_layers
    layers do not reach it."""
    n = gam.size
    Y = 1j * np.diag(gam).astype(np.complex128)
    R = np.zeros((n, n), dtype=np.complex128)
    for k in range(1, max_layers + 1):
        Y = layer_map(Mfun, gam, h, n_slices, tab, Y, threshold)
        Rn = reflection_of_state(Y, gam)
        done = np.max(np.abs(Rn - R)) <= tol
        R = Rn
        if done:
            return Y, R, k
    return Y, R, -1
