"""Single-beam homogeneous slab (oracle; test infrastructure).

One beam (n = 1) in a slab z in [-D, 0] of constant coupling U0, vacuum
outside.  With K^2 = Gamma^2 + U0 the field inside is a combination of
exp(+-iKz); matching c and c' at both faces under the boundary conditions
of Sec. 2.1 (tau(0) = 1, rho(-D) = 0, Eqs. vtau, vrho, bd0, bd1) gives

    r = -i U0 sin(KD) / (2 Gamma K cos(KD) + i (2 Gamma^2 + U0) sin(KD))
    t =  2 Gamma K    / (2 Gamma K cos(KD) + i (Gamma^2 + K^2) sin(KD))

with r = rho(0) and t = tau(-D).  Both are even in K, so no branch is
involved.  For D -> infinity with Im K < 0, r tends to the Fresnel value
(Gamma - K) / (Gamma + K).  This is the textbook step-barrier result, used
as an external pin for every solver.
"""
from __future__ import annotations

import numpy as np


def slab_rt(gam: complex, U0: complex, D: float):
    K = np.sqrt(complex(gam) ** 2 + U0)
    s = np.sin(K * D)
    c = np.cos(K * D)
    r = -1j * U0 * s / (2 * gam * K * c + 1j * (2 * gam ** 2 + U0) * s)
    t = 2 * gam * K / (2 * gam * K * c + 1j * (gam ** 2 + K ** 2) * s)
    return complex(r), complex(t)


def fresnel_r(gam: complex, U0: complex):
    K = np.sqrt(complex(gam) ** 2 + U0)
    if K.imag > 0:
        K = -K
    return complex((gam - K) / (gam + K))
