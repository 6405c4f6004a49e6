"""Beam constants and the incidence geometry (oracle; test infrastructure).

Paper: Sec. 2.1, Eqs. (sch1)-(sch3).  The paper does not print the
relation between beam energy and gamma, nor the factor that turns an
electrostatic potential in volts into the ``v`` of Eq. (sch1); both are
the standard relativistic expressions, written here from CODATA values.

Readings (paper silent or ambiguous):
* gamma = sqrt(2 m0 e E (1 + e E / (2 m0 c^2))) / hbar  (vacuum wavenumber).
* v = kappa * V with kappa = (2 m0 e / hbar^2) (1 + e E / (m0 c^2)), so a
  positive electrostatic potential attracts electrons (v > 0) and repels
  positrons (v < 0).
* b0 = gamma cos(theta0) (cos theta1, sin theta1), theta1 measured from b1.
* Gamma_j = sqrt(gamma^2 - |b0 + k_j|^2) for open beams; for evanescent
  beams the branch with Im Gamma_j < 0, i.e. -i sqrt(|b0+k_j|^2 - gamma^2).
  With tau ~ exp(+i Gamma z) travelling into the crystal this is the branch
  whose waves decay away from the slab on both sides.
"""
from __future__ import annotations

import math

import numpy as np

# CODATA 2018
M_E = 9.1093837015e-31      # kg
Q_E = 1.602176634e-19       # C
HBAR = 1.054571817e-34      # J s
C_LIGHT = 299792458.0       # m/s


def wavenumber(energy_eV: float) -> float:
    """Vacuum wavenumber gamma in 1/A for a lepton of kinetic energy E."""
    e = Q_E * energy_eV
    p2 = 2.0 * M_E * e * (1.0 + e / (2.0 * M_E * C_LIGHT ** 2))
    return math.sqrt(p2) / HBAR * 1e-10


def interaction_constant(energy_eV: float) -> float:
    """kappa in 1/(A^2 V): v(r) = charge * kappa * V(r) in Eq. (sch1)."""
    e = Q_E * energy_eV
    k = 2.0 * M_E * Q_E / HBAR ** 2 * (1.0 + e / (M_E * C_LIGHT ** 2))
    return k * 1e-20


def incident_b0(gamma: float, theta0: float, theta1: float) -> np.ndarray:
    """Projected incident wavevector b0 (1/A)."""
    return gamma * math.cos(theta0) * np.array([math.cos(theta1), math.sin(theta1)])


def beam_vectors(beams: np.ndarray, recip: np.ndarray) -> np.ndarray:
    """k_j = h_j b1 + k_j b2 for every rod, shape [N, 2]."""
    beams = np.asarray(beams, dtype=np.float64)
    return beams[:, :1] * recip[0][None, :] + beams[:, 1:2] * recip[1][None, :]


def gamma_diag(gamma: float, b0: np.ndarray, kvec: np.ndarray) -> np.ndarray:
    """Diagonal of Gamma, Eq. (sch3): (Gamma)_jj = sqrt(gamma^2 - |b0 + k_j|^2)."""
    q = b0[None, :] + kvec
    arg = gamma * gamma - np.einsum("ij,ij->i", q, q)
    out = np.empty(arg.shape, dtype=np.complex128)
    pos = arg >= 0
    out[pos] = np.sqrt(arg[pos])
    out[~pos] = -1j * np.sqrt(-arg[~pos])
    return out


def open_beams(gamma: float, b0: np.ndarray, kvec: np.ndarray) -> np.ndarray:
    """Mask of beams that propagate in vacuum: gamma^2 > |b0 + k_j|^2."""
    q = b0[None, :] + kvec
    return gamma * gamma > np.einsum("ij,ij->i", q, q)
