"""Fourier coefficients of the slab potential (oracle; test infrastructure).

Paper: Sec. 2.1.  The potential is expanded in the surface reciprocal
lattice, v = sum_g u_g(z) exp(i g.r_xy), and Eq. (sch2) couples beam j to
beam k through u_{l(j,k)}; with a Fourier series the index l(j,k) is the
rod g_j - g_k.  The paper takes the coefficients from its input files; the
workloads here build them from Gaussian atoms (one species):

    v_atom(r) = sum_{m=1..4} a_m exp(-b_m |r - r_a|^2)         (volts)

whose in-plane transform per unit cell area A is

    V_g(z) = (1/A) sum_a exp(-i g.rho_a)
             sum_m a_m (pi/b_m) exp(-|g|^2/(4 b_m)) exp(-b_m (z - z_a)^2).

The volts are rescaled so that the mean of V over the slab volume,
(1/(A D)) sum_a sum_m a_m (pi/b_m)^{3/2}, equals the requested mean inner
potential; the scale does not depend on the atom positions.  Finally
u_g = kappa * s * V_g * (charge - i * alpha): ``charge`` = +1 for
electrons, -1 for positrons, and ``alpha`` the relative absorption; with
the Gamma branch of ``physics`` a negative imaginary part removes flux.

Table layout (shared convention with the GPU library, written twice):
``U[node, (dh + Hd) * (2 Kd + 1) + (dk + Kd)]`` for rod differences
dh in [-Hd, Hd], dk in [-Kd, Kd] where Hd = max h - min h and
Kd = max k - min k over the beam set.  Node n of a tableau with distinct
fractional nodes ``cset`` sits at z = -D + (i + cset[m]) h with
n = i * len(cset) + m, plus a final node at z = 0.

Pins (tests/test_oracle_basics.py): the table against a direct real-space
evaluation of the Fourier integral (quadrature over the cell); the coupling
matrix U_jk = u_{l(j,k)} as a whole, orientation included, against a
quadrature of the matrix element (1/A) int exp(-i k_j.r) v(r) exp(i k_k.r)
d^2r on a cell without in-plane symmetry (where the transpose differs); the
derivatives against central differences.
"""
from __future__ import annotations

import math

import numpy as np


def difference_box(beams: np.ndarray):
    beams = np.asarray(beams)
    hd = int(beams[:, 0].max() - beams[:, 0].min())
    kd = int(beams[:, 1].max() - beams[:, 1].min())
    return hd, kd


def box_vectors(hd: int, kd: int, recip: np.ndarray):
    """Rod differences (dh, dk) in table order and their vectors g."""
    dh, dk = np.meshgrid(np.arange(-hd, hd + 1), np.arange(-kd, kd + 1), indexing="ij")
    dh = dh.ravel()
    dk = dk.ravel()
    g = dh[:, None] * recip[0][None, :] + dk[:, None] * recip[1][None, :]
    return dh, dk, g


def node_positions(thickness: float, n_slices: int, cset) -> np.ndarray:
    h = thickness / n_slices
    z = [-thickness + (i + c) * h for i in range(n_slices) for c in cset]
    z.append(0.0)
    return np.array(z)


def coupling_index(beams: np.ndarray, hd: int, kd: int) -> np.ndarray:
    """Table column of U_{jk} = u_{g_j - g_k} (the index l(j,k) of Eq. sch2)."""
    beams = np.asarray(beams, dtype=np.int64)
    dh = beams[:, None, 0] - beams[None, :, 0]
    dk = beams[:, None, 1] - beams[None, :, 1]
    return (dh + hd) * (2 * kd + 1) + (dk + kd)


def mip_scale(struct, mean_inner_potential: float) -> float:
    """Factor s making the slab-averaged potential equal the requested value."""
    a = np.asarray(struct.scat_a)
    b = np.asarray(struct.scat_b)
    per_atom = float(np.sum(a * (math.pi / b) ** 1.5))
    raw = struct.atoms.shape[0] * per_atom / (struct.cell_area * struct.thickness)
    return mean_inner_potential / raw


def _prefactor(struct, kappa, charge, absorption, mean_inner_potential):
    s = mip_scale(struct, mean_inner_potential)
    return kappa * s * (charge - 1j * absorption) / struct.cell_area


def potential_table(struct, z_nodes, kappa, charge, absorption, mean_inner_potential):
    """u_g(z) on the nodes, complex128 [n_nodes, box]."""
    hd, kd = difference_box(struct.beams)
    _, _, g = box_vectors(hd, kd, struct.recip)
    g2 = np.einsum("ij,ij->i", g, g)
    z = np.asarray(z_nodes)
    pref = _prefactor(struct, kappa, charge, absorption, mean_inner_potential)
    out = np.zeros((z.size, g.shape[0]), dtype=np.complex128)
    for (x, y, za) in struct.atoms:
        phase = np.exp(-1j * (g[:, 0] * x + g[:, 1] * y))
        dz2 = (z - za) ** 2
        acc = np.zeros((z.size, g.shape[0]))
        for am, bm in zip(struct.scat_a, struct.scat_b):
            acc += (am * math.pi / bm) * np.exp(-bm * dz2)[:, None] * np.exp(-g2 / (4 * bm))[None, :]
        out += acc * phase[None, :]
    return out * pref


def potential_table_direction(struct, z_nodes, kappa, charge, absorption,
                              mean_inner_potential, direction):
    """Directional derivative sum_{a,c} direction[a, c] d u_g(z) / d r_{a,c}.

    ``direction`` is [n_atoms, 3] (x, y, z components).
    d/dx_a brings -i g_x, d/dy_a brings -i g_y, and d/dz_a brings
    2 b_m (z - z_a) inside the Gaussian sum.
    """
    hd, kd = difference_box(struct.beams)
    _, _, g = box_vectors(hd, kd, struct.recip)
    g2 = np.einsum("ij,ij->i", g, g)
    z = np.asarray(z_nodes)
    pref = _prefactor(struct, kappa, charge, absorption, mean_inner_potential)
    out = np.zeros((z.size, g.shape[0]), dtype=np.complex128)
    direction = np.asarray(direction, dtype=np.float64)
    for ia, (x, y, za) in enumerate(struct.atoms):
        dx, dy, dzc = direction[ia]
        if dx == 0.0 and dy == 0.0 and dzc == 0.0:
            continue
        phase = np.exp(-1j * (g[:, 0] * x + g[:, 1] * y))
        dz = z - za
        acc = np.zeros((z.size, g.shape[0]))
        dacc = np.zeros((z.size, g.shape[0]))
        for am, bm in zip(struct.scat_a, struct.scat_b):
            term = (am * math.pi / bm) * np.exp(-bm * dz * dz)[:, None] * np.exp(-g2 / (4 * bm))[None, :]
            acc += term
            dacc += term * (2.0 * bm * dz)[:, None]
        lateral = -1j * (g[:, 0] * dx + g[:, 1] * dy)
        out += (acc * lateral[None, :] + dacc * dzc) * phase[None, :]
    return out * pref
