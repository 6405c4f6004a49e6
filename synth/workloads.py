"""Seeded synthetic workloads standing in for the paper's measured surfaces.

The paper times its method on a Si(111)-7x7 TRHEPD input (Table 2) whose
files are not public here, so every workload below is synthetic: a square
surface cell (a = 3.84 A), an m x m supercell, atoms in layers spaced
3.1 A, one atomic species with a four-Gaussian potential whose weights and
widths are drawn from a seeded generator, and glancing angles on a uniform
grid.  Everything is drawn with ``numpy.random.default_rng`` (PCG64).

Seeds: workload ``c`` uses ``1000 + c``; structure ``s`` of workload ``c``
uses ``100000 * (1000 + c) + s``; the perturbed target slab of the
gradient workload uses ``100000 * 1004 + 99999``.

Only inputs are produced here.  The potential's Fourier coefficients, the
wavenumbers and everything downstream are computed separately by the
oracle and by the GPU library.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

CELL = 3.84          # A, square surface cell edge
LAYER_D = 3.1        # A, layer spacing
LAYER_Z0 = 1.55      # A, depth of the first layer below the surface (z=0)
MEAN_INNER_POTENTIAL = 15.0  # V


@dataclasses.dataclass
class Structure:
    """One slab: beam set, atoms and slicing.  Lengths in A."""
    beams: np.ndarray          # int32 [N, 2] rod indices (h, k); beams[0] == (0, 0)
    recip: np.ndarray          # float64 [2, 2] rows b1, b2 (1/A) of the supercell
    cell_area: float           # A^2 of the supercell
    atoms: np.ndarray          # float64 [n_atoms, 3] (x, y, z), z < 0 inside the slab
    scat_a: np.ndarray         # float64 [4] Gaussian weights (V)
    scat_b: np.ndarray         # float64 [4] Gaussian exponents (1/A^2)
    thickness: float           # D: slab is z in [-D, 0]
    n_slices: int              # L
    grad_atoms: Optional[np.ndarray] = None  # int indices of atoms whose coordinates are differentiated

    @property
    def n_beams(self) -> int:
        return int(self.beams.shape[0])

    @property
    def step(self) -> float:
        return self.thickness / self.n_slices


@dataclasses.dataclass
class Workload:
    name: str
    structures: List[Structure]
    energy_eV: float
    charge: int                # +1 electron (attractive), -1 positron (repulsive)
    absorption: float          # alpha: U = kappa * s * V * (charge - i*alpha)
    theta0: np.ndarray         # float64 [A] glancing angles (rad)
    theta1: float              # azimuth (rad) measured from b1
    stepper: str = "rk4"
    mean_inner_potential: float = MEAN_INNER_POTENTIAL
    target: Optional[List[Structure]] = None   # gradient workload: slabs that make the target curve

    @property
    def n_pairs(self) -> int:
        return len(self.structures) * len(self.theta0)


def _recip(m: int) -> np.ndarray:
    b = 2.0 * math.pi / (CELL * m)
    return np.array([[b, 0.0], [0.0, b]])


def beams_nearest(n: int, recip: np.ndarray) -> np.ndarray:
    """The n reciprocal rods nearest to the origin.

    Order: |g|^2, then polar angle of g in [0, 2pi), then h, then k.  For a
    square lattice a disc cutoff cannot give every N (disc counts are
    1, 5, 9, 13, 21, 25, 29, 37, ...), so the set is "the N nearest rods";
    N = 61 and N = 121 are exact discs.
    """
    r = int(math.ceil(math.sqrt(n))) + 2
    cand = []
    for h in range(-r, r + 1):
        for k in range(-r, r + 1):
            g = h * recip[0] + k * recip[1]
            ang = math.atan2(g[1], g[0]) % (2.0 * math.pi)
            cand.append((round(float(g @ g), 12), round(ang, 12), h, k))
    cand.sort()
    out = np.array([[c[2], c[3]] for c in cand[:n]], dtype=np.int32)
    assert out[0, 0] == 0 and out[0, 1] == 0
    return out


def beams_row(hmax: int) -> np.ndarray:
    """The 1D row (h, 0), h = -hmax..hmax, ordered 0, 1, -1, 2, -2, ..."""
    hs = [0]
    for h in range(1, hmax + 1):
        hs += [h, -h]
    return np.array([[h, 0] for h in hs], dtype=np.int32)


def _layers(m: int, n_layers: int, sigma_xy: float, rng) -> np.ndarray:
    atoms = []
    for layer in range(n_layers):
        z = -(LAYER_Z0 + LAYER_D * layer)
        for i in range(m):
            for j in range(m):
                atoms.append((CELL * i, CELL * j, z))
    atoms = np.array(atoms, dtype=np.float64)
    if sigma_xy > 0:
        atoms[:, :2] += rng.normal(0.0, sigma_xy, size=(atoms.shape[0], 2))
    return atoms


def _scattering(rng):
    a = rng.uniform(1.0, 10.0, size=4)
    b = rng.uniform(0.5, 20.0, size=4)
    return a, b


def _deg(x):
    return np.deg2rad(np.asarray(x, dtype=np.float64))


def config1() -> Workload:
    """10 keV positrons on a 1D row of 13 beams, 1 atom per layer, 8 layers,
    25 A in 250 slices, 41 glancing angles 0.5..6.0 deg."""
    rng = np.random.default_rng(1001)
    a, b = _scattering(rng)
    atoms = np.array([[0.0, 0.0, -(LAYER_Z0 + LAYER_D * k)] for k in range(8)])
    s = Structure(beams=beams_row(6), recip=_recip(1), cell_area=CELL * CELL, atoms=atoms,
                  scat_a=a, scat_b=b, thickness=25.0, n_slices=250)
    return Workload("c1-positron-row-N13", [s], 10_000.0, -1, 0.1,
                    _deg(np.linspace(0.5, 6.0, 41)), float(_deg(90.0)))


def _c2_structure(n_beams=61, n_slices=400, thickness=40.0, seed=1002) -> Structure:
    rng = np.random.default_rng(seed)
    a, b = _scattering(rng)
    atoms = _layers(3, 10, 0.1, rng)
    rec = _recip(3)
    return Structure(beams=beams_nearest(n_beams, rec), recip=rec, cell_area=(3 * CELL) ** 2,
                     atoms=atoms, scat_a=a, scat_b=b, thickness=thickness, n_slices=n_slices)


def config2(stepper: str = "rk4") -> Workload:
    """15 keV electrons, N = 61 rods of a 3x3 supercell, 9 atoms x 10 layers,
    40 A in 400 slices, 128 angles 0.3..6.0 deg."""
    s = _c2_structure()
    return Workload("c2-electron-N61", [s], 15_000.0, +1, 0.1,
                    _deg(np.linspace(0.3, 6.0, 128)), 0.0, stepper=stepper)


def _perturbed(base: Structure, seed: int, n_beams: Optional[int] = None, sigma_z=0.2) -> Structure:
    rng = np.random.default_rng(seed)
    atoms = base.atoms.copy()
    atoms[:, 2] += rng.normal(0.0, sigma_z, size=atoms.shape[0])
    beams = base.beams if n_beams is None else beams_nearest(n_beams, base.recip)
    return dataclasses.replace(base, atoms=atoms, beams=beams)


# Slices of the 40 A slab per beam count in the uneven-N workload.  More beams
# reach more evanescent rods: the largest |Gamma_j| over the workload's angles
# is 15.7, 17.7, 19.5 and 21.1 1/A for N = 31, 61, 91, 121, and with h = 0.1 A
# (400 slices) the sixth-order step is off the physical solution for N >= 91
# (summed reflected intensities far above 1 under absorption).  Each N takes
# the smallest multiple of 20 slices, at least 400, with h max|Gamma_j| <= 1.45
# (a CPU test recomputes these from the oracle's Gamma).
UNEVEN_SLICES = {31: 440, 61: 500, 91: 540, 121: 600}
UNEVEN_H_GAMMA = 1.45


def config3(n_structures: int = 1024, slices=None) -> Workload:
    """1024 perturbed copies of the N=61 slab with N drawn from
    {31, 61, 91, 121}; 64 angles each; slices per N from ``slices``
    (default UNEVEN_SLICES; pass {n: 400} for the uniform 0.1 A grid)."""
    base = _c2_structure()
    rng = np.random.default_rng(1003)
    ns = rng.choice(np.array([31, 61, 91, 121]), size=n_structures)
    table = UNEVEN_SLICES if slices is None else slices
    structs = [dataclasses.replace(_perturbed(base, 100000 * 1003 + s, int(ns[s])), n_slices=table[int(ns[s])])
               for s in range(n_structures)]
    return Workload("c3-batched-uneven-N", structs, 15_000.0, +1, 0.1,
                    _deg(np.linspace(0.3, 6.0, 64)), 0.0)


def config4(n_structures: int = 1) -> Workload:
    """Gradient workload: the N=61 slab, 128 angles, R-factor against the
    curve of a perturbed copy; gradient w.r.t. the 27 atoms of the top three
    layers.  ``n_structures`` > 1 adds perturbed copies (batched variant)."""
    base = _c2_structure()
    base.grad_atoms = np.arange(27)
    structs = [base] + [_perturbed(base, 100000 * 1004 + s) for s in range(1, n_structures)]
    for s in structs:
        s.grad_atoms = np.arange(27)
    target = [_perturbed(s, 100000 * 1004 + 99999) for s in structs]
    return Workload("c4-grad-N61" if n_structures == 1 else f"c4-grad-N61-x{n_structures}",
                    structs, 15_000.0, +1, 0.1, _deg(np.linspace(0.3, 6.0, 128)), 0.0,
                    target=target)


def config5(n_structures: int = 64) -> Workload:
    """N = 199 rods of a 7x7 supercell, 49 atoms x 12 layers, 60 A in 1000
    slices, 256 angles, 64 structures, gradients for every atom z."""
    rec = _recip(7)
    beams = beams_nearest(199, rec)
    structs = []
    for s in range(n_structures):
        rng = np.random.default_rng(100000 * 1005 + s)
        a, b = _scattering(np.random.default_rng(1005))
        atoms = _layers(7, 12, 0.1, rng)
        structs.append(Structure(beams=beams, recip=rec, cell_area=(7 * CELL) ** 2, atoms=atoms,
                                 scat_a=a, scat_b=b, thickness=60.0, n_slices=1000,
                                 grad_atoms=np.arange(atoms.shape[0])))
    return Workload("c5-electron-N199", structs, 15_000.0, +1, 0.1,
                    _deg(np.linspace(0.3, 6.0, 256)), 0.0)


def single_angle_n521(n_slices: int = 661) -> Workload:
    """The single-angle case of the paper's timing table at its size (Sec. 4,
    Tables 2 and 3: n = 521 rods, one glancing angle of 1.3 deg at azimuth
    -30 deg, a 9.91 A domain without a bulk layer, RK4 at dz = 0.015 A):
    N = 521 rods of a 7x7 supercell, 49 atoms x 3 layers, 10 keV positrons,
    9.91 A in 661 slices.  The Si(111)-7x7 input itself is not available,
    so the cell, atoms and potential are synthetic like every other
    workload here (seeds of workload 6)."""
    rec = _recip(7)
    beams = beams_nearest(521, rec)
    a, b = _scattering(np.random.default_rng(1006))
    atoms = _layers(7, 3, 0.1, np.random.default_rng(100000 * 1006))
    s = Structure(beams=beams, recip=rec, cell_area=(7 * CELL) ** 2, atoms=atoms, scat_a=a, scat_b=b,
                  thickness=9.91, n_slices=n_slices)
    return Workload("paper-n521-single-angle", [s], 10_000.0, -1, 0.1, _deg(np.array([1.3])),
                    float(_deg(-30.0)))


def bulk_layer(surface: Workload, n_slices: int, images: int = 2) -> Workload:
    """The ideal bulk under a surface workload, one unit layer per structure.

    The unit layer is z in [-d, 0], d = 3.1 A (one layer spacing), with one
    atomic layer of the surface's supercell at z = -d/2 on the ideal lattice
    (no in-plane noise) and ``images`` periodic copies above and below, so
    that its table is the potential of the infinite stack up to Gaussian
    tails beyond ``images`` spacings.  The mean inner potential is counted
    over the 2 images + 1 layers placed in one spacing, so the potential
    scale equals that of a stack averaging the surface's value.  Beams,
    scattering factors, energy and angles are the surface's."""
    structs = []
    for s in surface.structures:
        m = int(round(math.sqrt(s.cell_area) / CELL))
        atoms = []
        for layer in range(-images, images + 1):
            z = -0.5 * LAYER_D + LAYER_D * layer
            for i in range(m):
                for j in range(m):
                    atoms.append((CELL * i, CELL * j, z))
        structs.append(Structure(beams=s.beams, recip=s.recip, cell_area=s.cell_area,
                                 atoms=np.array(atoms, dtype=np.float64), scat_a=s.scat_a, scat_b=s.scat_b,
                                 thickness=LAYER_D, n_slices=n_slices))
    return dataclasses.replace(surface, name=surface.name + "-bulk", structures=structs, target=None,
                               mean_inner_potential=surface.mean_inner_potential * (2 * images + 1))


def small_row(hmax=3, n_slices=50, n_angles=5, thickness=10.0, seed=7, n_layers=3,
              charge=-1, absorption=0.1) -> Workload:
    """A small positron row case for fast oracle checks."""
    rng = np.random.default_rng(seed)
    a, b = _scattering(rng)
    atoms = np.array([[0.0, 0.0, -(LAYER_Z0 + LAYER_D * k)] for k in range(n_layers)])
    s = Structure(beams=beams_row(hmax), recip=_recip(1), cell_area=CELL * CELL, atoms=atoms,
                  scat_a=a, scat_b=b, thickness=thickness, n_slices=n_slices,
                  grad_atoms=np.arange(atoms.shape[0]))
    return Workload(f"row-N{2 * hmax + 1}", [s], 10_000.0, charge, absorption,
                    _deg(np.linspace(0.7, 5.0, n_angles)), float(_deg(90.0)))


def small_2d(n_beams=21, n_slices=40, n_angles=4, thickness=8.0, seed=11, n_layers=2,
             m=3, n_structures=1, charge=+1, absorption=0.1, theta_range=(0.5, 5.0),
             sigma_xy=0.1, theta1_deg=0.0) -> Workload:
    """A small 2D electron case (m x m supercell) for parity at oracle speed."""
    rec = _recip(m)
    beams = beams_nearest(n_beams, rec)
    structs = []
    for s in range(n_structures):
        rng = np.random.default_rng(seed * 1000 + s)
        a, b = _scattering(np.random.default_rng(seed))
        atoms = _layers(m, n_layers, sigma_xy, rng)
        structs.append(Structure(beams=beams, recip=rec, cell_area=(m * CELL) ** 2, atoms=atoms,
                                 scat_a=a, scat_b=b, thickness=thickness, n_slices=n_slices,
                                 grad_atoms=np.arange(min(atoms.shape[0], 4))))
    return Workload(f"small2d-N{n_beams}", structs, 15_000.0, charge, absorption,
                    _deg(np.linspace(theta_range[0], theta_range[1], n_angles)),
                    float(_deg(theta1_deg)))


WORKLOADS = {"c1": config1, "c2": config2, "c3": config3, "c4": config4, "c5": config5}
