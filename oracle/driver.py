"""Glue from the seeded ``synth`` workloads to the oracle solvers (test infrastructure).

Builds, per structure, the potential table on the tableau's nodes, and per
angle the diagonal Gamma, then runs Algorithm 1 (``rk``), the conventional
method (``conventional``) or the tangent-linear method (``tangent``).
The R-factor of the gradient workload is sum_theta (eta_00 - target_00)^2.
"""
from __future__ import annotations

import numpy as np

from . import bulk, physics, potential, rk, tangent
from .conventional import eigen_multislice, ichimiya_recursion
from .tableaux import TABLEAUX


class StructureSetup:
    def __init__(self, wl, struct, tab):
        self.wl = wl
        self.s = struct
        self.tab = tab
        self.gamma = physics.wavenumber(wl.energy_eV)
        self.kappa = physics.interaction_constant(wl.energy_eV)
        self.hd, self.kd = potential.difference_box(struct.beams)
        self.z_nodes = potential.node_positions(struct.thickness, struct.n_slices, tab.cset)
        self.table = potential.potential_table(struct, self.z_nodes, self.kappa, wl.charge,
                                               wl.absorption, wl.mean_inner_potential)
        self.cidx = potential.coupling_index(struct.beams, self.hd, self.kd)
        self.kvec = physics.beam_vectors(struct.beams, struct.recip)
        self.h = struct.thickness / struct.n_slices

    def U_node(self, node, table=None):
        t = self.table if table is None else table
        return t[node][self.cidx]

    def angle(self, theta0):
        b0 = physics.incident_b0(self.gamma, theta0, self.wl.theta1)
        gam = physics.gamma_diag(self.gamma, b0, self.kvec)
        mask = physics.open_beams(self.gamma, b0, self.kvec)
        return gam, mask

    def mfun(self, gam, table=None):
        g2 = gam * gam
        tab = self.tab

        def M(i, r):
            return self.U_node(tab.node_index(i, r), table) + np.diag(g2)
        return M

    def solve(self, theta0, threshold=rk.THRESHOLD, literal_z0=False, track_transform=False, y_bottom=None):
        gam, mask = self.angle(theta0)
        rho, info = rk.solve_ode_str(self.mfun(gam), gam, self.h, self.s.n_slices, self.tab,
                                     threshold=threshold, literal_z0=literal_z0,
                                     track_transform=track_transform, y_bottom=y_bottom)
        return rho, gam, mask, info

    def midpoint_node(self, i):
        # the c = 1/2 node of slice i (present in the RK4 node set)
        return i * len(self.tab.cset) + self.tab.cset.index(0.5) if 0.5 in [float(c) for c in self.tab.cset] else None

    def solve_eigen(self, theta0):
        gam, mask = self.angle(theta0)
        g2 = np.diag(gam * gam)
        cs = [float(c) for c in self.tab.cset]
        m = cs.index(0.5)
        nc = len(cs)
        rho = eigen_multislice(lambda i: self.U_node(i * nc + m) + g2, gam, self.h, self.s.n_slices)
        return rho, gam, mask

    def solve_ichimiya(self, theta0):
        gam, mask = self.angle(theta0)
        cs = [float(c) for c in self.tab.cset]
        m = cs.index(0.5)
        nc = len(cs)
        rho = ichimiya_recursion(lambda i: self.U_node(i * nc + m), gam, self.h, self.s.n_slices)
        return rho, gam, mask


def rocking_curve(wl, s_idx=0, angle_idx=None, stepper=None, convention="flux", threshold=rk.THRESHOLD,
                  y_bottom=None):
    """eta [A, N] (float64), rho [A, N] (complex128), n_rhst [A].
    ``y_bottom``: bulk states [I; Y] below the slab as Y [A, N, N], one per
    angle of ``angle_idx`` (None: vacuum below)."""
    tab = TABLEAUX[stepper or wl.stepper]
    st = StructureSetup(wl, wl.structures[s_idx], tab)
    idx = range(len(wl.theta0)) if angle_idx is None else angle_idx
    etas, rhos, nr = [], [], []
    for k, a in enumerate(idx):
        th = float(wl.theta0[a])
        rho, gam, mask, info = st.solve(th, threshold=threshold,
                                        y_bottom=None if y_bottom is None else y_bottom[k])
        etas.append(rk.intensity(rho, gam, mask, th, convention))
        rhos.append(rho)
        nr.append(info["n_rhst"])
    return np.array(etas), np.array(rhos), np.array(nr)


def bulk_matrices(wl_bulk, s_idx=0, angle_idx=None, stepper=None, tol=1e-12, max_layers=200):
    """Y_bulk [A, N, N], R_bulk [A, N, N] and layers [A] for the unit layer
    of structure ``s_idx`` of a bulk workload, per angle (oracle.bulk)."""
    tab = TABLEAUX[stepper or wl_bulk.stepper]
    st = StructureSetup(wl_bulk, wl_bulk.structures[s_idx], tab)
    idx = range(len(wl_bulk.theta0)) if angle_idx is None else angle_idx
    Ys, Rs, layers = [], [], []
    for a in idx:
        gam, _ = st.angle(float(wl_bulk.theta0[a]))
        Y, R, n = bulk.bulk_reflection(st.mfun(gam), gam, st.h, st.s.n_slices, tab, tol, max_layers)
        Ys.append(Y)
        Rs.append(R)
        layers.append(n)
    return np.array(Ys), np.array(Rs), np.array(layers)


def rfactor(eta00, target00):
    d = np.asarray(eta00) - np.asarray(target00)
    return float(np.sum(d * d)), 2.0 * d


def rfactor_directional(wl, s_idx, direction, target00, angle_idx=None, stepper=None,
                        convention="flux", y_bottom=None):
    """Directional derivative of the R-factor along atom displacements
    ``direction`` [n_atoms, 3], by the tangent-linear method; ``y_bottom``
    as for ``rocking_curve`` (held fixed)."""
    tab = TABLEAUX[stepper or wl.stepper]
    st = StructureSetup(wl, wl.structures[s_idx], tab)
    dtable = potential.potential_table_direction(st.s, st.z_nodes, st.kappa, wl.charge,
                                                 wl.absorption, wl.mean_inner_potential, direction)
    idx = range(len(wl.theta0)) if angle_idx is None else angle_idx
    loss, dL = 0.0, 0.0
    for k, a in enumerate(idx):
        th = float(wl.theta0[a])
        gam, mask = st.angle(th)

        def dU(i, r):
            return dtable[tab.node_index(i, r)][st.cidx]
        rho, drho = tangent.solve_ode_str_tangent(st.mfun(gam), dU, gam, st.h, st.s.n_slices, tab,
                                                  y_bottom=None if y_bottom is None else y_bottom[k])
        eta = rk.intensity(rho, gam, mask, th, convention)
        deta = tangent.intensity_tangent(rho, drho, gam, mask, th, convention)
        diff = eta[0] - target00[k]
        loss += diff * diff
        dL += 2.0 * diff * deta[0]
    return loss, dL


def rfactor_directional_table(wl, s_idx, dtable, target00, angle_idx=None, stepper=None, convention="flux",
                              y_bottom=None):
    """Directional derivative of the R-factor along a perturbation ``dtable``
    of the potential table itself ([n_nodes, box] complex), tangent-linear;
    ``y_bottom`` as for ``rocking_curve`` (held fixed)."""
    tab = TABLEAUX[stepper or wl.stepper]
    st = StructureSetup(wl, wl.structures[s_idx], tab)
    idx = range(len(wl.theta0)) if angle_idx is None else angle_idx
    loss, dL = 0.0, 0.0
    for k, a in enumerate(idx):
        th = float(wl.theta0[a])
        gam, mask = st.angle(th)

        def dU(i, r):
            return dtable[tab.node_index(i, r)][st.cidx]
        rho, drho = tangent.solve_ode_str_tangent(st.mfun(gam), dU, gam, st.h, st.s.n_slices, tab,
                                                  y_bottom=None if y_bottom is None else y_bottom[k])
        eta = rk.intensity(rho, gam, mask, th, convention)
        deta = tangent.intensity_tangent(rho, drho, gam, mask, th, convention)
        diff = eta[0] - target00[k]
        loss += diff * diff
        dL += 2.0 * diff * deta[0]
    return loss, dL
