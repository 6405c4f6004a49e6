"""Pins for the oracle's building blocks: constants, tableaux, condition
estimate, potential table (CPU only)."""
import dataclasses
import itertools
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import physics, potential, rk
from oracle.tableaux import RK4, RK6, Tableau
from synth import small_2d, small_row, config2, beams_nearest, beams_row

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- constants
def test_wavenumber_and_kappa_against_handbook():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "textbook_constants.txt"))
            if l.strip() and not l.startswith("#")]
    for e, lam, sig in rows:
        e, lam, sig = float(e), float(lam), float(sig)
        assert physics.wavenumber(e) == pytest.approx(2 * math.pi / lam, rel=1e-4)
        assert physics.interaction_constant(e) == pytest.approx(4 * math.pi * sig / lam, rel=2e-4)


def test_gamma_branch_and_open_mask():
    g = 50.0
    b0 = physics.incident_b0(g, math.radians(2.0), 0.0)
    k = np.array([[0.0, 0.0], [3.0, 0.0], [-3.0, 0.0]])
    gam = physics.gamma_diag(g, b0, k)
    # specular: gamma sin(theta0)
    assert gam[0] == pytest.approx(g * math.sin(math.radians(2.0)), rel=1e-12)
    assert gam[1].real == 0 and gam[1].imag < 0      # evanescent, Im < 0
    assert gam[2].real > 0 and gam[2].imag == 0      # open
    mask = physics.open_beams(g, b0, k)
    assert list(mask) == [True, False, True]
    # Gamma^2 = gamma^2 - |b0 + k|^2 exactly on every branch
    q = b0[None, :] + k
    assert np.allclose(gam ** 2, g * g - (q * q).sum(1), rtol=1e-13, atol=1e-10)


# ---------------------------------------------------------------- tableaux
def _trees(order):
    """Rooted trees as sorted tuples of children, grouped by order."""
    by = {1: [()]}
    for n in range(2, order + 1):
        out = set()
        # children multiset with total order n-1
        def parts(rem, maxkey, acc):
            if rem == 0:
                out.add(tuple(sorted(acc)))
                return
            for m in range(1, rem + 1):
                for t in by[m]:
                    key = (m, t)
                    if maxkey is None or key <= maxkey:
                        parts(rem - m, key, acc + [t])
        parts(n - 1, None, [])
        by[n] = sorted(out)
    return by


def _order(t):
    return 1 + sum(_order(c) for c in t)


def _density(t):
    return _order(t) * math.prod(_density(c) for c in t)


def _weights(t, tab):
    s = tab.stages
    A = [[Fraction(x) for x in row] for row in tab.a_frac]
    g = [Fraction(1)] * s
    for c in t:
        gc = _weights(c, tab)
        Agc = [sum(A[i][j] * gc[j] for j in range(s)) for i in range(s)]
        g = [g[i] * Agc[i] for i in range(s)]
    return g


def _satisfies(tab, order):
    trees = _trees(order)
    for n in range(1, order + 1):
        for t in trees[n]:
            phi = sum(Fraction(b) * w for b, w in zip(tab.b_frac, _weights(t, tab)))
            if phi != Fraction(1, _density(t)):
                return False
    return True


def test_tree_enumeration_counts():
    # number of rooted trees of order 1..6: 1, 1, 2, 4, 9, 20 (OEIS A000081)
    by = _trees(6)
    assert [len(by[n]) for n in range(1, 7)] == [1, 1, 2, 4, 9, 20]


@pytest.mark.parametrize("tab", [RK4, RK6], ids=lambda t: t.name)
def test_tableau_order_conditions(tab):
    assert _satisfies(tab, tab.order)
    assert not _satisfies(tab, tab.order + 1)
    # internal consistency c_r = sum_j a_rj
    for r in range(tab.stages):
        assert sum(Fraction(x) for x in tab.a_frac[r]) == Fraction(tab.c_frac[r])


def test_tableau_node_grid():
    assert RK4.cset == [0, Fraction(1, 2)]
    assert RK4.node_index(3, 0) == 6 and RK4.node_index(3, 1) == 7 and RK4.node_index(3, 3) == 8
    assert RK6.cset == [0, Fraction(1, 3), Fraction(1, 2), Fraction(2, 3)]
    assert RK6.n_nodes(10) == 41


# ------------------------------------------------------------- xi estimate
def test_estcond_is_an_upper_bound_and_tight_at_identity():
    rng = np.random.default_rng(0)
    assert rk.estcond_gershgorin(np.eye(7, dtype=complex)) == 1.0
    for _ in range(50):
        n = 9
        Q = (rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))) * 0.05
        Q += np.diag(rng.uniform(0.5, 3.0, n) * np.exp(1j * rng.uniform(0, 6.28, n)))
        xi = rk.estcond_gershgorin(Q)
        cond = np.linalg.norm(Q, np.inf) * np.linalg.norm(np.linalg.inv(Q), np.inf)
        assert xi >= cond * (1 - 1e-12)
    Q = np.array([[1.0, 2.0], [0.0, 1.0]], dtype=complex)   # row 0 not dominant
    assert rk.estcond_gershgorin(Q) == math.inf


# ------------------------------------------------------------ beam sets
def test_beam_sets():
    b = beams_nearest(61, config2().structures[0].recip)
    assert len({tuple(x) for x in b}) == 61 and tuple(b[0]) == (0, 0)
    assert (b ** 2).sum(1).max() == 18          # N = 61 is the disc h^2 + k^2 <= 18
    assert np.all(np.diff((b ** 2).sum(1)) >= 0)
    r = beams_row(6)
    assert r.shape == (13, 2) and tuple(r[0]) == (0, 0) and set(r[:, 0]) == set(range(-6, 7))


# ---------------------------------------------------------- potential table
def test_potential_table_matches_real_space_fourier_integral():
    """u_g(z) against a direct quadrature of (1/A) int_cell v(r) exp(-i g.r) d^2r
    with the periodic sum of Gaussian atoms evaluated in real space."""
    wl = small_2d(n_beams=9, n_layers=1, m=1, sigma_xy=0.0)
    s = wl.structures[0]
    s.atoms = np.array([[0.7, 1.1, -1.3], [2.0, 3.1, -1.9]])
    s.scat_b = np.array([0.6, 0.9, 1.3, 2.0])            # wide enough for a coarse grid
    kappa = 0.27
    z = np.array([-1.0, -1.6, -2.4])
    tab = potential.potential_table(s, z, kappa, 1, 0.0, 15.0)
    sc = potential.mip_scale(s, 15.0)
    a = math.sqrt(s.cell_area)
    ng = 96
    xs = (np.arange(ng) + 0.5) * a / ng
    X, Y = np.meshgrid(xs, xs, indexing="ij")
    hd, kd = potential.difference_box(s.beams)
    dh, dk, g = potential.box_vectors(hd, kd, s.recip)
    for iz, zz in enumerate(z):
        V = np.zeros_like(X)
        for (x0, y0, z0) in s.atoms:
            for ix in range(-3, 4):
                for iy in range(-3, 4):
                    r2 = (X - x0 - ix * a) ** 2 + (Y - y0 - iy * a) ** 2 + (zz - z0) ** 2
                    for am, bm in zip(s.scat_a, s.scat_b):
                        V += am * np.exp(-bm * r2)
        for col in range(g.shape[0]):
            ref = np.mean(V * np.exp(-1j * (g[col, 0] * X + g[col, 1] * Y)))
            assert tab[iz, col] == pytest.approx(kappa * sc * ref, rel=1e-8, abs=1e-10)


def test_potential_hermitian_and_absorption_sign():
    wl = small_2d()
    s = wl.structures[0]
    z = potential.node_positions(s.thickness, 4, [0])
    kappa = 0.27
    t0 = potential.potential_table(s, z, kappa, 1, 0.0, 15.0)
    hd, kd = potential.difference_box(s.beams)
    ci = potential.coupling_index(s.beams, hd, kd)
    for n in range(z.size):
        U = t0[n][ci]
        assert np.allclose(U, U.conj().T, atol=1e-13)         # real potential -> Hermitian coupling
    ta = potential.potential_table(s, z, kappa, 1, 0.1, 15.0)
    assert np.allclose(ta, t0 * (1 - 0.1j), rtol=1e-14)
    tp = potential.potential_table(s, z, kappa, -1, 0.1, 15.0)
    assert np.allclose(tp, t0 * (-1 - 0.1j), rtol=1e-14)
    # mean inner potential: average of u_0 over a fine z grid of an infinitely
    # replicated slab equals kappa * 15 V when all atoms sit well inside
    # (checked on the closed Gaussian integral)
    s2 = small_row(n_layers=1).structures[0]
    s2.atoms = np.array([[0.0, 0.0, -5.0]])
    zz = np.linspace(-10.0, 0.0, 20001)
    u0 = potential.potential_table(s2, zz, 1.0, 1, 0.0, 15.0)[:, potential.box_vectors(*potential.difference_box(s2.beams), s2.recip)[0].size // 2]
    assert np.trapezoid(u0.real, zz) / s2.thickness == pytest.approx(15.0, rel=1e-6)


def test_potential_direction_matches_finite_differences():
    wl = small_2d(n_beams=13)
    s = wl.structures[0]
    z = potential.node_positions(s.thickness, 6, [0, 0.5])
    rng = np.random.default_rng(3)
    d = np.zeros_like(s.atoms)
    d[:4] = rng.normal(size=(4, 3))
    args = (0.27, 1, 0.1, 15.0)
    an = potential.potential_table_direction(s, z, *args, d)
    eps = 1e-5
    import copy
    sp, sm = copy.deepcopy(s), copy.deepcopy(s)
    sp.atoms = s.atoms + eps * d
    sm.atoms = s.atoms - eps * d
    fd = (potential.potential_table(sp, z, *args) - potential.potential_table(sm, z, *args)) / (2 * eps)
    assert np.abs(an - fd).max() <= 1e-7 * np.abs(an).max()


# ------------------------------------------------ coupling matrix orientation
def _asymmetric_cell():
    """One 1x1 cell with two atoms at general in-plane positions (no mirror,
    no inversion), so that u_g is complex and u_{-g} != u_g."""
    wl = small_2d(n_beams=9, n_slices=4, thickness=4.0, n_layers=1, m=1, sigma_xy=0.0,
                  absorption=0.1, n_angles=3)
    s = wl.structures[0]
    s.atoms = np.array([[0.7, 1.1, -1.3], [2.0, 3.1, -2.6]])
    s.scat_b = np.array([0.6, 0.9, 1.3, 2.0])            # wide enough for a coarse grid
    return wl, s


def test_coupling_matrix_is_the_matrix_element_of_the_potential():
    """Sec. 2.1, Eq. (sch2): inserting psi = sum_k c_k(z) exp(i (b0 + k_k).r)
    into the Schroedinger equation and projecting on exp(i (b0 + k_j).r)
    couples beam j to beam k through (1/A) int_cell exp(-i k_j.r) v(r)
    exp(+i k_k.r) d^2r.  That matrix element is evaluated here by direct
    quadrature of the real-space potential (periodic Gaussian atoms) and
    compared entry by entry with the U_jk the solver uses; the transposed
    orientation (u_{g_k - g_j}) fails on this cell."""
    from oracle import driver
    from oracle.tableaux import RK6
    wl, s = _asymmetric_cell()
    st = driver.StructureSetup(wl, s, RK6)
    sc = potential.mip_scale(s, wl.mean_inner_potential)
    pref = st.kappa * sc * (wl.charge - 1j * wl.absorption)
    a = math.sqrt(s.cell_area)
    ng = 96
    xs = (np.arange(ng) + 0.5) * a / ng
    X, Y = np.meshgrid(xs, xs, indexing="ij")
    kv = physics.beam_vectors(s.beams, s.recip)
    phase = np.exp(1j * (kv[:, 0, None, None] * X[None] + kv[:, 1, None, None] * Y[None]))  # exp(i k_k.r)
    N = s.n_beams
    for node in (0, 3, 7):
        zz = st.z_nodes[node]
        V = np.zeros_like(X)
        for (x0, y0, z0) in s.atoms:
            for ix in range(-3, 4):
                for iy in range(-3, 4):
                    r2 = (X - x0 - ix * a) ** 2 + (Y - y0 - iy * a) ** 2 + (zz - z0) ** 2
                    for am, bm in zip(s.scat_a, s.scat_b):
                        V += am * np.exp(-bm * r2)
        ref = np.empty((N, N), dtype=np.complex128)
        for j in range(N):
            for k in range(N):
                ref[j, k] = pref * np.mean(np.conj(phase[j]) * V * phase[k])
        U = st.U_node(node)
        scale = np.abs(ref).max()
        assert np.abs(U - ref).max() <= 1e-8 * scale
        # the orientation is observable on this cell: the transpose is far off
        assert np.abs(U.T - ref).max() > 1e-3 * scale


def test_transposed_coupling_changes_the_intensities():
    """The orientation of U_jk matters for the output: U^T (u_{g_k - g_j}) is
    the coupling of the in-plane point image v(-r) of the cell, which at the
    same incidence equals the original cell seen from the opposite azimuth;
    on a cell without in-plane symmetry the intensities, specular included,
    change off the specular beam, so a parity test over all beams on such a
    cell (the synthetic slabs carry random in-plane displacements) tells the
    two apart."""
    from oracle import driver
    from oracle.tableaux import RK6
    wl, s = _asymmetric_cell()
    s.n_slices, s.thickness = 40, 4.0
    st = driver.StructureSetup(wl, s, RK6)
    th = float(wl.theta0[1])
    gam, mask = st.angle(th)
    g2 = np.diag(gam * gam)

    def m_t(i, r):
        return st.U_node(RK6.node_index(i, r)).T + g2
    rho, _, _, _ = st.solve(th)
    rho_t, _ = rk.solve_ode_str(m_t, gam, st.h, s.n_slices, RK6)
    eta = rk.intensity(rho, gam, mask, th)
    eta_t = rk.intensity(rho_t, gam, mask, th)
    assert np.abs(eta_t[1:] - eta[1:]).max() > 1e-4 * eta.max()
    # the transpose at the opposite azimuth: the image cell seen from theta1 + pi
    # is the original cell seen from theta1, so U^T there gives eta back
    wl_b = dataclasses.replace(wl, theta1=wl.theta1 + math.pi)
    st_b = driver.StructureSetup(wl_b, s, RK6)
    gam_b, mask_b = st_b.angle(th)
    kv = physics.beam_vectors(s.beams, s.recip)
    # beam k_j at azimuth theta1 + pi corresponds to beam -k_j at theta1
    perm = [next(i for i in range(s.n_beams) if np.allclose(kv[i], -kv[j])) for j in range(s.n_beams)]
    g2b = np.diag(gam_b * gam_b)

    def m_bt(i, r):
        return st_b.U_node(RK6.node_index(i, r)).T + g2b
    rho_bt, _ = rk.solve_ode_str(m_bt, gam_b, st_b.h, s.n_slices, RK6)
    eta_bt = rk.intensity(rho_bt, gam_b, mask_b, th)
    assert np.allclose(eta_bt[perm], eta, rtol=1e-9, atol=1e-14)


def test_uneven_workload_slices_follow_the_step_rule():
    """The uneven-N workload's slices per N are the smallest multiple of 20
    (at least 400) with h max_j |Gamma_j| <= 1.45 over its angles, Gamma from
    the oracle (Sec. 2.1); 400 slices break that bound for N >= 61."""
    import math

    from synth import workloads as W
    wl = W.config3(8)
    gamma = physics.wavenumber(wl.energy_eV)
    seen = {}
    for st in wl.structures:
        kv = physics.beam_vectors(st.beams, st.recip)
        gmax = max(np.max(np.abs(physics.gamma_diag(gamma, physics.incident_b0(gamma, float(th), wl.theta1), kv)))
                   for th in wl.theta0)
        want = max(400, 20 * math.ceil(st.thickness * gmax / (W.UNEVEN_H_GAMMA * 20)))
        assert st.n_slices == want == W.UNEVEN_SLICES[st.n_beams]
        seen[st.n_beams] = st.thickness / 400 * gmax
    assert seen[31] < 1.6 and all(seen[n] > W.UNEVEN_H_GAMMA for n in (61, 91, 121) if n in seen)
