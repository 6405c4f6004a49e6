"""Parity of the splitting steppers (Sec. 3.4, BAB and ABA forms; the
fourth-order triple jump of the Stormer-Verlet step and the sixth-order
triple jump of that) on the GPU with the oracle's own splitting steps,
through the C ABI: N <= 64 on the one-workgroup kernel, N > 64 (fourth-order
BAB only) on the kernel that keeps the state in plan-owned memory; and their
adjoint (N <= 64) against the oracle's tangent-linear derivatives."""
import dataclasses

import numpy as np
import pytest

from oracle import driver
from oracle.tableaux import TABLEAUX
from synth import small_2d, small_row
from tests.gpu_util import eacc, gpu_forward, oracle_forward

pytestmark = pytest.mark.gpu

TOL = 1e-10


def _report(name, e):
    print(f"[parity] {name}: eacc={e:.3e}", flush=True)


@pytest.mark.parametrize("stepper", ["sp4", "sp6", "sp4a", "sp6a"])
def test_potential_tables_at_the_splitting_nodes(stepper):
    """The kick positions of every slice (for the BAB methods partly outside
    the slice) and the final node, against the oracle's table: the node
    order of the library is the oracle's."""
    wl = small_2d(n_beams=37, n_slices=10, n_layers=2)
    res = gpu_forward(wl, stepper=stepper)
    st = driver.StructureSetup(wl, wl.structures[0], TABLEAUX[stepper])
    assert res["plan"].info.nodes_per_slice == len(TABLEAUX[stepper].cset)
    ref = st.table.ravel()
    assert res["U"].shape == ref.shape
    assert np.abs(res["U"] - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("n_beams", [1, 21, 45, 64])
@pytest.mark.parametrize("stepper", ["sp4", "sp6", "sp4a", "sp6a"])
def test_forward_splitting_one_workgroup(stepper, n_beams):
    """Every splitting method on the one-workgroup kernel (N <= 64), several
    tiles and a ragged tail, against the oracle's splitting step: the same
    transformation decisions and 1e-10 in eacc."""
    wl = small_2d(n_beams=n_beams, n_slices=40, thickness=4.0, n_layers=2, n_angles=4)
    res = gpu_forward(wl, stepper=stepper, want_rho=True)
    assert res["plan"].info.large_pairs == 0 and not res["plan"].split
    ref, rho_ref, nr = oracle_forward(wl, stepper=stepper)
    got = res["intensity"][:, :n_beams]
    assert (res["status"] == 0).all()
    e = eacc(got, ref)
    _report(f"{stepper} N={n_beams} rhst={nr.tolist()} gpu_rhst={res['n_rhst'].tolist()}", e)
    assert e <= TOL
    assert res["n_rhst"].tolist() == nr.tolist()
    rho = res["rho"][:, :n_beams]
    assert np.abs(rho - rho_ref).max() <= 1e-9 * np.abs(rho_ref).max()


@pytest.mark.parametrize("stepper", ["sp6", "sp4a"])
def test_splitting_full_size_n61(stepper):
    """The N = 61 slab at full size (40 A, 128 angles) with a splitting
    method at the grid of the stepper comparison (800 slices), sampled
    angles against the oracle, every pair through the validity gate."""
    from synth import config2
    from tests.gpu_util import physical
    wl = config2()
    wl = dataclasses.replace(wl, structures=[dataclasses.replace(wl.structures[0], n_slices=800)])
    res = gpu_forward(wl, stepper=stepper)
    assert (res["status"] == 0).all()
    assert physical(res["intensity"][:, :61], wl.absorption).all()
    idx = [0, 64, 127]
    ref, _, _ = oracle_forward(wl, angle_idx=idx, stepper=stepper)
    e = eacc(res["intensity"][idx, :61], ref)
    _report(f"{stepper} N=61 800 slices (sampled angles)", e)
    assert e <= TOL


def test_splitting_for_large_n_is_fourth_order_bab_only():
    from paper_2306_00271_amd import api
    from paper_2306_00271_amd._lib import RheedError
    wl = small_2d(n_beams=69, n_slices=4, thickness=0.4, n_layers=2, n_angles=2)
    for stepper in ("sp6", "sp4a", "sp6a"):
        with pytest.raises(RheedError, match="RHEED_SP4"):
            api.plan_for(wl, stepper=stepper)


@pytest.mark.parametrize("n_beams", [65, 121])
def test_forward_sp4(n_beams):
    wl = small_2d(n_beams=n_beams, n_slices=40, thickness=4.0, n_layers=2, n_angles=4)
    res = gpu_forward(wl, stepper="sp4", want_rho=True)
    ref, rho_ref, nr = oracle_forward(wl, stepper="sp4")
    got = res["intensity"][:, :n_beams]
    assert (res["status"] == 0).all()
    e = eacc(got, ref)
    _report(f"sp4 N={n_beams} rhst={nr.tolist()} gpu_rhst={res['n_rhst'].tolist()}", e)
    assert e <= TOL
    assert res["n_rhst"].tolist() == nr.tolist()
    rho = res["rho"][:, :n_beams]
    assert np.abs(rho - rho_ref).max() <= 1e-9 * np.abs(rho_ref).max()


def test_forward_sp4_single_beam_and_row():
    """N = 1 (one column block of one k-step) and the 13-beam positron row."""
    wl = small_row(hmax=0, n_slices=60, thickness=6.0, n_layers=2, n_angles=5)
    res = gpu_forward(wl, stepper="sp4")
    ref, _, _ = oracle_forward(wl, stepper="sp4")
    e = eacc(res["intensity"][:, :1], ref)
    _report("sp4 N=1", e)
    assert e <= TOL
    wl = small_row(hmax=6, n_slices=80, thickness=12.0, n_layers=4, n_angles=6)
    res = gpu_forward(wl, stepper="sp4")
    ref, _, _ = oracle_forward(wl, stepper="sp4")
    e = eacc(res["intensity"][:, :13], ref)
    _report("sp4 row N=13", e)
    assert e <= TOL


def test_sp4_uneven_batch_in_one_launch():
    parts = [small_2d(n_beams=n, n_slices=L, thickness=0.1 * L, n_layers=2, n_angles=3, seed=70 + i)
             for i, (n, L) in enumerate(((13, 30), (61, 24), (91, 20)))]
    wl = dataclasses.replace(parts[0], structures=[p.structures[0] for p in parts])
    res = gpu_forward(wl, stepper="sp4")
    assert res["plan"].info.large_pairs == 3
    assert (res["status"] == 0).all()
    A = len(wl.theta0)
    for s, p in enumerate(parts):
        N = p.structures[0].n_beams
        ref, _, _ = oracle_forward(wl, s_idx=s, stepper="sp4")
        e = eacc(res["intensity"][s * A:(s + 1) * A, :N], ref)
        _report(f"sp4 batch structure {s} N={N}", e)
        assert e <= TOL
        assert np.all(res["intensity"][s * A:(s + 1) * A, N:] == 0.0)


def test_splitting_refuses_split_layout_and_large_n_adjoint():
    import torch
    from paper_2306_00271_amd import api
    from paper_2306_00271_amd._lib import RheedError
    wl = small_2d(n_beams=21, n_slices=4, thickness=0.4, n_layers=2, n_angles=2)
    for stepper in ("sp4", "sp6", "sp4a", "sp6a"):
        with pytest.raises(RheedError, match="one-workgroup"):
            api.plan_for(wl, stepper=stepper, layout="split")
    big = small_2d(n_beams=69, n_slices=4, thickness=0.4, n_layers=2, n_angles=2)
    plan = api.plan_for(big, stepper="sp4")
    assert plan.info.fwd_workspace == 0
    dev = torch.device("cuda:0")
    U = plan.potential(api.atoms_for(big, dev))
    ws = torch.empty(1024, dtype=torch.uint8, device=dev)
    with pytest.raises(RheedError, match="N <= 64"):
        plan.forward(U, api.angles_for(big, dev), workspace=ws)


def _grad(wl, stepper, target, every):
    import torch
    from paper_2306_00271_amd import api
    dev = torch.device("cuda:0")
    print(f"[adjoint-sp] {stepper} N={wl.structures[0].n_beams} K={every}", flush=True)
    plan = api.plan_for(wl, stepper=stepper, checkpoint_every=every)
    atoms = api.atoms_for(wl, dev)
    U = plan.potential(atoms)
    ang = api.angles_for(wl, dev)
    ws = plan.workspace(dev)
    out = plan.forward(U, ang, workspace=ws, want_nrhst=True)
    tgt = torch.from_numpy(np.asarray(target, dtype=np.float64)).to(dev)
    loss, dI = api.rfactor(out["intensity"], tgt)
    dU = plan.backward(U, ang, dI, ws)
    dA = plan.potential_backward(atoms, dU)
    torch.cuda.synchronize()
    res = {"loss": float(loss.item()), "dU": dU.cpu().numpy(), "datoms": dA.cpu().numpy(),
           "status": out["status"].cpu().numpy(), "n_rhst": out["n_rhst"].cpu().numpy()}
    del ws, plan
    return res


@pytest.mark.parametrize("every", [1, 7])
@pytest.mark.parametrize("stepper", ["sp4", "sp6", "sp4a", "sp6a"])
def test_splitting_table_gradient_matches_oracle_tangent(stepper, every):
    """The splitting adjoint (kicks as Hermitian table products on the
    adjoint vector, drifts as vector updates, the BAB method's merged end
    kicks) against the oracle's tangent-linear derivative along random
    table directions, over a slab with several transformations."""
    wl = small_2d(n_beams=21, n_slices=30, thickness=3.0, n_layers=1, n_angles=3)
    tgt = np.random.default_rng(3).uniform(0.0, 0.3, size=3)
    res = _grad(wl, stepper, tgt, every)
    assert (res["status"] == 0).all() and res["n_rhst"].min() >= 2
    st = driver.StructureSetup(wl, wl.structures[0], TABLEAUX[stepper])
    rng = np.random.default_rng(11)
    for _ in range(2):
        dt = rng.normal(size=st.table.shape) + 1j * rng.normal(size=st.table.shape)
        loss, dl = driver.rfactor_directional_table(wl, 0, dt, tgt, stepper=stepper)
        got = float(np.real(np.sum(np.conj(res["dU"]) * dt.ravel())))
        print(f"[adjoint-sp] {stepper} K={every} table direction: gpu {got:.12e} oracle {dl:.12e}", flush=True)
        assert res["loss"] == pytest.approx(loss, rel=1e-10)
        assert got == pytest.approx(dl, rel=1e-9)


@pytest.mark.parametrize("stepper,every", [("sp4", 1), ("sp6a", 20)])
def test_splitting_atom_gradient_every_coordinate(stepper, every):
    """Every coordinate of the 9 atoms of a small slab against the oracle's
    tangent-linear derivative along that coordinate, entry by entry."""
    from tests.gpu_util import assert_entrywise, oracle_atom_gradient
    wl = small_2d(n_beams=29, n_slices=40, thickness=4.0, n_layers=1, n_angles=3)
    tgt = np.random.default_rng(13).uniform(0.0, 0.3, size=3)
    res = _grad(wl, stepper, tgt, every)
    assert (res["status"] == 0).all()
    n_atoms = wl.structures[0].atoms.shape[0]
    coords = [(ia, c) for ia in range(n_atoms) for c in range(3)]
    ref = oracle_atom_gradient(wl, tgt, coords, stepper=stepper)
    got = np.array([res["datoms"][ia, c] for ia, c in coords])
    assert_entrywise(got, ref, what=f"{stepper} K={every}, all {len(coords)} coordinates")


@pytest.mark.parametrize("stepper", ["sp4", "sp6a"])
def test_splitting_checkpoint_segments_match_every_slice_states(stepper):
    wl = small_2d(n_beams=21, n_slices=50, thickness=5.0, n_layers=1, n_angles=3)
    tgt = np.random.default_rng(6).uniform(0.0, 0.3, size=3)
    ref = _grad(wl, stepper, tgt, 1)
    got = _grad(wl, stepper, tgt, 20)
    err = np.abs(got["dU"] - ref["dU"]).max() / np.abs(ref["dU"]).max()
    print(f"[adjoint-sp] {stepper} K=20 vs K=1: {err:.3e}", flush=True)
    np.testing.assert_allclose(got["dU"], ref["dU"], rtol=0.0, atol=1e-13 * np.abs(ref["dU"]).max())
