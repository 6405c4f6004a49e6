"""Parity of the forward pass for 128 < N <= 256 (the kernel that keeps the
state in plan-owned memory, stores its stage products there and streams the
rows of its eliminations) with the oracle's RK multi-slice, through the C
ABI: several tiles and a ragged tail (N = 129, 160, 199 and the full width
256), both RK steppers, a batch mixing all three kernels, the N = 199
workload's slab at full size on sampled angles, and the refusals."""
import dataclasses

import numpy as np
import pytest

from synth import small_2d
from tests.gpu_util import eacc, gpu_forward, oracle_forward, physical

pytestmark = pytest.mark.gpu

TOL = 1e-10


def _report(name, e):
    print(f"[parity-xl] {name}: eacc={e:.3e}", flush=True)


@pytest.mark.parametrize("layout", ["auto", "whole"])
@pytest.mark.parametrize("stepper,n_beams", [("rk6", 129), ("rk6", 160), ("rk4", 199), ("rk6", 199), ("rk6", 256)])
def test_forward_xl_matches_oracle(stepper, n_beams, layout):
    """Three pairs: with layout AUTO each on a group of workgroups (one per
    16-column block), with WHOLE each on one workgroup."""
    L = 20 if stepper == "rk6" else 32
    wl = small_2d(n_beams=n_beams, n_slices=L, thickness=0.1 * L, n_layers=1, n_angles=3)
    res = gpu_forward(wl, stepper=stepper, want_rho=True, layout=layout)
    assert res["plan"].info.xl_pairs == 3
    assert res["plan"].info.xl_group == (1 if layout == "whole" else (n_beams + 15) // 16)
    ref, rho_ref, nr = oracle_forward(wl, stepper=stepper)
    got = res["intensity"][:, :n_beams]
    assert (res["status"] == 0).all()
    e = eacc(got, ref)
    _report(f"{stepper} N={n_beams} {layout} rhst={nr.tolist()} gpu_rhst={res['n_rhst'].tolist()}", e)
    assert e <= TOL
    assert res["n_rhst"].tolist() == nr.tolist()
    rho = res["rho"][:, :n_beams]
    assert np.abs(rho - rho_ref).max() <= 1e-9 * np.abs(rho_ref).max()


def test_batch_mixing_three_kernels():
    """N = 45, 91 and 199 in one plan (one launch per kernel): each
    structure against the oracle, and zeros beyond each structure's N."""
    parts = [small_2d(n_beams=n, n_slices=L, thickness=0.1 * L, n_layers=1, n_angles=2, seed=80 + i)
             for i, (n, L) in enumerate(((45, 30), (91, 24), (199, 16)))]
    wl = dataclasses.replace(parts[0], structures=[p.structures[0] for p in parts])
    res = gpu_forward(wl, stepper="rk6")
    info = res["plan"].info
    assert info.large_pairs == 2 and info.xl_pairs == 2 and not info.queue
    assert (res["status"] == 0).all()
    A = len(wl.theta0)
    for s, p in enumerate(parts):
        N = p.structures[0].n_beams
        ref, _, _ = oracle_forward(wl, s_idx=s, stepper="rk6")
        e = eacc(res["intensity"][s * A:(s + 1) * A, :N], ref)
        _report(f"mixed batch structure {s} N={N}", e)
        assert e <= TOL
        assert np.all(res["intensity"][s * A:(s + 1) * A, N:] == 0.0)


@pytest.mark.parametrize("n_beams", [150, 199])
def test_group_and_one_workgroup_agree(n_beams):
    """The group launch (columns of a pair on several CUs, row sums summed
    across them) and the one-workgroup launch give the same curves and the
    same transformation counts."""
    wl = small_2d(n_beams=n_beams, n_slices=40, thickness=4.0, n_layers=2, n_angles=2, seed=5)
    grp = gpu_forward(wl, stepper="rk6", layout="auto")
    one = gpu_forward(wl, stepper="rk6", layout="whole")
    assert grp["plan"].info.xl_group > 1 and one["plan"].info.xl_group == 1
    assert (grp["status"] == 0).all() and (one["status"] == 0).all()
    assert grp["n_rhst"].tolist() == one["n_rhst"].tolist()
    d = np.abs(grp["intensity"] - one["intensity"]).max()
    print(f"[parity-xl] N={n_beams} group vs one workgroup: max |diff| = {d:.3e}", flush=True)
    np.testing.assert_allclose(grp["intensity"], one["intensity"], rtol=0.0, atol=1e-13)


def test_single_pair_group_matches_oracle():
    """One pair of N = 256 alone (16 workgroups on it) against the oracle."""
    wl = small_2d(n_beams=256, n_slices=24, thickness=2.4, n_layers=1, n_angles=1, theta_range=(2.0, 2.0))
    res = gpu_forward(wl, stepper="rk6")
    assert res["plan"].info.xl_group == 16
    ref, _, nr = oracle_forward(wl, stepper="rk6")
    assert (res["status"] == 0).all()
    e = eacc(res["intensity"][:, :256], ref)
    _report(f"single pair N=256 on 16 workgroups rhst={nr.tolist()} gpu={res['n_rhst'].tolist()}", e)
    assert e <= TOL
    assert res["n_rhst"].tolist() == nr.tolist()


def test_n199_workload_full_size_sampled():
    """The N = 199 slab of the large workload at full size (60 A in 1000
    slices, RK6) at four angles: every pair through the validity gate, and
    one angle against the oracle."""
    from synth import config5
    wl = config5(1)
    idx = [10, 100, 180, 250]
    sub = dataclasses.replace(wl, theta0=wl.theta0[idx])
    res = gpu_forward(sub, stepper="rk6")
    assert (res["status"] == 0).all()
    got = res["intensity"][:, :199]
    assert physical(got, sub.absorption).all()
    ref, _, nr = oracle_forward(sub, angle_idx=[1], stepper="rk6")
    e = eacc(got[[1]], ref)
    _report(f"N=199 full size, angle {idx[1]}, rhst gpu {res['n_rhst'][1]} oracle {nr.tolist()}", e)
    assert e <= TOL


def test_xl_refusals():
    import torch
    from paper_2306_00271_amd import api
    from paper_2306_00271_amd._lib import RheedError
    wl = small_2d(n_beams=150, n_slices=4, thickness=0.4, n_layers=1, n_angles=2)
    with pytest.raises(RheedError, match="N > 128 needs an RK stepper"):
        api.plan_for(wl, stepper="sp4")
    plan = api.plan_for(wl, stepper="rk6")
    # states padded to 256 beams: at least the final state and B^{-1} per pair
    assert plan.info.fwd_workspace >= plan.n_pairs * 3 * 256 * 256 * 16
    dev = torch.device("cuda:0")
    U = plan.potential(api.atoms_for(wl, dev))
    ws = torch.empty(1024, dtype=torch.uint8, device=dev)
    with pytest.raises(RheedError, match="workspace of"):
        plan.forward(U, api.angles_for(wl, dev), workspace=ws)


def test_group_of_two_matches_one_workgroup():
    """128 pairs of N = 150 get groups of 2 (the elimination pipeline with a
    single owner): the same curves and transformation counts as one
    workgroup per pair."""
    wl = small_2d(n_beams=150, n_slices=12, thickness=1.2, n_layers=1, n_angles=128, seed=9)
    grp = gpu_forward(wl, stepper="rk6", layout="auto")
    one = gpu_forward(wl, stepper="rk6", layout="whole")
    assert grp["plan"].info.xl_group == 2 and one["plan"].info.xl_group == 1
    assert (grp["status"] == 0).all() and (one["status"] == 0).all()
    assert grp["n_rhst"].tolist() == one["n_rhst"].tolist()
    d = np.abs(grp["intensity"] - one["intensity"]).max()
    print(f"[parity-xl] N=150, 128 pairs, groups of 2 vs one workgroup: max |diff| = {d:.3e}", flush=True)
    np.testing.assert_allclose(grp["intensity"], one["intensity"], rtol=0.0, atol=1e-13)


@pytest.mark.parametrize("half", [0, 1])
def test_group_wait_failure_is_reported(half):
    """The group launch's failure path, forced from the host: workgroup 0
    (which records the eliminations) or 1 (an owner in the elimination
    pipeline) of every pair's group waits for no other workgroup, as after
    a give-up.  Every pair must come back RHEED_PAIR_SYNC with NaN outputs
    from a call that succeeds; with the hook off the same plan is back to
    oracle parity."""
    import torch
    from paper_2306_00271_amd import api
    wl = small_2d(n_beams=150, n_slices=16, thickness=1.6, n_layers=1, n_angles=2)
    dev = torch.device("cuda:0")
    plan = api.plan_for(wl, stepper="rk6")
    assert plan.info.xl_group == 10
    U = plan.potential(api.atoms_for(wl, dev))
    ang = api.angles_for(wl, dev)
    plan.force_sync_failure(half)
    out = plan.forward(U, ang)
    torch.cuda.synchronize()
    st = out["status"].cpu().numpy()
    print(f"[parity-xl] forced give-up in workgroup {half}: status {st.tolist()}", flush=True)
    assert (st == 3).all()
    assert np.isnan(out["intensity"].cpu().numpy()[:, :150]).all()
    plan.force_sync_failure(-1)
    out = plan.forward(U, ang)
    torch.cuda.synchronize()
    assert (out["status"].cpu().numpy() == 0).all()
    ref, _, _ = oracle_forward(wl, stepper="rk6")
    e = eacc(out["intensity"].cpu().numpy()[:, :150], ref)
    _report("group launch after the forced failure", e)
    assert e <= TOL
