"""Parity of the forward pass for 256 < N <= 576 (every pair on a group of
workgroups stepping its 16-column blocks side by side; stage inputs formed
in row chunks, stage products and eliminations streamed through the pair's
memory) with the oracle's RK multi-slice, through the C ABI: N = 257, 300,
400, 521 and the full width 576, both RK steppers, one pair and several, a
plan that mixes it with the kernels for N <= 256, the paper's single-angle
n = 521 case at full size, and the refusals."""
import dataclasses

import numpy as np
import pytest

from synth import small_2d
from tests.gpu_util import eacc, gpu_forward, oracle_forward, physical

pytestmark = pytest.mark.gpu

TOL = 1e-10


def _report(name, e):
    print(f"[parity-xxl] {name}: eacc={e:.3e}", flush=True)


@pytest.mark.parametrize("stepper,n_beams,n_angles", [("rk4", 257, 2), ("rk6", 300, 2), ("rk6", 400, 1),
                                                      ("rk4", 521, 1), ("rk6", 576, 1)])
def test_forward_xxl_matches_oracle(stepper, n_beams, n_angles):
    """Thin slabs of a 7x7 cell (12 RK6 or 20 RK4 slices of 0.1 A): every
    pair on ceil(N / 16) workgroups, against the oracle."""
    L = 12 if stepper == "rk6" else 20
    wl = small_2d(n_beams=n_beams, n_slices=L, thickness=0.1 * L, n_layers=1, n_angles=n_angles, m=7)
    print(f"[parity-xxl] start {stepper} N={n_beams} angles={n_angles}", flush=True)
    res = gpu_forward(wl, stepper=stepper, want_rho=True)
    info = res["plan"].info
    assert info.xxl_pairs == n_angles and info.xxl_group == (n_beams + 15) // 16
    ref, rho_ref, nr = oracle_forward(wl, stepper=stepper)
    assert (res["status"] == 0).all()
    e = eacc(res["intensity"][:, :n_beams], ref)
    _report(f"{stepper} N={n_beams} rhst={nr.tolist()} gpu_rhst={res['n_rhst'].tolist()}", e)
    assert e <= TOL
    assert res["n_rhst"].tolist() == nr.tolist()
    rho = res["rho"][:, :n_beams]
    assert np.abs(rho - rho_ref).max() <= 1e-9 * np.abs(rho_ref).max()


def test_plan_mixing_n199_and_n300():
    """N = 45, 199 and 300 in one plan (three kernels, one launch each):
    each structure against the oracle, and zeros beyond each structure's N."""
    parts = [small_2d(n_beams=n, n_slices=L, thickness=0.1 * L, n_layers=1, n_angles=2, m=m, seed=90 + i)
             for i, (n, L, m) in enumerate(((45, 24, 3), (199, 16, 7), (300, 12, 7)))]
    wl = dataclasses.replace(parts[0], structures=[p.structures[0] for p in parts])
    res = gpu_forward(wl, stepper="rk6")
    info = res["plan"].info
    assert info.xl_pairs == 2 and info.xxl_pairs == 2
    assert (res["status"] == 0).all()
    A = len(wl.theta0)
    for s, p in enumerate(parts):
        N = p.structures[0].n_beams
        ref, _, _ = oracle_forward(wl, s_idx=s, stepper="rk6")
        e = eacc(res["intensity"][s * A:(s + 1) * A, :N], ref)
        _report(f"mixed plan structure {s} N={N}", e)
        assert e <= TOL
        assert np.all(res["intensity"][s * A:(s + 1) * A, N:] == 0.0)


def test_single_angle_n521_full_size():
    """The paper's single-angle case at its size (n = 521, 9.91 A in 661
    RK4 slices of 0.015 A, 10 keV positrons at 1.3 deg, azimuth -30 deg):
    through the validity gate and against the oracle."""
    from synth import single_angle_n521
    wl = single_angle_n521()
    res = gpu_forward(wl, stepper="rk4")
    assert res["plan"].info.xxl_group == 33
    assert (res["status"] == 0).all()
    got = res["intensity"][:, :521]
    assert physical(got, wl.absorption).all()
    ref, _, nr = oracle_forward(wl, stepper="rk4")
    e = eacc(got, ref)
    _report(f"n=521 full size rhst gpu {res['n_rhst'].tolist()} oracle {nr.tolist()}, "
            f"specular {got[0, 0]:.6e} sum {got.sum():.6e}", e)
    assert e <= TOL
    assert res["n_rhst"].tolist() == nr.tolist()


def test_xxl_refusals():
    import torch
    from paper_2306_00271_amd import api
    from paper_2306_00271_amd._lib import RheedError
    wl = small_2d(n_beams=300, n_slices=4, thickness=0.4, n_layers=1, n_angles=2, m=7)
    with pytest.raises(RheedError, match="N > 128"):
        api.plan_for(wl, stepper="sp4")
    plan = api.plan_for(wl, stepper="rk6")
    assert plan.info.fwd_workspace == 0 and plan.info.bwd_workspace == 0
    dev = torch.device("cuda:0")
    U = plan.potential(api.atoms_for(wl, dev))
    ws = torch.empty(1 << 20, dtype=torch.uint8, device=dev)
    with pytest.raises(RheedError, match="N <= 256"):
        plan.forward(U, api.angles_for(wl, dev), workspace=ws)


@pytest.mark.parametrize("n_angles,group", [(100, 2), (200, 1), (300, 1)])
def test_many_pairs_small_groups(n_angles, group):
    """Enough pairs that each gets a group of 2 (one owner in the
    elimination pipeline) or of 1 (the one-workgroup elimination), and more
    pairs than the device holds at once (two launches): N = 257 on a thin
    slab, sampled pairs against the oracle, every pair valid."""
    wl = small_2d(n_beams=257, n_slices=6, thickness=0.6, n_layers=1, n_angles=n_angles, m=7)
    res = gpu_forward(wl, stepper="rk6")
    assert res["plan"].info.xxl_group == group
    assert (res["status"] == 0).all()
    assert physical(res["intensity"][:, :257], wl.absorption).all()
    idx = [0, n_angles // 2, n_angles - 1]
    ref, _, nr = oracle_forward(wl, angle_idx=idx, stepper="rk6")
    e = eacc(res["intensity"][idx, :257], ref)
    _report(f"N=257, {n_angles} pairs on groups of {group}, rhst gpu {res['n_rhst'][idx].tolist()} "
            f"oracle {nr.tolist()}", e)
    assert e <= TOL
    assert res["n_rhst"][idx].tolist() == nr.tolist()


@pytest.mark.parametrize("half", [0, 1])
def test_group_wait_failure_is_reported(half):
    """As for N <= 256: a workgroup of every pair's group forced to wait
    for no other; every pair RHEED_PAIR_SYNC from a call that succeeds, then
    oracle parity again with the hook off."""
    import torch
    from paper_2306_00271_amd import api
    wl = small_2d(n_beams=300, n_slices=8, thickness=0.8, n_layers=1, n_angles=2, m=7)
    dev = torch.device("cuda:0")
    plan = api.plan_for(wl, stepper="rk6")
    assert plan.info.xxl_group == 19
    U = plan.potential(api.atoms_for(wl, dev))
    ang = api.angles_for(wl, dev)
    plan.force_sync_failure(half)
    out = plan.forward(U, ang)
    torch.cuda.synchronize()
    st = out["status"].cpu().numpy()
    print(f"[parity-xxl] forced give-up in workgroup {half}: status {st.tolist()}", flush=True)
    assert (st == 3).all()
    assert np.isnan(out["intensity"].cpu().numpy()[:, :300]).all()
    plan.force_sync_failure(-1)
    out = plan.forward(U, ang)
    torch.cuda.synchronize()
    assert (out["status"].cpu().numpy() == 0).all()
    ref, _, _ = oracle_forward(wl, stepper="rk6")
    e = eacc(out["intensity"].cpu().numpy()[:, :300], ref)
    _report("group launch after the forced failure", e)
    assert e <= TOL
