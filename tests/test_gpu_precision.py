"""Lower-precision evaluation (the paper's Sec. 6 names single and half
precision as future work): the RK stage products U X in FP32 on the FP32
matrix cores, everything else in FP64, for every N <= 256 (the kernels for
N <= 64, 64 < N <= 128 and both launches of the one for 128 < N <= 256).
The reference is the FP64 oracle.
FP32 rounds each operand to a relative 6e-8 and a 64-term product
accumulates a few times that, so a slab's curve moves by ~1e-7 relative:
the bound is 1e-5 in eacc (the paper's accuracy target for its steppers is
eacc ~1e-4), and the curve must move by more than 1e-11 (the FP32 path is
really taken)."""
import dataclasses

import numpy as np
import pytest

from synth import config2, small_2d
from tests.gpu_util import eacc, gpu_forward, oracle_forward, physical

pytestmark = pytest.mark.gpu

BOUND = 1e-5


def _report(name, e):
    print(f"[fp32] {name}: eacc={e:.3e}", flush=True)


def _run(wl, stepper, precision, layout="auto", threshold=1000.0):
    import torch
    from paper_2306_00271_amd import api
    dev = torch.device("cuda:0")
    plan = api.plan_for(wl, stepper=stepper, layout=layout, stage_precision=precision, threshold=threshold)
    U = plan.potential(api.atoms_for(wl, dev))
    out = plan.forward(U, api.angles_for(wl, dev), want_nrhst=True)
    torch.cuda.synchronize()
    res = {k: (v.cpu().numpy() if v is not None else None) for k, v in out.items()}
    res["plan"] = plan
    return res


@pytest.mark.parametrize("layout", ["whole", "split"])
@pytest.mark.parametrize("stepper", ["rk4", "rk6"])
def test_fp32_stages_against_the_oracle(stepper, layout):
    wl = small_2d(n_beams=45, n_slices=80 if stepper == "rk4" else 40, thickness=4.0, n_layers=2, n_angles=4)
    res = _run(wl, stepper, "fp32", layout=layout)
    assert res["plan"].split == (layout == "split")
    assert (res["status"] == 0).all()
    ref, _, _ = oracle_forward(wl, stepper=stepper)
    e = eacc(res["intensity"][:, :45], ref)
    _report(f"small2d N=45 {stepper} {layout}", e)
    assert 1e-11 < e <= BOUND


def test_fp32_stages_full_size_n61():
    """The N = 61 slab of the gradient workload (400 slices, 128 angles,
    RK6, split layout): the FP32-stage curves against the FP64 ones on every
    angle and against the oracle on sampled ones; the FP32 rounding must stay
    far below the step's own discretisation error (RK6 at 400 slices against
    1600 slices), and every pair must pass the validity gate."""
    wl = config2(stepper="rk6")
    f32 = _run(wl, "rk6", "fp32")
    f64 = _run(wl, "rk6", "fp64")
    assert (f32["status"] == 0).all() and physical(f32["intensity"][:, :61], wl.absorption).all()
    e = eacc(f32["intensity"][:, :61], f64["intensity"][:, :61])
    fine = dataclasses.replace(wl, structures=[dataclasses.replace(wl.structures[0], n_slices=1600)])
    f64_fine = _run(fine, "rk6", "fp64")
    disc = eacc(f64["intensity"][:, :61], f64_fine["intensity"][:, :61])
    idx = [0, 64, 127]
    ref, _, _ = oracle_forward(wl, angle_idx=idx)
    eo = eacc(f32["intensity"][idx, :61], ref)
    _report(f"N=61 full size: FP32 vs FP64 stages {e:.3e}, FP32 vs oracle (sampled) {eo:.3e}, "
            f"discretisation error of the grid {disc:.3e}", e)
    assert 1e-11 < e <= BOUND and eo <= BOUND
    assert e < 1e-3 * disc


@pytest.mark.parametrize("layout", ["whole", "auto"])
@pytest.mark.parametrize("stepper,n_beams", [("rk4", 150), ("rk6", 199)])
def test_fp32_stages_wide_against_the_oracle(stepper, n_beams, layout):
    """128 < N <= 256 on one workgroup per pair and on a group per pair:
    the FP32-stage curves against the oracle within the bound, and moved
    from the FP64 ones (the FP32 instance really runs)."""
    L = 24 if stepper == "rk6" else 40
    wl = small_2d(n_beams=n_beams, n_slices=L, thickness=0.1 * L, n_layers=1, n_angles=3)
    f32 = _run(wl, stepper, "fp32", layout=layout)
    f64 = _run(wl, stepper, "fp64", layout=layout)
    assert f32["plan"].info.xl_group == (1 if layout == "whole" else (n_beams + 15) // 16)
    assert (f32["status"] == 0).all()
    ref, _, _ = oracle_forward(wl, stepper=stepper)
    e = eacc(f32["intensity"][:, :n_beams], ref)
    moved = eacc(f32["intensity"][:, :n_beams], f64["intensity"][:, :n_beams])
    _report(f"small2d N={n_beams} {stepper} {layout}: vs oracle {e:.3e}, vs FP64 stages {moved:.3e}", e)
    assert e <= BOUND and 1e-11 < moved <= BOUND


@pytest.mark.parametrize("stepper,n_beams", [("rk4", 91), ("rk6", 121)])
def test_fp32_stages_n_up_to_128_against_the_oracle(stepper, n_beams):
    """64 < N <= 128 (the slot-based kernel): the FP32-stage curves against
    the oracle within the bound, and moved from the FP64 ones."""
    L = 24 if stepper == "rk6" else 40
    wl = small_2d(n_beams=n_beams, n_slices=L, thickness=0.1 * L, n_layers=1, n_angles=3, m=7)
    f32 = _run(wl, stepper, "fp32")
    f64 = _run(wl, stepper, "fp64")
    assert f32["plan"].info.large_pairs == 3
    assert (f32["status"] == 0).all()
    ref, _, _ = oracle_forward(wl, stepper=stepper)
    e = eacc(f32["intensity"][:, :n_beams], ref)
    moved = eacc(f32["intensity"][:, :n_beams], f64["intensity"][:, :n_beams])
    _report(f"small2d N={n_beams} {stepper}: vs oracle {e:.3e}, vs FP64 stages {moved:.3e}", e)
    assert e <= BOUND and 1e-11 < moved <= BOUND


def test_fp32_stages_full_size_n199():
    """The N = 199 slab at full size (1000 slices, RK6) at 16 angles: the
    FP32-stage curves against the FP64 ones within the bound and far below
    the grid's discretisation error (1000 against 2000 slices, two angles),
    every pair through the validity gate."""
    from synth import config5
    wl = config5(1)
    sub = dataclasses.replace(wl, theta0=wl.theta0[::16])
    f32 = _run(sub, "rk6", "fp32")
    f64 = _run(sub, "rk6", "fp64")
    assert (f32["status"] == 0).all() and physical(f32["intensity"][:, :199], wl.absorption).all()
    e = eacc(f32["intensity"][:, :199], f64["intensity"][:, :199])
    two = dataclasses.replace(sub, theta0=sub.theta0[[3, 9]])
    fine = dataclasses.replace(two, structures=[dataclasses.replace(two.structures[0], n_slices=2000)])
    disc = eacc(_run(two, "rk6", "fp64")["intensity"][:, :199], _run(fine, "rk6", "fp64")["intensity"][:, :199])
    _report(f"N=199 full size: FP32 vs FP64 stages {e:.3e}, discretisation error of the grid {disc:.3e}", e)
    assert 1e-11 < e <= BOUND
    assert e < 1e-2 * disc


def test_fp32_stages_refusals():
    from paper_2306_00271_amd import api
    from paper_2306_00271_amd._lib import RheedError
    import torch
    small = small_2d(n_beams=21, n_slices=4, thickness=0.4, n_layers=1, n_angles=2)
    wider = small_2d(n_beams=300, n_slices=4, thickness=0.4, n_layers=1, n_angles=2, m=7)
    with pytest.raises(RheedError, match="RK stepper"):
        api.plan_for(small, stepper="sp4", stage_precision="fp32")
    with pytest.raises(RheedError, match="N <= 256"):
        api.plan_for(wider, stepper="rk6", stage_precision="fp32")
    plan = api.plan_for(small, stepper="rk6", stage_precision="fp32")
    assert plan.info.fwd_workspace == 0
    dev = torch.device("cuda:0")
    U = plan.potential(api.atoms_for(small, dev))
    ws = torch.empty(1024, dtype=torch.uint8, device=dev)
    with pytest.raises(RheedError, match="FP64 stages"):
        plan.forward(U, api.angles_for(small, dev), workspace=ws)
