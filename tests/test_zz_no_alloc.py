"""rheed_potential_backward_noalloc (the entry point for callers that cannot
allocate) against rheed_potential_backward, both called through the C ABI:
the same kernels in the same order, so the atom gradients must agree bit for
bit, on two calls in a row, the second on a plan with fewer atoms."""
import ctypes as C

import numpy as np
import pytest

from synth import small_2d

pytestmark = pytest.mark.gpu


def _both(wl, seed):
    import torch
    from paper_2306_00271_amd import _lib, api
    dev = torch.device("cuda:0")
    plan = api.plan_for(wl, stepper="rk4")
    atoms = api.atoms_for(wl, dev)
    n_tab = int(plan.info.table_elems)
    rng = np.random.default_rng(seed)
    dU = torch.from_numpy(rng.normal(size=n_tab) + 1j * rng.normal(size=n_tab)).to(dev)
    ref = torch.full_like(atoms, float("nan"))
    got = torch.full_like(atoms, float("nan"))
    lib = _lib.lib()
    st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    _lib.check(lib.rheed_potential_backward(plan._handle(), C.c_void_p(atoms.data_ptr()),
                                            C.c_void_p(dU.data_ptr()), C.c_void_p(ref.data_ptr()), st),
               "potential_backward")
    _lib.check(lib.rheed_potential_backward_noalloc(plan._handle(), C.c_void_p(atoms.data_ptr()),
                                                    C.c_void_p(dU.data_ptr()), C.c_void_p(got.data_ptr()), st),
               "potential_backward_noalloc")
    torch.cuda.synchronize()
    plan.close()
    return ref.cpu().numpy(), got.cpu().numpy()


def test_noalloc_matches_plan_buffers_on_two_calls():
    big = small_2d(n_beams=21, n_slices=20, thickness=8.0, n_layers=3, n_angles=2, n_structures=3, seed=5)
    small = small_2d(n_beams=13, n_slices=10, thickness=4.0, n_layers=1, n_angles=2, seed=6)
    for wl, seed in ((big, 1), (small, 2)):
        ref, got = _both(wl, seed)
        print(f"noalloc: {ref.shape[0]} atoms, max |grad| {np.max(np.abs(ref)):.3e}", flush=True)
        assert np.all(np.isfinite(ref)) and np.max(np.abs(ref)) > 0.0
        assert np.array_equal(ref, got)


def test_noalloc_refuses_more_atoms_than_the_array_holds():
    import torch
    from paper_2306_00271_amd import _lib, api
    wl = small_2d(n_beams=5, n_slices=2, thickness=1.0, n_layers=1, n_angles=1, m=1,
                  n_structures=_lib.RHEED_NOALLOC_MAX_ATOMS + 1)
    dev = torch.device("cuda:0")
    plan = api.plan_for(wl, stepper="rk4")
    assert plan.info.n_atoms_total == _lib.RHEED_NOALLOC_MAX_ATOMS + 1
    atoms = api.atoms_for(wl, dev)
    dU = torch.zeros(int(plan.info.table_elems), dtype=torch.complex128, device=dev)
    out = torch.empty_like(atoms)
    code = _lib.lib().rheed_potential_backward_noalloc(plan._handle(), C.c_void_p(atoms.data_ptr()),
                                                       C.c_void_p(dU.data_ptr()), C.c_void_p(out.data_ptr()),
                                                       C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert code == _lib.RHEED_E_UNSUPPORTED
    assert b"4096" in _lib.lib().rheed_last_error()
    plan.close()
