"""Thin Python binding over librheed: marshals torch tensors to the C ABI.

Every computation runs in the library's HIP kernels; this module only
allocates output tensors, passes pointers and the current HIP stream, and
checks status codes.  Device tensors must live on the current HIP device.
"""
from __future__ import annotations

import atexit
import ctypes as C
import sys
import weakref
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib

STEPPERS = {"rk4": _lib.RHEED_RK4, "rk6": _lib.RHEED_RK6, "sp4": _lib.RHEED_SP4, "sp6": _lib.RHEED_SP6,
            "sp4a": _lib.RHEED_SP4_ABA, "sp6a": _lib.RHEED_SP6_ABA}
CONVENTIONS = {"flux": _lib.RHEED_INTENSITY_FLUX, "paper": _lib.RHEED_INTENSITY_PAPER}
LAYOUTS = {"auto": _lib.RHEED_LAYOUT_AUTO, "whole": _lib.RHEED_LAYOUT_WHOLE, "split": _lib.RHEED_LAYOUT_SPLIT}
PRECISIONS = {"fp64": _lib.RHEED_STAGES_FP64, "fp32": _lib.RHEED_STAGES_FP32}


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: Optional[torch.Tensor]):
    return C.c_void_p(0) if t is None else C.c_void_p(t.data_ptr())


def _dev(t: torch.Tensor, dtype, name):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def beam_constants(energy_eV: float):
    """(gamma in 1/A, kappa in 1/(A^2 V)) from the library."""
    g, k = C.c_double(), C.c_double()
    _lib.check(_lib.lib().rheed_beam_constants(float(energy_eV), C.byref(g), C.byref(k)), "beam_constants")
    return g.value, k.value


# Plans still open; closed by an exit hook while the HIP runtime is alive, so
# that no plan's device memory is freed from a finalizer during interpreter
# teardown.
_LIVE_PLANS: "weakref.WeakSet[Plan]" = weakref.WeakSet()


@atexit.register
def _close_live_plans():
    for plan in list(_LIVE_PLANS):
        plan.close()


class Plan:
    """A set of structures, each with a number of angles (pairs are numbered
    structure-major).  ``structures`` are objects with the attributes
    ``beams`` [N,2] int, ``recip`` [2,2], ``n_slices``, ``thickness``,
    ``atoms`` [n_atoms,3], ``cell_area``, ``scat_a`` [4], ``scat_b`` [4].

    ``close()`` (or leaving a ``with`` block) releases the plan's device
    memory; a plan still open at interpreter exit is closed by an exit hook."""

    def __init__(self, structures: Sequence, angles_per_struct: Sequence[int], *, energy_eV: float,
                 charge: float, absorption: float, mean_inner_potential: float = 15.0, stepper: str = "rk6",
                 threshold: float = 1000.0, checkpoint_every: int = 1, convention: str = "flux",
                 layout: str = "auto", stage_precision: str = "fp64"):
        L = _lib.lib()
        self.gamma, self.kappa = beam_constants(energy_eV)
        self.stepper = stepper
        n = len(structures)
        arr = (_lib.Structure * n)()
        self._keep = []
        for i, s in enumerate(structures):
            beams = np.ascontiguousarray(np.asarray(s.beams, dtype=np.int32))
            self._keep.append(beams)
            st = arr[i]
            st.n_beams = beams.shape[0]
            st.beam_hk = beams.ctypes.data_as(C.POINTER(C.c_int32))
            rec = np.asarray(s.recip, dtype=np.float64)
            st.recip = (C.c_double * 4)(rec[0, 0], rec[0, 1], rec[1, 0], rec[1, 1])
            st.n_slices = int(s.n_slices)
            st.thickness = float(s.thickness)
            st.wavenumber = self.gamma
            st.n_atoms = int(np.asarray(s.atoms).shape[0])
            st.cell_area = float(s.cell_area)
            st.scat_a = (C.c_double * 4)(*[float(x) for x in s.scat_a])
            st.scat_b = (C.c_double * 4)(*[float(x) for x in s.scat_b])
            st.kappa = self.kappa
            st.charge = float(charge)
            st.absorption = float(absorption)
            st.mean_inner_potential = float(mean_inner_potential)
        aps = (C.c_int32 * n)(*[int(a) for a in angles_per_struct])
        opts = _lib.Opts(STEPPERS[stepper], float(threshold), int(checkpoint_every), CONVENTIONS[convention],
                         LAYOUTS[layout], PRECISIONS[stage_precision])
        h = C.c_void_p()
        _lib.check(L.rheed_plan_create(C.byref(h), C.byref(opts), n, arr, aps), "plan_create")
        self._h = h
        _LIVE_PLANS.add(self)
        info = _lib.PlanInfo()
        _lib.check(L.rheed_plan_get_info(h, C.byref(info)), "plan_get_info")
        self.info = info
        self.n_pairs = info.n_pairs
        self.max_beams = info.max_beams
        self.split = bool(info.split)
        offs = (C.c_int64 * (n + 1))()
        _lib.check(L.rheed_plan_table_offsets(h, offs), "plan_table_offsets")
        self.table_offsets = np.array(offs[:], dtype=np.int64)
        aoffs = (C.c_int64 * (n + 1))()
        _lib.check(L.rheed_plan_atom_offsets(h, aoffs), "plan_atom_offsets")
        self.atom_offsets = np.array(aoffs[:], dtype=np.int64)

    def close(self) -> None:
        """Destroys the plan (rheed_plan_destroy); later calls on it raise."""
        h = getattr(self, "_h", None)
        self._h = None
        _LIVE_PLANS.discard(self)
        if h is not None and h.value:
            _lib.lib().rheed_plan_destroy(h)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self, _finalizing=sys.is_finalizing):
        # no HIP call once the interpreter is shutting down: the exit hook
        # has closed every plan by then (the check is bound at definition,
        # since module globals may already be gone at that point)
        if not _finalizing():
            self.close()

    def force_sync_failure(self, half: int) -> None:
        """rheed_plan_force_sync_failure: the failure path of the split layout and
        of the group launches, for tests."""
        _lib.check(_lib.lib().rheed_plan_force_sync_failure(self._handle(), int(half)), "plan_force_sync_failure")

    def _handle(self):
        if self._h is None:
            raise ValueError("the plan is closed")
        return self._h

    # ------------------------------------------------------------------
    def potential(self, atoms: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        _dev(atoms, torch.float64, "atoms")
        if out is None:
            out = torch.empty(int(self.info.table_elems), dtype=torch.complex128, device=atoms.device)
        _lib.check(_lib.lib().rheed_potential(self._handle(), _ptr(atoms), _ptr(out), _stream()), "potential")
        return out

    def potential_backward(self, atoms: torch.Tensor, dL_dU: torch.Tensor) -> torch.Tensor:
        _dev(atoms, torch.float64, "atoms")
        _dev(dL_dU, torch.complex128, "dL_dU")
        out = torch.empty_like(atoms)
        _lib.check(_lib.lib().rheed_potential_backward(self._handle(), _ptr(atoms), _ptr(dL_dU), _ptr(out), _stream()),
                   "potential_backward")
        return out

    def workspace(self, device) -> torch.Tensor:
        nbytes = int(self.info.fwd_workspace + self.info.bwd_workspace)
        return torch.empty(max(nbytes, 1), dtype=torch.uint8, device=device)

    def forward(self, U: torch.Tensor, angles: torch.Tensor, *, want_rho: bool = False,
                workspace: Optional[torch.Tensor] = None, want_nrhst: bool = False,
                y_bottom: Optional[torch.Tensor] = None):
        """rheed_forward, or rheed_forward_bulk when ``y_bottom`` (complex
        [n_pairs, max_beams, max_beams]: the state [I; Y] of a bulk below) is given."""
        _dev(U, torch.complex128, "U")
        _dev(angles, torch.float64, "angles")
        if angles.shape != (self.n_pairs, 2):
            raise ValueError(f"angles must be [{self.n_pairs}, 2]")
        dev = U.device
        inten = torch.empty((self.n_pairs, self.max_beams), dtype=torch.float64, device=dev)
        rho = torch.empty((self.n_pairs, self.max_beams), dtype=torch.complex128, device=dev) if want_rho else None
        status = torch.empty(self.n_pairs, dtype=torch.int32, device=dev)
        nrhst = torch.empty(self.n_pairs, dtype=torch.int32, device=dev) if want_nrhst else None
        ws_bytes = 0 if workspace is None else workspace.numel()
        if y_bottom is None:
            _lib.check(_lib.lib().rheed_forward(self._handle(), _ptr(U), _ptr(angles), _ptr(inten), _ptr(rho),
                                                _ptr(status), _ptr(nrhst), _ptr(workspace), ws_bytes, _stream()),
                       "forward")
        else:
            _dev(y_bottom, torch.complex128, "y_bottom")
            if y_bottom.shape != (self.n_pairs, self.max_beams, self.max_beams):
                raise ValueError(f"y_bottom must be [{self.n_pairs}, {self.max_beams}, {self.max_beams}]")
            _lib.check(_lib.lib().rheed_forward_bulk(self._handle(), _ptr(U), _ptr(angles), _ptr(y_bottom), _ptr(inten),
                                                     _ptr(rho), _ptr(status), _ptr(nrhst), _ptr(workspace),
                                                     ws_bytes, _stream()), "forward_bulk")
        return {"intensity": inten, "rho": rho, "status": status, "n_rhst": nrhst}

    def bulk_reflection(self, U: torch.Tensor, angles: torch.Tensor, *, tol: float = 1e-6,
                        max_layers: int = 2000):
        """The bulk whose unit layers this plan's structures are, stacked from
        the vacuum until R converges (rheed_bulk_reflection): {"y": state
        [n_pairs, M, M] for ``forward(y_bottom=...)``, "r": reflection
        matrices, "layers": [n_pairs] int32, "status": [n_pairs] int32}."""
        _dev(U, torch.complex128, "U")
        _dev(angles, torch.float64, "angles")
        dev = U.device
        M = self.max_beams
        y = torch.empty((self.n_pairs, M, M), dtype=torch.complex128, device=dev)
        r = torch.empty_like(y)
        layers = torch.empty(self.n_pairs, dtype=torch.int32, device=dev)
        status = torch.empty(self.n_pairs, dtype=torch.int32, device=dev)
        nbytes = int(self.info.fwd_workspace + self.info.bulk_workspace)
        ws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=dev)
        _lib.check(_lib.lib().rheed_bulk_reflection(self._handle(), _ptr(U), _ptr(angles), float(tol), int(max_layers),
                                                    _ptr(y), _ptr(r), _ptr(layers), _ptr(status), _ptr(ws),
                                                    ws.numel(), _stream()), "bulk_reflection")
        return {"y": y, "r": r, "layers": layers, "status": status}

    def autotune(self, U: torch.Tensor, angles: torch.Tensor, reps: int = 3) -> dict:
        """Times the launch configurations of forward on these inputs and keeps
        the fastest for later calls (rheed_autotune); returns the timings."""
        _dev(U, torch.complex128, "U")
        _dev(angles, torch.float64, "angles")
        dev = U.device
        inten = torch.empty((self.n_pairs, self.max_beams), dtype=torch.float64, device=dev)
        status = torch.empty(self.n_pairs, dtype=torch.int32, device=dev)
        rep = _lib.TuneReport()
        _lib.check(_lib.lib().rheed_autotune(self._handle(), _ptr(U), _ptr(angles), _ptr(inten), _ptr(status), int(reps),
                                             _stream(), C.byref(rep)), "autotune")
        info = _lib.PlanInfo()
        _lib.check(_lib.lib().rheed_plan_get_info(self._handle(), C.byref(info)), "plan_get_info")
        self.info = info
        self.split = bool(info.split)
        n = rep.n_candidates
        return {"chosen": rep.chosen,
                "candidates": [{"split": bool(rep.split[c]), "large_cost_order": bool(rep.large_cost_order[c]),
                                "queue": bool(rep.queue[c]), "ms": float(rep.ms[c])} for c in range(n)]}

    def backward(self, U: torch.Tensor, angles: torch.Tensor, dL_dI: torch.Tensor,
                 workspace: torch.Tensor) -> torch.Tensor:
        _dev(U, torch.complex128, "U")
        _dev(angles, torch.float64, "angles")
        _dev(dL_dI, torch.float64, "dL_dI")
        dU = torch.empty_like(U)
        _lib.check(_lib.lib().rheed_backward(self._handle(), _ptr(U), _ptr(angles), _ptr(dL_dI), _ptr(dU),
                                             _ptr(workspace), workspace.numel(), _stream()), "backward")
        return dU


def rfactor(intensity: torch.Tensor, target: torch.Tensor):
    """loss = sum_p (I[p,0] - target[p])^2 (device scalar) and dL/dI."""
    _dev(intensity, torch.float64, "intensity")
    _dev(target, torch.float64, "target")
    P, ld = intensity.shape
    loss = torch.empty((), dtype=torch.float64, device=intensity.device)
    dI = torch.empty_like(intensity)
    _lib.check(_lib.lib().rheed_rfactor(P, ld, _ptr(intensity), _ptr(target), _ptr(loss), _ptr(dI), _stream()),
               "rfactor")
    return loss, dI


class _Intensity(torch.autograd.Function):
    """Intensities of every pair as a differentiable function of the atom
    coordinates: tables (rheed_potential) -> propagation (rheed_forward) on
    the way forward; rheed_backward -> rheed_potential_backward on the way
    back.  The forward keeps the workspace only when a gradient is needed.
    With ``y_bottom`` (a bulk's state below the slab) the bulk is held fixed."""

    @staticmethod
    def forward(ctx, atoms, plan, angles, y_bottom):
        U = plan.potential(atoms)
        ws = plan.workspace(atoms.device) if ctx.needs_input_grad[0] else None
        out = plan.forward(U, angles, workspace=ws, y_bottom=y_bottom)
        ctx.plan = plan
        if ws is not None:
            ctx.save_for_backward(atoms, U, angles, ws)
        ctx.mark_non_differentiable(out["status"])
        return out["intensity"], out["status"]

    @staticmethod
    def backward(ctx, dI, _dstatus):
        atoms, U, angles, ws = ctx.saved_tensors
        dU = ctx.plan.backward(U, angles, dI.contiguous(), ws)
        return ctx.plan.potential_backward(atoms, dU), None, None, None


def intensity(plan: Plan, atoms: torch.Tensor, angles: torch.Tensor, y_bottom: Optional[torch.Tensor] = None):
    """(intensity [n_pairs][max_beams], pair status [n_pairs]) with autograd
    support: a loss built from the intensities back-propagates to `atoms`.
    ``y_bottom``: the state of a bulk below the slab (``Plan.bulk_reflection``),
    held fixed; None for the vacuum."""
    return _Intensity.apply(atoms, plan, angles, y_bottom)


def mfma_f64_peak(blocks: int = 1024, iters: int = 4000) -> float:
    """Measured FP64 matrix-core TFLOP/s of the current device."""
    out = C.c_double()
    _lib.check(_lib.lib().rheed_mfma_f64_peak(int(blocks), int(iters), C.byref(out)), "mfma_f64_peak")
    return out.value


# ----------------------------------------------------------------- helpers
def plan_for(workload, stepper: Optional[str] = None, **kw) -> Plan:
    """Plan over every structure of a workload, each with all its angles."""
    return Plan(workload.structures, [len(workload.theta0)] * len(workload.structures),
                energy_eV=workload.energy_eV, charge=workload.charge, absorption=workload.absorption,
                mean_inner_potential=workload.mean_inner_potential, stepper=stepper or workload.stepper, **kw)


def angles_for(workload, device) -> torch.Tensor:
    th = np.asarray(workload.theta0, dtype=np.float64)
    a = np.stack([th, np.full_like(th, workload.theta1)], axis=1)
    a = np.tile(a, (len(workload.structures), 1))
    return torch.from_numpy(a).to(device)


def atoms_for(workload, device, structures=None) -> torch.Tensor:
    structs = workload.structures if structures is None else structures
    return torch.from_numpy(np.concatenate([np.asarray(s.atoms, dtype=np.float64) for s in structs])).to(device)
