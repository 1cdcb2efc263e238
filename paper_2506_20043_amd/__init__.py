"""MI355X (gfx950) docking hot path of PocketVina (arXiv 2506.20043).

A thin Python binding over the C ABI of ``include/pvdock.h``
(``_lib/libpvdock.so``): argument marshalling only.  Every step of the hot
path -- grid maps, forward kinematics, score and gradient, BFGS, Monte Carlo
chains -- runs in the library's HIP kernels.  PyTorch provides device memory
and streams.  There is no CPU fallback: when the library is missing, the
first call raises.

    ctx = Context(0)
    grids = build_grids(ctx, rec_xyz, rec_type, boxes)
    ligs = Ligands(ctx, molecules)
    out = score_grad(ctx, grids, ligs, lig_of_pose, box_of_pose, dof)
    res = dock(ctx, grids, ligs, jobs, params)
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libpvdock.so")
_lib = None

PV_DOCK_TIMESTAMPS = 1
PV_DOCK_GRAPH = 2
PV_DOCK_LARGEST_FIRST = 4
PV_DOCK_BOX_ORDER = 8
PV_DOCK_NO_INTRA_BOUND = 16
PV_JOB_NONFINITE, PV_JOB_BUDGET, PV_JOB_OUTSIDE = 1, 2, 4
MAX_ATOMS, MAX_TORS = 128, 32


class PvError(RuntimeError):
    """A pvdock call returned an error status."""


class Box(C.Structure):
    _fields_ = [("center", C.c_float * 3), ("size", C.c_float * 3), ("spacing", C.c_float)]


class DockParams(C.Structure):
    _fields_ = [("chains", C.c_int32), ("steps", C.c_int32), ("bfgs_max_iter", C.c_int32),
                ("bfgs_m", C.c_int32), ("ls_max_trials", C.c_int32), ("refine_max_iter", C.c_int32),
                ("ls_rho", C.c_float), ("ls_sigma", C.c_float), ("eps_grad", C.c_float),
                ("eps_curv", C.c_float), ("temperature", C.c_float), ("mut_pos_amp", C.c_float),
                ("mut_rot_amp", C.c_float), ("flags", C.c_uint32), ("seed", C.c_uint64),
                ("workgroups", C.c_int32), ("consistency", C.c_int32), ("max_evals", C.c_int64)]


class Job(C.Structure):
    _fields_ = [("ligand", C.c_int32), ("box", C.c_int32)]


class DockOut(C.Structure):
    _fields_ = [("chain_best_e", C.c_void_p), ("chain_best_dof", C.c_void_p),
                ("chain_evals", C.c_void_p), ("chain_pairs", C.c_void_p),
                ("job_best_e", C.c_void_p), ("job_best_chain", C.c_void_p),
                ("job_evals", C.c_void_p), ("job_status", C.c_void_p),
                ("job_t_start", C.c_void_p), ("job_t_end", C.c_void_p), ("dof_stride", C.c_int32),
                ("chain_grads", C.c_void_p), ("chain_status", C.c_void_p), ("chain_bounded", C.c_void_p)]


class OutputParams(C.Structure):
    _fields_ = [("modes", C.c_int32), ("refine_max_iter", C.c_int32), ("rmsd_cut", C.c_float),
                ("affinity_w", C.c_float)]


class Schedule(C.Structure):
    _fields_ = [("variant", C.c_int32), ("workgroups", C.c_int32), ("lds_bytes", C.c_int32),
                ("per_cu", C.c_int32), ("n_jobs", C.c_int32)]


class TuneResult(C.Structure):
    _fields_ = [("group", C.c_int32), ("variant", C.c_int32), ("workgroups", C.c_int32), ("chosen", C.c_int32),
                ("cached", C.c_int32), ("ms", C.c_float), ("evals_per_s", C.c_double)]


class ModesOut(C.Structure):
    _fields_ = [("n_modes", C.c_void_p), ("mode_chain", C.c_void_p), ("mode_e", C.c_void_p),
                ("mode_affinity", C.c_void_p), ("mode_dof", C.c_void_p), ("dof_stride", C.c_int32)]


_vp = C.c_void_p
_ip = C.POINTER(C.c_int32)
_i32 = C.c_int32

# name: (restype, argtypes); every declared symbol is exported by the library
SIGNATURES = {
    "pv_last_error": (C.c_char_p, []),
    "pv_version": (C.c_int32, []),
    "pv_create": (C.c_int, [_i32, C.POINTER(_vp)]),
    "pv_destroy": (None, [_vp]),
    "pv_box_lattice": (C.c_int, [C.POINTER(Box), _ip, C.POINTER(C.c_float)]),
    "pv_build_grids": (C.c_int, [_vp, _i32, _vp, _vp, C.POINTER(Box), _i32, C.c_float, _vp, C.POINTER(_vp)]),
    "pv_grids_info": (C.c_int, [_vp, _i32, _ip, C.POINTER(C.c_float), C.POINTER(_vp)]),
    "pv_grids_copy": (C.c_int, [_vp, _i32, _vp, _vp]),
    "pv_grids_rebuild": (C.c_int, [_vp, _vp]),
    "pv_grids_free": (None, [_vp]),
    "pv_ligands_create": (C.c_int, [_vp, _i32, _vp, _vp, _vp, _vp, _vp, _vp, C.POINTER(_vp)]),
    "pv_ligands_info": (C.c_int, [_vp, _i32, _ip]),
    "pv_ligands_free": (None, [_vp]),
    "pv_ligand_describe": (C.c_int, [_i32, _vp, _vp, _i32, _vp, _vp, _ip, _ip, _i32, _ip]),
    "pv_score_grad": (C.c_int, [_vp, _vp, _vp, _i32, _vp, _vp, _vp, _i32, _vp, _vp, _vp, _vp, _vp, _vp, _i32, _vp]),
    "pv_score_grad_xyz": (C.c_int, [_vp, _vp, _vp, _i32, _vp, _vp, _vp, _i32, _vp, _vp, _vp, _vp, _vp]),
    "pv_dock_params_default": (None, [C.POINTER(DockParams)]),
    "pv_dock_plan": (C.c_int, [_vp, _vp, _vp, C.POINTER(Job), _i32, C.POINTER(DockParams), C.POINTER(_vp)]),
    "pv_dock_run": (C.c_int, [_vp, C.POINTER(DockOut), _vp]),
    "pv_dock_run_plain": (C.c_int, [_vp, C.POINTER(DockOut), _vp]),
    "pv_plan_free": (None, [_vp]),
    "pv_plan_groups": (C.c_int, [_vp, _ip]),
    "pv_plan_schedule": (C.c_int, [_vp, _i32, C.POINTER(Schedule)]),
    "pv_plan_set_schedule": (C.c_int, [_vp, _i32, _i32, _i32]),
    "pv_dock_autotune": (C.c_int, [_vp, _i32, _i32, _vp, C.POINTER(TuneResult), _i32, _ip]),
    "pv_dock": (C.c_int, [_vp, _vp, _vp, C.POINTER(Job), _i32, C.POINTER(DockParams), C.POINTER(DockOut), _vp]),
    "pv_dock_noalloc": (C.c_int, [_vp, _vp, _vp, C.POINTER(Job), _i32, C.POINTER(DockParams), C.POINTER(DockOut),
                                  _vp]),
    "pv_local_opt": (C.c_int, [_vp, _vp, _vp, _i32, _vp, _vp, _vp, _i32, C.POINTER(DockParams), _vp, _vp, _vp, _vp]),
    "pv_launch_info": (C.c_int, [_vp, _vp, _i32, C.c_int64, _ip, _ip, _ip]),
    "pv_sas_build": (C.c_int, [_vp, _i32, _vp, _vp, _i32, _vp, C.c_float, _vp, C.POINTER(C.c_void_p)]),
    "pv_sas_info": (C.c_int, [_vp, _ip]),
    "pv_sas_copy": (C.c_int, [_vp, _vp, _vp, _vp]),
    "pv_sas_features": (C.c_int, [_vp, _vp, _vp]),
    "pv_sas_free": (None, [_vp]),
    "pv_output_params_default": (None, [C.POINTER(OutputParams)]),
    "pv_output_stage": (C.c_int, [_vp, _vp, _vp, _i32, C.POINTER(OutputParams), C.POINTER(ModesOut), _vp]),
    "pv_fma_peak": (C.c_int, [_vp, _i32, _vp, _i32, _vp]),
}


def lib():
    """The loaded HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise PvError("native library %s is missing: build it with "
                          "`python -c 'import __graft_entry__ as g; g.build()'`" % LIB_PATH)
        # torch carries its own HIP runtime; loading it first makes the
        # library bind to that same runtime (one runtime, one set of streams)
        _torch()
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(rc, what):
    if rc != 0:
        msg = lib().pv_last_error()
        raise PvError("%s failed (status %d): %s" % (what, rc, msg.decode() if msg else ""))


def _torch():
    import torch
    return torch


def _stream(stream=None):
    """The HIP stream of a launch: torch's current stream, or `stream`, which
    then first waits for the current stream's work (the inputs were prepared
    there).  Results on `stream` are the caller's to wait for."""
    torch = _torch()
    cur = torch.cuda.current_stream()
    if stream is None:
        return C.c_void_p(cur.cuda_stream)
    if stream.cuda_stream != cur.cuda_stream:
        stream.wait_stream(cur)
    return C.c_void_p(stream.cuda_stream)


def _ptr(t):
    return C.c_void_p(0 if t is None else t.data_ptr())


def _used_on(stream, *tensors):
    """Tensors a launch on `stream` reads or writes.  torch's allocator ties a
    block to the stream current when it was allocated; on another stream the
    block could be handed out again while the launch still uses it, so it is
    recorded on that stream too."""
    if stream is None:
        return
    for t in tensors:
        if t is not None:
            t.record_stream(stream)


def _dev_tensor(a, dtype, device):
    torch = _torch()
    if isinstance(a, torch.Tensor):
        t = a.to(device=device, dtype=dtype)
    else:
        t = torch.as_tensor(np.asarray(a), device=device).to(dtype)
    return t.contiguous()


# ---------------------------------------------------------------- handles
class Context:
    def __init__(self, device: int = 0):
        h = C.c_void_p()
        _check(lib().pv_create(int(device), C.byref(h)), "pv_create")
        self.h = h
        self.device = int(device)

    @property
    def torch_device(self):
        return _torch().device("cuda", self.device)

    def close(self):
        if self.h:
            lib().pv_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def make_boxes(boxes):
    """[(center, size, spacing)] or objects with .center/.size/.spacing -> Box array."""
    arr = (Box * len(boxes))()
    for i, b in enumerate(boxes):
        c, s, h = (b.center, b.size, b.spacing) if hasattr(b, "center") else b
        s = np.broadcast_to(np.asarray(s, np.float32), (3,))
        for a in range(3):
            arr[i].center[a] = float(np.float32(c[a]))
            arr[i].size[a] = float(s[a])
        arr[i].spacing = float(h)
    return arr


def box_lattice(center, size, spacing):
    """Host-only: (dims, origin) of one box's lattice."""
    b = make_boxes([(center, size, spacing)])
    dims = (C.c_int32 * 3)()
    org = (C.c_float * 3)()
    _check(lib().pv_box_lattice(b, dims, org), "pv_box_lattice")
    return np.array(dims[:], np.int32), np.array(org[:], np.float32)


def describe_ligand(xyz, types, bonds, rotatable):
    """Host-only: (info, pairs [P,2] in input atom indices, frag [N]) of one ligand."""
    x = np.ascontiguousarray(xyz, np.float32).reshape(-1, 3)
    t = np.ascontiguousarray(types, np.uint8).reshape(-1)
    b = np.ascontiguousarray(bonds, np.int32).reshape(-1, 2)
    r = np.ascontiguousarray(rotatable, np.uint8).reshape(-1)
    n = len(t)
    cap = max(n * (n - 1) // 2, 1)
    info = (C.c_int32 * 8)()
    pairs = np.zeros((cap, 2), np.int32)
    frag = np.zeros(n, np.int32)
    _check(lib().pv_ligand_describe(n, x.ctypes.data_as(_vp), t.ctypes.data_as(_vp), len(b), b.ctypes.data_as(_vp),
                                    r.ctypes.data_as(_vp), info, pairs.ctypes.data_as(_ip), cap,
                                    frag.ctypes.data_as(_ip)), "pv_ligand_describe")
    info = list(info)
    return info, pairs[:info[3]].copy(), frag


class Grids:
    """Grid maps of every box, resident on the device (build_grids)."""

    def __init__(self, ctx: Context, handle, n_boxes):
        self.ctx, self.h, self.n_boxes = ctx, handle, n_boxes

    def info(self, box: int):
        dims = (C.c_int32 * 3)()
        org = (C.c_float * 3)()
        _check(lib().pv_grids_info(self.h, int(box), dims, org, None), "pv_grids_info")
        return np.array(dims[:], np.int32), np.array(org[:], np.float32)

    def maps(self, box: int, stream=None):
        """Copy of the 8 maps of one box as a device tensor [8, nz, ny, nx]."""
        torch = _torch()
        dims, _ = self.info(box)
        out = torch.empty((8, int(dims[2]), int(dims[1]), int(dims[0])), dtype=torch.float32,
                          device=self.ctx.torch_device)
        _check(lib().pv_grids_copy(self.h, int(box), _ptr(out), _stream(stream)), "pv_grids_copy")
        _used_on(stream, out)
        return out

    def rebuild(self, stream=None):
        """Recompute every map in place (same kernel, no allocation)."""
        _check(lib().pv_grids_rebuild(self.h, _stream(stream)), "pv_grids_rebuild")

    def close(self):
        if self.h:
            lib().pv_grids_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def build_grids(ctx: Context, rec_xyz, rec_type, boxes, penalty_slope: float = 10.0, stream=None) -> Grids:
    """Grid maps of every box over one receptor (the paper's grid cache)."""
    x = np.ascontiguousarray(rec_xyz, np.float32).reshape(-1, 3)
    t = np.ascontiguousarray(rec_type, np.uint8).reshape(-1)
    if len(x) != len(t):
        raise ValueError("rec_xyz and rec_type differ in length")
    bx = make_boxes(boxes)
    h = C.c_void_p()
    _check(lib().pv_build_grids(ctx.h, len(t), x.ctypes.data_as(_vp), t.ctypes.data_as(_vp), bx, len(bx),
                                float(penalty_slope), _stream(stream), C.byref(h)), "pv_build_grids")
    return Grids(ctx, h, len(bx))


class Ligands:
    """Packed torsion trees and intra pair lists of a set of ligands.

    molecules: objects with .xyz [N,3], .types [N], .bonds [B,2], .rotatable [B]
    """

    def __init__(self, ctx: Context, molecules):
        mols = list(molecules)
        na = np.array([len(m.types) for m in mols], np.int64)
        nb = np.array([len(m.bonds) for m in mols], np.int64)
        atom_off = np.concatenate([[0], np.cumsum(na)]).astype(np.int32)
        bond_off = np.concatenate([[0], np.cumsum(nb)]).astype(np.int32)
        xyz = np.ascontiguousarray(np.concatenate([np.asarray(m.xyz, np.float32).reshape(-1, 3) for m in mols]))
        ty = np.ascontiguousarray(np.concatenate([np.asarray(m.types).reshape(-1) for m in mols]).astype(np.uint8))
        bonds = np.ascontiguousarray(np.concatenate([np.asarray(m.bonds, np.int32).reshape(-1, 2) for m in mols]))
        rot = np.ascontiguousarray(np.concatenate([np.asarray(m.rotatable).reshape(-1) for m in mols]).astype(np.uint8))
        h = C.c_void_p()
        _check(lib().pv_ligands_create(ctx.h, len(mols), atom_off.ctypes.data_as(_vp), xyz.ctypes.data_as(_vp),
                                       ty.ctypes.data_as(_vp), bond_off.ctypes.data_as(_vp),
                                       bonds.ctypes.data_as(_vp), rot.ctypes.data_as(_vp), C.byref(h)),
               "pv_ligands_create")
        self.ctx, self.h, self.n = ctx, h, len(mols)
        self.infos = np.array([self.info(i) for i in range(self.n)], np.int32)
        self.max_atoms = int(self.infos[:, 0].max())
        self.max_tors = int(self.infos[:, 2].max())

    def info(self, i: int):
        v = (C.c_int32 * 8)()
        _check(lib().pv_ligands_info(self.h, int(i), v), "pv_ligands_info")
        return list(v)

    @property
    def dof_stride(self):
        return 7 + self.max_tors

    def close(self):
        if self.h:
            lib().pv_ligands_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- score + grad
def score_grad(ctx: Context, grids: Grids, ligs: Ligands, lig_of_pose, box_of_pose, dof, *, grad=True,
               parts=False, xyz=False, grad_energy=None, stream=None):
    """SF = e_inter + e_intra of B poses and its gradient (device tensors)."""
    torch = _torch()
    dev = ctx.torch_device
    dof = _dev_tensor(dof, torch.float32, dev)
    B, stride = dof.shape
    lp = _dev_tensor(lig_of_pose, torch.int32, dev)
    bp = _dev_tensor(box_of_pose, torch.int32, dev)
    ge = None if grad_energy is None else _dev_tensor(grad_energy, torch.float32, dev)
    out = {"energy": torch.empty(B, dtype=torch.float32, device=dev)}
    if parts:
        out["e_parts"] = torch.empty((B, 2), dtype=torch.float32, device=dev)
    if grad:
        out["grad_dof"] = torch.empty((B, stride), dtype=torch.float32, device=dev)
    ma = ligs.max_atoms
    if xyz:
        out["xyz"] = torch.empty((B, ma, 3), dtype=torch.float32, device=dev)
        out["grad_xyz"] = torch.empty((B, ma, 3), dtype=torch.float32, device=dev)
    _check(lib().pv_score_grad(ctx.h, grids.h, ligs.h, int(B), _ptr(lp), _ptr(bp), _ptr(dof), int(stride),
                               _ptr(ge), _ptr(out["energy"]), _ptr(out.get("e_parts")), _ptr(out.get("grad_dof")),
                               _ptr(out.get("xyz")), _ptr(out.get("grad_xyz")), int(ma), _stream(stream)),
           "pv_score_grad")
    _used_on(stream, dof, lp, bp, ge, *out.values())
    return out


def score_grad_xyz(ctx: Context, grids: Grids, ligs: Ligands, lig_of_pose, box_of_pose, xyz, *,
                   grad_energy=None, parts=False, stream=None):
    """The score on given coordinates xyz [B, stride, 3] and dSF/dxyz."""
    torch = _torch()
    dev = ctx.torch_device
    x = _dev_tensor(xyz, torch.float32, dev)
    B, stride, _ = x.shape
    lp = _dev_tensor(lig_of_pose, torch.int32, dev)
    bp = _dev_tensor(box_of_pose, torch.int32, dev)
    ge = None if grad_energy is None else _dev_tensor(grad_energy, torch.float32, dev)
    out = {"energy": torch.empty(B, dtype=torch.float32, device=dev),
           "grad_xyz": torch.zeros((B, stride, 3), dtype=torch.float32, device=dev)}
    if parts:
        out["e_parts"] = torch.empty((B, 2), dtype=torch.float32, device=dev)
    _check(lib().pv_score_grad_xyz(ctx.h, grids.h, ligs.h, int(B), _ptr(lp), _ptr(bp), _ptr(x), int(stride),
                                   _ptr(ge), _ptr(out["energy"]), _ptr(out.get("e_parts")), _ptr(out["grad_xyz"]),
                                   _stream(stream)), "pv_score_grad_xyz")
    _used_on(stream, x, lp, bp, ge, *out.values())
    return out


def _autograd_classes():
    torch = _torch()

    class ScoreGrad(torch.autograd.Function):
        """E(pose) with the hand-written gradient kernel as its backward.

        apply(dof [B, stride], handles) -> energy [B]; the gradient reaches
        dof as dE/d(t, raw q, psi)."""

        @staticmethod
        def forward(fctx, dof, handles):
            ctx, grids, ligs, lp, bp = handles
            fctx.save_for_backward(dof)
            fctx.handles = handles
            return score_grad(ctx, grids, ligs, lp, bp, dof.detach(), grad=False)["energy"]

        @staticmethod
        def backward(fctx, g):
            (dof,) = fctx.saved_tensors
            ctx, grids, ligs, lp, bp = fctx.handles
            r = score_grad(ctx, grids, ligs, lp, bp, dof.detach(), grad=True, grad_energy=g.contiguous())
            return r["grad_dof"], None

    class ScoreGradXYZ(torch.autograd.Function):
        """E(xyz) with dE/dxyz from the same kernel."""

        @staticmethod
        def forward(fctx, xyz, handles):
            ctx, grids, ligs, lp, bp = handles
            fctx.save_for_backward(xyz)
            fctx.handles = handles
            return score_grad_xyz(ctx, grids, ligs, lp, bp, xyz.detach())["energy"]

        @staticmethod
        def backward(fctx, g):
            (xyz,) = fctx.saved_tensors
            ctx, grids, ligs, lp, bp = fctx.handles
            r = score_grad_xyz(ctx, grids, ligs, lp, bp, xyz.detach(), grad_energy=g.contiguous())
            return r["grad_xyz"], None

    return ScoreGrad, ScoreGradXYZ


def __getattr__(name):
    if name in ("ScoreGrad", "ScoreGradXYZ"):
        sg, sx = _autograd_classes()
        globals()["ScoreGrad"], globals()["ScoreGradXYZ"] = sg, sx
        return globals()[name]
    raise AttributeError(name)


# ---------------------------------------------------------------- search
def dock_params(**kw) -> DockParams:
    p = DockParams()
    lib().pv_dock_params_default(C.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


class Plan:
    """A dock plan: the job table on the device plus checked parameters."""

    def __init__(self, ctx: Context, grids: Grids, ligs: Ligands, jobs, params: DockParams):
        jobs = np.ascontiguousarray(jobs, np.int32).reshape(-1, 2)
        arr = (Job * max(len(jobs), 1))()
        for i, (l, b) in enumerate(jobs):
            arr[i].ligand, arr[i].box = int(l), int(b)
        h = C.c_void_p()
        _check(lib().pv_dock_plan(ctx.h, grids.h, ligs.h, arr, len(jobs), C.byref(params), C.byref(h)),
               "pv_dock_plan")
        self.ctx, self.grids, self.ligs, self.h = ctx, grids, ligs, h
        self.n_jobs, self.params = len(jobs), params
        self._out = None

    def outputs(self):
        """Device tensors for every output of the plan (allocated once)."""
        if self._out is None:
            torch = _torch()
            dev = self.ctx.torch_device
            nj, ch = self.n_jobs, self.params.chains
            stride = self.ligs.dof_stride
            self._out = dict(
                chain_best_e=torch.empty(nj * ch, dtype=torch.float32, device=dev),
                chain_best_dof=torch.zeros((nj * ch, stride), dtype=torch.float32, device=dev),
                chain_evals=torch.empty(nj * ch, dtype=torch.int64, device=dev),
                chain_pairs=torch.empty(nj * ch, dtype=torch.int64, device=dev),
                chain_grads=torch.empty(nj * ch, dtype=torch.int64, device=dev),
                chain_status=torch.empty(nj * ch, dtype=torch.int32, device=dev),
                chain_bounded=torch.empty(nj * ch, dtype=torch.int64, device=dev),
                job_best_e=torch.empty(nj, dtype=torch.float32, device=dev),
                job_best_chain=torch.empty(nj, dtype=torch.int32, device=dev),
                job_evals=torch.empty(nj, dtype=torch.int64, device=dev),
                job_status=torch.empty(nj, dtype=torch.int32, device=dev),
                job_t_start=torch.empty(nj, dtype=torch.int64, device=dev),
                job_t_end=torch.empty(nj, dtype=torch.int64, device=dev),
            )
            o = DockOut()
            for k, v in self._out.items():
                setattr(o, k, v.data_ptr())
            o.dof_stride = stride
            self._c_out = o
        return self._out

    def run(self, plain: bool = False, stream=None):
        self.outputs()
        fn = lib().pv_dock_run_plain if plain else lib().pv_dock_run
        _check(fn(self.h, C.byref(self._c_out), _stream(stream)), "pv_dock_run")
        _used_on(stream, *self._out.values())
        return self._out

    def groups(self) -> int:
        """Size classes of the plan's jobs (each runs one persistent launch)."""
        n = C.c_int32()
        _check(lib().pv_plan_groups(self.h, C.byref(n)), "pv_plan_groups")
        return n.value

    def schedule(self, group: int = 0) -> dict:
        """Variant, width, LDS bytes, workgroups per CU and jobs of a size class."""
        sc = Schedule()
        _check(lib().pv_plan_schedule(self.h, group, C.byref(sc)), "pv_plan_schedule")
        return {k: getattr(sc, k) for k, _ in Schedule._fields_}

    def set_schedule(self, group: int, variant: int, workgroups: int = 0):
        _check(lib().pv_plan_set_schedule(self.h, group, variant, workgroups), "pv_plan_set_schedule")

    def autotune(self, steps: int = 20, repeats: int = 2, stream=None) -> list:
        """Times the candidate schedules of every size class on a short run
        and keeps the fastest; returns one dict per candidate."""
        cap = 16 * max(self.groups(), 1)
        res = (TuneResult * cap)()
        n = C.c_int32()
        _check(lib().pv_dock_autotune(self.h, steps, repeats, _stream(stream), res, cap, C.byref(n)),
               "pv_dock_autotune")
        return [{k: getattr(res[i], k) for k, _ in TuneResult._fields_} for i in range(n.value)]

    def close(self):
        if self.h:
            lib().pv_plan_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def dock(ctx: Context, grids: Grids, ligs: Ligands, jobs, params: DockParams | None = None, *, plain=False,
         stream=None):
    """Monte Carlo + BFGS docking of every (ligand, box) job; returns device tensors."""
    plan = Plan(ctx, grids, ligs, jobs, params if params is not None else dock_params())
    out = plan.run(plain=plain, stream=stream)
    _torch().cuda.synchronize(ctx.device)
    plan.close()
    return out


NOALLOC_MAX_JOBS, NOALLOC_MAX_CHAINS = 65536, 1 << 20


def _job_array(jobs):
    jobs = np.ascontiguousarray(jobs, np.int32).reshape(-1, 2)
    arr = (Job * max(len(jobs), 1))()
    for i, (l, b) in enumerate(jobs):
        arr[i].ligand, arr[i].box = int(l), int(b)
    return arr, len(jobs)


def _dock_outputs(ctx, ligs, n_jobs, chains, chain_outputs=True):
    """Device tensors for a dock's outputs and the pv_dock_out that names
    them; without chain_outputs the per-chain arrays are left out (NULL)."""
    torch = _torch()
    dev = ctx.torch_device
    nc = n_jobs * chains
    out = dict(job_best_e=torch.empty(n_jobs, dtype=torch.float32, device=dev),
               job_best_chain=torch.empty(n_jobs, dtype=torch.int32, device=dev),
               job_evals=torch.empty(n_jobs, dtype=torch.int64, device=dev),
               job_status=torch.empty(n_jobs, dtype=torch.int32, device=dev))
    if chain_outputs:
        out.update(chain_best_e=torch.empty(nc, dtype=torch.float32, device=dev),
                   chain_best_dof=torch.zeros((nc, ligs.dof_stride), dtype=torch.float32, device=dev),
                   chain_evals=torch.empty(nc, dtype=torch.int64, device=dev),
                   chain_pairs=torch.empty(nc, dtype=torch.int64, device=dev),
                   chain_grads=torch.empty(nc, dtype=torch.int64, device=dev),
                   chain_status=torch.empty(nc, dtype=torch.int32, device=dev),
                   chain_bounded=torch.empty(nc, dtype=torch.int64, device=dev))
    o = DockOut()
    for k, v in out.items():
        setattr(o, k, v.data_ptr())
    o.dof_stride = ligs.dof_stride
    return out, o


def dock_call(ctx: Context, grids: Grids, ligs: Ligands, jobs, params: DockParams, stream=None):
    """pv_dock: plan, batched run and release in one call (returns after the
    dock has completed); returns device tensors."""
    arr, n = _job_array(jobs)
    out, o = _dock_outputs(ctx, ligs, n, params.chains)
    _check(lib().pv_dock(ctx.h, grids.h, ligs.h, arr, n, C.byref(params), C.byref(o), _stream(stream)), "pv_dock")
    return out


def dock_noalloc(ctx: Context, grids: Grids, ligs: Ligands, jobs, params: DockParams, chain_outputs=True,
                 stream=None):
    """pv_dock_noalloc: the same dock with no device allocation by the
    library (its scratch is a static device array); returns the device
    tensors allocated here for its outputs.  Without chain_outputs only the
    per-job outputs are asked for."""
    arr, n = _job_array(jobs)
    out, o = _dock_outputs(ctx, ligs, n, params.chains, chain_outputs)
    _check(lib().pv_dock_noalloc(ctx.h, grids.h, ligs.h, arr, n, C.byref(params), C.byref(o), _stream(stream)),
           "pv_dock_noalloc")
    return out


def local_opt(ctx: Context, grids: Grids, ligs: Ligands, lig_of_pose, box_of_pose, dof,
              params: DockParams | None = None, stream=None):
    """One BFGS run from each pose; returns (dof_out, energy, n_evals)."""
    torch = _torch()
    dev = ctx.torch_device
    p = params if params is not None else dock_params()
    dof = _dev_tensor(dof, torch.float32, dev)
    B, stride = dof.shape
    lp = _dev_tensor(lig_of_pose, torch.int32, dev)
    bp = _dev_tensor(box_of_pose, torch.int32, dev)
    out = torch.empty_like(dof)
    e = torch.empty(B, dtype=torch.float32, device=dev)
    ne = torch.empty(B, dtype=torch.int64, device=dev)
    _check(lib().pv_local_opt(ctx.h, grids.h, ligs.h, int(B), _ptr(lp), _ptr(bp), _ptr(dof), int(stride),
                              C.byref(p), _ptr(out), _ptr(e), _ptr(ne), _stream(stream)), "pv_local_opt")
    _used_on(stream, dof, lp, bp, out, e, ne)
    return out, e, ne


def fma_peak(ctx: Context, iters: int, out, stream=None) -> float:
    """Launches the FP32 multiply-add throughput kernel over out (a device
    float32 tensor whose length is a multiple of 256); returns the launch's
    floating-point operation count."""
    n = int(out.numel())
    _check(lib().pv_fma_peak(ctx.h, int(iters), _ptr(out), n, _stream(stream)), "pv_fma_peak")
    _used_on(stream, out)
    return 2.0 * 16 * int(iters) * n


KIND_DOCK, KIND_SCORE, KIND_LOCAL_OPT = 0, 1, 2
VARIANT_SLOTS, VARIANT_GATHER, VARIANT_GATHER2 = 0, 1, 2


def launch_info(ctx: Context, ligs: Ligands, kind: int, items: int):
    """(variant, LDS bytes, workgroups per CU) of a launch of `kind` over
    `items` waves on these ligands (host-side, no device work)."""
    v, lds, occ = C.c_int32(), C.c_int32(), C.c_int32()
    _check(lib().pv_launch_info(ctx.h, ligs.h, int(kind), int(items), C.byref(v), C.byref(lds), C.byref(occ)),
           "pv_launch_info")
    return v.value, lds.value, occ.value


def output_params(**kw) -> OutputParams:
    p = OutputParams()
    lib().pv_output_params_default(C.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def output_stage(plan: Plan, chain_best_e, chain_best_dof, params: OutputParams | None = None, stream=None):
    """Cluster, refine, rescore, filter and sort every job's chain bests
    (device tensors [n_jobs*chains] and [n_jobs*chains, stride]); returns
    device tensors n_modes [n_jobs], mode_chain / mode_e / mode_affinity
    [n_jobs, modes] and mode_dof [n_jobs, modes, stride]."""
    torch = _torch()
    dev = plan.ctx.torch_device
    p = params if params is not None else output_params()
    e = _dev_tensor(chain_best_e, torch.float32, dev)
    d = _dev_tensor(chain_best_dof, torch.float32, dev)
    stride = int(d.shape[-1])
    nj, m = plan.n_jobs, int(p.modes)
    out = {"n_modes": torch.empty(nj, dtype=torch.int32, device=dev),
           "mode_chain": torch.empty((nj, m), dtype=torch.int32, device=dev),
           "mode_e": torch.empty((nj, m), dtype=torch.float32, device=dev),
           "mode_affinity": torch.empty((nj, m), dtype=torch.float32, device=dev),
           "mode_dof": torch.empty((nj, m, stride), dtype=torch.float32, device=dev)}
    o = ModesOut(out["n_modes"].data_ptr(), out["mode_chain"].data_ptr(), out["mode_e"].data_ptr(),
                 out["mode_affinity"].data_ptr(), out["mode_dof"].data_ptr(), stride)
    _check(lib().pv_output_stage(plan.h, _ptr(e), _ptr(d), stride, C.byref(p), C.byref(o), _stream(stream)),
           "pv_output_stage")
    _used_on(stream, e, d, *out.values())
    return out


class SurfacePoints:
    """Solvent-accessible surface points of a receptor and their Eq.
    prank_eq_1 features (pv_sas_build / pv_sas_features)."""

    def __init__(self, ctx: Context, rec_xyz, rec_type, dirs, probe: float = 1.6, stream=None):
        x = np.ascontiguousarray(rec_xyz, np.float32).reshape(-1, 3)
        t = np.ascontiguousarray(rec_type, np.uint8).reshape(-1)
        d = np.ascontiguousarray(dirs, np.float32).reshape(-1, 3)
        h = C.c_void_p()
        _check(lib().pv_sas_build(ctx.h, len(t), x.ctypes.data_as(_vp), t.ctypes.data_as(_vp), len(d),
                                  d.ctypes.data_as(_vp), float(probe), _stream(stream), C.byref(h)), "pv_sas_build")
        self.ctx, self.h = ctx, h
        n = C.c_int32()
        _check(lib().pv_sas_info(h, C.byref(n)), "pv_sas_info")
        self.n_points = n.value

    def points(self, stream=None):
        torch = _torch()
        dev = self.ctx.torch_device
        xyz = torch.empty((self.n_points, 3), dtype=torch.float32, device=dev)
        atom = torch.empty(self.n_points, dtype=torch.int32, device=dev)
        _check(lib().pv_sas_copy(self.h, _ptr(xyz), _ptr(atom), _stream(stream)), "pv_sas_copy")
        _used_on(stream, xyz, atom)
        return xyz, atom

    def features(self, out=None, stream=None):
        torch = _torch()
        f = out if out is not None else torch.empty((self.n_points, 12), dtype=torch.float32,
                                                    device=self.ctx.torch_device)
        _check(lib().pv_sas_features(self.h, _ptr(f), _stream(stream)), "pv_sas_features")
        _used_on(stream, f)
        return f

    def close(self):
        if self.h:
            lib().pv_sas_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
