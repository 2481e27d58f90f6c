"""Python binding of the MI355X Newton linearisation and solve library.

Argument marshalling only: every step of the path runs in the HIP kernels of
``libopm_gpu.so`` (C ABI declared in ``include/opm_gpu.h``).  torch provides
device memory and the stream; nothing here computes any part of the method.
The library must be built (``__graft_entry__.build()``); importing this
module on a machine without the built library or without a gfx950 GPU raises
instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np
import torch

from . import cases as _cases

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libopm_gpu.so")

OK, EINVAL, ESINGULAR, ENOTCONV, EBREAKDOWN, ENONFINITE, EHIP = 0, -1, -2, -3, -4, -5, -6
PREC_FP64, PREC_MIXED = 0, 1
KRYLOV_BICGSTAB, KRYLOV_GMRES = 0, 1
GMRES_MAX_RESTART = 32
PRECOND_ILU0, PRECOND_CPR = 0, 1

_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_ip = ctypes.POINTER(ctypes.c_int32)
_dp = ctypes.POINTER(ctypes.c_double)


class Fluid(ctypes.Structure):
    _fields_ = [("rho_s", ctypes.c_double * 3), ("c", ctypes.c_double * 3),
                ("p_ref", ctypes.c_double), ("mu", ctypes.c_double * 3),
                ("swc", ctypes.c_double), ("n_corey", ctypes.c_double), ("g", ctypes.c_double),
                ("rs_c", ctypes.c_double), ("bo_r", ctypes.c_double), ("muo_r", ctypes.c_double),
                ("eps_switch", ctypes.c_double), ("live", _i32), ("pad", _i32),
                ("rv_c", ctypes.c_double)]


class Topology(ctypes.Structure):
    _fields_ = [(name, _ip) for name in (
        "cell_box", "face_cells", "face_dir", "row_ptr", "col_idx", "blk_face", "diag_pos",
        "level_ptr", "perm", "iperm", "lo_blk", "lo_tblk", "lo_pos", "up_blk", "up_pos")] + [
        ("n_levels", _i32), ("max_level", _i32), ("sweep_span", _i32)]


class IluBlocks(ctypes.Structure):
    _fields_ = [("bx", _i32), ("by", _i32), ("bz", _i32), ("sub_level_ptr", _ip), ("slot", _ip),
                ("n_sub", _i32), ("max_sub", _i32), ("max_width", _i32)]


class Problem(ctypes.Structure):
    _fields_ = [("n_cells", _i32), ("n_faces", _i32), ("nnzb", _i32), ("n_levels", _i32),
                ("max_level", _i32), ("n_conns", _i32),
                ("trans", _vp), ("pore_vol", _vp), ("depth", _vp),
                ("row_ptr", _vp), ("col_idx", _vp), ("blk_face", _vp), ("face_cells", _vp),
                ("diag_pos", _vp), ("level_ptr", _vp), ("level_ptr_h", _vp), ("perm", _vp),
                ("iperm", _vp), ("lo_blk", _vp), ("lo_tblk", _vp), ("lo_pos", _vp),
                ("up_blk", _vp), ("up_pos", _vp), ("cell_conn_ptr", _vp), ("cell_conn", _vp),
                ("conn_kind", _vp), ("conn_phase", _vp), ("conn_wi", _vp), ("conn_rate", _vp),
                ("conn_bhp", _vp), ("fluid", Fluid), ("sweep_span", _i32),
                ("n_sub", _i32), ("max_sub", _i32), ("max_width", _i32),
                ("sub_level_ptr", _vp), ("slot", _vp), ("meaning", _vp),
                ("n_wells", _i32), ("pad_w", _i32), ("well_conn_ptr", _vp), ("conn_cell", _vp),
                ("conn_well", _vp), ("well_kind", _vp), ("well_phase", _vp), ("well_target", _vp),
                ("well_vol", _vp), ("well_state", _vp), ("amg", _vp), ("well_limit", _vp),
                ("well_ctrl", _vp), ("nx", _i32), ("ny", _i32), ("nz", _i32), ("pad_l", _i32),
                ("box_cell", _vp), ("cell_box", _vp)]


AMG_MAX_LEVELS, AMG_COARSE = 12, 64


class Amg(ctypes.Structure):
    _fields_ = [("n_levels", _i32), ("n", _i32 * AMG_MAX_LEVELS),
                ("nnz", _i32 * AMG_MAX_LEVELS)] + [
        (name, _vp * AMG_MAX_LEVELS) for name in (
            "row_ptr", "col", "dpos", "agg", "child_ptr", "child", "gmap_ptr", "gmap")]


class SolveReport(ctypes.Structure):
    _fields_ = [("status", _i32), ("half", _i32), ("its", _i32), ("pad", _i32),
                ("rel_res", ctypes.c_double)]


class NewtonOpts(ctypes.Structure):
    _fields_ = [("tol_cnv", ctypes.c_double), ("tol_mb", ctypes.c_double),
                ("ds_max", ctypes.c_double), ("dp_max_rel", ctypes.c_double),
                ("lin_rtol", ctypes.c_double), ("max_newton", _i32), ("lin_maxit", _i32),
                ("precision", _i32), ("max_cuts", _i32), ("krylov", _i32), ("restart", _i32),
                ("precond", _i32), ("pad", _i32)]


class NewtonReport(ctypes.Structure):
    _fields_ = [("status", _i32), ("newton_its", _i32), ("lin_its", _i32), ("substeps", _i32),
                ("cuts", _i32), ("pad", _i32), ("cnv", ctypes.c_double * 3),
                ("mb", ctypes.c_double * 3), ("cell_newton_its", ctypes.c_double),
                ("t_assemble", ctypes.c_double), ("t_factor", ctypes.c_double),
                ("t_krylov", ctypes.c_double), ("t_update", ctypes.c_double)]

    def as_dict(self):
        return {k: (list(getattr(self, k)) if k in ("cnv", "mb") else getattr(self, k))
                for k, _ in self._fields_ if k != "pad"}


EXPORTS = [
    "opm_init", "opm_strerror", "opm_topology_count", "opm_topology_build",
    "opm_ilu_blocks_count", "opm_topology_build_blocks", "opm_geometry",
    "opm_well_index", "opm_well_groups", "opm_accumulation", "opm_norms_bytes", "opm_assemble",
    "opm_assemble_noalloc",
    "opm_ilu0_bytes", "opm_ilu0_factor", "opm_ilu0_apply", "opm_spmv", "opm_krylov_bytes",
    "opm_bicgstab", "opm_gmres_bytes", "opm_gmres", "opm_newton_bytes", "opm_newton_work_bytes",
    "opm_newton_step", "opm_advance", "opm_set_option", "opm_wells_bytes", "opm_assemble_wells",
    "opm_ensemble_bytes", "opm_ensemble_prepare", "opm_ensemble_launch",
    "opm_amg_count", "opm_amg_build", "opm_cpr_bytes", "opm_cpr_setup", "opm_cpr_vcycle",
    "opm_cpr_apply", "opm_cpr_values", "opm_bicgstab_cpr",
]

OPT_SWEEP_MODE, OPT_KRYLOV_CHUNK, OPT_SWEEP_KERNEL, OPT_BLOCK_DEPTH, OPT_KRYLOV_GRAPH = 1, 2, 3, 4, 5
OPT_ASSEMBLY, OPT_PLANE_SWEEP, OPT_PLANE_SPIN, OPT_ENSEMBLE_SPIN = 6, 7, 8, 9

_lib = None


class OpmError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what}: {_strerror(code)} ({code})")
        self.code = code


def _strerror(code):
    try:
        return lib().opm_strerror(code).decode()
    except Exception:
        return "error"


def lib():
    """Load libopm_gpu.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"HIP library {LIB_PATH} is not built; run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        L.opm_strerror.restype = ctypes.c_char_p
        L.opm_strerror.argtypes = [ctypes.c_int]
        L.opm_init.restype = ctypes.c_int
        L.opm_set_option.argtypes = [ctypes.c_int, ctypes.c_int]
        L.opm_topology_count.argtypes = [_i32, _i32, _i32, _vp, _ip, _ip]
        L.opm_topology_build.argtypes = [_i32, _i32, _i32, _vp, ctypes.POINTER(Topology)]
        L.opm_ilu_blocks_count.argtypes = [_i32, _i32, _i32, _vp, _i32, _i32, _i32, _ip, _ip]
        L.opm_topology_build_blocks.argtypes = [_i32, _i32, _i32, _vp, ctypes.POINTER(IluBlocks),
                                                ctypes.POINTER(Topology)]
        L.opm_geometry.argtypes = [_i32, _i32, _i32, ctypes.c_double, ctypes.c_double, _vp, _vp,
                                   ctypes.c_double, _vp, _i32, _i32, _vp, _vp, _vp, _vp, _vp,
                                   _vp, _vp]
        L.opm_well_index.argtypes = [_i32, _i32, ctypes.c_double, ctypes.c_double, _vp, _vp, _vp,
                                     _i32, _vp, _vp, _vp, _vp, _i32, _vp, _vp, _vp, _vp, _vp,
                                     _vp, _vp, _vp]
        L.opm_well_groups.argtypes = [_i32, _i32, _vp, _vp, _vp]
        P = ctypes.POINTER(Problem)
        L.opm_accumulation.argtypes = [P, _vp, _vp, _vp]
        L.opm_norms_bytes.argtypes = [P]
        L.opm_norms_bytes.restype = ctypes.c_size_t
        L.opm_assemble.argtypes = [P, _vp, _vp, ctypes.c_double, _vp, _vp, _vp, _vp]
        L.opm_assemble_noalloc.argtypes = [P, _vp, _vp, ctypes.c_double, _vp, _vp, _vp, _vp]
        L.opm_ilu0_bytes.argtypes = [P, ctypes.c_int]
        L.opm_ilu0_bytes.restype = ctypes.c_size_t
        L.opm_ilu0_factor.argtypes = [P, _vp, _vp, ctypes.c_int, _vp, _vp]
        L.opm_ilu0_apply.argtypes = [P, _vp, ctypes.c_int, _vp, _vp, _vp]
        L.opm_spmv.argtypes = [P, _vp, _vp, _vp, _vp]
        L.opm_krylov_bytes.argtypes = [P]
        L.opm_krylov_bytes.restype = ctypes.c_size_t
        L.opm_bicgstab.argtypes = [P, _vp, _vp, ctypes.c_int, _vp, _vp, ctypes.c_double, _i32,
                                   _vp, ctypes.POINTER(SolveReport), _vp]
        L.opm_gmres_bytes.argtypes = [P, _i32]
        L.opm_gmres_bytes.restype = ctypes.c_size_t
        L.opm_gmres.argtypes = [P, _vp, _vp, ctypes.c_int, _vp, _vp, ctypes.c_double, _i32, _i32,
                                _vp, ctypes.POINTER(SolveReport), _vp]
        L.opm_newton_bytes.argtypes = [P, ctypes.c_int]
        L.opm_newton_bytes.restype = ctypes.c_size_t
        L.opm_newton_work_bytes.argtypes = [P, ctypes.POINTER(NewtonOpts)]
        L.opm_newton_work_bytes.restype = ctypes.c_size_t
        L.opm_wells_bytes.argtypes = [P]
        L.opm_wells_bytes.restype = ctypes.c_size_t
        L.opm_assemble_wells.argtypes = [P, _vp, _vp, _vp, ctypes.c_double, _vp, _vp, _vp, _vp,
                                         _vp, _vp, _vp, _vp]
        L.opm_newton_step.argtypes = [P, _vp, _vp, ctypes.c_double, ctypes.POINTER(NewtonOpts),
                                      _vp, ctypes.POINTER(NewtonReport), _vp]
        L.opm_advance.argtypes = [P, _vp, ctypes.c_double, ctypes.POINTER(NewtonOpts), _vp, _vp,
                                  ctypes.POINTER(NewtonReport), _vp]
        A = ctypes.POINTER(Amg)
        L.opm_amg_count.argtypes = [_i32, _i32, _i32, _vp, _i32, _vp, _vp, A]
        L.opm_amg_build.argtypes = [_i32, _i32, _i32, _vp, _i32, _vp, _vp, A]
        L.opm_cpr_bytes.argtypes = [P]
        L.opm_cpr_bytes.restype = ctypes.c_size_t
        L.opm_cpr_setup.argtypes = [P, _vp, _vp, _vp, _vp]
        L.opm_cpr_vcycle.argtypes = [P, _vp, _vp, _vp, _vp]
        L.opm_cpr_apply.argtypes = [P, _vp, _vp, ctypes.c_int, _vp, _vp, _vp, _vp]
        L.opm_cpr_values.argtypes = [P, _vp, _i32, _vp, _vp, _vp]
        L.opm_bicgstab_cpr.argtypes = [P, _vp, _vp, ctypes.c_int, _vp, _vp, _vp, ctypes.c_double,
                                       _i32, _vp, ctypes.POINTER(SolveReport), _vp]
        _lib = L
    return _lib


def _check(code, what):
    if code != OK:
        raise OpmError(code, what)


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


_initialised = set()


def init(device=None):
    """opm_init on the current device (once per device)."""
    dev = torch.cuda.current_device() if device is None else device
    if dev not in _initialised:
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device: the MI355X path cannot run here")
        with torch.cuda.device(dev):
            _check(lib().opm_init(), "opm_init (needs a gfx950 device)")
        _initialised.add(dev)


def set_option(option: int, value: int) -> None:
    """Set a tuning knob (OPT_SWEEP_MODE, OPT_KRYLOV_CHUNK)."""
    _check(lib().opm_set_option(option, value), "opm_set_option")


def default_opts(case=None, precision=PREC_FP64, **kw) -> NewtonOpts:
    o = NewtonOpts(tol_cnv=1e-8, tol_mb=1e-11, ds_max=0.2, dp_max_rel=0.3, lin_rtol=1e-6,
                   max_newton=20, lin_maxit=500, precision=precision, max_cuts=8,
                   krylov=KRYLOV_BICGSTAB, restart=30, precond=PRECOND_ILU0)
    if case is not None:
        o.tol_cnv, o.tol_mb, o.lin_rtol = case.tol_cnv, case.tol_mb, case.lin_rtol
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def build_topology(nx: int, ny: int, nz: int, mask: np.ndarray,
                   ilu_blocks: Optional[Sequence[int]] = None):
    """Host topology (opm_topology_build, or opm_topology_build_blocks for a
    block ILU0 over subdomain boxes of ilu_blocks = (bx, by, bz) cells).
    Returns (n, nf, host arrays, Topology, IluBlocks or None)."""
    L = lib()
    mask = np.ascontiguousarray(mask, dtype=np.uint8).ravel()
    n, nf = _i32(), _i32()
    _check(L.opm_topology_count(nx, ny, nz, mask.ctypes.data, ctypes.byref(n), ctypes.byref(nf)),
           "opm_topology_count")
    n, nf = n.value, nf.value
    nnzb = n + 2 * nf
    sizes = dict(cell_box=n, face_cells=2 * nf, face_dir=nf, row_ptr=n + 1, col_idx=nnzb,
                 blk_face=nnzb, diag_pos=n, level_ptr=n + 1, perm=n, iperm=n, lo_blk=3 * n,
                 lo_tblk=3 * n, lo_pos=3 * n, up_blk=3 * n, up_pos=3 * n)
    host = {k: np.zeros(max(v, 1), np.int32) for k, v in sizes.items()}
    topo = Topology(**{k: a.ctypes.data_as(_ip) for k, a in host.items()})
    if ilu_blocks is None:
        _check(L.opm_topology_build(nx, ny, nz, mask.ctypes.data, ctypes.byref(topo)),
               "opm_topology_build")
        return n, nf, host, topo, None
    bx, by, bz = (int(b) for b in ilu_blocks)
    ns, nl = _i32(), _i32()
    _check(L.opm_ilu_blocks_count(nx, ny, nz, mask.ctypes.data, bx, by, bz, ctypes.byref(ns),
                                  ctypes.byref(nl)), "opm_ilu_blocks_count")
    host["sub_level_ptr"] = np.zeros(max(nl.value * (ns.value + 1), 1), np.int32)
    host["slot"] = np.zeros(max(n, 1), np.int32)
    blk = IluBlocks(bx=bx, by=by, bz=bz, sub_level_ptr=host["sub_level_ptr"].ctypes.data_as(_ip),
                    slot=host["slot"].ctypes.data_as(_ip))
    _check(L.opm_topology_build_blocks(nx, ny, nz, mask.ctypes.data, ctypes.byref(blk),
                                       ctypes.byref(topo)), "opm_topology_build_blocks")
    return n, nf, host, topo, blk


def amg_hierarchy(nx: int, ny: int, nz: int, mask: np.ndarray, n: int, row_ptr: np.ndarray,
                  col_idx: np.ndarray):
    """opm_amg_count + opm_amg_build (host only): the Amg struct (host
    pointers) and its arrays {(name, level): int32 array}."""
    L = lib()
    mask = np.ascontiguousarray(mask, dtype=np.uint8).ravel()
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    g = Amg()
    _check(L.opm_amg_count(nx, ny, nz, mask.ctypes.data, n, rp.ctypes.data, ci.ctypes.data,
                           ctypes.byref(g)), "opm_amg_count")
    nl = g.n_levels
    arrays = {}
    for l in range(nl):
        nl_, nnz = g.n[l], g.nnz[l]
        if l >= 1:
            for k, size in (("row_ptr", nl_ + 1), ("col", nnz), ("dpos", nl_),
                            ("gmap_ptr", nnz + 1), ("gmap", g.nnz[l - 1])):
                arrays[k, l] = np.zeros(size, np.int32)
        if l + 1 < nl:
            for k, size in (("agg", nl_), ("child_ptr", g.n[l + 1] + 1), ("child", nl_)):
                arrays[k, l] = np.zeros(size, np.int32)
    for (k, l), a in arrays.items():
        getattr(g, k)[l] = a.ctypes.data
    _check(L.opm_amg_build(nx, ny, nz, mask.ctypes.data, n, rp.ctypes.data, ci.ctypes.data,
                           ctypes.byref(g)), "opm_amg_build")
    return g, arrays


class GpuModel:
    """A case laid out on the GPU: topology, geometry and wells on device.
    ilu_blocks = (bx, by, bz) selects the block ILU0 over subdomain boxes of
    that many cells per axis (one block per subdomain) instead of the
    single-block ILU(0).  amg builds the CPR-AMG hierarchy (needed for
    precond = PRECOND_CPR)."""

    def __init__(self, case: _cases.Case, device: str = "cuda",
                 ilu_blocks: Optional[Sequence[int]] = None, amg: bool = True):
        L = lib()
        init()
        self.case = case
        self.dev = torch.device(device)
        nx, ny, nz = case.nx, case.ny, case.nz
        n, nf, host, topo, blk = build_topology(nx, ny, nz, case.mask, ilu_blocks)
        nnzb = n + 2 * nf
        self.ilu_blocks = None if ilu_blocks is None else tuple(int(b) for b in ilu_blocks)
        self.blocks = blk
        self.n, self.nf, self.nnzb = n, nf, nnzb
        self.n_levels, self.max_level = topo.n_levels, topo.max_level
        self.sweep_span = topo.sweep_span
        self.host = host
        self.level_ptr_h = np.ascontiguousarray(host["level_ptr"][:self.n_levels + 1])
        d = {k: torch.from_numpy(a).to(self.dev) for k, a in host.items()}
        self.t = d
        cell_box = host["cell_box"][:n]
        box_cell = np.full(case.n_box, -1, np.int64)
        box_cell[cell_box] = np.arange(n)
        self.cell_box, self.box_cell = cell_box, box_cell
        f64 = dict(dtype=torch.float64, device=self.dev)
        self.perm_h = torch.from_numpy(np.ascontiguousarray(case.perm_h.ravel()[cell_box])).to(self.dev)
        self.poro = torch.from_numpy(np.ascontiguousarray(case.poro.ravel()[cell_box])).to(self.dev)
        self.dz = torch.tensor(np.asarray(case.dz, dtype=np.float64), **f64)
        self.trans = torch.zeros(max(nf, 1), **f64)
        self.pore_vol = torch.zeros(n, **f64)
        self.depth = torch.zeros(n, **f64)
        st = _stream()
        _check(L.opm_geometry(nx, ny, nz, case.dx, case.dy, _ptr(self.dz), _ptr(self.perm_h),
                              case.kv_kh, _ptr(self.poro), n, nf, _ptr(d["cell_box"]),
                              _ptr(d["face_cells"]), _ptr(d["face_dir"]), _ptr(self.trans),
                              _ptr(self.pore_vol), _ptr(self.depth), st), "opm_geometry")
        # wells
        wells = case.wells
        nw = len(wells)
        conn_cell = np.array([box_cell[case.box_index(*c)] for w in wells for c in w.cells],
                             dtype=np.int32)
        if np.any(conn_cell < 0):
            raise ValueError("well connection in an inactive cell")
        conn_well = np.array([k for k, w in enumerate(wells) for _ in w.cells], dtype=np.int32)
        nc = len(conn_cell)
        self.nc = nc
        i32 = dict(dtype=torch.int32, device=self.dev)
        self.well_kind = torch.tensor([w.kind for w in wells] + [0], **i32)
        self.well_phase = torch.tensor([w.phase for w in wells] + [0], **i32)
        self.well_target = torch.tensor([w.target for w in wells] + [0.0], **f64)
        self.well_rw = torch.tensor([w.rw for w in wells] + [1.0], **f64)
        self.conn_cell = torch.from_numpy(np.append(conn_cell, 0).astype(np.int32)).to(self.dev)
        self.conn_well = torch.from_numpy(np.append(conn_well, 0).astype(np.int32)).to(self.dev)
        m = max(nc, 1)
        self.conn_wi = torch.zeros(m, **f64)
        self.conn_rate = torch.zeros(m, **f64)
        self.conn_bhp = torch.zeros(m, **f64)
        self.conn_kind = torch.zeros(m, **i32)
        self.conn_phase = torch.zeros(m, **i32)
        _check(L.opm_well_index(nx, ny, case.dx, case.dy, _ptr(self.dz), _ptr(self.perm_h),
                                _ptr(d["cell_box"]), nw, _ptr(self.well_kind),
                                _ptr(self.well_phase), _ptr(self.well_target), _ptr(self.well_rw),
                                nc, _ptr(self.conn_cell), _ptr(self.conn_well), _ptr(self.conn_wi),
                                _ptr(self.conn_rate), _ptr(self.conn_kind), _ptr(self.conn_phase),
                                _ptr(self.conn_bhp), st), "opm_well_index")
        ccp = np.zeros(n + 1, np.int32)
        cc = np.zeros(m, np.int32)
        cc_src = np.append(conn_cell, 0).astype(np.int32)
        _check(L.opm_well_groups(n, nc, cc_src.ctypes.data, ccp.ctypes.data, cc.ctypes.data),
               "opm_well_groups")
        self.cell_conn_ptr = torch.from_numpy(ccp).to(self.dev)
        self.cell_conn = torch.from_numpy(cc).to(self.dev)
        f = case.fluid
        fl = Fluid((ctypes.c_double * 3)(*f.rho_s), (ctypes.c_double * 3)(*f.c), f.p_ref,
                   (ctypes.c_double * 3)(*f.mu), f.swc, f.n_corey, f.g, f.rs_c, f.bo_r, f.muo_r,
                   f.eps_switch, int(f.live), 0, float(getattr(f, "rv_c", 0.0)))
        self.pb = Problem(
            n_cells=n, n_faces=nf, nnzb=nnzb, n_levels=self.n_levels, max_level=self.max_level,
            n_conns=nc, trans=self.trans.data_ptr(), pore_vol=self.pore_vol.data_ptr(),
            depth=self.depth.data_ptr(), row_ptr=d["row_ptr"].data_ptr(),
            col_idx=d["col_idx"].data_ptr(), blk_face=d["blk_face"].data_ptr(),
            face_cells=d["face_cells"].data_ptr(), diag_pos=d["diag_pos"].data_ptr(),
            level_ptr=d["level_ptr"].data_ptr(), level_ptr_h=self.level_ptr_h.ctypes.data,
            perm=d["perm"].data_ptr(), iperm=d["iperm"].data_ptr(), lo_blk=d["lo_blk"].data_ptr(),
            lo_tblk=d["lo_tblk"].data_ptr(), lo_pos=d["lo_pos"].data_ptr(),
            up_blk=d["up_blk"].data_ptr(), up_pos=d["up_pos"].data_ptr(),
            cell_conn_ptr=self.cell_conn_ptr.data_ptr(), cell_conn=self.cell_conn.data_ptr(),
            conn_kind=self.conn_kind.data_ptr(), conn_phase=self.conn_phase.data_ptr(),
            conn_wi=self.conn_wi.data_ptr(), conn_rate=self.conn_rate.data_ptr(),
            conn_bhp=self.conn_bhp.data_ptr(), fluid=fl, sweep_span=topo.sweep_span)
        # the lattice, for the LDS-tiled assembly
        self.box_cell_t = torch.from_numpy(box_cell.astype(np.int32)).to(self.dev)
        self.pb.nx, self.pb.ny, self.pb.nz = nx, ny, nz
        self.pb.box_cell = self.box_cell_t.data_ptr()
        self.pb.cell_box = d["cell_box"].data_ptr()
        if blk is not None:
            self.pb.n_sub, self.pb.max_sub, self.pb.max_width = blk.n_sub, blk.max_sub, blk.max_width
            self.pb.sub_level_ptr = d["sub_level_ptr"].data_ptr()
            self.pb.slot = d["slot"].data_ptr()
        # meaning of the third variable per cell (0 s_g, 1 r_go): live oil only
        self.live = bool(f.live)
        self.meaning_t = torch.from_numpy(case.initial_meaning()).to(self.dev)
        if self.live:
            self.pb.meaning = self.meaning_t.data_ptr()
        # standard wells: well unknowns (Q_t, F_w, F_g, p_bhp) per well
        self.nw = nw
        self.std_wells = bool(getattr(case, "standard_wells", False))
        if self.std_wells:
            vol, x0 = case.standard_well_init()
            wcp = np.zeros(nw + 1, np.int32)
            wcp[1:] = np.cumsum([len(w.cells) for w in wells])
            self.well_conn_ptr = torch.from_numpy(wcp).to(self.dev)
            self.well_vol = torch.tensor(vol, **f64)
            self.well_state_t = torch.tensor(x0, **f64).contiguous()
            self.pb.n_wells = nw
            self.pb.well_conn_ptr = self.well_conn_ptr.data_ptr()
            self.pb.conn_cell = self.conn_cell.data_ptr()
            self.pb.conn_well = self.conn_well.data_ptr()
            self.pb.well_kind = self.well_kind.data_ptr()
            self.pb.well_phase = self.well_phase.data_ptr()
            self.pb.well_target = self.well_target.data_ptr()
            self.pb.well_vol = self.well_vol.data_ptr()
            self.pb.well_state = self.well_state_t.data_ptr()
            # control limits (zero = none) and the active controls
            lim = case.standard_well_limits()
            self.well_ctrl_t = torch.zeros(max(nw, 1), dtype=torch.int32, device=self.dev)
            if (lim > 0).any():
                self.well_limit = torch.tensor(lim, **f64)
                self.pb.well_limit = self.well_limit.data_ptr()
                self.pb.well_ctrl = self.well_ctrl_t.data_ptr()
        self._work = {}
        self.amg = self._build_amg(host) if amg else None
        if amg:
            self.pb.amg = ctypes.addressof(self.amg)
        torch.cuda.current_stream().synchronize()

    def _build_amg(self, host):
        """The CPR-AMG hierarchy (opm_amg_build on the host, arrays copied to
        the device); the struct handed to the library holds device pointers."""
        c = self.case
        g, arrays = amg_hierarchy(c.nx, c.ny, c.nz, c.mask, self.n, host["row_ptr"],
                                  host["col_idx"])
        self.amg_host = arrays
        self.amg_dev = {key: torch.from_numpy(a).to(self.dev) for key, a in arrays.items()}
        d = Amg()
        d.n_levels = g.n_levels
        for l in range(g.n_levels):
            d.n[l], d.nnz[l] = g.n[l], g.nnz[l]
        for (k, l), t in self.amg_dev.items():
            getattr(d, k)[l] = t.data_ptr()
        return d

    def amg_levels(self):
        """(n, nnz) per level of the CPR hierarchy."""
        return [(self.amg.n[l], self.amg.nnz[l]) for l in range(self.amg.n_levels)]

    def cpr_setup(self, J):
        """opm_cpr_setup: the CPR workspace for the Jacobian J, and the
        device status word."""
        L = lib()
        nb = L.opm_cpr_bytes(self._pbp())
        if nb == 0:
            raise OpmError(EINVAL, "opm_cpr_bytes")
        cpr = torch.zeros(nb, dtype=torch.uint8, device=self.dev)
        status = torch.zeros(1, dtype=torch.int32, device=self.dev)
        _check(L.opm_cpr_setup(self._pbp(), _ptr(J), _ptr(cpr), _ptr(status), _stream()),
               "opm_cpr_setup")
        return cpr, status

    def cpr_values(self, cpr, level):
        """(level matrix values, weights [n][3]) of a set-up CPR workspace."""
        a = torch.zeros(self.amg.nnz[level], dtype=torch.float64, device=self.dev)
        w = self.zeros_state()
        _check(lib().opm_cpr_values(self._pbp(), _ptr(cpr), level, _ptr(a), _ptr(w), _stream()),
               "opm_cpr_values")
        return a, w

    def cpr_vcycle(self, cpr, b):
        x = torch.zeros(self.n, dtype=torch.float64, device=self.dev)
        _check(lib().opm_cpr_vcycle(self._pbp(), _ptr(cpr), _ptr(b), _ptr(x), _stream()),
               "opm_cpr_vcycle")
        return x

    def cpr_apply(self, J, ilu, cpr, r, precision=PREC_FP64):
        z = self.zeros_state()
        _check(lib().opm_cpr_apply(self._pbp(), _ptr(J), _ptr(ilu), precision, _ptr(cpr), _ptr(r),
                                   _ptr(z), _stream()), "opm_cpr_apply")
        return z

    def bicgstab_cpr(self, J, ilu, cpr, b, rtol=1e-6, maxit=500, precision=PREC_FP64):
        L = lib()
        x = self.zeros_state()
        work = self.workspace("krylov", L.opm_krylov_bytes(self._pbp()))
        rep = SolveReport()
        _check(L.opm_bicgstab_cpr(self._pbp(), _ptr(J), _ptr(ilu), precision, _ptr(cpr), _ptr(b),
                                  _ptr(x), rtol, maxit, _ptr(work), ctypes.byref(rep), _stream()),
               "opm_bicgstab_cpr")
        return x, rep

    # ------------------------------------------------------------ helpers
    def _pbp(self):
        return ctypes.byref(self.pb)

    def zeros_state(self):
        return torch.zeros((self.n, 3), dtype=torch.float64, device=self.dev)

    def state(self, y) -> torch.Tensor:
        return torch.as_tensor(np.ascontiguousarray(y, dtype=np.float64)).to(self.dev).contiguous()

    def initial_state(self) -> torch.Tensor:
        """The case's initial state; also resets the variable meanings to the
        case's initial ones (live oil) and the well unknowns (standard wells)."""
        self.set_meaning(self.case.initial_meaning())
        if self.std_wells:
            self.set_well_state(self.case.standard_well_init()[1])
            self.well_ctrl_t.zero_()
        return self.state(self.case.initial_state())

    def set_well_state(self, x) -> None:
        """Well unknowns [n_wells][4] = (Q_t, F_w, F_g, p_bhp) (standard wells)."""
        self.well_state_t.copy_(torch.as_tensor(np.ascontiguousarray(x, dtype=np.float64)))

    def well_state(self) -> np.ndarray:
        return self.well_state_t.cpu().numpy().copy()

    def well_ctrl(self) -> np.ndarray:
        """Active control per standard well: 0 its own, 1 its limit."""
        return self.well_ctrl_t.cpu().numpy()[:self.nw].copy()

    def set_well_ctrl(self, c) -> None:
        self.well_ctrl_t[:self.nw].copy_(torch.as_tensor(np.ascontiguousarray(c, dtype=np.int32)))

    def assemble_wells(self, y, acc0, well_state0, dt):
        """opm_assemble_wells: (R, J, Rw, B, C, D) on the device."""
        L = lib()
        R = self.zeros_state()
        J = torch.zeros((self.nnzb, 3, 3), dtype=torch.float64, device=self.dev)
        f64 = dict(dtype=torch.float64, device=self.dev)
        Rw = torch.zeros((self.nw, 4), **f64)
        B = torch.zeros((max(self.nc, 1), 4, 3), **f64)
        C = torch.zeros((max(self.nc, 1), 3, 4), **f64)
        D = torch.zeros((self.nw, 4, 4), **f64)
        x0 = torch.as_tensor(np.ascontiguousarray(well_state0, dtype=np.float64)).to(self.dev)
        work = self.workspace("wells", L.opm_wells_bytes(self._pbp()))
        _check(L.opm_assemble_wells(self._pbp(), _ptr(y), _ptr(acc0), _ptr(x0), dt, _ptr(R),
                                    _ptr(J), _ptr(Rw), _ptr(B), _ptr(C), _ptr(D), _ptr(work),
                                    _stream()), "opm_assemble_wells")
        return R, J, Rw, B[:self.nc], C[:self.nc], D

    def set_meaning(self, mean) -> None:
        """Meaning of the third variable per cell (0 s_g, 1 r_go), the state
        that goes with y for live oil."""
        m = torch.as_tensor(np.ascontiguousarray(mean, dtype=np.uint8))
        wet = self.live and self.case.fluid.rv_c > 0.0
        if (m.shape != (self.n,) or (not self.live and bool(m.any())) or
                bool((m > (2 if wet else 1)).any())):
            raise ValueError("meaning: one value per cell (0 s_g, 1 r_go, 2 r_og with wet gas), "
                             "all 0 for dead oil")
        self.meaning_t.copy_(m.to(self.dev))

    def meaning(self) -> np.ndarray:
        return self.meaning_t.cpu().numpy().copy()

    def pattern(self):
        return (self.host["row_ptr"][:self.n + 1].copy(), self.host["col_idx"][:self.nnzb].copy())

    def workspace(self, kind: str, nbytes: int) -> torch.Tensor:
        w = self._work.get(kind)
        if w is None or w.numel() < nbytes:
            w = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=self.dev)
            self._work[kind] = w
        return w

    # ------------------------------------------------------------ path steps
    def accumulation(self, y: torch.Tensor) -> torch.Tensor:
        acc = self.zeros_state()
        _check(lib().opm_accumulation(self._pbp(), _ptr(y), _ptr(acc), _stream()),
               "opm_accumulation")
        return acc

    def assemble(self, y, acc0, dt, jacobian=True, norms=True):
        L = lib()
        R = self.zeros_state()
        J = torch.zeros((self.nnzb, 3, 3), dtype=torch.float64, device=self.dev) if jacobian else None
        nb = None
        if norms:
            nb = torch.zeros(L.opm_norms_bytes(self._pbp()) // 8, dtype=torch.float64,
                             device=self.dev)
        _check(L.opm_assemble(self._pbp(), _ptr(y), _ptr(acc0), dt, _ptr(R), _ptr(J), _ptr(nb),
                              _stream()), "opm_assemble")
        return R, J, (nb[:8] if norms else None)

    def assemble_noalloc(self, y, acc0, dt, R, J, norms):
        """opm_assemble_noalloc into caller-given tensors (J and norms may be
        None); returns the status code."""
        return lib().opm_assemble_noalloc(self._pbp(), _ptr(y), _ptr(acc0), dt, _ptr(R), _ptr(J),
                                          _ptr(norms), _stream())

    def ilu0_factor(self, J, precision=PREC_FP64):
        L = lib()
        ilu = torch.zeros(L.opm_ilu0_bytes(self._pbp(), precision), dtype=torch.uint8,
                          device=self.dev)
        status = torch.zeros(1, dtype=torch.int32, device=self.dev)
        _check(L.opm_ilu0_factor(self._pbp(), _ptr(J), _ptr(ilu), precision, _ptr(status),
                                 _stream()), "opm_ilu0_factor")
        return ilu, status

    def ilu0_apply(self, ilu, r, precision=PREC_FP64):
        x = self.zeros_state()
        _check(lib().opm_ilu0_apply(self._pbp(), _ptr(ilu), precision, _ptr(r), _ptr(x),
                                    _stream()), "opm_ilu0_apply")
        return x

    def spmv(self, J, x):
        y = self.zeros_state()
        _check(lib().opm_spmv(self._pbp(), _ptr(J), _ptr(x), _ptr(y), _stream()), "opm_spmv")
        return y

    def bicgstab(self, J, ilu, b, rtol=1e-6, maxit=500, precision=PREC_FP64):
        L = lib()
        x = self.zeros_state()
        work = self.workspace("krylov", L.opm_krylov_bytes(self._pbp()))
        rep = SolveReport()
        _check(L.opm_bicgstab(self._pbp(), _ptr(J), _ptr(ilu), precision, _ptr(b), _ptr(x), rtol,
                              maxit, _ptr(work), ctypes.byref(rep), _stream()), "opm_bicgstab")
        return x, rep

    def gmres(self, J, ilu, b, rtol=1e-6, maxit=500, restart=30, precision=PREC_FP64):
        L = lib()
        x = self.zeros_state()
        work = self.workspace("gmres", L.opm_gmres_bytes(self._pbp(), restart))
        rep = SolveReport()
        _check(L.opm_gmres(self._pbp(), _ptr(J), _ptr(ilu), precision, _ptr(b), _ptr(x), rtol,
                           maxit, restart, _ptr(work), ctypes.byref(rep), _stream()), "opm_gmres")
        return x, rep

    def newton_work(self, o: NewtonOpts) -> torch.Tensor:
        nbytes = lib().opm_newton_work_bytes(self._pbp(), ctypes.byref(o))
        if nbytes == 0:
            raise OpmError(EINVAL, "opm_newton_work_bytes")
        return self.workspace(f"newton{o.precision}", nbytes)

    def newton_step(self, y, y_prev, dt, opts: Optional[NewtonOpts] = None):
        L = lib()
        o = opts or default_opts(self.case)
        work = self.newton_work(o)
        rep = NewtonReport()
        st = L.opm_newton_step(self._pbp(), _ptr(y), _ptr(y_prev), dt, ctypes.byref(o),
                               _ptr(work), ctypes.byref(rep), _stream())
        if st in (EINVAL, EHIP):
            _check(st, "opm_newton_step")
        return st, rep

    def advance(self, y, dt, opts: Optional[NewtonOpts] = None):
        L = lib()
        o = opts or default_opts(self.case)
        work = self.newton_work(o)
        ysave = self.workspace("ysave", 24 * self.n).view(torch.float64)[:3 * self.n].view(self.n, 3)
        rep = NewtonReport()
        st = L.opm_advance(self._pbp(), _ptr(y), dt, ctypes.byref(o), _ptr(work), _ptr(ysave),
                           ctypes.byref(rep), _stream())
        if st in (EINVAL, EHIP):
            _check(st, "opm_advance")
        return st, rep

    def run(self, y=None, n_steps=None, opts=None, keep_states=True):
        """Advance over the case's report schedule (raises on a failed step);
        with live oil the meanings after each step are in ``run_meanings``."""
        y = self.initial_state() if y is None else y
        states, reps = [], []
        self.run_meanings = []
        self.run_well_states = []
        self.run_well_ctrls = []
        for dt in self.case.report_dt[:n_steps]:
            st, rep = self.advance(y, dt, opts)
            if st != OK:
                raise OpmError(st, "opm_advance")
            if keep_states:
                states.append(y.detach().cpu().numpy().copy())
                if self.live:
                    self.run_meanings.append(self.meaning())
                if self.std_wells:
                    self.run_well_states.append(self.well_state())
                    self.run_well_ctrls.append(self.well_ctrl())
            reps.append(rep.as_dict())
        return y, states, reps

    # ------------------------------------------------ learned initial guess
    def guess_features(self, net, y_n, y_nm1):
        c = self.case
        s = net.struct(self)
        feats = torch.zeros((guess_act_rows(c.nx, c.ny, c.nz), GUESS_CH), dtype=torch.int16,
                            device=self.dev)
        _check(_guess_lib().opm_guess_features(self._pbp(), ctypes.byref(s), _ptr(y_n), _ptr(y_nm1),
                                               _ptr(feats), _stream()), "opm_guess_features")
        return feats


    def guess_infer(self, net, y_n, y_nm1):
        s, work = _model_guess_work(self, net)
        yg = self.zeros_state()
        _check(_guess_lib().opm_guess_infer(self._pbp(), ctypes.byref(s), _ptr(y_n), _ptr(y_nm1),
                                            _ptr(yg), _ptr(work), _stream()), "opm_guess_infer")
        return yg


    def guess_train_step(self, net, y_n, y_nm1, y_next, lr, loss_out=None):
        """One Adam step on one sample; returns the device loss (before the step)."""
        s, work = _model_guess_work(self, net)
        loss = loss_out if loss_out is not None else torch.zeros(1, dtype=torch.float64,
                                                                 device=self.dev)
        net.step += 1
        _check(_guess_lib().opm_guess_train_step(self._pbp(), ctypes.byref(s), _ptr(y_n), _ptr(y_nm1),
                                                 _ptr(y_next), _ptr(net.adam_m), _ptr(net.adam_v),
                                                 net.step, float(lr), _ptr(loss), _ptr(work),
                                                 _stream()), "opm_guess_train_step")
        return loss


    def guess_select(self, y, y_prev, y_guess, dt, precision=PREC_FP64):
        L = _guess_lib()
        work = self.workspace(f"newton{precision}", L.opm_newton_bytes(self._pbp(), precision))
        chosen = _i32()
        cnv = (ctypes.c_double * 2)()
        _check(L.opm_guess_select(self._pbp(), _ptr(y), _ptr(y_prev), _ptr(y_guess), dt, _ptr(work),
                                  ctypes.byref(chosen), cnv, _stream()), "opm_guess_select")
        return chosen.value, (cnv[0], cnv[1])


    def advance_guess(self, y, y_nm1, dt, net=None, opts: Optional[NewtonOpts] = None):
        """opm_advance_guess: (status, report, guess_used)."""
        L = _guess_lib()
        o = opts or default_opts(self.case)
        work = self.newton_work(o)
        ysave = self.workspace("ysave", 24 * self.n).view(torch.float64)[:3 * self.n].view(self.n, 3)
        rep = NewtonReport()
        used = _i32()
        if net is not None:
            s, gwork = _model_guess_work(self, net)
            yg = self.workspace("yguess", 24 * self.n).view(torch.float64)[:3 * self.n]
            st = L.opm_advance_guess(self._pbp(), _ptr(y), _ptr(y_nm1), dt, ctypes.byref(o),
                                     ctypes.byref(s), _ptr(gwork), _ptr(yg), _ptr(work), _ptr(ysave),
                                     ctypes.byref(rep), ctypes.byref(used), _stream())
        else:
            st = L.opm_advance_guess(self._pbp(), _ptr(y), None, dt, ctypes.byref(o), None, None,
                                     None, _ptr(work), _ptr(ysave), ctypes.byref(rep),
                                     ctypes.byref(used), _stream())
        if st in (EINVAL, EHIP):
            _check(st, "opm_advance_guess")
        return st, rep, used.value


class EnsembleReport(ctypes.Structure):
    _fields_ = [("status", _i32), ("newton_its", _i32), ("lin_its", _i32), ("substeps", _i32),
                ("cuts", _i32), ("steps_done", _i32), ("cell_newton_its", ctypes.c_double),
                ("cnv", ctypes.c_double * 3), ("mb", ctypes.c_double * 3)]


_ENS_REPORT_DOUBLES = ctypes.sizeof(EnsembleReport) // 8


class EnsembleConfig(ctypes.Structure):
    _fields_ = [("threads", _i32), ("fac_window", _i32), ("ring", _i32), ("sweep_bytes", _i32),
                ("wgs", _i32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


EXPORTS += ["opm_ensemble_default_config", "opm_ensemble_configure",
            "opm_ensemble_launch_config", "opm_ensemble_autotune"]


def _ensemble_lib():
    L = lib()
    if not getattr(L, "_ens_ready", False):
        P = ctypes.POINTER(Problem)
        L.opm_ensemble_bytes.argtypes = [P, _i32, ctypes.c_int]
        L.opm_ensemble_bytes.restype = ctypes.c_size_t
        L.opm_ensemble_prepare.argtypes = [P, ctypes.POINTER(ctypes.c_void_p), _i32, ctypes.c_int,
                                           _vp, ctypes.c_size_t]
        L.opm_ensemble_launch.argtypes = [_vp, _i32, ctypes.c_int, _i32, ctypes.c_double, _i32,
                                          ctypes.POINTER(NewtonOpts), _vp, _vp]
        C = ctypes.POINTER(EnsembleConfig)
        L.opm_ensemble_default_config.argtypes = [P, _i32, ctypes.c_int, C]
        L.opm_ensemble_configure.argtypes = [P, _i32, ctypes.c_int, _vp, C]
        L.opm_ensemble_launch_config.argtypes = [_vp, _i32, ctypes.c_int, _i32, C, ctypes.c_double,
                                                 _i32, ctypes.POINTER(NewtonOpts), _vp, _vp]
        L.opm_ensemble_autotune.argtypes = [P, _i32, ctypes.c_int, _vp, ctypes.c_double,
                                            ctypes.POINTER(NewtonOpts), C, _dp, _ip, _vp]
        L._ens_ready = True
    return L


def member_blocks(case: _cases.Case, split: Optional[Sequence[int]]):
    """Subdomain box (bx, by, bz) of an a x b split of the case's columns
    (None: the member's ILU(0) of the whole system)."""
    if split is None:
        return None
    a, b = (int(v) for v in split)
    return (-(-case.nx // a), -(-case.ny // b), case.nz)


class Ensemble:
    """Independent members advanced together by one persistent kernel launch
    per call (one workgroup per member).  member_split = (a, b) gives every
    member the block ILU0 over a x b whole-column subdomains (boxes of
    ceil(nx / a) x ceil(ny / b) x nz cells, sec. 2.5): the workgroup walks the
    subdomains' local levels together, nx/a + ny/b + nz - 2 of them instead of
    the nx + ny + nz - 2 levels of the member's ILU(0)."""

    def __init__(self, member_cases, precision=PREC_MIXED, device="cuda",
                 member_split: Optional[Sequence[int]] = None):
        L = _ensemble_lib()
        self.member_split = None if member_split is None else tuple(int(v) for v in member_split)
        self.members = [GpuModel(c, device=device, ilu_blocks=member_blocks(c, self.member_split))
                        for c in member_cases]
        self.precision = precision
        self.dev = self.members[0].dev
        nm = len(self.members)
        self.n_members = nm
        self.problems = (Problem * nm)(*[m.pb for m in self.members])
        self.y = [m.initial_state() for m in self.members]
        self.yptr = (ctypes.c_void_p * nm)(*[t.data_ptr() for t in self.y])
        self.max_level = max(m.max_level for m in self.members)
        nbytes = L.opm_ensemble_bytes(self.problems, nm, precision)
        if nbytes == 0:
            raise OpmError(EINVAL, "opm_ensemble_bytes")
        self.work = torch.empty(nbytes, dtype=torch.uint8, device=self.dev)
        _check(L.opm_ensemble_prepare(self.problems, self.yptr, nm, precision,
                                      ctypes.c_void_p(self.work.data_ptr()), nbytes),
               "opm_ensemble_prepare")
        self.reports = torch.zeros((nm, _ENS_REPORT_DOUBLES), dtype=torch.float64, device=self.dev)
        self.n_cells = [m.n for m in self.members]
        # the default shape (one workgroup per member); None when it does not
        # fit in LDS (split members then need configure or autotune)
        self.config = EnsembleConfig()
        if L.opm_ensemble_default_config(self.problems, nm, precision,
                                         ctypes.byref(self.config)) != OK:
            self.config = None
        self.tuning = None

    def signature(self) -> str:
        """Key of the tuning cache: precision and the members' grids."""
        import hashlib
        dims = ";".join(f"{m.case.nx}x{m.case.ny}x{m.case.nz}:{m.n}:{m.ilu_blocks}"
                        for m in self.members)
        return f"p{self.precision}-" + hashlib.sha256(dims.encode()).hexdigest()[:16]

    def configure(self, threads: int, fac_window: int, ring: int, wgs: int = 0) -> None:
        c = EnsembleConfig(threads=threads, fac_window=fac_window, ring=ring, sweep_bytes=0,
                           wgs=wgs)
        _check(_ensemble_lib().opm_ensemble_configure(
            self.problems, self.n_members, self.precision, ctypes.c_void_p(self.work.data_ptr()),
            ctypes.byref(c)), "opm_ensemble_configure")
        self.config = c

    def autotune(self, dt_report, opts: Optional[NewtonOpts] = None,
                 cache: Optional[str] = None) -> dict:
        """Pick the launch shape with opm_ensemble_autotune (one trial report
        step per shape; states are restored), or reuse the shape stored for
        this ensemble's signature in the JSON file `cache`."""
        import json
        key = self.signature()
        if cache and os.path.exists(cache):
            entry = json.load(open(cache)).get(key)
            if entry:
                self.configure(entry["threads"], entry["fac_window"], entry["ring"],
                               entry.get("wgs", 0))
                self.tuning = {"cached": True, **entry}
                return self.tuning
        o = opts or default_opts(self.members[0].case, precision=self.precision)
        best = EnsembleConfig()
        secs = (ctypes.c_double * 16)()
        tried = _i32()
        _check(_ensemble_lib().opm_ensemble_autotune(
            self.problems, self.n_members, self.precision, ctypes.c_void_p(self.work.data_ptr()),
            dt_report, ctypes.byref(o), ctypes.byref(best), secs, ctypes.byref(tried), _stream()),
            "opm_ensemble_autotune")
        self.config = best
        self.tuning = {"cached": False, **best.as_dict(),
                       "trial_seconds": [round(secs[k], 4) for k in range(tried.value)]}
        if cache:
            table = json.load(open(cache)) if os.path.exists(cache) else {}
            table[key] = {k: v for k, v in best.as_dict().items() if k != "sweep_bytes"}
            with open(cache, "w") as f:
                json.dump(table, f, indent=1, sort_keys=True)
        return self.tuning

    def launch(self, dt_report, n_steps, opts: Optional[NewtonOpts] = None):
        """Enqueue one launch with the current shape (asynchronous)."""
        o = opts or default_opts(self.members[0].case, precision=self.precision)
        if self.config is None:
            raise OpmError(EINVAL, "Ensemble.launch: no launch shape fits (configure or autotune)")
        _check(_ensemble_lib().opm_ensemble_launch_config(
            ctypes.c_void_p(self.work.data_ptr()), self.n_members, self.precision, self.max_level,
            ctypes.byref(self.config), dt_report, n_steps, ctypes.byref(o),
            ctypes.c_void_p(self.reports.data_ptr()), _stream()), "opm_ensemble_launch_config")

    def read_reports(self):
        raw = self.reports.cpu().numpy().tobytes()
        size = ctypes.sizeof(EnsembleReport)
        out = []
        for m in range(self.n_members):
            r = EnsembleReport.from_buffer_copy(raw[m * size:(m + 1) * size])
            out.append({"status": r.status, "newton_its": r.newton_its, "lin_its": r.lin_its,
                        "substeps": r.substeps, "cuts": r.cuts, "steps_done": r.steps_done,
                        "cell_newton_its": r.cell_newton_its, "cnv": list(r.cnv), "mb": list(r.mb)})
        return out

    def states(self):
        return [t.detach().cpu().numpy().copy() for t in self.y]


# ------------------------------------------------ learned Newton initial guess
GUESS_CH = _cases.GUESS_CH
GUESS_LAYER_W = _cases.GUESS_LAYER_W
GUESS_LAYER = _cases.GUESS_LAYER
GUESS_PARAMS = _cases.GUESS_PARAMS

EXPORTS += ["opm_guess_pack_weights", "opm_guess_conv", "opm_guess_conv_backward_bytes",
            "opm_guess_conv_backward", "opm_guess_features", "opm_guess_work_bytes",
            "opm_guess_infer", "opm_guess_train_step", "opm_guess_select", "opm_advance_guess"]


class GuessNetStruct(ctypes.Structure):
    _fields_ = [("nx", _i32), ("ny", _i32), ("nz", _i32), ("pad", _i32), ("cell_box", _vp),
                ("perm_h", _vp), ("master", _vp), ("wbf16", _vp)]


def _guess_lib():
    L = lib()
    if not getattr(L, "_guess_ready", False):
        P = ctypes.POINTER(Problem)
        N = ctypes.POINTER(GuessNetStruct)
        sz = ctypes.c_size_t
        L.opm_guess_pack_weights.argtypes = [_vp, _vp, _vp]
        L.opm_guess_conv.argtypes = [_i32, _i32, _i32, _vp, _vp, _vp, _i32, _vp, _vp, _vp]
        L.opm_guess_conv_backward_bytes.argtypes = [_i32, _i32, _i32]
        L.opm_guess_conv_backward_bytes.restype = sz
        L.opm_guess_conv_backward.argtypes = [_i32, _i32, _i32, _vp, _vp, _vp, _vp, _vp, _vp,
                                              _vp, sz, _vp]
        L.opm_guess_features.argtypes = [P, N, _vp, _vp, _vp, _vp]
        L.opm_guess_work_bytes.argtypes = [P, N]
        L.opm_guess_work_bytes.restype = sz
        L.opm_guess_infer.argtypes = [P, N, _vp, _vp, _vp, _vp, _vp]
        L.opm_guess_train_step.argtypes = [P, N, _vp, _vp, _vp, _vp, _vp, _i32, ctypes.c_float,
                                           _vp, _vp, _vp]
        L.opm_guess_select.argtypes = [P, _vp, _vp, _vp, ctypes.c_double, _vp, _ip, _dp, _vp]
        L.opm_advance_guess.argtypes = [P, _vp, _vp, ctypes.c_double, ctypes.POINTER(NewtonOpts),
                                        N, _vp, _vp, _vp, _vp, ctypes.POINTER(NewtonReport), _ip,
                                        _vp]
        L._guess_ready = True
    return L


def guess_act_rows(nx, ny, nz) -> int:
    """Rows of a BF16 activation buffer: the box padded to 16 cells."""
    return (nx * ny * nz + 15) // 16 * 16


def guess_pack_weights(master: torch.Tensor, wbf16: torch.Tensor) -> None:
    _check(_guess_lib().opm_guess_pack_weights(_ptr(master), _ptr(wbf16), _stream()),
           "opm_guess_pack_weights")


def guess_conv(shape, x: torch.Tensor, w_fwd: torch.Tensor, bias: torch.Tensor, relu: bool):
    """One layer on the box (nz, ny, nx): BF16 out (int16 view) if relu, else FP32."""
    nz, ny, nx = shape
    rows = guess_act_rows(nx, ny, nz)
    if relu:
        out = torch.zeros((rows, GUESS_CH), dtype=torch.int16, device=x.device)
        args = (_ptr(out), None)
    else:
        out = torch.zeros((rows, GUESS_CH), dtype=torch.float32, device=x.device)
        args = (None, _ptr(out))
    _check(_guess_lib().opm_guess_conv(nx, ny, nz, _ptr(x), _ptr(w_fwd), _ptr(bias), int(relu),
                                       *args, _stream()), "opm_guess_conv")
    return out


def guess_conv_backward(shape, x, dout, w_bwd=None, act_in=None):
    """(grad [27*16*16 + 16] FP32, din BF16 or None) of one layer."""
    nz, ny, nx = shape
    L = _guess_lib()
    nbytes = L.opm_guess_conv_backward_bytes(nx, ny, nz)
    work = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=x.device)
    grad = torch.zeros(GUESS_LAYER, dtype=torch.float32, device=x.device)
    din = None
    if w_bwd is not None:
        din = torch.zeros((guess_act_rows(nx, ny, nz), GUESS_CH), dtype=torch.int16,
                          device=x.device)
    _check(L.opm_guess_conv_backward(nx, ny, nz, _ptr(x), _ptr(dout), _ptr(w_bwd), _ptr(act_in),
                                     _ptr(din), _ptr(grad), _ptr(work), nbytes, _stream()),
           "opm_guess_conv_backward")
    return grad, din


class GuessNet:
    """Parameters of the learned guess on the device: FP32 master copy, BF16
    operand copies and Adam moments."""

    def __init__(self, params: Optional[np.ndarray] = None, seed: int = 0, device="cuda"):
        init()
        p = _cases.guess_init_params(seed) if params is None else np.asarray(params, np.float32)
        if p.shape != (GUESS_PARAMS,):
            raise ValueError("guess parameters must have %d entries" % GUESS_PARAMS)
        self.dev = torch.device(device)
        self.master = torch.from_numpy(p.copy()).to(self.dev)
        self.wbf16 = torch.zeros(2 * 3 * GUESS_LAYER_W, dtype=torch.int16, device=self.dev)
        self.adam_m = torch.zeros(GUESS_PARAMS, dtype=torch.float32, device=self.dev)
        self.adam_v = torch.zeros(GUESS_PARAMS, dtype=torch.float32, device=self.dev)
        self.step = 0
        guess_pack_weights(self.master, self.wbf16)

    def params(self) -> np.ndarray:
        return self.master.detach().cpu().numpy().copy()

    def w_fwd(self, layer):
        return self.wbf16[layer * GUESS_LAYER_W:(layer + 1) * GUESS_LAYER_W]

    def w_bwd(self, layer):
        base = 3 * GUESS_LAYER_W
        return self.wbf16[base + layer * GUESS_LAYER_W:base + (layer + 1) * GUESS_LAYER_W]

    def bias(self, layer):
        return self.master[layer * GUESS_LAYER + GUESS_LAYER_W:(layer + 1) * GUESS_LAYER]

    def struct(self, model: "GpuModel") -> GuessNetStruct:
        c = model.case
        return GuessNetStruct(nx=c.nx, ny=c.ny, nz=c.nz, pad=0,
                              cell_box=model.t["cell_box"].data_ptr(),
                              perm_h=model.perm_h.data_ptr(), master=self.master.data_ptr(),
                              wbf16=self.wbf16.data_ptr())


def _model_guess_work(model, net):
    s = net.struct(model)
    nbytes = _guess_lib().opm_guess_work_bytes(model._pbp(), ctypes.byref(s))
    if nbytes == 0:
        raise OpmError(EINVAL, "opm_guess_work_bytes")
    return s, model.workspace("guess", nbytes)
