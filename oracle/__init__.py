"""Plain FP64 CPU oracle of the TPFA black-oil Newton path (ctypes wrapper).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py``.  The GPU library never calls it.
The C sources (``oracle.c``) are compiled with gcc into ``liboracle.so``
next to this file; ``build()`` recompiles them.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SOURCES = [os.path.join(_HERE, "oracle.c")]
_libs = {}

OK, EINVAL, ESINGULAR, ENOTCONV, EBREAKDOWN, ENONFINITE = 0, -1, -2, -3, -4, -5

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)
_u8p = ctypes.POINTER(ctypes.c_uint8)


class Fluid(ctypes.Structure):
    _fields_ = [("rho_s", ctypes.c_double * 3), ("c", ctypes.c_double * 3),
                ("p_ref", ctypes.c_double), ("mu", ctypes.c_double * 3),
                ("swc", ctypes.c_double), ("n_corey", ctypes.c_double), ("g", ctypes.c_double),
                ("rs_c", ctypes.c_double), ("bo_r", ctypes.c_double), ("muo_r", ctypes.c_double),
                ("eps_switch", ctypes.c_double), ("live", ctypes.c_int), ("pad", ctypes.c_int),
                ("rv_c", ctypes.c_double)]


class Opts(ctypes.Structure):
    _fields_ = [("tol_cnv", ctypes.c_double), ("tol_mb", ctypes.c_double),
                ("ds_max", ctypes.c_double), ("dp_max_rel", ctypes.c_double),
                ("lin_rtol", ctypes.c_double), ("max_newton", ctypes.c_int),
                ("lin_maxit", ctypes.c_int), ("max_cuts", ctypes.c_int),
                ("krylov", ctypes.c_int), ("restart", ctypes.c_int),
                ("precond", ctypes.c_int), ("pad", ctypes.c_int)]


class Report(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("newton_its", ctypes.c_int),
                ("substeps", ctypes.c_int), ("cuts", ctypes.c_int),
                ("lin_its", ctypes.c_double), ("cnv", ctypes.c_double * 3),
                ("mb", ctypes.c_double * 3), ("mass_err", ctypes.c_double * 3),
                ("t_assemble", ctypes.c_double), ("t_factor", ctypes.c_double),
                ("t_krylov", ctypes.c_double), ("t_update", ctypes.c_double),
                ("cell_newton_its", ctypes.c_double)]

    def as_dict(self):
        return {"status": self.status, "newton_its": self.newton_its, "substeps": self.substeps,
                "cuts": self.cuts, "lin_its": self.lin_its, "cnv": list(self.cnv),
                "mb": list(self.mb), "mass_err": list(self.mass_err),
                "t_assemble": self.t_assemble, "t_factor": self.t_factor,
                "t_krylov": self.t_krylov, "t_update": self.t_update,
                "cell_newton_its": self.cell_newton_its}


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc (plain -O2, IEEE semantics, single thread)."""
    if not force and os.path.exists(_LIB_PATH) and all(
            os.path.getmtime(_LIB_PATH) >= os.path.getmtime(s) for s in _SOURCES
            + [os.path.join(_HERE, "oracle.h")]):
        return _LIB_PATH
    tmp = _LIB_PATH + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fPIC", "-shared", "-o", tmp] + _SOURCES + ["-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_BASELINE_PATH = os.path.join(_HERE, "liboracle_omp.so")


def build_baseline(path: Optional[str] = None) -> str:
    """Compile the same sources as the CPU baseline: -O3 -march=native for
    the host it runs on, OpenMP over the cells of the accumulation, the
    faces of the flux evaluation and the rows of the Jacobian product, and
    no floating-point contraction, so that it computes the plain build's
    bits with any number of threads."""
    out = path or _BASELINE_PATH
    tmp = out + ".tmp"
    cmd = ["gcc", "-O3", "-march=native", "-ffp-contract=off", "-fopenmp", "-std=c11",
           "-D_GNU_SOURCE", "-fPIC", "-shared", "-o", tmp] + _SOURCES + ["-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def set_threads(n: int, lib_path: Optional[str] = None) -> int:
    """Threads of an OpenMP build (the plain build stays at one); returns the
    number the library will use."""
    L = lib(lib_path)
    L.ora_set_threads(int(n))
    return int(L.ora_threads())


def lib(path: Optional[str] = None):
    """Load the oracle library (``path`` selects another build of the same
    sources, e.g. a deliberately mutated copy used by the pin tests)."""
    key = path or _LIB_PATH
    if key not in _libs:
        if path is None:
            build(force=False)
        L = ctypes.CDLL(key)
        L.ora_create.restype = ctypes.c_void_p
        L.ora_create.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                 ctypes.c_double, _dp, _dp, ctypes.c_double, _dp, _u8p,
                                 ctypes.POINTER(Fluid), ctypes.c_int, _ip, _ip, _dp, _dp, _ip, _ip]
        L.ora_destroy.argtypes = [ctypes.c_void_p]
        for name in ("ora_n_cells", "ora_n_faces", "ora_nnzb", "ora_n_conns"):
            getattr(L, name).argtypes = [ctypes.c_void_p]
            getattr(L, name).restype = ctypes.c_int
        L.ora_geometry.argtypes = [ctypes.c_void_p, _ip, _dp, _dp, _dp, _ip]
        L.ora_pattern.argtypes = [ctypes.c_void_p, _ip, _ip]
        L.ora_conns.argtypes = [ctypes.c_void_p, _ip, _dp, _ip]
        L.ora_accumulation.argtypes = [ctypes.c_void_p, _dp, _dp]
        L.ora_well_rates.argtypes = [ctypes.c_void_p, _dp, _dp]
        L.ora_assemble.argtypes = [ctypes.c_void_p, _dp, _dp, ctypes.c_double, _dp, _dp]
        L.ora_norms.argtypes = [ctypes.c_void_p, _dp, _dp, ctypes.c_double, _dp, _dp]
        L.ora_ilu0.argtypes = [ctypes.c_void_p, _dp, _dp]
        L.ora_ilu0_apply.argtypes = [ctypes.c_void_p, _dp, _dp, _dp]
        L.ora_set_ilu_blocks.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.ora_set_ilu_blocks.restype = ctypes.c_int
        L.ora_spmv.argtypes = [ctypes.c_void_p, _dp, _dp, _dp]
        L.ora_gmres.argtypes = [ctypes.c_void_p, _dp, _dp, _dp, _dp, ctypes.c_double, ctypes.c_int,
                                ctypes.c_int, _dp, _dp]
        L.ora_gmres.restype = ctypes.c_int
        L.ora_bicgstab.argtypes = [ctypes.c_void_p, _dp, _dp, _dp, _dp, ctypes.c_double,
                                   ctypes.c_int, _dp, _dp]
        L.ora_newton_step.argtypes = [ctypes.c_void_p, _dp, _dp, ctypes.c_double,
                                      ctypes.POINTER(Opts), ctypes.POINTER(Report)]
        L.ora_advance.argtypes = [ctypes.c_void_p, _dp, ctypes.c_double, ctypes.POINTER(Opts),
                                  ctypes.POINTER(Report)]
        L.ora_advance_log.argtypes = [ctypes.c_void_p, _dp, ctypes.c_double, ctypes.POINTER(Opts),
                                      ctypes.POINTER(Report), _dp, _ip, ctypes.c_int, _ip]
        L.ora_dense_solve.argtypes = [ctypes.c_int, _dp, _dp]
        L.ora_set_threads.argtypes = [ctypes.c_int]
        L.ora_threads.restype = ctypes.c_int
        L.ora_set_standard_wells.argtypes = [ctypes.c_void_p, _dp, _dp, _dp]
        L.ora_get_well_ctrl.argtypes = [ctypes.c_void_p, _ip]
        L.ora_set_well_ctrl.argtypes = [ctypes.c_void_p, _ip]
        L.ora_set_standard_wells.restype = ctypes.c_int
        L.ora_get_well_state.argtypes = [ctypes.c_void_p, _dp]
        L.ora_set_well_state.argtypes = [ctypes.c_void_p, _dp]
        L.ora_well_storage_start.argtypes = [ctypes.c_void_p]
        L.ora_well_system.argtypes = [ctypes.c_void_p, _dp, ctypes.c_double, _dp, _dp, _dp, _dp]
        L.ora_well_system.restype = ctypes.c_int
        L.ora_schur_solve.argtypes = [ctypes.c_void_p, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp,
                                      ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                      _dp, _dp]
        L.ora_schur_solve.restype = ctypes.c_int
        vp = ctypes.c_void_p
        L.ora_cpr_setup.argtypes = [vp, _dp, ctypes.POINTER(vp)]
        L.ora_cpr_setup.restype = ctypes.c_int
        L.ora_cpr_destroy.argtypes = [vp]
        L.ora_cpr_levels.argtypes = [vp]
        L.ora_cpr_levels.restype = ctypes.c_int
        L.ora_cpr_level_size.argtypes = [vp, ctypes.c_int, _ip, _ip]
        L.ora_cpr_level.argtypes = [vp, ctypes.c_int, _ip, _ip, _dp, _ip]
        L.ora_cpr_weights.argtypes = [vp, _dp]
        L.ora_cpr_vcycle.argtypes = [vp, _dp, _dp]
        L.ora_cpr_apply.argtypes = [vp, vp, _dp, _dp, _dp, _dp]
        L.ora_bicgstab_cpr.argtypes = [vp, _dp, _dp, vp, _dp, _dp, ctypes.c_double, ctypes.c_int,
                                       _dp, _dp]
        L.ora_bicgstab_cpr.restype = ctypes.c_int
        L.ora_set_meaning.argtypes = [ctypes.c_void_p, _u8p]
        L.ora_set_meaning.restype = ctypes.c_int
        L.ora_get_meaning.argtypes = [ctypes.c_void_p, _u8p]
        _libs[key] = L
    return _libs[key]


def _d(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_dp)


def _i(a: np.ndarray):
    assert a.dtype == np.int32 and a.flags.c_contiguous
    return a.ctypes.data_as(_ip)


def default_opts(case=None, **kw) -> Opts:
    o = Opts(tol_cnv=1e-8, tol_mb=1e-11, ds_max=0.2, dp_max_rel=0.3, lin_rtol=1e-6,
             max_newton=20, lin_maxit=500, max_cuts=8, krylov=0, restart=30, precond=0)
    if case is not None:
        o.tol_cnv, o.tol_mb, o.lin_rtol = case.tol_cnv, case.tol_mb, case.lin_rtol
    for k, v in kw.items():
        setattr(o, k, v)
    return o


class Model:
    """Oracle model of one case (owns the C handle)."""

    def __init__(self, case, lib_path: Optional[str] = None):
        L = lib(lib_path)
        f = case.fluid
        self.fluid = Fluid((ctypes.c_double * 3)(*f.rho_s), (ctypes.c_double * 3)(*f.c), f.p_ref,
                           (ctypes.c_double * 3)(*f.mu), f.swc, f.n_corey, f.g,
                           getattr(f, "rs_c", 0.0), getattr(f, "bo_r", 0.0),
                           getattr(f, "muo_r", 0.0), getattr(f, "eps_switch", 0.0),
                           int(getattr(f, "live", False)), 0, getattr(f, "rv_c", 0.0))
        dz = np.ascontiguousarray(case.dz, dtype=np.float64)
        perm = np.ascontiguousarray(case.perm_h, dtype=np.float64).ravel()
        poro = np.ascontiguousarray(case.poro, dtype=np.float64).ravel()
        mask = np.ascontiguousarray(case.mask, dtype=np.uint8).ravel()
        nw = len(case.wells)
        kind = np.array([w.kind for w in case.wells] + [0], dtype=np.int32)
        phase = np.array([w.phase for w in case.wells] + [0], dtype=np.int32)
        target = np.array([w.target for w in case.wells] + [0.0], dtype=np.float64)
        rw = np.array([w.rw for w in case.wells] + [1.0], dtype=np.float64)
        nconn = np.array([len(w.cells) for w in case.wells] + [0], dtype=np.int32)
        ijk = np.array([c for w in case.wells for c in w.cells] + [(0, 0, 0)], dtype=np.int32)
        self._keep = (dz, perm, poro, mask, kind, phase, target, rw, nconn, ijk)
        h = L.ora_create(case.nx, case.ny, case.nz, case.dx, case.dy, _d(dz), _d(perm), case.kv_kh,
                         _d(poro), mask.ctypes.data_as(_u8p), ctypes.byref(self.fluid), nw,
                         _i(kind), _i(phase), _d(target), _d(rw), _i(nconn), _i(ijk))
        if not h:
            raise ValueError("oracle: invalid case")
        self.h = ctypes.c_void_p(h)
        self.L = L
        self.case = case
        self.n = L.ora_n_cells(self.h)
        self.nf = L.ora_n_faces(self.h)
        self.nnzb = L.ora_nnzb(self.h)
        self.nc = L.ora_n_conns(self.h)
        if hasattr(case, "initial_meaning"):
            self.set_meaning(case.initial_meaning())
        self.nw = nw
        self.std_wells = bool(getattr(case, "standard_wells", False))
        if self.std_wells:
            vol, x0 = case.standard_well_init()
            lim = np.ascontiguousarray(case.standard_well_limits(), dtype=np.float64)
            st = L.ora_set_standard_wells(self.h, _d(np.ascontiguousarray(vol, dtype=np.float64)),
                                          _d(np.ascontiguousarray(x0, dtype=np.float64)),
                                          _d(lim))
            if st != OK:
                raise ValueError("oracle: invalid standard wells")

    def __del__(self):
        try:
            self.L.ora_destroy(self.h)
        except Exception:
            pass

    # ---- geometry / pattern
    def geometry(self):
        fc = np.zeros((max(self.nf, 1), 2), np.int32)
        T = np.zeros(max(self.nf, 1))
        pv = np.zeros(self.n)
        z = np.zeros(self.n)
        cb = np.zeros(self.n, np.int32)
        self.L.ora_geometry(self.h, _i(fc), _d(T), _d(pv), _d(z), _i(cb))
        return {"face_cells": fc[:self.nf], "trans": T[:self.nf], "pore_vol": pv, "depth": z,
                "cell_box": cb}

    def pattern(self):
        rp = np.zeros(self.n + 1, np.int32)
        ci = np.zeros(self.nnzb, np.int32)
        self.L.ora_pattern(self.h, _i(rp), _i(ci))
        return rp, ci

    def conns(self):
        cell = np.zeros(max(self.nc, 1), np.int32)
        wi = np.zeros(max(self.nc, 1))
        well = np.zeros(max(self.nc, 1), np.int32)
        self.L.ora_conns(self.h, _i(cell), _d(wi), _i(well))
        return cell[:self.nc], wi[:self.nc], well[:self.nc]

    # ---- CPR-AMG (two-stage preconditioner with an aggregation AMG)
    def cpr(self, J) -> "Cpr":
        return Cpr(self, J)

    # ---- state: meaning of the third variable per cell (0 s_g, 1 r_go)
    def set_meaning(self, mean):
        mean = np.ascontiguousarray(mean, dtype=np.uint8)
        assert mean.shape == (self.n,)
        st = self.L.ora_set_meaning(self.h, mean.ctypes.data_as(_u8p))
        if st != OK:
            raise ValueError("oracle: invalid variable meaning")

    def meaning(self) -> np.ndarray:
        out = np.zeros(max(self.n, 1), np.uint8)
        self.L.ora_get_meaning(self.h, out.ctypes.data_as(_u8p))
        return out[:self.n]

    # ---- standard wells (well unknowns Q_t, F_w, F_g, p_bhp per well)
    def well_state(self) -> np.ndarray:
        x = np.zeros((max(self.nw, 1), 4))
        self.L.ora_get_well_state(self.h, _d(x))
        return x[:self.nw]

    def set_well_state(self, x):
        self.L.ora_set_well_state(self.h, _d(np.ascontiguousarray(x, dtype=np.float64)))

    def well_ctrl(self) -> np.ndarray:
        """Active control per well: 0 its own, 1 its limit."""
        c = np.zeros(max(self.nw, 1), np.int32)
        self.L.ora_get_well_ctrl(self.h, _i(c))
        return c[:self.nw]

    def set_well_ctrl(self, c):
        self.L.ora_set_well_ctrl(self.h, _i(np.ascontiguousarray(c, dtype=np.int32)))

    def well_storage_start(self):
        self.L.ora_well_storage_start(self.h)

    def well_system(self, y, dt):
        y = np.ascontiguousarray(y, dtype=np.float64)
        Rw = np.zeros((self.nw, 4))
        B = np.zeros((max(self.nc, 1), 4, 3))
        C = np.zeros((max(self.nc, 1), 3, 4))
        D = np.zeros((self.nw, 4, 4))
        st = self.L.ora_well_system(self.h, _d(y), dt, _d(Rw), _d(B), _d(C), _d(D))
        return st, Rw, B[:self.nc], C[:self.nc], D

    def schur_solve(self, J, F, B, C, D, Rr, Rw, rtol=1e-10, maxit=500, krylov=0, restart=30):
        xr = np.zeros((self.n, 3))
        xw = np.zeros((self.nw, 4))
        its = ctypes.c_double()
        rr = ctypes.c_double()
        f = lambda a: _d(np.ascontiguousarray(a, dtype=np.float64))
        st = self.L.ora_schur_solve(self.h, f(J), f(F), f(B), f(C), f(D), f(Rr), f(Rw), _d(xr),
                                    _d(xw), rtol, maxit, krylov, restart, ctypes.byref(its),
                                    ctypes.byref(rr))
        return st, xr, xw, its.value

    # ---- path steps
    def accumulation(self, y):
        y = np.ascontiguousarray(y, dtype=np.float64)
        acc = np.zeros((self.n, 3))
        self.L.ora_accumulation(self.h, _d(y), _d(acc))
        return acc

    def well_rates(self, y):
        y = np.ascontiguousarray(y, dtype=np.float64)
        q = np.zeros((self.n, 3))
        self.L.ora_well_rates(self.h, _d(y), _d(q))
        return q

    def assemble(self, y, acc0, dt, jacobian=True):
        y = np.ascontiguousarray(y, dtype=np.float64)
        acc0 = np.ascontiguousarray(acc0, dtype=np.float64)
        R = np.zeros((self.n, 3))
        J = np.zeros((self.nnzb, 3, 3)) if jacobian else None
        st = self.L.ora_assemble(self.h, _d(y), _d(acc0), dt, _d(R),
                                 _d(J) if jacobian else ctypes.cast(None, _dp))
        return st, R, J

    def norms(self, y, R, dt):
        cnv = np.zeros(3)
        mb = np.zeros(3)
        self.L.ora_norms(self.h, _d(np.ascontiguousarray(y)), _d(np.ascontiguousarray(R)), dt,
                         _d(cnv), _d(mb))
        return cnv, mb

    def set_ilu_blocks(self, bx: int, by: int, bz: int):
        """Block ILU0 over boxes of bx x by x bz cells (0, 0, 0: one block)."""
        st = self.L.ora_set_ilu_blocks(self.h, bx, by, bz)
        if st != OK:
            raise ValueError(f"oracle: invalid ILU blocks {(bx, by, bz)}")

    def ilu0(self, J):
        F = np.zeros_like(J)
        st = self.L.ora_ilu0(self.h, _d(np.ascontiguousarray(J)), _d(F))
        return st, F

    def ilu0_apply(self, F, r):
        x = np.zeros((self.n, 3))
        self.L.ora_ilu0_apply(self.h, _d(F), _d(np.ascontiguousarray(r, dtype=np.float64)), _d(x))
        return x

    def spmv(self, J, x):
        y = np.zeros((self.n, 3))
        self.L.ora_spmv(self.h, _d(J), _d(np.ascontiguousarray(x, dtype=np.float64)), _d(y))
        return y

    def bicgstab(self, J, F, b, rtol=1e-6, maxit=500):
        x = np.zeros((self.n, 3))
        its = ctypes.c_double()
        rr = ctypes.c_double()
        st = self.L.ora_bicgstab(self.h, _d(J), _d(F), _d(np.ascontiguousarray(b, dtype=np.float64)),
                                 _d(x), rtol, maxit, ctypes.byref(its), ctypes.byref(rr))
        return st, x, its.value, rr.value

    def gmres(self, J, F, b, rtol=1e-6, maxit=500, restart=30):
        x = np.zeros((self.n, 3))
        its = ctypes.c_double()
        rr = ctypes.c_double()
        st = self.L.ora_gmres(self.h, _d(J), _d(F), _d(np.ascontiguousarray(b, dtype=np.float64)),
                              _d(x), rtol, maxit, restart, ctypes.byref(its), ctypes.byref(rr))
        return st, x, its.value, rr.value

    def newton_step(self, y, y_prev, dt, opts: Optional[Opts] = None):
        y = np.array(y, dtype=np.float64, order="C")
        yp = np.ascontiguousarray(y_prev, dtype=np.float64)
        rep = Report()
        o = opts or default_opts(self.case)
        st = self.L.ora_newton_step(self.h, _d(y), _d(yp), dt, ctypes.byref(o), ctypes.byref(rep))
        return st, y, rep

    def advance(self, y, dt, opts: Optional[Opts] = None):
        y = np.array(y, dtype=np.float64, order="C")
        rep = Report()
        o = opts or default_opts(self.case)
        st = self.L.ora_advance(self.h, _d(y), dt, ctypes.byref(o), ctypes.byref(rep))
        return st, y, rep

    def advance_log(self, y, dt, opts: Optional[Opts] = None, cap: int = 4096):
        """advance() that also returns every attempted substep: (status, y,
        report, lengths [k], Newton statuses [k])."""
        y = np.array(y, dtype=np.float64, order="C")
        rep = Report()
        o = opts or default_opts(self.case)
        dts = np.zeros(cap)
        sts = np.zeros(cap, np.int32)
        n = ctypes.c_int()
        st = self.L.ora_advance_log(self.h, _d(y), dt, ctypes.byref(o), ctypes.byref(rep), _d(dts),
                                    _i(sts), cap, ctypes.byref(n))
        k = min(n.value, cap)
        return st, y, rep, dts[:k], sts[:k]

    def run(self, y0=None, n_steps=None, opts=None):
        """Advance over the case's report schedule; returns states after each
        report step (their variable meanings in ``self.run_meanings``).
        Without y0 the run starts from the case's initial state and meaning."""
        if y0 is None:
            y = self.case.initial_state()
            if hasattr(self.case, "initial_meaning"):
                self.set_meaning(self.case.initial_meaning())
            if self.std_wells:
                self.set_well_state(self.case.standard_well_init()[1])
                self.set_well_ctrl(np.zeros(self.nw, np.int32))
        else:
            y = np.array(y0, dtype=np.float64)
        states, reps = [], []
        self.run_meanings = []
        self.run_well_states = []
        self.run_well_ctrls = []
        for dt in self.case.report_dt[:n_steps]:
            st, y, rep = self.advance(y, dt, opts)
            if st != OK:
                raise RuntimeError(f"oracle advance failed with status {st}")
            states.append(y.copy())
            self.run_meanings.append(self.meaning().copy())
            if self.std_wells:
                self.run_well_states.append(self.well_state().copy())
                self.run_well_ctrls.append(self.well_ctrl().copy())
            reps.append(rep.as_dict())
        return states, reps


class Cpr:
    """The oracle's CPR-AMG hierarchy for one Jacobian (owns the C handle)."""

    def __init__(self, model: Model, J):
        self.m = model
        self.L = model.L
        self.J = np.ascontiguousarray(J, dtype=np.float64)
        h = ctypes.c_void_p()
        st = self.L.ora_cpr_setup(model.h, _d(self.J), ctypes.byref(h))
        if st != OK:
            raise ValueError(f"oracle: CPR setup failed ({st})")
        self.h = h
        self.nl = self.L.ora_cpr_levels(h)

    def __del__(self):
        try:
            self.L.ora_cpr_destroy(self.h)
        except Exception:
            pass

    def level(self, l):
        """(rp, ci, a, agg) of level l (agg None on the coarsest)."""
        n, nnz = ctypes.c_int(), ctypes.c_int()
        self.L.ora_cpr_level_size(self.h, l, ctypes.byref(n), ctypes.byref(nnz))
        n, nnz = n.value, nnz.value
        rp = np.zeros(n + 1, np.int32)
        ci = np.zeros(max(nnz, 1), np.int32)
        a = np.zeros(max(nnz, 1))
        agg = np.zeros(max(n, 1), np.int32)
        last = l == self.nl - 1
        self.L.ora_cpr_level(self.h, l, _i(rp), _i(ci), _d(a),
                             ctypes.cast(None, _ip) if last else _i(agg))
        return rp, ci[:nnz], a[:nnz], (None if last else agg[:n])

    def weights(self):
        w = np.zeros((self.m.n, 3))
        self.L.ora_cpr_weights(self.h, _d(w))
        return w

    def vcycle(self, b):
        b = np.ascontiguousarray(b, dtype=np.float64)
        x = np.zeros(self.m.n)
        self.L.ora_cpr_vcycle(self.h, _d(b), _d(x))
        return x

    def apply(self, F, r):
        z = np.zeros((self.m.n, 3))
        self.L.ora_cpr_apply(self.m.h, self.h, _d(self.J), _d(np.ascontiguousarray(F)),
                             _d(np.ascontiguousarray(r, dtype=np.float64)), _d(z))
        return z

    def bicgstab(self, F, b, rtol=1e-6, maxit=500):
        x = np.zeros((self.m.n, 3))
        its = ctypes.c_double()
        rr = ctypes.c_double()
        st = self.L.ora_bicgstab_cpr(self.m.h, _d(self.J), _d(np.ascontiguousarray(F)), self.h,
                                     _d(np.ascontiguousarray(b, dtype=np.float64)), _d(x), rtol,
                                     maxit, ctypes.byref(its), ctypes.byref(rr))
        return st, x, its.value, rr.value


def dense_solve(A: np.ndarray, b: np.ndarray, lib_path: Optional[str] = None) -> np.ndarray:
    A = np.array(A, dtype=np.float64, order="C")
    x = np.array(b, dtype=np.float64, order="C")
    st = lib(lib_path).ora_dense_solve(A.shape[0], _d(A), _d(x))
    if st != OK:
        raise np.linalg.LinAlgError("singular")
    return x
