"""C-ABI library: exports and host-side set-up (no GPU needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from paper_1910_06059_amd import cases

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _opm():
    from paper_1910_06059_amd import opm
    try:
        opm.lib()
    except ImportError as e:
        pytest.fail(f"library not built: {e}")
    return opm


def test_header_declarations_are_exported():
    """Every function declared in include/opm_gpu.h is exported by the library."""
    opm = _opm()
    src = open(os.path.join(ROOT, "include", "opm_gpu.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = set(re.findall(r"\b(opm_[a-z0-9_]+)\s*\(", src))
    assert len(names) >= 20
    L = opm.lib()
    missing = [nm for nm in sorted(names) if not hasattr(L, nm)]
    assert not missing, missing
    assert set(opm.EXPORTS) <= names


def test_strerror_and_options():
    opm = _opm()
    L = opm.lib()
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert L.opm_strerror(code)
    assert L.opm_set_option(opm.OPT_SWEEP_MODE, 7) == opm.EINVAL
    assert L.opm_set_option(999, 0) == opm.EINVAL
    assert L.opm_set_option(opm.OPT_SWEEP_MODE, -1) == opm.OK


def _topology(case):
    opm = _opm()
    L = opm.lib()
    mask = np.ascontiguousarray(case.mask, dtype=np.uint8).ravel()
    n, nf = ctypes.c_int32(), ctypes.c_int32()
    assert L.opm_topology_count(case.nx, case.ny, case.nz, mask.ctypes.data, ctypes.byref(n),
                                ctypes.byref(nf)) == 0
    n, nf = n.value, nf.value
    nnzb = n + 2 * nf
    sizes = dict(cell_box=n, face_cells=2 * nf, face_dir=nf, row_ptr=n + 1, col_idx=nnzb,
                 blk_face=nnzb, diag_pos=n, level_ptr=n + 1, perm=n, iperm=n, lo_blk=3 * n,
                 lo_tblk=3 * n, lo_pos=3 * n, up_blk=3 * n, up_pos=3 * n)
    h = {k: np.zeros(max(v, 1), np.int32) for k, v in sizes.items()}
    topo = opm.Topology(**{k: a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)) for k, a in h.items()})
    assert L.opm_topology_build(case.nx, case.ny, case.nz, mask.ctypes.data, ctypes.byref(topo)) == 0
    return n, nf, h, topo


@pytest.mark.parametrize("make", [
    lambda: cases.box_case(4, 3, 2, seed=1),
    lambda: cases.box_case(7, 1, 1, seed=1),
    lambda: cases.config1(),
    lambda: cases.box_case(6, 5, 4, seed=2, mask=np.random.default_rng(5).random((4, 5, 6)) > 0.35,
                           wells=[]),
], ids=["box", "chain", "C1", "masked"])
def test_topology_matches_oracle(make):
    """The library's host set-up numbers cells, faces and the block pattern
    exactly as the oracle's independent code does; the level schedule is a
    valid topological order of the lower-triangular dependency graph."""
    case = make()
    n, nf, h, topo = _topology(case)
    m = oracle.Model(case)
    g = m.geometry()
    assert n == m.n and nf == m.nf
    assert np.array_equal(h["cell_box"][:n], g["cell_box"])
    assert np.array_equal(h["face_cells"][:2 * nf].reshape(-1, 2), g["face_cells"])
    rp, ci = m.pattern()
    assert np.array_equal(h["row_ptr"][:n + 1], rp)
    assert np.array_equal(h["col_idx"][:n + 2 * nf], ci)
    # diagonal positions and face of every off-diagonal block
    for i in range(n):
        assert ci[h["diag_pos"][i]] == i
        for q in range(rp[i], rp[i + 1]):
            f = h["blk_face"][q]
            if ci[q] == i:
                assert f == -1
            else:
                assert sorted(g["face_cells"][f]) == sorted([i, ci[q]])
    # level schedule: permutation, levels strictly after all lower neighbours
    L = topo.n_levels
    lp = h["level_ptr"][:L + 1]
    perm = h["perm"][:n]
    assert lp[0] == 0 and lp[-1] == n and np.all(np.diff(lp) > 0)
    assert np.array_equal(np.sort(perm), np.arange(n))
    assert np.array_equal(h["iperm"][perm], np.arange(n))
    level = np.zeros(n, int)
    for l in range(L):
        level[perm[lp[l]:lp[l + 1]]] = l
        assert np.all(np.diff(perm[lp[l]:lp[l + 1]]) > 0)
    # levels are the non-empty hyperplanes i + j + k in increasing order, and
    # every lower neighbour lies on the previous level
    hyper = np.array([b % case.nx + (b // case.nx) % case.ny + b // (case.nx * case.ny)
                      for b in g["cell_box"]])
    assert np.array_equal(np.unique(hyper, return_inverse=True)[1], level)
    for i in range(n):
        lower = [ci[q] for q in range(rp[i], rp[i + 1]) if ci[q] < i]
        assert all(level[k] == level[i] - 1 for k in lower)
    assert topo.max_level == np.diff(lp).max()
    # sweep index tables
    for pos in range(n):
        i = perm[pos]
        lower = [q for q in range(rp[i], rp[i + 1]) if ci[q] < i]
        upper = [q for q in range(rp[i], rp[i + 1]) if ci[q] > i]
        lb = h["lo_blk"][3 * pos:3 * pos + 3]
        assert list(lb[:len(lower)]) == lower and np.all(lb[len(lower):] == -1)
        for s, q in enumerate(lower):
            k = ci[q]
            assert h["lo_pos"][3 * pos + s] == h["iperm"][k]
            tq = h["lo_tblk"][3 * pos + s]
            assert ci[tq] == i and rp[k] <= tq < rp[k + 1]
        ub = h["up_blk"][3 * pos:3 * pos + 3]
        assert list(ub[:len(upper)]) == upper and np.all(ub[len(upper):] == -1)
        for s, q in enumerate(upper):
            assert h["up_pos"][3 * pos + s] == h["iperm"][ci[q]]


def test_topology_levels_are_hyperplanes():
    """On a full box every lower neighbour sits on the previous level, so the
    levels are the hyperplanes i + j + k = const: nx + ny + nz - 2 of them."""
    case = cases.box_case(5, 4, 3, seed=0)
    n, nf, h, topo = _topology(case)
    assert topo.n_levels == 5 + 4 + 3 - 2
    lp = h["level_ptr"]
    for l in range(topo.n_levels):
        for c in h["perm"][lp[l]:lp[l + 1]]:
            b = h["cell_box"][c]
            assert b % 5 + (b // 5) % 4 + b // 20 == l


def test_topology_edge_cases():
    opm = _opm()
    L = opm.lib()
    n, nf = ctypes.c_int32(), ctypes.c_int32()
    assert L.opm_topology_count(0, 1, 1, None, ctypes.byref(n), ctypes.byref(nf)) == opm.EINVAL
    mask = np.zeros(8, np.uint8)
    assert L.opm_topology_count(2, 2, 2, mask.ctypes.data, ctypes.byref(n), ctypes.byref(nf)) == 0
    assert n.value == 0 and nf.value == 0
    n1, nf1, h, topo = _topology(cases.box_case(1, 1, 1, wells=[]))
    assert n1 == 1 and nf1 == 0 and topo.n_levels == 1
    # a connection in a cell index out of range is rejected by the grouping
    ccp = np.zeros(3, np.int32)
    cc = np.zeros(1, np.int32)
    bad = np.array([5], np.int32)
    assert L.opm_well_groups(2, 1, bad.ctypes.data, ccp.ctypes.data, cc.ctypes.data) == opm.EINVAL
    good = np.array([1, 0, 1], np.int32)
    ccp = np.zeros(3, np.int32)
    cc = np.zeros(3, np.int32)
    assert L.opm_well_groups(2, 3, good.ctypes.data, ccp.ctypes.data, cc.ctypes.data) == 0
    assert list(ccp) == [0, 1, 3] and list(cc) == [1, 0, 2]


def test_invalid_problem_rejected_without_gpu():
    """Argument checks happen on the host before any device work."""
    opm = _opm()
    L = opm.lib()
    pb = opm.Problem()
    pb.n_cells, pb.n_faces, pb.nnzb = 4, 1, 5   # nnzb must be n + 2 nf = 6
    R = ctypes.c_void_p(1)
    assert L.opm_assemble(ctypes.byref(pb), R, R, 1.0, R, R, None, None) == opm.EINVAL
    pb.nnzb = 6   # consistent sizes but null device arrays
    assert L.opm_assemble(ctypes.byref(pb), R, R, 1.0, R, R, None, None) == opm.EINVAL
    assert L.opm_newton_bytes(None, 0) == 0
