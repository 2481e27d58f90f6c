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
    assert L.opm_set_option(opm.OPT_PLANE_SWEEP, 2) == opm.EINVAL
    assert L.opm_set_option(opm.OPT_PLANE_SPIN, -1) == opm.EINVAL


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


def _subdomains(case, cell_box, blk):
    """Dense subdomain index of every cell, computed here from the box
    formula: box (i // bx, j // by, k // bz), nonempty boxes numbered in box
    order."""
    nx, ny, nz = case.nx, case.ny, case.nz
    bx, by, bz = (min(b, e) for b, e in zip(blk, (nx, ny, nz)))
    i, j, k = cell_box % nx, (cell_box // nx) % ny, cell_box // (nx * ny)
    nbx, nby = -(-nx // bx), -(-ny // by)
    box = i // bx + nbx * (j // by + nby * (k // bz))
    used = np.unique(box)
    dense = {int(b): q for q, b in enumerate(used)}
    hyper = i % bx + j % by + k % bz
    return np.array([dense[int(b)] for b in box]), hyper, len(used)


@pytest.mark.parametrize("blk", [(2, 3, 2), (3, 2, 5), (1, 1, 1), (20, 20, 20)])
@pytest.mark.parametrize("masked", [False, True])
def test_block_topology(blk, masked):
    """Block ILU0 topology: same connectivity as the single-block one; the
    ILU neighbour lists hold exactly the neighbours in the same subdomain;
    positions ordered by (local hyperplane level, subdomain, cell), each
    lower neighbour of a row on the previous level; the subdomain ranges
    and slots index every row once."""
    opm = _opm()
    mask = np.random.default_rng(8).random((5, 4, 6)) > 0.3 if masked else None
    case = cases.box_case(6, 4, 5, seed=3, mask=mask, wells=[])
    n, nf, h0, t0 = _topology(case)
    n1, nf1, h, topo, b = opm.build_topology(case.nx, case.ny, case.nz, case.mask, blk)
    assert (n1, nf1) == (n, nf)
    for k in ("cell_box", "face_cells", "face_dir", "row_ptr", "col_idx", "blk_face", "diag_pos"):
        assert np.array_equal(h[k], h0[k]), k
    sub, hyper, nsub = _subdomains(case, h["cell_box"][:n], blk)
    assert b.n_sub == nsub
    levels = np.unique(hyper)
    lev_of = {int(v): q for q, v in enumerate(levels)}
    assert topo.n_levels == len(levels)
    perm, iperm, lp = h["perm"][:n], h["iperm"][:n], h["level_ptr"]
    key = [(lev_of[int(hyper[c])], sub[c], c) for c in perm]
    assert key == sorted(key) and np.array_equal(iperm[perm], np.arange(n))
    for l in range(topo.n_levels):
        assert all(key[p][0] == l for p in range(lp[l], lp[l + 1]))
    slp = h["sub_level_ptr"][:topo.n_levels * (nsub + 1)].reshape(topo.n_levels, nsub + 1)
    slot, counts, widths = h["slot"][:n], np.zeros(nsub, int), []
    for l in range(topo.n_levels):
        assert slp[l, 0] == lp[l] and slp[l, nsub] == lp[l + 1]
        for sb in range(nsub):
            rows = range(slp[l, sb], slp[l, sb + 1])
            widths.append(len(rows))
            for q, p in enumerate(rows):
                assert sub[perm[p]] == sb and slot[p] == counts[sb] + q
            counts[sb] += len(rows)
    assert b.max_sub == counts.max() and b.max_width == max(widths)
    rp, ci = h["row_ptr"], h["col_idx"]
    for p in range(n):
        c = perm[p]
        lo = [q for q in range(rp[c], rp[c + 1]) if ci[q] < c and sub[ci[q]] == sub[c]]
        up = [q for q in range(rp[c], rp[c + 1]) if ci[q] > c and sub[ci[q]] == sub[c]]
        assert list(h["lo_blk"][3 * p:3 * p + len(lo)]) == lo
        assert list(h["up_blk"][3 * p:3 * p + len(up)]) == up
        assert (h["lo_blk"][3 * p + len(lo):3 * p + 3] == -1).all()
        assert (h["up_blk"][3 * p + len(up):3 * p + 3] == -1).all()
        for s_, q in enumerate(lo):
            kp = h["lo_pos"][3 * p + s_]
            assert kp == iperm[ci[q]] and key[kp][0] == key[p][0] - 1
            assert ci[h["lo_tblk"][3 * p + s_]] == c
        for s_, q in enumerate(up):
            assert h["up_pos"][3 * p + s_] == iperm[ci[q]]
    if blk == (20, 20, 20):
        for k in ("level_ptr", "perm", "iperm", "lo_blk", "lo_tblk", "lo_pos", "up_blk", "up_pos"):
            assert np.array_equal(h[k], h0[k]), k


def test_block_topology_invalid():
    opm = _opm()
    L = opm.lib()
    ns, nl = ctypes.c_int32(), ctypes.c_int32()
    for blk in [(0, 1, 1), (1, -2, 1), (1, 1, 0)]:
        assert L.opm_ilu_blocks_count(3, 3, 3, None, *blk, ctypes.byref(ns), ctypes.byref(nl)) == opm.EINVAL
        with pytest.raises(opm.OpmError):
            opm.build_topology(3, 3, 3, np.ones((3, 3, 3), np.uint8), blk)
    assert L.opm_ilu_blocks_count(3, 3, 3, None, 2, 2, 2, ctypes.byref(ns), ctypes.byref(nl)) == 0
    assert (ns.value, nl.value) == (8, 4)
    blk = opm.IluBlocks(bx=2, by=2, bz=2)   # NULL output arrays
    t = opm.Topology()
    assert L.opm_topology_build_blocks(3, 3, 3, None, ctypes.byref(blk), ctypes.byref(t)) == opm.EINVAL


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


def test_gmres_sizes_and_option_checks_without_gpu():
    """GMRes workspace sizes and the Krylov option checks are host-only."""
    opm = _opm()
    L = opm.lib()
    pb = opm.Problem()
    pb.n_cells, pb.n_faces, pb.nnzb = 4, 1, 6
    assert L.opm_gmres_bytes(None, 30) == 0
    for bad in (0, -1, opm.GMRES_MAX_RESTART + 1):
        assert L.opm_gmres_bytes(ctypes.byref(pb), bad) == 0
    # restart + 1 basis vectors of 3 n (padded to 32 doubles) at least
    for m in (1, 8, opm.GMRES_MAX_RESTART):
        assert L.opm_gmres_bytes(ctypes.byref(pb), m) >= 8 * 32 * (m + 1)
    assert L.opm_gmres_bytes(ctypes.byref(pb), 8) < L.opm_gmres_bytes(ctypes.byref(pb), 9)
    o = opm.default_opts()
    assert o.krylov == opm.KRYLOV_BICGSTAB
    assert L.opm_newton_work_bytes(ctypes.byref(pb), ctypes.byref(o)) == \
        L.opm_newton_bytes(ctypes.byref(pb), o.precision)
    o.krylov = opm.KRYLOV_GMRES
    assert L.opm_newton_work_bytes(ctypes.byref(pb), ctypes.byref(o)) > \
        L.opm_newton_bytes(ctypes.byref(pb), o.precision)
    for krylov, restart in ((opm.KRYLOV_GMRES, 0), (opm.KRYLOV_GMRES, 33), (2, 30)):
        o.krylov, o.restart = krylov, restart
        assert L.opm_newton_work_bytes(ctypes.byref(pb), ctypes.byref(o)) == 0
    # a solve with restart out of range or null buffers is rejected before any device work
    rep = opm.SolveReport()
    R = ctypes.c_void_p(1)
    for restart in (0, 33):
        assert L.opm_gmres(ctypes.byref(pb), R, R, 0, R, R, 1e-6, 10, restart, R,
                           ctypes.byref(rep), None) == opm.EINVAL


def test_oracle_baseline_build_same_bits(tmp_path):
    """The CPU baseline is the oracle's own sources built with -O3
    -march=native and OpenMP: with one thread and with four it computes the
    plain test build's bits (assembly of the 9000-cell case and a Newton
    step of C1)."""
    import oracle
    from paper_1910_06059_amd import cases
    so = oracle.build_baseline(str(tmp_path / "liboracle_omp.so"))
    c2 = cases.config2()
    y = cases.random_state(c2, seed=3)
    y0 = cases.random_state(c2, seed=4)
    plain = oracle.Model(c2)
    _, R0, J0 = plain.assemble(y, plain.accumulation(y0), 86400.0)
    c1 = cases.config1()
    _, ys0, _ = oracle.Model(c1).newton_step(c1.initial_state(), c1.initial_state(),
                                              c1.report_dt[0])
    for threads in (1, 4):
        assert oracle.set_threads(threads, so) == threads
        omp = oracle.Model(c2, lib_path=so)
        _, R1, J1 = omp.assemble(y, omp.accumulation(y0), 86400.0)
        assert np.array_equal(R0, R1) and np.array_equal(J0, J1)
        _, ys1, _ = oracle.Model(c1, lib_path=so).newton_step(c1.initial_state(),
                                                              c1.initial_state(), c1.report_dt[0])
        assert np.array_equal(ys0, ys1)
