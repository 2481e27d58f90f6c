"""The CPR-AMG hierarchy built by the library on the host (opm_amg_count,
opm_amg_build; no GPU needed) against the oracle's hierarchy: the same
levels, patterns and aggregates, child lists that invert the aggregate map,
diagonal positions, and gather lists whose in-order sums reproduce the
oracle's Galerkin coarse values bit for bit (sec. 2.3.1, the CPR pressure
stage's AMG)."""
import numpy as np
import pytest

import oracle
from paper_1910_06059_amd import cases
from paper_1910_06059_amd.cases import DAY


def _opm():
    from paper_1910_06059_amd import opm
    try:
        opm.lib()
    except ImportError as e:
        pytest.fail(f"library not built: {e}")
    return opm


def _masked():
    return cases.box_case(9, 7, 4, seed=5, mask=cases.masked_mask(
        np.random.default_rng(8), (4, 7, 9), 150), wells=[])


CASES = {
    "tiny": lambda: cases.box_case(4, 3, 2, seed=7, wells=[]),   # one level (n <= 64)
    "box": lambda: cases.box_case(11, 9, 5, seed=3, wells=[]),
    "masked": _masked,
    "C1": cases.config1,
    "C2": cases.config2,
}


def _seq_sum(vals):
    s = 0.0
    for v in vals:
        s += v
    return s


@pytest.mark.parametrize("name", list(CASES))
def test_amg_hierarchy_matches_oracle(name):
    opm = _opm()
    c = CASES[name]()
    m = oracle.Model(c)
    rp0, ci0 = m.pattern()
    g, arr = opm.amg_hierarchy(c.nx, c.ny, c.nz, c.mask, m.n, rp0, ci0)
    y = cases.random_state(c, seed=2)
    st, R, J = m.assemble(y, m.accumulation(cases.random_state(c, seed=3)), 2 * DAY)
    cp = m.cpr(J)
    assert g.n_levels == cp.nl
    assert g.n[g.n_levels - 1] <= opm.AMG_COARSE
    prev_a = None
    for l in range(cp.nl):
        rp, ci, a, agg = cp.level(l)
        assert g.n[l] == len(rp) - 1 and g.nnz[l] == len(ci)
        if l >= 1:
            assert np.array_equal(arr["row_ptr", l], rp) and np.array_equal(arr["col", l], ci)
            n = g.n[l]
            for i in range(n):   # the diagonal entry of each row
                assert ci[arr["dpos", l][i]] == i and rp[i] <= arr["dpos", l][i] < rp[i + 1]
            gp, gm = arr["gmap_ptr", l], arr["gmap", l]
            assert gp[-1] == g.nnz[l - 1]   # every fine entry lands in one coarse entry
            assert np.array_equal(np.sort(gm), np.arange(g.nnz[l - 1]))
            got = np.array([_seq_sum(prev_a[gm[gp[e]:gp[e + 1]]]) for e in range(len(ci))])
            assert np.array_equal(got, a), f"level {l}: Galerkin sums differ"
        if l + 1 < cp.nl:
            assert np.array_equal(arr["agg", l], agg)
            cptr, ch = arr["child_ptr", l], arr["child", l]
            assert np.array_equal(ch, np.argsort(agg, kind="stable"))
            assert np.array_equal(np.diff(cptr), np.bincount(agg, minlength=g.n[l + 1]))
        prev_a = a


def test_amg_invalid_arguments():
    opm = _opm()
    L = opm.lib()
    import ctypes
    g = opm.Amg()
    c = cases.box_case(4, 3, 2, seed=7, wells=[])
    rp, ci = oracle.Model(c).pattern()
    mask = np.ascontiguousarray(c.mask, dtype=np.uint8).ravel()
    # a cell count that does not match the mask
    assert L.opm_amg_count(c.nx, c.ny, c.nz, mask.ctypes.data, 5, rp.ctypes.data, ci.ctypes.data,
                           ctypes.byref(g)) == opm.EINVAL
    assert L.opm_amg_count(0, c.ny, c.nz, mask.ctypes.data, 24, rp.ctypes.data, ci.ctypes.data,
                           ctypes.byref(g)) == opm.EINVAL
    # build needs the arrays of every level
    c2 = cases.box_case(11, 9, 5, seed=3, wells=[])
    rp2, ci2 = oracle.Model(c2).pattern()
    m2 = np.ascontiguousarray(c2.mask, dtype=np.uint8).ravel()
    g2 = opm.Amg()
    assert L.opm_amg_build(c2.nx, c2.ny, c2.nz, m2.ctypes.data, len(rp2) - 1, rp2.ctypes.data,
                           ci2.ctypes.data, ctypes.byref(g2)) == opm.EINVAL
    # the CPR entry points reject a problem without a hierarchy on the host
    pb = opm.Problem()
    pb.n_cells, pb.n_faces, pb.nnzb = 4, 1, 6
    assert L.opm_cpr_bytes(ctypes.byref(pb)) == 0
    o = opm.default_opts(precond=opm.PRECOND_CPR)
    R = ctypes.c_void_p(1)
    rep = opm.NewtonReport()
    assert L.opm_newton_step(ctypes.byref(pb), R, R, 1.0, ctypes.byref(o), R, ctypes.byref(rep),
                             None) == opm.EINVAL
