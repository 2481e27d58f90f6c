"""CPR-AMG (sec. 2.3.1, the two-stage CPR preconditioner) on the GPU,
through the C ABI, against the oracle's CPR.

Every device computation starts from the oracle's Jacobian, so each stage is
checked on its own:
  - weights and every level's matrix: same operations in the same order as
    the oracle (3x3 partial-pivot elimination, in-order Galerkin sums), to
    1e-13 of the largest entry of the row;
  - the V-cycle: the coarsest level is applied through its inverse on the
    device and by elimination in the oracle, so results agree to rounding
    amplified by the coarsest matrix's condition: 1e-8 of max |x|;
  - z = CPR(r) with FP64 ILU(0): 1e-8 of the largest entry per component;
    with the FP32 ILU(0) second stage: 1e-4;
  - BiCGStab with CPR: iterations within one of the oracle's, true residual
    at the tolerance;
  - Newton runs with CPR: states after every report step to 1e-6 (relative
    pressure, absolute saturations), as for the ILU(0) runs.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1910_06059_amd import cases
from paper_1910_06059_amd.cases import DAY, PSI

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def opm():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    from paper_1910_06059_amd import opm as _opm
    _opm.init()
    return _opm


def _masked():
    return cases.box_case(9, 7, 4, seed=5, mask=cases.masked_mask(
        np.random.default_rng(8), (4, 7, 9), 150), wells=[])


CASES = {
    "one_cell": lambda: cases.box_case(1, 1, 1, seed=2, wells=[]),
    "column": lambda: cases.box_case(1, 1, 7, seed=2, wells=[]),   # one column, one level
    "tiny": lambda: cases.box_case(4, 3, 2, seed=7, wells=[]),   # one level
    "box": lambda: cases.box_case(11, 9, 5, seed=3, wells=[]),
    "masked": _masked,
    "C2": cases.config2,
    "C6_live": cases.config_live,
}


def _state(c, seed):
    if c.fluid.live:
        rng = np.random.default_rng(seed)
        n = c.n_active
        y = np.empty((n, 3))
        y[:, 0] = rng.uniform(3300, 3700, n) * PSI
        y[:, 1] = rng.uniform(0.15, 0.5, n)
        y[:, 2] = rng.uniform(0.3, 0.9, n) * c.fluid.rs_c * y[:, 0]
        return y
    return cases.random_state(c, seed=seed)


def _system(c, seed=1):
    m = oracle.Model(c)
    y = _state(c, seed)
    st, R, J = m.assemble(y, m.accumulation(_state(c, seed + 1)), 2 * DAY)
    assert st == 0
    st, F = m.ilu0(J)
    assert st == 0
    return m, R, J, F


def _dev(g, a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).to(g.dev).contiguous()


@pytest.mark.parametrize("name", list(CASES))
def test_cpr_setup_parity(opm, name):
    c = CASES[name]()
    m, R, J, F = _system(c)
    g = opm.GpuModel(c)
    cpr, status = g.cpr_setup(_dev(g, J))
    assert int(status.item()) == 0
    cp = m.cpr(J)
    assert g.amg.n_levels == cp.nl
    w_o = cp.weights()
    for l in range(cp.nl):
        a_g, w_g = g.cpr_values(cpr, l)
        rp, ci, a_o, _ = cp.level(l)
        a_g = a_g.cpu().numpy()
        rowmax = np.maximum.reduceat(np.abs(a_o), rp[:-1]) + 1e-300
        scale = np.repeat(rowmax, np.diff(rp))
        assert (np.abs(a_g - a_o) / scale).max() <= 1e-13, f"level {l}"
    w_g = w_g.cpu().numpy()
    assert (np.abs(w_g - w_o) / (np.abs(w_o).max(axis=1, keepdims=True) + 1e-300)).max() <= 1e-13


@pytest.mark.parametrize("name", list(CASES))
def test_cpr_vcycle_and_apply_parity(opm, name):
    c = CASES[name]()
    m, R, J, F = _system(c, seed=4)
    g = opm.GpuModel(c)
    Jd = _dev(g, J)
    cpr, status = g.cpr_setup(Jd)
    cp = m.cpr(J)
    rng = np.random.default_rng(9)
    b = rng.standard_normal(m.n) * np.abs(R[:, 0]).max()
    x_o = cp.vcycle(b)
    x_g = g.cpr_vcycle(cpr, _dev(g, b)).cpu().numpy()
    assert np.abs(x_g - x_o).max() <= 1e-8 * np.abs(x_o).max()
    ilu, st = g.ilu0_factor(Jd)
    assert int(st.item()) == 0
    z_o = cp.apply(F, R)
    z_g = g.cpr_apply(Jd, ilu, cpr, _dev(g, R)).cpu().numpy()
    scale = np.abs(z_o).max(axis=0) + 1e-300
    assert (np.abs(z_g - z_o) / scale).max() <= 1e-8
    ilu32, st = g.ilu0_factor(Jd, precision=opm.PREC_MIXED)
    z_m = g.cpr_apply(Jd, ilu32, cpr, _dev(g, R), precision=opm.PREC_MIXED).cpu().numpy()
    assert (np.abs(z_m - z_o) / scale).max() <= 1e-4


@pytest.mark.parametrize("name", ["box", "masked", "C2", "C6_live"])
def test_bicgstab_cpr_parity(opm, name):
    c = CASES[name]()
    m, R, J, F = _system(c, seed=6)
    g = opm.GpuModel(c)
    Jd = _dev(g, J)
    cpr, _ = g.cpr_setup(Jd)
    ilu, _ = g.ilu0_factor(Jd)
    cp = m.cpr(J)
    st, x_o, its_o, rr_o = cp.bicgstab(F, -R, rtol=1e-6)
    assert st == 0
    x_g, rep = g.bicgstab_cpr(Jd, ilu, cpr, _dev(g, -R), rtol=1e-6)
    assert rep.status == 0
    its_g = rep.its - 0.5 * rep.half
    assert abs(its_g - its_o) <= 1.0, (its_g, its_o)
    x_g = x_g.cpu().numpy()
    res = -R - m.spmv(J, x_g)
    assert np.linalg.norm(res) <= 1e-6 * np.linalg.norm(R) * 1.001
    x_i, rep_i = g.bicgstab(Jd, ilu, _dev(g, -R), rtol=1e-6)
    assert rep.its <= rep_i.its


def _compare_states(c, gstates, ostates, what):
    for s, (yg, yo) in enumerate(zip(gstates, ostates)):
        ep = np.abs(yg[:, 0] - yo[:, 0]).max() / np.abs(yo[:, 0]).max()
        if c.fluid.live:
            es = np.abs(yg[:, 1] - yo[:, 1]).max()
        else:
            es = np.abs(yg[:, 1:] - yo[:, 1:]).max()
        assert ep <= 1e-6 and es <= 1e-6, f"{what} step {s}: p {ep:.2e} s {es:.2e}"


@pytest.mark.parametrize("precision", [0, 1])
def test_newton_cpr_run_c1(opm, precision):
    c = cases.config1()
    g = opm.GpuModel(c)
    m = oracle.Model(c)
    ostates, oreps = m.run(opts=oracle.default_opts(c, precond=1))
    y, gstates, greps = g.run(opts=opm.default_opts(c, precision=precision,
                                                    precond=opm.PRECOND_CPR))
    _compare_states(c, gstates, ostates, "C1")
    for rg, ro in zip(greps, oreps):
        assert abs(rg["newton_its"] - ro["newton_its"]) <= 1


@pytest.mark.parametrize("blk", [None, (4, 4, 5)], ids=["single", "blocks"])
def test_newton_cpr_run_c2(opm, blk):
    """Three report steps of the 9000-cell waterflood with CPR (single and
    block ILU(0) second stage): the oracle's states, fewer linear
    iterations than with the ILU(0) alone."""
    c = cases.config2()
    g = opm.GpuModel(c, ilu_blocks=blk)
    m = oracle.Model(c)
    ostates, oreps = m.run(n_steps=3, opts=oracle.default_opts(c, precond=1))
    y, gstates, greps = g.run(n_steps=3, opts=opm.default_opts(c, precond=opm.PRECOND_CPR))
    _compare_states(c, gstates, ostates, "C2")
    y2, _, greps_ilu = g.run(n_steps=3, opts=opm.default_opts(c))
    assert sum(r["lin_its"] for r in greps) < sum(r["lin_its"] for r in greps_ilu)


def test_newton_cpr_live_and_wells(opm):
    """CPR with live oil (variable switching) and with standard wells (the
    preconditioner of the Schur-complement system)."""
    c = cases.config_live()
    g = opm.GpuModel(c)
    m = oracle.Model(c)
    ostates, _ = m.run(n_steps=6, opts=oracle.default_opts(c, precond=1))
    y, gstates, _ = g.run(n_steps=6, opts=opm.default_opts(c, precond=opm.PRECOND_CPR))
    rs = c.fluid.rs_c
    for s, (yg, mg, yo, mo) in enumerate(zip(gstates, g.run_meanings, ostates, m.run_meanings)):
        r_g = np.where(mg == 0, rs * yg[:, 0], yg[:, 2])
        r_o = np.where(mo == 0, rs * yo[:, 0], yo[:, 2])
        assert np.abs(yg[:, 0] - yo[:, 0]).max() <= 1e-6 * np.abs(yo[:, 0]).max()
        assert np.abs(r_g - r_o).max() <= 1e-6 * np.abs(r_o).max(), f"live step {s}"
    c = cases.config1()
    c.standard_wells = True
    g = opm.GpuModel(c)
    m = oracle.Model(c)
    ostates, _ = m.run(n_steps=4, opts=oracle.default_opts(c, precond=1))
    y, gstates, _ = g.run(n_steps=4, opts=opm.default_opts(c, precond=opm.PRECOND_CPR))
    _compare_states(c, gstates, ostates, "C1 standard wells")
    for xg, xo in zip(g.run_well_states, m.run_well_states):
        assert np.abs(xg[:, 3] - xo[:, 3]).max() <= 1e-6 * np.abs(xo[:, 3]).max()


def test_newton_cpr_gmres(opm):
    c = cases.config1()
    g = opm.GpuModel(c)
    m = oracle.Model(c)
    ostates, _ = m.run(n_steps=4, opts=oracle.default_opts(c, precond=1, krylov=1, restart=20))
    y, gstates, _ = g.run(n_steps=4, opts=opm.default_opts(
        c, precond=opm.PRECOND_CPR, krylov=opm.KRYLOV_GMRES, restart=20))
    _compare_states(c, gstates, ostates, "C1 GMRes")


def test_cpr_rejections(opm):
    c = cases.config1()
    g = opm.GpuModel(c, amg=False)
    y = g.initial_state()
    with pytest.raises(opm.OpmError):   # no hierarchy: OPM_EINVAL
        g.newton_step(y, g.initial_state(), DAY, opm.default_opts(c, precond=opm.PRECOND_CPR))
    with pytest.raises(opm.OpmError):
        g.newton_step(y, g.initial_state(), DAY, opm.default_opts(c, precond=2))


def test_cpr_full_size_c5(opm):
    """The 500k-cell system at full size: every level's matrix and the
    weights against the oracle's, the V-cycle and z = CPR(r) with the
    single-block ILU(0) against the oracle's, and BiCGStab with CPR and the
    block ILU0 on 4x4x50 columns (the benchmark's launch configuration)
    solving to the tolerance on the oracle's operator."""
    c = cases.config5(seed=5008)
    m = oracle.Model(c)
    y = cases.random_state(c, seed=9)
    st, R, J = m.assemble(y, m.accumulation(cases.random_state(c, seed=10)), c.report_dt[0])
    assert st == 0
    cp = m.cpr(J)
    g = opm.GpuModel(c)
    Jd = _dev(g, J)
    cpr, status = g.cpr_setup(Jd)
    assert int(status.item()) == 0
    assert g.amg.n_levels == cp.nl == 6
    for l in range(cp.nl):
        a_g, w_g = g.cpr_values(cpr, l)
        rp, ci, a_o, _ = cp.level(l)
        rowmax = np.maximum.reduceat(np.abs(a_o), rp[:-1]) + 1e-300
        err = np.abs(a_g.cpu().numpy() - a_o) / np.repeat(rowmax, np.diff(rp))
        assert err.max() <= 1e-13, f"level {l}"
    w_o = cp.weights()
    assert (np.abs(w_g.cpu().numpy() - w_o) / np.abs(w_o).max(axis=1, keepdims=True)).max() <= 1e-13
    b = np.random.default_rng(9).standard_normal(m.n)
    x_o = cp.vcycle(b)
    x_g = g.cpr_vcycle(cpr, _dev(g, b)).cpu().numpy()
    assert np.abs(x_g - x_o).max() <= 1e-8 * np.abs(x_o).max()
    st, F = m.ilu0(J)
    assert st == 0
    ilu, st = g.ilu0_factor(Jd)
    z_o = cp.apply(F, R)
    z_g = g.cpr_apply(Jd, ilu, cpr, _dev(g, R)).cpu().numpy()
    assert (np.abs(z_g - z_o) / (np.abs(z_o).max(axis=0) + 1e-300)).max() <= 1e-8
    del ilu, F
    gb = opm.GpuModel(c, ilu_blocks=(4, 4, 50))
    Jb = _dev(gb, J)
    cprb, _ = gb.cpr_setup(Jb)
    bilu, _ = gb.ilu0_factor(Jb)
    x, rep = gb.bicgstab_cpr(Jb, bilu, cprb, _dev(gb, -R), rtol=1e-6)
    assert rep.status == 0
    res = -R - m.spmv(J, x.cpu().numpy())
    assert np.linalg.norm(res) <= 1.01e-6 * np.linalg.norm(R)
