"""GPU path (through the C ABI) against the CPU oracle, step by step.

Tolerances: residual and Jacobian entries agree to 1e-11 of the largest
entry of the same (equation, variable) column over the system, since the two
sides sum the same terms in different orders; ILU(0) factors and sweeps to
1e-9 relative (FP64) and 1e-4 (FP32 factors); converged Newton states to
1e-6 relative in pressure and 1e-6 absolute in saturation after every report
step, the parity bar of the path.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1910_06059_amd import cases
from paper_1910_06059_amd.cases import DAY, PSI, STB, Well

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def opm():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    from paper_1910_06059_amd import opm as _opm
    _opm.init()
    return _opm


def _cases_small():
    return {
        "box_wells": cases.box_case(5, 4, 3, seed=3, wells=[
            Well("I", cases.WELL_RATE_INJ, [(0, 0, k) for k in range(3)], 800 * STB / DAY),
            Well("G", cases.WELL_RATE_INJ, [(2, 2, 0)], 3e3 * cases.MSCF / DAY, phase=cases.GAS),
            Well("P", cases.WELL_BHP_PROD, [(4, 3, 2)], 3000 * PSI),
            Well("P2", cases.WELL_BHP_PROD, [(4, 3, 2), (4, 0, 0)], 3500 * PSI)]),
        "C1": cases.config1(),
        "masked": cases.box_case(9, 7, 4, seed=5, mask=cases.masked_mask(
            np.random.default_rng(8), (4, 7, 9), 150), wells=[]),
    }


def _masked_with_wells():
    c = _cases_small()["masked"]
    act = np.argwhere(c.mask)
    k, j, i = act[0]
    k2, j2, i2 = act[-1]
    c.wells = [Well("I", cases.WELL_RATE_INJ, [(int(i), int(j), int(k))], 300 * STB / DAY),
               Well("P", cases.WELL_BHP_PROD, [(int(i2), int(j2), int(k2))], 3000 * PSI)]
    return c


CASES = dict(_cases_small(), masked=_masked_with_wells())


def _colscale(J):
    return np.abs(J).max(axis=0) + 1e-300


def _state_pair(case, kind, m):
    if kind == "initial":
        y = case.initial_state()
        return y, y
    if kind == "random":
        return cases.random_state(case, seed=1), cases.random_state(case, seed=2)
    st, y, rep = m.newton_step(case.initial_state(), case.initial_state(), case.report_dt[0])
    assert st == 0
    return y, case.initial_state()


@pytest.mark.parametrize("name", list(CASES))
def test_geometry_parity(opm, name):
    case = CASES[name]
    g = opm.GpuModel(case)
    m = oracle.Model(case)
    geo = m.geometry()
    np.testing.assert_allclose(g.trans.cpu().numpy()[:m.nf], geo["trans"], rtol=1e-14, atol=0)
    np.testing.assert_allclose(g.pore_vol.cpu().numpy(), geo["pore_vol"], rtol=1e-14, atol=0)
    np.testing.assert_allclose(g.depth.cpu().numpy(), geo["depth"], rtol=1e-14, atol=1e-14)
    cell, wi, well = m.conns()
    np.testing.assert_array_equal(g.conn_cell.cpu().numpy()[:m.nc], cell)
    np.testing.assert_allclose(g.conn_wi.cpu().numpy()[:m.nc], wi, rtol=1e-13, atol=0)


@pytest.mark.parametrize("kind", ["initial", "random", "converged"])
@pytest.mark.parametrize("name", list(CASES))
def test_assembly_parity(opm, name, kind):
    case = CASES[name]
    g = opm.GpuModel(case)
    m = oracle.Model(case)
    y, y0 = _state_pair(case, kind, m)
    dt = case.report_dt[0]
    acc0 = m.accumulation(y0)
    st, Ro, Jo = m.assemble(y, acc0, dt)
    acc0_g = g.accumulation(g.state(y0))
    np.testing.assert_allclose(acc0_g.cpu().numpy(), acc0, rtol=1e-14, atol=0)
    R, J, nrm = g.assemble(g.state(y), acc0_g, dt)
    R, J, nrm = R.cpu().numpy(), J.cpu().numpy(), nrm.cpu().numpy()
    # scale of the terms that are summed into R (a converged residual is a
    # near-cancelling sum of accumulation, fluxes and well terms)
    pv = m.geometry()["pore_vol"]
    acc_term = pv[:, None] / dt * np.abs(m.accumulation(y) - acc0)
    scale = np.maximum.reduce([np.abs(Ro).max(axis=0), acc_term.max(axis=0),
                               np.abs(m.well_rates(y)).max(axis=0),
                               (pv[:, None] / dt * np.abs(acc0)).max(axis=0) * 1e-6])
    assert np.all(np.abs(R - Ro) <= 1e-11 * scale[None, :]), np.abs(R - Ro).max(axis=0) / scale
    err = np.abs(J - Jo) / _colscale(Jo)[None]
    assert err.max() <= 1e-11, err.max()
    _check_norms(m, y, dt, R, Ro, nrm, 1e-11 * scale)


def _check_norms(m, y, dt, R, Ro, nrm, r_tol):
    """CNV/MB (sec. 2.3) of the GPU against the oracle.  (1) On the same
    residual (the GPU's R fed to the oracle's norms) the reductions agree to
    rounding: CNV_a = dt max|R_a|/(b_a PV) takes the same maximum (rtol 1e-13
    covers b's last bits), and MB's sum differs only by summation order,
    |d sum| <= n eps sum_i |R_a,i| (Higham's bound for recursive summation).
    (2) Against the oracle's own residual, the norms may move as far as the
    residual itself is allowed to: |R - Ro| <= r_tol[a] per cell gives
    |d CNV_a| <= dt r_tol[a] / min_i(b_a,i PV_i) and
    |d MB_a| <= dt n r_tol[a] / (mean b_a sum PV)."""
    geo = m.geometry()
    pv = geo["pore_vol"]
    n = len(pv)
    b = np.exp(np.asarray(m.case.fluid.c)[None, :] * (y[:, :1] - m.case.fluid.p_ref))
    cnv_s, mb_s = m.norms(y, np.ascontiguousarray(R), dt)
    np.testing.assert_allclose(nrm[:3], cnv_s, rtol=1e-13, atol=0)
    eps = np.finfo(np.float64).eps
    sum_bound = dt * n * eps * np.abs(R).sum(axis=0) / (b.mean(axis=0) * pv.sum())
    assert np.all(np.abs(nrm[3:6] - mb_s) <= sum_bound + 1e-13 * mb_s), (nrm[3:6], mb_s)
    cnv, mb = m.norms(y, Ro, dt)
    live = bool(getattr(m.case.fluid, "live", False))
    if not live:   # b_a(p) as above only for the dead-oil fluid
        cnv_tol = dt * r_tol / (b * pv[:, None]).min(axis=0)
        mb_tol = dt * n * r_tol / (b.mean(axis=0) * pv.sum())
        assert np.all(np.abs(nrm[:3] - cnv) <= cnv_tol + 1e-13 * cnv), (nrm[:3], cnv, cnv_tol)
        assert np.all(np.abs(nrm[3:6] - mb) <= mb_tol + 1e-13 * mb), (nrm[3:6], mb, mb_tol)


def test_assembly_deterministic(opm):
    case = CASES["box_wells"]
    g = opm.GpuModel(case)
    y = g.state(cases.random_state(case, 3))
    acc0 = g.accumulation(g.state(cases.random_state(case, 4)))
    R1, J1, n1 = g.assemble(y, acc0, DAY)
    R2, J2, n2 = g.assemble(y, acc0, DAY)
    assert torch.equal(R1, R2) and torch.equal(J1, J2) and torch.equal(n1, n2)


def _oracle_system(case, seed=1):
    m = oracle.Model(case)
    y = cases.random_state(case, seed=seed)
    st, R, J = m.assemble(y, m.accumulation(cases.random_state(case, seed=seed + 1)), 2 * DAY)
    st, F = m.ilu0(J)
    assert st == 0
    return m, R, J, F


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("name", list(CASES))
def test_ilu0_parity(opm, name, mode):
    case = CASES[name]
    g = opm.GpuModel(case)
    m, R, J, F = _oracle_system(case)
    opm.set_option(opm.OPT_SWEEP_MODE, mode)
    try:
        Jg = torch.from_numpy(J).to(g.dev)
        ilu, status = g.ilu0_factor(Jg, opm.PREC_FP64)
        assert int(status.item()) == 0
        ns = (g.n + 63) // 64 * 64
        dinv = ilu.view(torch.float64)[:9 * ns].view(9, ns).cpu().numpy()[:, :g.n]
        rp, ci = m.pattern()
        perm = g.host["perm"][:g.n]
        for pos in range(g.n):
            i = perm[pos]
            q = [k for k in range(rp[i], rp[i + 1]) if ci[k] == i][0]
            ref = np.linalg.inv(F[q])
            got = dinv[:, pos].reshape(3, 3)
            assert np.abs(got - ref).max() <= 1e-9 * np.abs(ref).max()
        r = np.random.default_rng(4).standard_normal((g.n, 3))
        xo = m.ilu0_apply(F, r)
        xg = g.ilu0_apply(ilu, g.state(r)).cpu().numpy()
        assert np.abs(xg - xo).max() <= 1e-9 * np.abs(xo).max()
        # mixed precision: FP32 factors and sweeps
        ilu32, status = g.ilu0_factor(Jg, opm.PREC_MIXED)
        assert int(status.item()) == 0
        x32 = g.ilu0_apply(ilu32, g.state(r), opm.PREC_MIXED).cpu().numpy()
        assert np.abs(x32 - xo).max() <= 1e-4 * np.abs(xo).max()
    finally:
        opm.set_option(opm.OPT_SWEEP_MODE, -1)


def test_sweep_modes_bitwise_equal(opm):
    case = cases.config2()
    g = opm.GpuModel(case)
    y = g.state(cases.random_state(case, 5))
    acc0 = g.accumulation(g.state(cases.random_state(case, 6)))
    R, J, _ = g.assemble(y, acc0, DAY)
    out = []
    # the factors (FP64 inverse pivots, lower and upper blocks: 9 + 27 + 27
    # values per padded row) lead the ILU buffer; sweep scratch and the
    # record sweep's copy follow them
    ns = (g.n + 63) // 64 * 64
    nfac = 8 * (9 + 27 + 27) * ns
    for mode in (0, 1):
        opm.set_option(opm.OPT_SWEEP_MODE, mode)
        ilu, status = g.ilu0_factor(J)
        out.append((ilu[:nfac].clone(), g.ilu0_apply(ilu, R)))
    opm.set_option(opm.OPT_SWEEP_MODE, -1)
    assert torch.equal(out[0][0], out[1][0]) and torch.equal(out[0][1], out[1][1])


@pytest.mark.parametrize("precision", [0, 1])
def test_sweep_kernels_bitwise_equal(opm, precision):
    """Every one-workgroup ring-sweep kernel (gather inside the sweep;
    branch-free prefetch with 512, 256, 128 threads; idle wavefronts
    skipping) gives bitwise the same result, including levels wider than
    the workgroup (the 30x30x12 box has up to 360 rows per level)."""
    for case in (cases.config2(), cases.box_case(30, 30, 12, seed=9)):
        g = opm.GpuModel(case)
        y = g.state(cases.random_state(case, 5))
        acc0 = g.accumulation(g.state(cases.random_state(case, 6)))
        R, J, _ = g.assemble(y, acc0, DAY)
        ilu, status = g.ilu0_factor(J, precision)
        assert int(status.item()) == 0
        out = []
        try:
            for kind in range(1, 7):
                opm.set_option(opm.OPT_SWEEP_KERNEL, kind)
                out.append(g.ilu0_apply(ilu, R, precision))
        finally:
            opm.set_option(opm.OPT_SWEEP_KERNEL, 0)
        for kind, x in enumerate(out[1:], start=2):
            assert torch.equal(x, out[0]), (case.name, precision, kind)
    assert g.max_level > 256


@pytest.mark.parametrize("name", list(CASES))
def test_spmv_parity(opm, name):
    case = CASES[name]
    g = opm.GpuModel(case)
    m, R, J, F = _oracle_system(case)
    x = np.random.default_rng(2).standard_normal((g.n, 3)) * np.array([1e5, 0.1, 0.1])
    yo = m.spmv(J, x)
    yg = g.spmv(torch.from_numpy(J).to(g.dev), g.state(x)).cpu().numpy()
    scale = np.abs(yo).max(axis=0)
    assert np.all(np.abs(yg - yo) <= 1e-12 * scale[None, :])


def _dense(m, J):
    rp, ci = m.pattern()
    D = np.zeros((3 * m.n, 3 * m.n))
    for i in range(m.n):
        for q in range(rp[i], rp[i + 1]):
            D[3 * i:3 * i + 3, 3 * ci[q]:3 * ci[q] + 3] = J[q]
    return D


@pytest.mark.parametrize("dims", [(2, 2, 2), (3, 3, 3), (4, 3, 2), (7, 1, 1), (1, 1, 1)])
@pytest.mark.parametrize("precision", [0, 1])
def test_bicgstab_dense_solve(opm, dims, precision):
    nx, ny, nz = dims
    wells = [Well("I", cases.WELL_RATE_INJ, [(0, 0, 0)], 500 * STB / DAY),
             Well("P", cases.WELL_BHP_PROD, [(nx - 1, ny - 1, nz - 1)], 3000 * PSI)]
    case = cases.box_case(nx, ny, nz, seed=sum(dims), wells=wells)
    g = opm.GpuModel(case)
    m, R, J, F = _oracle_system(case, seed=sum(dims))
    Jg = torch.from_numpy(J).to(g.dev)
    ilu, status = g.ilu0_factor(Jg, precision)
    x, rep = g.bicgstab(Jg, ilu, g.state(-R), rtol=1e-13, maxit=300, precision=precision)
    assert rep.status == 0, rep.status
    xd = np.linalg.solve(_dense(m, J), -R.ravel()).reshape(-1, 3)
    err = np.abs(x.cpu().numpy() - xd) / np.abs(xd).max(axis=0)[None, :]
    assert err.max() <= 1e-9, err.max()
    if dims[1] == dims[2] == 1 and precision == 0:
        assert rep.its == 1 and rep.half == 1   # exact LU on a chain: half an iteration


def test_bicgstab_matches_oracle_iterations(opm):
    case = cases.config2()
    g = opm.GpuModel(case)
    m, R, J, F = _oracle_system(case)
    st, xo, its_o, rr = m.bicgstab(J, F, -R, rtol=1e-6)
    Jg = torch.from_numpy(J).to(g.dev)
    ilu, _ = g.ilu0_factor(Jg)
    x, rep = g.bicgstab(Jg, ilu, g.state(-R), rtol=1e-6)
    assert rep.status == 0 and st == 0
    its_g = rep.its - 0.5 * rep.half
    assert abs(its_g - its_o) <= 1.0, (its_g, its_o)
    # both meet the tolerance on the oracle's own operator
    res = -R - m.spmv(J, x.cpu().numpy())
    assert np.linalg.norm(res) <= 1e-6 * np.linalg.norm(R) * 1.0001


def _compare_states(yg, yo, what):
    ep = np.abs(yg[:, 0] - yo[:, 0]).max() / np.abs(yo[:, 0]).max()
    es = np.abs(yg[:, 1:] - yo[:, 1:]).max()
    assert ep <= 1e-6 and es <= 1e-6, f"{what}: p rel err {ep:.2e}, s abs err {es:.2e}"
    return ep, es


@pytest.mark.parametrize("precision", [0, 1])
def test_newton_run_c1(opm, precision):
    case = cases.config1()
    g = opm.GpuModel(case)
    m = oracle.Model(case)
    ostates, oreps = m.run()
    y, gstates, greps = g.run(opts=opm.default_opts(case, precision=precision))
    for s, (yg, yo) in enumerate(zip(gstates, ostates)):
        _compare_states(yg, yo, f"C1 step {s}")
    for rg, ro in zip(greps, oreps):
        assert abs(rg["newton_its"] - ro["newton_its"]) <= 1


@pytest.mark.parametrize("precision", [0, 1])
def test_newton_run_c2(opm, precision):
    """The benchmark workload: 24x25x15, 30 report steps of 10 days."""
    case = cases.config2()
    g = opm.GpuModel(case)
    m = oracle.Model(case)
    y = case.initial_state()
    yg = g.initial_state()
    opts = opm.default_opts(case, precision=precision)
    for s, dt in enumerate(case.report_dt):
        st, y, rep = m.advance(y, dt)
        assert st == 0
        stg, repg = g.advance(yg, dt, opts)
        assert stg == 0, stg
        _compare_states(yg.cpu().numpy(), y, f"C2 step {s}")


def test_newton_masked(opm):
    case = cases.config3()
    g = opm.GpuModel(case)
    m = oracle.Model(case)
    y = case.initial_state()
    yg = g.initial_state()
    for s, dt in enumerate(case.report_dt[:2]):
        st, y, rep = m.advance(y, dt)
        stg, repg = g.advance(yg, dt)
        assert st == 0 and stg == 0
        _compare_states(yg.cpu().numpy(), y, f"C3 step {s}")


def test_failure_paths(opm):
    case = cases.box_case(4, 3, 2, seed=2)
    g = opm.GpuModel(case)
    y0 = g.initial_state()
    # BiCGStab iteration cap
    st, rep = g.newton_step(y0.clone(), y0, 30 * DAY, opm.default_opts(case, lin_maxit=1))
    assert st == opm.ENOTCONV
    # a tight Newton cap forces the time-step cut path; the cut decisions
    # are the oracle's
    y = y0.clone()
    st, rep = g.advance(y, 90 * DAY, opm.default_opts(case, max_newton=2))
    m = oracle.Model(case)
    ost, yo, orep = m.advance(case.initial_state(), 90 * DAY, oracle.default_opts(case, max_newton=2))
    assert rep.cuts >= 1 and rep.cuts == orep.cuts and (st == 0) == (ost == 0)
    if st == 0:
        _compare_states(y.cpu().numpy(), yo, "cut path")
    # non-finite state
    y = y0.clone()
    y[1, 0] = float("nan")
    st, rep = g.newton_step(y, y0, DAY)
    assert st == opm.ENONFINITE


def test_singular_pivot(opm):
    """A cell with no pore volume and no connections gives a zero diagonal
    block: ILU(0) reports a singular pivot."""
    case = cases.box_case(3, 1, 1, seed=1, wells=[])
    case.poro[0, 0, 2] = 0.0
    case.perm_h[0, 0, 2] = 0.0
    g = opm.GpuModel(case)
    y0 = g.initial_state()
    R, J, _ = g.assemble(y0, g.accumulation(y0), DAY)
    ilu, status = g.ilu0_factor(J)
    assert int(status.item()) == opm.ESINGULAR
    y = y0.clone()
    y[0, 0] += 1e5   # not at rest: Newton has to factor
    st, rep = g.newton_step(y, y0, DAY)
    assert st == opm.ESINGULAR


def test_full_size_c5_sampled(opm):
    """500k-cell system at full size: residual and Jacobian rows sampled
    against the oracle's assembly, and the GPU BiCGStab solution checked by
    its true residual on the oracle's operator."""
    case = cases.config5(seed=5008)
    g = opm.GpuModel(case)
    m = oracle.Model(case)
    y = cases.random_state(case, seed=9)
    y0 = cases.random_state(case, seed=10)
    dt = case.report_dt[0]
    st, Ro, Jo = m.assemble(y, m.accumulation(y0), dt)
    R, J, _ = g.assemble(g.state(y), g.accumulation(g.state(y0)), dt)
    rows = np.random.default_rng(0).choice(g.n, 4000, replace=False)
    Rg = R.cpu().numpy()
    scale = np.abs(Ro).max(axis=0)
    assert np.all(np.abs(Rg[rows] - Ro[rows]) <= 1e-11 * scale[None, :])
    Jg = J.cpu().numpy()
    rp, _ = m.pattern()
    blocks = np.concatenate([np.arange(rp[i], rp[i + 1]) for i in rows])
    assert (np.abs(Jg[blocks] - Jo[blocks]) / _colscale(Jo)[None]).max() <= 1e-11
    ilu, status = g.ilu0_factor(J)
    assert int(status.item()) == 0
    x, rep = g.bicgstab(J, ilu, -R, rtol=1e-6)
    assert rep.status == 0
    res = -Ro - m.spmv(Jo, x.cpu().numpy())
    assert np.linalg.norm(res) <= 1.01e-6 * np.linalg.norm(Ro)


def _plane_systems():
    masked = cases.box_case(19, 13, 6, seed=6, mask=cases.masked_mask(
        np.random.default_rng(9), (6, 13, 19), 900), wells=[])
    return [cases.config2(), masked, cases.box_case(30, 30, 12, seed=9),
            cases.box_case(7, 40, 5, seed=4), cases.box_case(1, 1, 9, seed=2)]


@pytest.mark.parametrize("precision", [0, 1])
def test_plane_sweep_bitwise_equal(opm, precision):
    """The plane-pipelined factorisation and sweeps (one workgroup per
    z-plane, the values exchanged between planes through marked vectors)
    give the per-level launches' bits: the same row arithmetic in the same
    order, on full, masked, tall and one-column grids."""
    for case in _plane_systems():
        print(f"plane sweep: {case.name} precision {precision}", flush=True)
        g = opm.GpuModel(case)
        y = g.state(cases.random_state(case, 5))
        acc0 = g.accumulation(g.state(cases.random_state(case, 6)))
        R, J, _ = g.assemble(y, acc0, DAY)
        ns = (g.n + 63) // 64 * 64
        npiv = 8 * 9 * ns if precision == 0 else 8 * 9 * ns + 4 * 9 * ns
        opm.set_option(opm.OPT_SWEEP_MODE, 1)
        try:
            facs = []
            for planes in (0, 1):
                opm.set_option(opm.OPT_PLANE_SWEEP, planes)
                ilu, status = g.ilu0_factor(J, precision)
                assert int(status.item()) == 0
                facs.append(ilu[:npiv].clone())
            assert torch.equal(facs[0], facs[1]), (case.name, "pivots")
            xs = []
            for planes in (0, 1):
                opm.set_option(opm.OPT_PLANE_SWEEP, planes)
                xs.append(g.ilu0_apply(ilu, R, precision))
            # repeated applications reset the exchange vectors
            for _ in range(3):
                xs.append(g.ilu0_apply(ilu, R, precision))
        finally:
            opm.set_option(opm.OPT_SWEEP_MODE, -1)
            opm.set_option(opm.OPT_PLANE_SWEEP, 1)
        assert torch.isfinite(xs[0]).all()
        for q, xq in enumerate(xs[1:]):
            assert torch.equal(xs[0], xq), (case.name, q)


def test_plane_sweep_gives_up_with_nan(opm):
    """A plane sweep whose wait gives up (forced from the host: a spin limit
    of zero polls) returns NaN for every row instead of hanging, and
    BiCGStab reports it; the next solve with the normal limit is exact
    again."""
    case = cases.box_case(12, 10, 6, seed=3)
    g = opm.GpuModel(case)
    y = g.state(cases.random_state(case, 5))
    acc0 = g.accumulation(g.state(cases.random_state(case, 6)))
    R, J, _ = g.assemble(y, acc0, DAY)
    opm.set_option(opm.OPT_SWEEP_MODE, 1)
    try:
        ilu, status = g.ilu0_factor(J)
        ref = g.ilu0_apply(ilu, R)
        opm.set_option(opm.OPT_PLANE_SPIN, 0)
        bad = g.ilu0_apply(ilu, R)
        assert torch.isnan(bad).all()
        x, rep = g.bicgstab(J, ilu, -R, rtol=1e-6)
        assert rep.status != 0
        opm.set_option(opm.OPT_PLANE_SPIN, 1 << 18)
        assert torch.equal(g.ilu0_apply(ilu, R), ref)
    finally:
        opm.set_option(opm.OPT_PLANE_SPIN, 1 << 18)
        opm.set_option(opm.OPT_SWEEP_MODE, -1)
