"""Live oil with variable switching on the GPU (through the C ABI) against the
oracle's live-oil model.

Tolerances as for dead oil: accumulation to 1e-14 relative, residual and
Jacobian to 1e-11 of the largest entry of the same column, converged states
to 1e-6 (relative pressure, absolute saturations, dissolved ratio relative
to its largest value).  States are compared through the physical quantities
(p, s_w, s_g, r_go), which are continuous across a switch; the meanings
themselves must agree except in cells within 1e-4 of the switching point.
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


def _live_box(nx, ny, nz, seed, masked=False):
    fl = cases.live_fluid()
    mask = None
    if masked:
        mask = cases.masked_mask(np.random.default_rng(seed), (nz, ny, nx), int(0.7 * nx * ny * nz))
    c = cases.box_case(nx, ny, nz, seed=seed, fluid=fl, mask=mask, wells=[])
    act = np.argwhere(c.mask)
    k, j, i = act[0]
    k2, j2, i2 = act[-1]
    c.wells = [Well("I", cases.WELL_RATE_INJ, [(int(i), int(j), int(k))], 300 * STB / DAY),
               Well("P", cases.WELL_BHP_PROD, [(int(i2), int(j2), int(k2))], 2500 * PSI)]
    return c


def _live_state(c, seed):
    rng = np.random.default_rng(seed)
    n = c.n_active
    mean = rng.integers(0, 2, n).astype(np.uint8)
    y = np.empty((n, 3))
    y[:, 0] = rng.uniform(2800, 3200, n) * PSI
    y[:, 1] = rng.uniform(0.15, 0.5, n)
    rs = c.fluid.rs_c * y[:, 0]
    y[:, 2] = np.where(mean == 0, rng.uniform(0.03, 0.2, n), rng.uniform(0.3, 0.9, n) * rs)
    return y, mean


CASES = {
    "box": lambda: _live_box(5, 4, 3, seed=3),
    "masked": lambda: _live_box(9, 7, 4, seed=5, masked=True),
    "C6": cases.config_live,
}


def _colscale(J):
    return np.abs(J).max(axis=0) + 1e-300


@pytest.mark.parametrize("name", list(CASES))
def test_live_assembly_parity(opm, name):
    c = CASES[name]()
    g = opm.GpuModel(c)
    m = oracle.Model(c)
    y0, mean0 = _live_state(c, seed=11)
    y, mean = _live_state(c, seed=12)
    m.set_meaning(mean0)
    g.set_meaning(mean0)
    a_o = m.accumulation(y0)
    a_g = g.accumulation(g.state(y0)).cpu().numpy()
    assert np.abs(a_g - a_o).max() <= 1e-14 * np.abs(a_o).max()
    m.set_meaning(mean)
    g.set_meaning(mean)
    st, R, J = m.assemble(y, a_o, 2 * DAY)
    Rg, Jg, norms = g.assemble(g.state(y), g.state(a_o), 2 * DAY)
    Rg, Jg = Rg.cpu().numpy(), Jg.cpu().numpy()
    rs = np.abs(R).max(axis=0) + 1e-300
    assert (np.abs(Rg - R) / rs).max() <= 1e-11
    Jf, Jgf = J.reshape(-1, 9), Jg.reshape(-1, 9)
    assert (np.abs(Jgf - Jf) / _colscale(Jf)).max() <= 1e-11
    cnv, mb = m.norms(y, R, 2 * DAY)
    ng = norms.cpu().numpy()
    assert np.allclose(ng[:3], cnv, rtol=1e-9, atol=0) and np.allclose(ng[3:6], mb, rtol=1e-9,
                                                                        atol=1e-300)


def test_live_dead_limit_bitwise(opm):
    """The live-oil kernels with no dissolution (r_s = 0, every cell s_g)
    give the bits of the dead-oil row-per-lane kernel (the same instruction
    sequence with the live terms zero; the LDS-tiled dead-oil kernel sums in
    another order and is compared with it in test_gpu_assembly)."""
    dead = cases.box_case(5, 4, 3, seed=3)
    live = cases.box_case(5, 4, 3, seed=3)
    live.fluid = cases.Fluid(live=True, rs_c=0.0, bo_r=0.5, muo_r=0.2)
    gd, gl = opm.GpuModel(dead), opm.GpuModel(live)
    y = gd.state(cases.random_state(dead, seed=4))
    a0 = gd.accumulation(gd.state(cases.random_state(dead, seed=5)))
    assert torch.equal(gl.accumulation(y), gd.accumulation(y))
    opm.lib().opm_set_option(opm.OPT_ASSEMBLY, 0)
    try:
        Rd, Jd, _ = gd.assemble(y, a0, DAY)
    finally:
        opm.lib().opm_set_option(opm.OPT_ASSEMBLY, 1)
    Rl, Jl, _ = gl.assemble(y, a0, DAY)
    assert torch.equal(Rd, Rl) and torch.equal(Jd, Jl)


def _physical(c, y, mean):
    rs = c.fluid.rs_c * y[:, 0]
    sg = np.where(mean == 0, y[:, 2], 0.0)
    r = np.where(mean == 0, rs, y[:, 2])
    return y[:, 0], y[:, 1], sg, r


def _compare_live(c, yg, mg, yo, mo, what):
    pg, swg, sgg, rg = _physical(c, yg, mg)
    po, swo, sgo, ro = _physical(c, yo, mo)
    ep = np.abs(pg - po).max() / np.abs(po).max()
    es = max(np.abs(swg - swo).max(), np.abs(sgg - sgo).max())
    er = np.abs(rg - ro).max() / np.abs(ro).max()
    assert ep <= 1e-6 and es <= 1e-6 and er <= 1e-6, f"{what}: p {ep:.2e} s {es:.2e} r {er:.2e}"
    differ = mg != mo
    borderline = (np.abs(sgg) <= 1e-4) & (np.abs(sgo) <= 1e-4)
    assert np.all(borderline[differ]), f"{what}: meanings differ away from the switching point"


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("blk", [None, (4, 4, 5)], ids=["single", "blocks"])
def test_live_run_c6(opm, precision, blk):
    """The live-oil depletion with phase appearance: 20 report steps of 15
    days; after each one the state and meanings match the oracle's run."""
    c = cases.config_live()
    g = opm.GpuModel(c, ilu_blocks=blk)
    m = oracle.Model(c)
    ostates, oreps = m.run()
    y, gstates, greps = g.run(opts=opm.default_opts(c, precision=precision))
    for s, (yg, mg, yo, mo) in enumerate(zip(gstates, g.run_meanings, ostates, m.run_meanings)):
        _compare_live(c, yg, mg, yo, mo, f"C6 step {s}")
    assert (g.run_meanings[-1] == 0).sum() > 100   # free gas has appeared
    for rg, ro in zip(greps, oreps):
        assert abs(rg["newton_its"] - ro["newton_its"]) <= 1


def test_live_newton_switches(opm):
    """One Newton step from an undersaturated state to a pressure below the
    bubble point: the same cells switch to free gas as in the oracle."""
    c = cases.config_live()
    g = opm.GpuModel(c)
    m = oracle.Model(c)
    y0 = c.initial_state()
    st, yo, rep = m.newton_step(y0, y0, 15 * DAY)
    assert st == 0
    yg = g.initial_state()
    st, grep = g.newton_step(yg, g.initial_state(), 15 * DAY)
    assert st == 0
    _compare_live(c, yg.cpu().numpy(), g.meaning(), yo, m.meaning(), "step 1")
    assert (m.meaning() == 0).any()


def test_live_restrictions(opm):
    """The ensemble and the learned-guess start selection are dead oil only."""
    import ctypes
    c = cases.config_live()
    g = opm.GpuModel(c)
    y = g.initial_state()
    with pytest.raises(opm.OpmError):
        g.guess_select(y, y, y, DAY)
    L = opm._ensemble_lib()
    members = (opm.Problem * 1)(g.pb)
    ys = (ctypes.c_void_p * 1)(y.data_ptr())
    nb = L.opm_ensemble_bytes(members, 1, 0)
    ens = torch.empty(max(nb, 256), dtype=torch.uint8, device=g.dev)
    assert L.opm_ensemble_prepare(members, ys, 1, 0, ens.data_ptr(), nb) == opm.EINVAL


# ------------------------------------------------------------- wet gas
def _wet_case(name):
    fl = cases.live_fluid()
    fl.rv_c = 0.05 / (3000 * PSI)
    if name == "C6_wet":
        c = cases.config_live()
        c.fluid = fl
        return c
    c = _live_box(*((5, 4, 3, 3) if name == "box" else (9, 7, 4, 5)), masked=name == "masked")
    c.fluid = fl
    return c


def _wet_state(c, seed):
    rng = np.random.default_rng(seed)
    n = c.n_active
    mean = rng.integers(0, 3, n).astype(np.uint8)
    y = np.empty((n, 3))
    y[:, 0] = rng.uniform(2800, 3200, n) * PSI
    y[:, 1] = rng.uniform(0.15, 0.4, n)
    rs, rv = c.fluid.rs_c * y[:, 0], c.fluid.rv_c * y[:, 0]
    y[:, 2] = np.where(mean == 0, rng.uniform(0.05, 0.3, n),
                       np.where(mean == 1, rng.uniform(0.3, 0.9, n) * rs,
                                rng.uniform(0.3, 0.9, n) * rv))
    return y, mean


@pytest.mark.parametrize("name", ["box", "masked", "C6_wet"])
def test_wet_assembly_parity(opm, name):
    """Wet gas (oil vaporised in the gas): accumulation, residual, Jacobian
    and norms with all three meanings against the oracle, at the live-oil
    tolerances."""
    c = _wet_case(name)
    g = opm.GpuModel(c)
    m = oracle.Model(c)
    y0, mean0 = _wet_state(c, seed=11)
    y, mean = _wet_state(c, seed=12)
    m.set_meaning(mean0)
    g.set_meaning(mean0)
    a_o = m.accumulation(y0)
    a_g = g.accumulation(g.state(y0)).cpu().numpy()
    assert np.abs(a_g - a_o).max() <= 1e-14 * np.abs(a_o).max()
    m.set_meaning(mean)
    g.set_meaning(mean)
    st, R, J = m.assemble(y, a_o, 2 * DAY)
    Rg, Jg, norms = g.assemble(g.state(y), g.state(a_o), 2 * DAY)
    Rg, Jg = Rg.cpu().numpy(), Jg.cpu().numpy()
    assert (np.abs(Rg - R) / (np.abs(R).max(axis=0) + 1e-300)).max() <= 1e-11
    Jf, Jgf = J.reshape(-1, 9), Jg.reshape(-1, 9)
    assert (np.abs(Jgf - Jf) / _colscale(Jf)).max() <= 1e-11
    cnv, mb = m.norms(y, R, 2 * DAY)
    ng = norms.cpu().numpy()
    assert np.allclose(ng[:3], cnv, rtol=1e-9, atol=0)


def test_wet_newton_iterates(opm):
    """Two Newton iterations from a state with all three meanings (linear
    solves to 1e-12): the iterates, meanings and switches equal the
    oracle's."""
    c = _wet_case("C6_wet")
    g = opm.GpuModel(c)
    m = oracle.Model(c)
    y, mean = _wet_state(c, seed=21)
    m.set_meaning(mean)
    g.set_meaning(mean)
    o_o = oracle.default_opts(c, max_newton=2, lin_rtol=1e-12)
    o_g = opm.default_opts(c, max_newton=2, lin_rtol=1e-12)
    st_o, yo, rep_o = m.newton_step(y, y, DAY, o_o)
    yg = g.state(y)
    st_g, rep_g = g.newton_step(yg, g.state(y), DAY, o_g)
    assert st_o == st_g and rep_o.newton_its == rep_g.newton_its == 2
    mg, mo = g.meaning(), m.meaning()
    assert np.array_equal(mg, mo)
    yg = yg.cpu().numpy()
    assert np.abs(yg[:, 0] - yo[:, 0]).max() <= 1e-8 * np.abs(yo[:, 0]).max()
    assert np.abs(yg[:, 1] - yo[:, 1]).max() <= 1e-8
    x_scale = np.where(mo == 0, 1.0, np.abs(yo[:, 2]).max())
    assert (np.abs(yg[:, 2] - yo[:, 2]) / x_scale).max() <= 1e-8


def _wet_physical(c, y, mean):
    sg = np.where(mean == 0, y[:, 2], np.where(mean == 2, 1.0 - y[:, 1], 0.0))
    r = np.where(mean == 1, y[:, 2], c.fluid.rs_c * y[:, 0])
    rv = np.where(mean == 2, y[:, 2], c.fluid.rv_c * y[:, 0])
    return sg, 1.0 - y[:, 1] - sg, r, rv


@pytest.mark.parametrize("blk", [None, (4, 4, 5)], ids=["single", "blocks"])
def test_wet_run(opm, blk):
    """Dry gas into undersaturated oil with wet gas, twelve 30-day steps:
    after each the pressure, saturations and both ratios match the oracle's
    run to 1e-6 (ratios relative to their largest value), the meanings
    agree away from the switching points, and oil-free cells have
    appeared."""
    c = cases.config_wet()
    g = opm.GpuModel(c, ilu_blocks=blk)
    m = oracle.Model(c)
    ostates, oreps = m.run()
    y, gstates, greps = g.run()
    for s, (yg, mg, yo, mo) in enumerate(zip(gstates, g.run_meanings, ostates, m.run_meanings)):
        sgg, sog, rg, rvg = _wet_physical(c, yg, mg)
        sgo, soo, ro, rvo = _wet_physical(c, yo, mo)
        assert np.abs(yg[:, 0] - yo[:, 0]).max() <= 1e-6 * np.abs(yo[:, 0]).max(), s
        assert np.abs(yg[:, 1] - yo[:, 1]).max() <= 1e-6, s
        assert np.abs(sgg - sgo).max() <= 1e-6 and np.abs(sog - soo).max() <= 1e-6, s
        assert np.abs(rg - ro).max() <= 1e-6 * np.abs(ro).max(), s
        assert np.abs(rvg - rvo).max() <= 1e-6 * np.abs(rvo).max(), s
        differ = mg != mo
        border = ((np.abs(sgo) <= 1e-4) | (np.abs(soo) <= 1e-4)) & \
                 ((np.abs(sgg) <= 1e-4) | (np.abs(sog) <= 1e-4))
        assert np.all(border[differ]), f"step {s}: meanings differ away from a switching point"
    assert (g.run_meanings[-1] == 2).sum() > 0
    for rg_, ro_ in zip(greps, oreps):
        assert abs(rg_["newton_its"] - ro_["newton_its"]) <= 1
