"""The benchmarked configurations against the oracle, report step by report
step, at the parity bar of the path: pressure within 1e-6 of the oracle's
largest pressure, saturations within 1e-6 absolute (after every report step).

* the 9000-cell waterflood as benchmarked (block ILU0 on 4x4x15 columns, FP64)
  for all 30 steps;
* the masked 45k-cell case in mixed precision (FP32 ILU(0) factors and
  sweeps inside FP64 BiCGStab) for all 10 steps, with the ILU(0) of the whole
  system and with block ILU0 on 8x8x22 columns;
* the 500k-cell waterflood as benchmarked (block ILU0 on 4x4x50 columns) for
  three report steps, at 4000 sampled cells against the oracle's states
  stored by tests/golden/make_golden.py;
* the three largest members of the 64-member ensemble (108k, 100k and 98k
  cells, levels wider than the factor's LDS window) for one report step in
  the batched launch, FP64 and FP32 factors, one workgroup per member with
  each member's ILU(0) and in the benchmarked launch (block ILU0 on 6x6
  whole-column subdomains per member, 256 workgroups), against stored
  oracle states; all 64 members in the benchmarked launch against the
  single-system path on the same partition;
* forced time-step cuts (a tight Newton cap) on live oil and on standard wells
  with binding limits, against the oracle's runs with the same cap.
The oracle runs use its OpenMP build (the plain build's bits).
"""
import os

import numpy as np
import pytest
import torch

import oracle
from paper_1910_06059_amd import cases
from paper_1910_06059_amd.cases import DAY, PSI, STB

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def opm():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    from paper_1910_06059_amd import opm as _opm
    _opm.init()
    return _opm


def _errors(yg, yo):
    return (np.abs(yg[:, 0] - yo[:, 0]).max() / np.abs(yo[:, 0]).max(),
            np.abs(yg[:, 1:] - yo[:, 1:]).max())


def _compare(yg, yo, what):
    ep, es = _errors(yg, yo)
    assert ep <= 1e-6 and es <= 1e-6, f"{what}: p rel {ep:.2e}, s abs {es:.2e}"


def _oracle_run(case, so, steps=None, blocks=None):
    m = oracle.Model(case, lib_path=so)
    if blocks:
        m.set_ilu_blocks(*blocks)
    states, _ = m.run(n_steps=steps)
    return states


def test_c2_block_ilu0_all_steps(opm, oracle_omp):
    case = cases.config2()
    print("C2 block ILU0 4x4x15, 30 steps", flush=True)
    ostates = _oracle_run(case, oracle_omp)
    g = opm.GpuModel(case, ilu_blocks=(4, 4, case.nz))
    _, gstates, greps = g.run()
    assert len(gstates) == len(ostates) == 30
    for s, (yg, yo) in enumerate(zip(gstates, ostates)):
        _compare(yg, yo, f"C2 block ILU0 step {s}")


@pytest.fixture(scope="module")
def c3_oracle(oracle_omp):
    case = cases.config3()
    return case, _oracle_run(case, oracle_omp)


@pytest.mark.parametrize("blocks", [None, (8, 8, 22)], ids=["ilu0", "block_8x8x22"])
def test_c3_mixed_precision_all_steps(opm, c3_oracle, blocks):
    case, ostates = c3_oracle
    print(f"C3 mixed precision, blocks {blocks}", flush=True)
    g = opm.GpuModel(case, ilu_blocks=blocks)
    _, gstates, greps = g.run(opts=opm.default_opts(case, precision=opm.PREC_MIXED))
    assert len(gstates) == len(ostates) == 10
    for s, (yg, yo) in enumerate(zip(gstates, ostates)):
        _compare(yg, yo, f"C3 mixed step {s}")


def _golden(name):
    path = os.path.join(GOLDEN, name)
    if not os.path.exists(path):
        pytest.fail(f"{path} missing: run tests/golden/make_golden.py")
    return np.load(path)


@pytest.mark.slow
def test_c5_block_ilu0_three_steps(opm):
    d = _golden("c5_block_ilu0.npz")
    case = cases.config5(5008)
    print("C5 block ILU0 4x4x50, 3 steps", flush=True)
    g = opm.GpuModel(case, ilu_blocks=(4, 4, case.nz))
    _, gstates, _ = g.run(n_steps=3)
    idx = d["idx"]
    for s, yg in enumerate(gstates):
        yo = np.stack([d["p"][s], d["sw"][s], d["sg"][s]], axis=1)
        _compare(yg[idx], yo, f"C5 step {s} (4000 sampled cells)")


@pytest.mark.slow
@pytest.mark.parametrize("split", [None, (6, 6)], ids=["whole", "split6x6"])
@pytest.mark.parametrize("precision", [0, 1])
def test_c4_largest_members(opm, precision, split):
    """The three largest ensemble members, one report step, against the
    oracle's states: one workgroup per member with each member's ILU(0), and
    the benchmarked launch (6x6 whole-column block ILU0 per member, the
    members' workgroups in proportion to their rows over 256)."""
    d = _golden("c4_largest.npz")
    members = [int(m) for m in d["members"]]
    ms = [cases.config4_member(m) for m in members]
    print(f"C4 members {members} ({[c.n_active for c in ms]} cells), precision {precision}, "
          f"split {split}", flush=True)
    ens = opm.Ensemble(ms, precision=precision, member_split=split)
    if split is not None:
        ens.configure(256, 0, 0, 256)
    ens.launch(ms[0].report_dt[0], 1)
    torch.cuda.synchronize()
    reps = ens.read_reports()
    states = ens.states()
    for k, m in enumerate(members):
        assert reps[k]["status"] == 0 and reps[k]["steps_done"] == 1, reps[k]
        idx = d[f"m{m}_idx"]
        yo = np.stack([d[f"m{m}_p"][0], d[f"m{m}_sw"][0], d[f"m{m}_sg"][0]], axis=1)
        _compare(states[k][idx], yo, f"C4 member {m}")


@pytest.mark.slow
def test_c4_split_members_match_single_system_path(opm):
    """All 64 ensemble members in the benchmarked launch shape (FP64, 6x6
    whole-column block ILU0 per member, 256 workgroups) against the
    single-system path's run of every member on the same partition: the same
    Newton iterations, states within 1e-9 (only the order of summation in
    the reductions differs)."""
    split = (6, 6)
    ms = [cases.config4_member(m) for m in range(64)]
    ens = opm.Ensemble(ms, precision=0, member_split=split)
    ens.configure(256, 0, 0, 256)
    dt = ms[0].report_dt[0]
    ens.launch(dt, 1)
    torch.cuda.synchronize()
    reps = ens.read_reports()
    states = ens.states()
    worst = (0.0, 0.0)
    for m, case in enumerate(ms):
        assert reps[m]["status"] == 0 and reps[m]["steps_done"] == 1, (m, reps[m])
        g = opm.GpuModel(case, ilu_blocks=opm.member_blocks(case, split))
        y = g.initial_state()
        st, rep = g.advance(y, dt)
        assert st == 0, m
        yg = y.cpu().numpy()
        ep = np.abs(states[m][:, 0] - yg[:, 0]).max() / np.abs(yg[:, 0]).max()
        es = np.abs(states[m][:, 1:] - yg[:, 1:]).max()
        worst = (max(worst[0], ep), max(worst[1], es))
        assert ep <= 1e-9 and es <= 1e-9, (m, ep, es)
        assert reps[m]["newton_its"] == rep.newton_its, m
    print(f"64 members: max p_rel {worst[0]:.2e}, max s_abs {worst[1]:.2e}", flush=True)


def _switch_case(inj_psi, prod_stb):
    c = cases.config1()
    c.standard_wells = True
    c.wells[0].limit = inj_psi * PSI
    c.wells[1].limit = prod_stb * STB / DAY
    return c


@pytest.mark.parametrize("which", ["live", "std_wells"])
def test_forced_cuts_match_oracle(opm, which):
    """A tight Newton cap forces time-step cuts (sec. 2.3): the GPU's report
    steps meet the oracle's run with the same cap, and both cut."""
    if which == "live":
        case, cap = cases.config_live(), 3
        steps = list(case.report_dt[:2])
    else:
        case, cap = _switch_case(7000, 1500), 7
        steps = [30 * DAY] * 2
    m = oracle.Model(case)
    g = opm.GpuModel(case)
    y = case.initial_state()
    yg = g.initial_state()
    o_cuts = g_cuts = 0
    for s, dt in enumerate(steps):
        st, y, orep = m.advance(y, dt, oracle.default_opts(case, max_newton=cap))
        stg, grep = g.advance(yg, dt, opm.default_opts(case, max_newton=cap))
        assert st == 0 and stg == 0, (st, stg)
        o_cuts += orep.cuts
        g_cuts += grep.cuts
        _compare(yg.cpu().numpy(), y, f"{which} step {s}")
    assert o_cuts >= 1 and g_cuts >= 1, (o_cuts, g_cuts)
