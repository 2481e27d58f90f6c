"""Batched ensemble (one persistent launch, one workgroup per member) against
the oracle run of every member on its own, and against the single-system GPU
path.  Parity bar as for single systems: pressure 1e-6 relative, saturations
1e-6 absolute after every launch of report steps."""
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


def _members():
    ms = [
        cases.box_case(6, 5, 3, seed=11, name="m0"),
        cases.box_case(9, 4, 5, seed=12, name="m1", wells=[
            Well("G", cases.WELL_RATE_INJ, [(0, 0, 0)], 2e3 * cases.MSCF / DAY, phase=cases.GAS),
            Well("P", cases.WELL_BHP_PROD, [(8, 3, 4)], 3000 * PSI)]),
        cases.config1(),
        cases.box_case(3, 3, 3, seed=13, name="m3"),
        cases.box_case(12, 10, 2, seed=14, name="m4", mask=cases.masked_mask(
            np.random.default_rng(3), (2, 10, 12), 150), wells=[]),
    ]
    act = np.argwhere(ms[4].mask)
    k, j, i = act[0]
    k2, j2, i2 = act[-1]
    ms[4].wells = [Well("I", cases.WELL_RATE_INJ, [(int(i), int(j), int(k))], 200 * STB / DAY),
                   Well("P", cases.WELL_BHP_PROD, [(int(i2), int(j2), int(k2))], 3000 * PSI)]
    return ms


def _check(yg, yo, what):
    ep = np.abs(yg[:, 0] - yo[:, 0]).max() / np.abs(yo[:, 0]).max()
    es = np.abs(yg[:, 1:] - yo[:, 1:]).max()
    assert ep <= 1e-6 and es <= 1e-6, f"{what}: p {ep:.2e} s {es:.2e}"


@pytest.mark.parametrize("precision", [0, 1])
def test_ensemble_matches_oracle(opm, precision):
    ms = _members()
    ens = opm.Ensemble(ms, precision=precision)
    dt = 10 * DAY
    ens.launch(dt, 2)
    torch.cuda.synchronize()
    reps = ens.read_reports()
    states = ens.states()
    for m, case in enumerate(ms):
        assert reps[m]["status"] == 0 and reps[m]["steps_done"] == 2, reps[m]
        om = oracle.Model(case)
        y = case.initial_state()
        its = 0
        for _ in range(2):
            st, y, r = om.advance(y, dt)
            assert st == 0
            its += r.newton_its
        _check(states[m], y, f"member {m}")
        assert abs(reps[m]["newton_its"] - its) <= 2
    # a second launch continues from the states left by the first
    ens.launch(dt, 1)
    torch.cuda.synchronize()
    states2 = ens.states()
    om = oracle.Model(ms[0])
    st, y, r = om.advance(states[0], dt)
    _check(states2[0], y, "member 0, second launch")


def test_ensemble_matches_single_system_path(opm):
    ms = _members()[:3]
    ens = opm.Ensemble(ms, precision=opm.PREC_FP64)
    dt = 10 * DAY
    ens.launch(dt, 1)
    torch.cuda.synchronize()
    reps = ens.read_reports()
    for m, case in enumerate(ms):
        g = opm.GpuModel(case)
        y = g.initial_state()
        st, rep = g.advance(y, dt)
        assert st == 0
        yg = y.cpu().numpy()
        ye = ens.states()[m]
        assert np.abs(ye[:, 0] - yg[:, 0]).max() <= 1e-9 * np.abs(yg[:, 0]).max()
        assert np.abs(ye[:, 1:] - yg[:, 1:]).max() <= 1e-9
        assert reps[m]["newton_its"] == rep.newton_its


def test_ensemble_graph_capture(opm):
    """The launch is one graph node: replays equal eager launches."""
    ms = _members()[:2]
    dt = 5 * DAY
    eager = opm.Ensemble(ms, precision=opm.PREC_MIXED)
    for _ in range(3):
        eager.launch(dt, 1)
        torch.cuda.synchronize()
    ref = eager.states()
    ens = opm.Ensemble(ms, precision=opm.PREC_MIXED)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            ens.launch(dt, 1)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    # capture does not run the kernel: states are still initial
    assert np.array_equal(ens.states()[0], ms[0].initial_state())
    for _ in range(3):
        g.replay()
        torch.cuda.synchronize()
        _ = ens.read_reports()   # eager work between replays
    got = ens.states()
    for m in range(2):
        assert np.array_equal(got[m], ref[m]), f"member {m}: graph replay differs from eager"


def test_ensemble_c4_members(opm):
    """Three of the 64 ensemble members (the smallest), one 15-day report step,
    against the oracle."""
    sizes = []
    for m in range(64):
        c = cases.config4_member(m)
        sizes.append((c.n_active, m))
    picks = [m for _, m in sorted(sizes)[:3]]
    ms = [cases.config4_member(m) for m in picks]
    ens = opm.Ensemble(ms, precision=opm.PREC_MIXED)
    ens.launch(15 * DAY, 1)
    torch.cuda.synchronize()
    reps = ens.read_reports()
    for k, case in enumerate(ms):
        assert reps[k]["status"] == 0
        st, y, r = oracle.Model(case).advance(case.initial_state(), 15 * DAY)
        assert st == 0
        _check(ens.states()[k], y, case.name)


_ORACLE_ONE_STEP = {}


def _oracle_step(case, dt):
    key = (case.name, dt)
    if key not in _ORACLE_ONE_STEP:
        st, y, _ = oracle.Model(case).advance(case.initial_state(), dt)
        assert st == 0
        _ORACLE_ONE_STEP[key] = y
    return _ORACLE_ONE_STEP[key]


SHAPES = [(t, f, r) for t in (256, 128) for f in (1, 0) for r in (0, 1)]


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "t%d-fw%d-ring%d" % s)
def test_ensemble_shapes_match_oracle(opm, shape, precision):
    """Every launch shape the autotuner can pick gives oracle-matching states."""
    ms = _members()
    ens = opm.Ensemble(ms, precision=precision)
    ens.configure(*shape)
    if shape[2]:
        # the ring holds sweep_span + max_level + 1 rows rounded up to a power of two
        ts = 4 if precision else 8
        rings = []
        for m in ens.members:
            c = 1
            while c < m.sweep_span + m.max_level + 1:
                c <<= 1
            rings.append(3 * ts * c)
        assert ens.config.sweep_bytes >= max(rings)
    dt = 10 * DAY
    ens.launch(dt, 1)
    torch.cuda.synchronize()
    reps = ens.read_reports()
    for m, case in enumerate(ms):
        assert reps[m]["status"] == 0 and reps[m]["steps_done"] == 1, (m, reps[m])
        _check(ens.states()[m], _oracle_step(case, dt), f"{shape} member {m}")


def test_ensemble_autotune(opm, tmp_path):
    """The autotuner times every shape, restores the states, configures the
    fastest; a cached choice is reused without trials."""
    ms = _members()
    ens = opm.Ensemble(ms, precision=opm.PREC_MIXED)
    y0 = ens.states()
    cache = str(tmp_path / "ensemble_tuning.json")
    dt = 10 * DAY
    t = ens.autotune(dt, cache=cache)
    assert not t["cached"] and len(t["trial_seconds"]) == 8
    assert t["threads"] in (128, 256) and t["ring"] in (0, 1) and t["fac_window"] in (0, 1)
    for m, y in enumerate(ens.states()):
        assert np.array_equal(y, y0[m]), f"member {m} not restored"
    ens.launch(dt, 1)
    torch.cuda.synchronize()
    for m, case in enumerate(ms):
        assert ens.read_reports()[m]["status"] == 0
        _check(ens.states()[m], _oracle_step(case, dt), f"tuned member {m}")
    ens2 = opm.Ensemble(ms, precision=opm.PREC_MIXED)
    t2 = ens2.autotune(dt, cache=cache)
    assert t2["cached"] and (t2["threads"], t2["ring"], t2["fac_window"]) == (
        t["threads"], t["ring"], t["fac_window"])


def test_ensemble_graph_capture_tuned_shape(opm):
    """A configured shape is captured and replayed like the default one."""
    ms = _members()[:3]
    dt = 5 * DAY
    eager = opm.Ensemble(ms, precision=opm.PREC_FP64)
    eager.configure(128, 0, 1)
    for _ in range(2):
        eager.launch(dt, 1)
        torch.cuda.synchronize()
    ref = eager.states()
    ens = opm.Ensemble(ms, precision=opm.PREC_FP64)
    ens.configure(128, 0, 1)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            ens.launch(dt, 1)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    for _ in range(2):
        g.replay()
        torch.cuda.synchronize()
        _ = ens.read_reports()
    for m in range(3):
        assert np.array_equal(ens.states()[m], ref[m])


SPLIT = (2, 2)


def _split_ensemble(opm, ms, precision, wgs):
    ens = opm.Ensemble(ms, precision=precision, member_split=SPLIT)
    ens.configure(256, 0, 0, wgs)
    return ens


def test_split_members_match_single_system_path(opm):
    """Several workgroups per member (each a range of the member's 2x2
    block-ILU0 column subdomains, meeting at device-memory barriers) give the
    single-system path's block-ILU0 run of every member: the same Newton
    iterations, states within 1e-9 (only the order of summation in the
    reductions differs)."""
    ms = _members()
    ens = _split_ensemble(opm, ms, opm.PREC_FP64, 12)
    # the larger members got more than one workgroup
    assert ens.config.wgs > len(ms)
    dt = 10 * DAY
    ens.launch(dt, 1)
    torch.cuda.synchronize()
    reps = ens.read_reports()
    for m, case in enumerate(ms):
        assert reps[m]["status"] == 0 and reps[m]["steps_done"] == 1, (m, reps[m])
        g = opm.GpuModel(case, ilu_blocks=opm.member_blocks(case, SPLIT))
        y = g.initial_state()
        st, rep = g.advance(y, dt)
        assert st == 0
        yg = y.cpu().numpy()
        ye = ens.states()[m]
        assert np.abs(ye[:, 0] - yg[:, 0]).max() <= 1e-9 * np.abs(yg[:, 0]).max(), m
        assert np.abs(ye[:, 1:] - yg[:, 1:]).max() <= 1e-9, m
        assert reps[m]["newton_its"] == rep.newton_its, m


@pytest.mark.parametrize("precision", [0, 1])
def test_split_members_match_oracle(opm, precision):
    """Split members, FP64 and FP32 factors, two report steps, against the
    oracle's run of every member (1e-6)."""
    ms = _members()
    ens = _split_ensemble(opm, ms, precision, 256)
    dt = 10 * DAY
    ens.launch(dt, 2)
    torch.cuda.synchronize()
    reps = ens.read_reports()
    for m, case in enumerate(ms):
        assert reps[m]["status"] == 0 and reps[m]["steps_done"] == 2, (m, reps[m])
        om = oracle.Model(case)
        y = case.initial_state()
        for _ in range(2):
            st, y, _ = om.advance(y, dt)
            assert st == 0
        _check(ens.states()[m], y, f"split member {m}")


def test_split_members_graph_replay(opm):
    """The launch with several workgroups per member (a reset of the barrier
    words and the persistent kernel) replays from a graph with the eager
    launches' bits."""
    ms = _members()[:3]
    dt = 5 * DAY
    eager = _split_ensemble(opm, ms, opm.PREC_MIXED, 8)
    for _ in range(2):
        eager.launch(dt, 1)
        torch.cuda.synchronize()
    ref = eager.states()
    ens = _split_ensemble(opm, ms, opm.PREC_MIXED, 8)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            ens.launch(dt, 1)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    for _ in range(2):
        g.replay()
        torch.cuda.synchronize()
        _ = ens.read_reports()
    for m in range(3):
        assert np.array_equal(ens.states()[m], ref[m]), m


def test_split_members_barrier_gives_up(opm):
    """A member barrier that gives up (forced from the host: a spin limit of
    zero polls) fails exactly the members with several workgroups, with
    OPM_EHIP, instead of hanging; the next launch with the normal limit
    works again."""
    ms = _members()
    ens = _split_ensemble(opm, ms, opm.PREC_MIXED, 12)
    assert ens.config.wgs > len(ms)
    dt = 10 * DAY
    try:
        opm.set_option(opm.OPT_ENSEMBLE_SPIN, 0)
        ens.launch(dt, 1)
        torch.cuda.synchronize()
        reps = ens.read_reports()
    finally:
        opm.set_option(opm.OPT_ENSEMBLE_SPIN, 1 << 22)
    failed = [m for m in range(len(ms)) if reps[m]["status"] == opm.EHIP]
    assert failed
    for m in range(len(ms)):
        assert reps[m]["status"] in (0, opm.EHIP), (m, reps[m])
        if m in failed:   # only members with subdomains to share out
            assert ens.members[m].pb.n_sub > 1, m
    for t, mm in zip(ens.y, ens.members):
        t.copy_(mm.initial_state())
    ens.launch(dt, 1)
    torch.cuda.synchronize()
    for m, case in enumerate(ms):
        assert ens.read_reports()[m]["status"] == 0, m
        _check(ens.states()[m], _oracle_step(case, dt), f"member {m} after the failed launch")
