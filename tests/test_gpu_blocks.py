"""Block ILU0 over subdomain boxes (one block per subdomain, one workgroup per
subdomain on the GPU) against the oracle's block ILU0 on the same partition.

Tolerances as for the single-block path: inverse pivots and sweeps to 1e-9
relative in FP64 and 1e-4 with FP32 factors; converged Newton states to 1e-6
(relative pressure, absolute saturation) against the oracle's single-block
run, since the preconditioner changes the linear iterations only.  The launch
shapes (one workgroup per subdomain, one workgroup for all levels, one launch
per level) compute each row in the same order: bitwise equal results.
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


def _masked():
    c = cases.box_case(9, 7, 4, seed=5, mask=cases.masked_mask(
        np.random.default_rng(8), (4, 7, 9), 150), wells=[])
    act = np.argwhere(c.mask)
    k, j, i = act[0]
    k2, j2, i2 = act[-1]
    c.wells = [Well("I", cases.WELL_RATE_INJ, [(int(i), int(j), int(k))], 300 * STB / DAY),
               Well("P", cases.WELL_BHP_PROD, [(int(i2), int(j2), int(k2))], 3000 * PSI)]
    return c


CASES = {
    "box_ragged": (lambda: cases.box_case(5, 4, 3, seed=3, wells=[
        Well("I", cases.WELL_RATE_INJ, [(0, 0, k) for k in range(3)], 800 * STB / DAY),
        Well("P", cases.WELL_BHP_PROD, [(4, 3, 2)], 3000 * PSI)]), (2, 3, 2)),
    "C1_columns": (cases.config1, (4, 4, 3)),
    "masked": (_masked, (3, 3, 4)),
    "jacobi": (lambda: cases.box_case(5, 4, 3, seed=4), (1, 1, 1)),
    "C2_columns": (cases.config2, (4, 4, 15)),
}


def _system(case, blk, seed=1):
    m = oracle.Model(case)
    m.set_ilu_blocks(*blk)
    y = cases.random_state(case, seed=seed)
    st, R, J = m.assemble(y, m.accumulation(cases.random_state(case, seed=seed + 1)), 2 * DAY)
    st, F = m.ilu0(J)
    assert st == 0
    return m, R, J, F


def _pivot_bytes(g, precision):
    """The inverse pivots lead the ILU buffer: FP64 [9][ns], then with FP32
    factors their FP32 copy [9][ns]."""
    ns = (g.n + 63) // 64 * 64
    return 8 * 9 * ns if precision == 0 else 8 * 9 * ns + 4 * 9 * ns


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("name", list(CASES))
def test_block_ilu0_parity(opm, name, precision):
    make, blk = CASES[name]
    case = make()
    g = opm.GpuModel(case, ilu_blocks=blk)
    assert g.pb.n_sub > 1
    m, R, J, F = _system(case, blk)
    Jg = torch.from_numpy(J).to(g.dev)
    ilu, status = g.ilu0_factor(Jg, precision)
    assert int(status.item()) == 0
    ns = (g.n + 63) // 64 * 64
    dinv = ilu.view(torch.float64)[:9 * ns].view(9, ns).cpu().numpy()[:, :g.n]
    rp, ci = m.pattern()
    perm = g.host["perm"][:g.n]
    for pos in range(g.n):
        i = perm[pos]
        q = [k for k in range(rp[i], rp[i + 1]) if ci[k] == i][0]
        ref = np.linalg.inv(F[q])
        assert np.abs(dinv[:, pos].reshape(3, 3) - ref).max() <= 1e-9 * np.abs(ref).max()
    r = np.random.default_rng(4).standard_normal((g.n, 3))
    xo = m.ilu0_apply(F, r)
    xg = g.ilu0_apply(ilu, g.state(r), precision).cpu().numpy()
    tol = 1e-9 if precision == 0 else 1e-4
    assert np.abs(xg - xo).max() <= tol * np.abs(xo).max()


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("name", ["C2_columns", "masked", "box_ragged"])
def test_block_launch_shapes_bitwise_equal(opm, name, precision):
    """One workgroup per subdomain (automatic), one workgroup for all levels
    and one launch per level give bitwise equal inverse pivots and sweeps;
    so do one and two levels of sweep data in flight."""
    make, blk = CASES[name]
    case = make()
    g = opm.GpuModel(case, ilu_blocks=blk)
    y = g.state(cases.random_state(case, 5))
    acc0 = g.accumulation(g.state(cases.random_state(case, 6)))
    R, J, _ = g.assemble(y, acc0, DAY)
    nfac = _pivot_bytes(g, precision)
    out = []
    try:
        for mode in (-1, 2, 1, 0):
            opm.set_option(opm.OPT_SWEEP_MODE, mode)
            ilu, status = g.ilu0_factor(J, precision)
            assert int(status.item()) == 0
            out.append((ilu[:nfac].clone(), g.ilu0_apply(ilu, R, precision)))
    finally:
        opm.set_option(opm.OPT_SWEEP_MODE, -1)
    for mode, (f, x) in zip((2, 1, 0), out[1:]):
        assert torch.equal(f, out[0][0]), (name, precision, mode, "factors")
        assert torch.equal(x, out[0][1]), (name, precision, mode, "sweep")
    ilu, _ = g.ilu0_factor(J, precision)
    try:
        for depth in (1, 2):
            opm.set_option(opm.OPT_BLOCK_DEPTH, depth)
            assert torch.equal(g.ilu0_apply(ilu, R, precision), out[0][1]), (name, depth)
    finally:
        opm.set_option(opm.OPT_BLOCK_DEPTH, 0)


def test_block_wide_subdomain(opm):
    """A subdomain whose levels are wider than the 256-thread workgroup
    (17 x 17 x 33: up to 289 rows per level; one subdomain, forced to the
    one-workgroup-per-subdomain shape, FP32 so that its vector fits in LDS)
    against the oracle and bitwise against the per-level launches."""
    case = cases.box_case(17, 17, 33, seed=12, wells=[])
    blk = (17, 17, 33)
    g = opm.GpuModel(case, ilu_blocks=blk)
    assert g.pb.n_sub == 1 and g.pb.max_width > 256
    m, R, J, F = _system(case, blk)
    Jg = torch.from_numpy(J).to(g.dev)
    r = np.random.default_rng(6).standard_normal((g.n, 3))
    out = []
    try:
        for mode in (2, 1):
            opm.set_option(opm.OPT_SWEEP_MODE, mode)
            ilu, status = g.ilu0_factor(Jg, opm.PREC_MIXED)
            assert int(status.item()) == 0
            out.append(g.ilu0_apply(ilu, g.state(r), opm.PREC_MIXED))
    finally:
        opm.set_option(opm.OPT_SWEEP_MODE, -1)
    assert torch.equal(out[0], out[1])
    xo = m.ilu0_apply(F, r)
    assert np.abs(out[0].cpu().numpy() - xo).max() <= 1e-4 * np.abs(xo).max()


def test_block_bicgstab_matches_oracle_iterations(opm):
    make, blk = CASES["C2_columns"]
    case = make()
    g = opm.GpuModel(case, ilu_blocks=blk)
    m, R, J, F = _system(case, blk)
    st, xo, its_o, rr = m.bicgstab(J, F, -R, rtol=1e-6)
    assert st == 0
    Jg = torch.from_numpy(J).to(g.dev)
    ilu, _ = g.ilu0_factor(Jg)
    x, rep = g.bicgstab(Jg, ilu, g.state(-R), rtol=1e-6)
    assert rep.status == 0
    its_g = rep.its - 0.5 * rep.half
    assert abs(its_g - its_o) <= 1.0, (its_g, its_o)
    res = -R - m.spmv(J, x.cpu().numpy())
    assert np.linalg.norm(res) <= 1e-6 * np.linalg.norm(R) * 1.0001


@pytest.mark.parametrize("depth", [1, 2], ids=["depth1", "depth2"])
@pytest.mark.parametrize("precision", [0, 1])
def test_block_fused_krylov(opm, precision, depth):
    """With one workgroup per subdomain the p and s updates of BiCGStab (and
    the tests before them) run inside the preconditioner sweeps; the solve
    takes the same iterations as the unfused sequence of kernels (the same
    preconditioner by per-level launches) and the same solution to the
    rounding of the reordered dot products, with one level of loads in
    flight or two (the automatic choice for the fused sweeps)."""
    make, blk = CASES["C2_columns"]
    case = make()
    g = opm.GpuModel(case, ilu_blocks=blk)
    m, R, J, F = _system(case, blk, seed=3)
    Jg = torch.from_numpy(J).to(g.dev)
    out = []
    try:
        opm.set_option(opm.OPT_BLOCK_DEPTH, depth)
        for mode in (-1, 1):
            opm.set_option(opm.OPT_SWEEP_MODE, mode)
            ilu, _ = g.ilu0_factor(Jg, precision)
            x, rep = g.bicgstab(Jg, ilu, g.state(-R), rtol=1e-6, precision=precision)
            assert rep.status == 0
            out.append((x.cpu().numpy(), rep.its, rep.half))
    finally:
        opm.set_option(opm.OPT_SWEEP_MODE, -1)
        opm.set_option(opm.OPT_BLOCK_DEPTH, 0)
    (x0, i0, h0), (x1, i1, h1) = out
    assert (i0, h0) == (i1, h1)
    # FP32 sweeps pass the last-bit differences of the dot products on at
    # their own rounding (about 1e-7 relative)
    tol = 1e-9 if precision == 0 else 1e-7
    assert np.abs(x0 - x1).max() <= tol * np.abs(x1).max()


@pytest.mark.parametrize("blk", [None, (4, 4, 15)], ids=["single", "blocks"])
def test_krylov_chunks_queued_ahead(opm, blk):
    """After a long solve the next one queues chunks of iterations ahead of
    its state reads, past its own end: its solution and report equal those of
    the same solve after a short one (no chunk queued ahead), bitwise, also
    when it stops at the iteration cap."""
    case = cases.config2()
    g = opm.GpuModel(case, ilu_blocks=blk)
    y = g.state(cases.random_state(case, 11))
    acc0 = g.accumulation(g.state(cases.random_state(case, 12)))
    R, J, _ = g.assemble(y, acc0, DAY)
    b = -R
    ilu, _ = g.ilu0_factor(J)

    def after(rtol_before, rtol, maxit):
        g.bicgstab(J, ilu, b, rtol=rtol_before)
        x, rep = g.bicgstab(J, ilu, b, rtol=rtol, maxit=maxit)
        torch.cuda.synchronize()
        return x.clone(), (rep.status, rep.its, rep.half, rep.rel_res)

    for rtol, maxit in ((1e-3, 500), (1e-12, 5)):
        x_short, r_short = after(0.9, rtol, maxit)
        x_long, r_long = after(1e-12, rtol, maxit)
        assert r_short == r_long
        assert torch.equal(x_short, x_long)
        if maxit == 5:
            assert r_long[0] == opm.ENOTCONV and r_long[1] == 5


@pytest.mark.parametrize("blk", [None, (4, 4, 15)], ids=["single", "blocks"])
def test_krylov_graph_replay(opm, blk):
    """Chunks of BiCGStab iterations replayed from a captured HIP graph give
    bitwise the solutions of the kernel-by-kernel enqueue, over several
    solves with other work and synchronisations between the replays."""
    case = cases.config2()
    g = opm.GpuModel(case, ilu_blocks=blk)
    systems = []
    for seed in (5, 7, 9):
        y = g.state(cases.random_state(case, seed))
        acc0 = g.accumulation(g.state(cases.random_state(case, seed + 1)))
        R, J, _ = g.assemble(y, acc0, DAY)
        systems.append((R.clone(), J.clone()))
    def solve_all():
        out = []
        for R, J in systems:
            ilu, _ = g.ilu0_factor(J)
            x, rep = g.bicgstab(J, ilu, -R, rtol=1e-8)
            assert rep.status == 0
            out.append((x.clone(), rep.its, rep.half))
            torch.cuda.synchronize()
        return out
    try:
        opm.set_option(opm.OPT_KRYLOV_CHUNK, 4)   # several chunks per solve
        opm.set_option(opm.OPT_KRYLOV_GRAPH, 0)
        eager = solve_all()
        opm.set_option(opm.OPT_KRYLOV_GRAPH, 1)
        for _ in range(2):
            got = solve_all()
            for (xe, ie, he), (xg, ig, hg) in zip(eager, got):
                assert (ie, he) == (ig, hg) and ie > 4
                assert torch.equal(xe, xg)
    finally:
        opm.set_option(opm.OPT_KRYLOV_GRAPH, 1)
        opm.set_option(opm.OPT_KRYLOV_CHUNK, 0)


def _compare_states(yg, yo, what):
    ep = np.abs(yg[:, 0] - yo[:, 0]).max() / np.abs(yo[:, 0]).max()
    es = np.abs(yg[:, 1:] - yo[:, 1:]).max()
    assert ep <= 1e-6 and es <= 1e-6, f"{what}: p rel err {ep:.2e}, s abs err {es:.2e}"


@pytest.mark.parametrize("precision", [0, 1])
def test_block_newton_c2(opm, precision):
    """Report steps of the 24x25x15 workload with column subdomains: states
    against the oracle's single-block run (the preconditioner does not move
    the converged state), Newton iterations against the oracle's block run."""
    case = cases.config2()
    blk = (4, 4, 15)
    g = opm.GpuModel(case, ilu_blocks=blk)
    m = oracle.Model(case)
    mb = oracle.Model(case)
    mb.set_ilu_blocks(*blk)
    y = case.initial_state()
    yb = case.initial_state()
    yg = g.initial_state()
    opts = opm.default_opts(case, precision=precision)
    for s, dt in enumerate(case.report_dt[:4]):
        st, y, rep = m.advance(y, dt)
        st2, yb, repb = mb.advance(yb, dt)
        assert st == 0 and st2 == 0
        stg, repg = g.advance(yg, dt, opts)
        assert stg == 0, stg
        _compare_states(yg.cpu().numpy(), y, f"C2 blocks step {s}")
        assert abs(repg.newton_its - repb.newton_its) <= 1


def test_block_full_size_c5(opm):
    """500k cells with 8 x 8 x 50 column subdomains (169 workgroups): the
    preconditioner solve against the oracle's block ILU0 on the whole
    system, and the BiCGStab solution by its true residual on the oracle's
    operator."""
    case = cases.config5(seed=5008)
    blk = (8, 8, 50)
    g = opm.GpuModel(case, ilu_blocks=blk)
    assert g.pb.n_sub == 169
    m, R, J, F = _system(case, blk, seed=9)
    Jg = torch.from_numpy(J).to(g.dev)
    ilu, status = g.ilu0_factor(Jg)
    assert int(status.item()) == 0
    r = np.random.default_rng(3).standard_normal((g.n, 3))
    xo = m.ilu0_apply(F, r)
    xg = g.ilu0_apply(ilu, g.state(r)).cpu().numpy()
    assert np.abs(xg - xo).max() <= 1e-9 * np.abs(xo).max()
    x, rep = g.bicgstab(Jg, ilu, g.state(-R), rtol=1e-6)
    assert rep.status == 0
    res = -R - m.spmv(J, x.cpu().numpy())
    assert np.linalg.norm(res) <= 1.01e-6 * np.linalg.norm(R)
