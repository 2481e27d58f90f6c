"""Pins of the CPU oracle against what the paper and mathematics fix.

Each ``pin_*`` function raises AssertionError when the oracle built at
``lib_path`` (default: the real oracle) disagrees with an independent
statement: a closed form, a worked value, an invariant, a special case that
reduces to a textbook result, brute force on a tiny input, or a library
routine (numpy's dense solver).  ``test_oracle_pins.py`` runs them on the real
oracle; ``test_oracle_mutants.py`` runs them on deliberately broken copies of
the oracle and requires every planted mistake to be caught.

Paper sections: residual and fluxes sec. 2.1.1 (eqs. materialbalance, flux1,
head); relative permeability sec. 2.1.5 (eq. gwseg); PVT sec. 2.1.6; wells
sec. 2.2.1 (eq. wellinflow); Newton sec. 2.3 (eq. linsystem); ILU0/BiCGStab
sec. 2.3.1; transmissibility appendix B.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.optimize import brentq

import oracle
from paper_1910_06059_amd import cases
from paper_1910_06059_amd.cases import DAY, FT, MD, PSI, STB, Well


def _model(case, lib_path):
    return oracle.Model(case, lib_path=lib_path)


def _dense(m, J):
    rp, ci = m.pattern()
    n = m.n
    D = np.zeros((3 * n, 3 * n))
    for i in range(n):
        for q in range(rp[i], rp[i + 1]):
            j = ci[q]
            D[3 * i:3 * i + 3, 3 * j:3 * j + 3] = J[q]
    return D


def _b(fl, a, p):
    """Constant-compressibility factor: the solution of (1/b) db/dp = c, b(p_ref) = 1."""
    return math.exp(fl.c[a] * (p - fl.p_ref))


# ---------------------------------------------------------------- geometry
def pin_series_transmissibility(lib_path=None):
    """Appendix B: T_ij is the series (harmonic) combination of the two half
    transmissibilities, so the resistances 1/T along a 1-D chain add up to the
    textbook series resistance between the first and last cell centres."""
    k = np.array([50.0, 400.0, 20.0, 150.0]) * MD
    c = cases.box_case(4, 1, 1, dx=10.0, dy=2.0, dz=3.0, wells=[], name="chain_x")
    c.perm_h = k.reshape(1, 1, 4).copy()
    m = _model(c, lib_path)
    T = m.geometry()["trans"]
    A = 2.0 * 3.0
    series = (5.0 / (k[0] * A) + 10.0 / (k[1] * A) + 10.0 / (k[2] * A) + 5.0 / (k[3] * A))
    assert len(T) == 3
    assert abs(np.sum(1.0 / T) - series) <= 1e-12 * series
    # vertical chain: kv = kv_kh * kh, unequal layer thicknesses
    kz = np.array([100.0, 30.0, 250.0]) * MD
    c = cases.box_case(1, 1, 3, dx=4.0, dy=5.0, dz=[1.0, 2.0, 4.0], wells=[], name="chain_z")
    c.perm_h = kz.reshape(3, 1, 1).copy()
    m = _model(c, lib_path)
    T = m.geometry()["trans"]
    kv = 0.1 * kz
    A = 20.0
    series = 0.5 / (kv[0] * A) + 2.0 / (kv[1] * A) + 2.0 / (kv[2] * A)
    assert abs(np.sum(1.0 / T) - series) <= 1e-12 * series
    # equal permeabilities: T = k A / d
    c = cases.box_case(2, 1, 1, dx=8.0, dy=2.0, dz=1.0, wells=[], sigma_ln=0.0, median_md=10.0)
    T = _model(c, lib_path).geometry()["trans"]
    assert abs(T[0] - 10.0 * MD * 2.0 / 8.0) <= 1e-14 * T[0]


def pin_depth_pore_volume(lib_path=None):
    """Cell-centre depth of layered cells and pore volume phi * V."""
    c = cases.box_case(2, 1, 3, dx=3.0, dy=2.0, dz=[1.0, 2.0, 4.0], poro=0.25, wells=[])
    g = _model(c, lib_path).geometry()
    assert np.allclose(g["depth"], [0.5, 0.5, 2.0, 2.0, 5.0, 5.0], rtol=0, atol=1e-14)
    assert np.allclose(g["pore_vol"], 0.25 * 6.0 * np.array([1, 1, 2, 2, 4, 4.0]), rtol=1e-15)


def pin_peaceman_worked_value(lib_path=None):
    """Peaceman index 2 pi k h / ln(r_o / r_w), r_o = 0.14 sqrt(dx^2 + dy^2):
    k = 100 mD, h = 20 ft, dx = dy = 1000 ft, r_w = 0.25 ft -> 5.66355101e-13 m^3."""
    c = cases.box_case(1, 1, 1, dx=1000 * FT, dy=1000 * FT, dz=20 * FT, sigma_ln=0.0,
                       median_md=100.0, wells=[Well("P", cases.WELL_BHP_PROD, [(0, 0, 0)], 1e7)])
    _, wi, _ = _model(c, lib_path).conns()
    assert abs(wi[0] - 5.663551011069723e-13) <= 1e-12 * 5.663551011069723e-13


# -------------------------------------------------------------- properties
def pin_compressibility(lib_path=None):
    """b = exp(c (p - p_ref)) solves (1/b) db/dp = c exactly: the log of b is
    linear in p with slope c; b(p_ref) = 1.  Worked values at 4800 psi."""
    c = cases.box_case(1, 1, 1, wells=[])
    m = _model(c, lib_path)
    fl = c.fluid
    s = np.array([0.5, 0.3, 0.2])   # s_w, s_o, s_g
    ps = np.array([fl.p_ref, 1000 * PSI, 3000 * PSI, 4800 * PSI, 9000 * PSI])
    bs = []
    for p in ps:
        acc = m.accumulation(np.array([[p, 0.5, 0.2]]))[0]
        bs.append(acc / s)
    bs = np.array(bs)
    assert np.allclose(bs[0], 1.0, rtol=0, atol=1e-15)
    slopes = np.diff(np.log(bs), axis=0) / np.diff(ps)[:, None]
    assert np.allclose(slopes, np.array(fl.c)[None, :], rtol=1e-9)
    assert abs(bs[3][2] - 119.7378) < 5e-5
    assert abs(bs[3][1] - 1.049016) < 5e-7
    assert abs(bs[3][0] - 1.014459) < 5e-7


def _two_cell(lib_path, y, g=0.0):
    fl = cases.Fluid(g=g)
    c = cases.box_case(2, 1, 1, dx=50.0, dy=10.0, dz=4.0, wells=[], fluid=fl)
    c.perm_h = np.array([[[80.0 * MD, 240.0 * MD]]])
    m = _model(c, lib_path)
    acc0 = m.accumulation(y)
    st, R, J = m.assemble(y, acc0, 10 * DAY)
    assert st == 0
    T = 10.0 * 4.0 / (25.0 / (80.0 * MD) + 25.0 / (240.0 * MD))
    return fl, R, J, T


def pin_darcy_flux_upwind(lib_path=None):
    """Eqs. (flux1), (head), upwind rule and eq. (gwseg) on two cells with g=0:
    F_alpha = b_alpha(p_U) k_r,alpha(s_U) / mu_alpha * T * (p_i - p_j).  Worked
    relative permeabilities: s_w = 0.56, s_g = 0.22 give normalised
    saturations 0.5, 0.25, 0.25 -> k_rw = 0.25, k_ro = k_rg = 0.0625."""
    y = np.array([[5000 * PSI, 0.56, 0.22], [4900 * PSI, 0.30, 0.10]])
    fl, R, J, T = _two_cell(lib_path, y)
    kr = np.array([0.25, 0.0625, 0.0625])
    for a in range(3):
        F = _b(fl, a, y[0, 0]) * kr[a] / fl.mu[a] * T * (y[0, 0] - y[1, 0])
        assert abs(R[0, a] - F) <= 1e-12 * abs(F), (a, R[0, a], F)
        assert abs(R[1, a] + F) <= 1e-12 * abs(F)
    # flow reversed: cell 1 is upwind; k_ro by gwseg with weights 0.18 and 0.10
    y2 = y.copy()
    y2[0, 0], y2[1, 0] = 4900 * PSI, 5000 * PSI
    fl, R, J, T = _two_cell(lib_path, y2)
    kr = np.array([(0.18 / 0.88) ** 2, (0.6 / 0.88) ** 2, (0.10 / 0.88) ** 2])
    for a in range(3):
        F = _b(fl, a, y2[1, 0]) * kr[a] / fl.mu[a] * T * (y2[0, 0] - y2[1, 0])
        assert abs(R[0, a] - F) <= 1e-12 * abs(F), (a, R[0, a], F)
    # upwind cell without gas carries no gas, whatever the downstream cell holds
    y3 = np.array([[4900 * PSI, 0.3, 0.3], [5000 * PSI, 0.3, 0.0]])
    fl, R, J, T = _two_cell(lib_path, y3)
    assert R[0, 2] == 0.0 and R[1, 2] == 0.0
    assert R[0, 1] < 0.0   # oil flows from cell 1 into cell 0


def pin_hydrostatic_column(lib_path=None):
    """Gravity term of eq. (head) with the average density: an oil column in
    discrete hydrostatic equilibrium p_{k+1} - p_k = g (rho_k + rho_{k+1})/2 dz
    has zero flux through every face (R = 0 up to round-off)."""
    dz = np.array([10.0, 20.0, 5.0, 15.0, 30.0])
    fl = cases.Fluid(c=(3e-6 / PSI, 3e-4 / PSI, 1e-3 / PSI))   # strongly compressible oil
    c = cases.box_case(1, 1, 5, dx=30.0, dy=30.0, dz=dz, wells=[], fluid=fl, sigma_ln=0.7)
    m = _model(c, lib_path)
    zc = np.cumsum(dz) - dz / 2

    def rho(p):
        return fl.rho_s[1] * math.exp(fl.c[1] * (p - fl.p_ref))

    p = [3000 * PSI]
    for k in range(4):
        hk = zc[k + 1] - zc[k]
        f = lambda q, pk=p[-1]: q - pk - fl.g * 0.5 * (rho(pk) + rho(q)) * hk
        p.append(brentq(f, p[-1], p[-1] + 1e7, xtol=1e-12, rtol=1e-15))
    y = np.array([[pk, 0.0, 0.0] for pk in p])
    st, R, _ = m.assemble(y, m.accumulation(y), DAY)
    T = m.geometry()["trans"]
    scale = T.max() * fl.g * rho(p[0]) * 30.0 / fl.mu[1]
    assert np.all(np.abs(R) <= 1e-12 * scale), (np.abs(R).max(), scale)
    # the same column at uniform pressure is not at rest: oil leaves the top
    # cell (positive outflux) and enters the bottom one
    y[:, 0] = p[0]
    st, R, _ = m.assemble(y, m.accumulation(y), DAY)
    assert R[0, 1] > 1e-6 * scale and R[4, 1] < -1e-6 * scale


def pin_pressure_block(lib_path=None):
    """Single mobile phase (oil), uniform state, g = 0, no wells: the pressure
    derivatives of the oil equation are b_o lambda_o times the TPFA graph
    Laplacian of T plus PV c_o b_o s_o / dt on the diagonal; the water row
    holds only its accumulation derivative PV c_w b_w s_w / dt."""
    fl = cases.Fluid(g=0.0)
    c = cases.box_case(3, 2, 2, dz=[5.0, 9.0], wells=[], fluid=fl, sigma_ln=1.2, seed=4)
    m = _model(c, lib_path)
    p0 = 4000 * PSI
    y = np.tile([p0, fl.swc, 0.0], (m.n, 1))
    dt = 3 * DAY
    st, R, J = m.assemble(y, m.accumulation(y), dt)
    g = m.geometry()
    rp, ci = m.pattern()
    bo, bw = _b(fl, 1, p0), _b(fl, 0, p0)
    lam = 1.0 / fl.mu[1]   # k_ro(s_o = 1 - swc) = 1
    L = np.zeros((m.n, m.n))
    for f, (i, j) in enumerate(g["face_cells"]):
        t = g["trans"][f]
        L[i, i] += t; L[j, j] += t; L[i, j] -= t; L[j, i] -= t
    for i in range(m.n):
        for q in range(rp[i], rp[i + 1]):
            j = ci[q]
            exp_o = bo * lam * L[i, j]
            exp_w = 0.0
            if i == j:
                exp_o += g["pore_vol"][i] * fl.c[1] * bo * (1 - fl.swc) / dt
                exp_w = g["pore_vol"][i] * fl.c[0] * bw * fl.swc / dt
            sc = abs(bo * lam * L[i, i])
            assert abs(J[q][1, 0] - exp_o) <= 1e-12 * sc, (i, j, J[q][1, 0], exp_o)
            assert abs(J[q][0, 0] - exp_w) <= 1e-12 * abs(exp_w if i == j else sc)


def _wells_case(nx, ny, nz, seed):
    wells = [Well("I", cases.WELL_RATE_INJ, [(0, 0, k) for k in range(nz)], 500 * STB / DAY,
                  phase=cases.GAS),
             Well("P", cases.WELL_BHP_PROD, [(nx - 1, ny - 1, nz - 1)], 3000 * PSI)]
    return cases.box_case(nx, ny, nz, seed=seed, wells=wells, dz=[6.0 + 3 * k for k in range(nz)])


# ---------------------------------------------------------------- Jacobian
def pin_jacobian_fd(lib_path=None):
    """Forward-mode AD Jacobian against central finite differences of the
    residual on random states away from relative-permeability kinks."""
    c = _wells_case(3, 3, 2, seed=7)
    m = _model(c, lib_path)
    y = cases.random_state(c, seed=11)
    y0 = cases.random_state(c, seed=12)
    acc0 = m.accumulation(y0)
    dt = 2 * DAY
    st, R, J = m.assemble(y, acc0, dt)
    D = _dense(m, J)
    FD = np.zeros_like(D)
    for cidx in range(m.n):
        for v in range(3):
            h = 1e-7 * (abs(y[cidx, 0]) + 1e5) if v == 0 else 1e-7
            yp, ym = y.copy(), y.copy()
            yp[cidx, v] += h
            ym[cidx, v] -= h
            Rp = m.assemble(yp, acc0, dt, jacobian=False)[1].ravel()
            Rm = m.assemble(ym, acc0, dt, jacobian=False)[1].ravel()
            FD[:, 3 * cidx + v] = (Rp - Rm) / (2 * h)
    # compare column-scaled (variables have different units) per block
    colscale = np.abs(D).max(axis=0) + 1e-300
    err = np.abs(D - FD) / colscale[None, :]
    assert err.max() <= 1e-6, err.max()


def pin_conservation(lib_path=None):
    """Each connection flux leaves one cell and enters the other (u_ij = -u_ji),
    so the residuals sum to accumulation change plus well terms."""
    c = _wells_case(4, 3, 3, seed=3)
    m = _model(c, lib_path)
    y = cases.random_state(c, seed=5)
    y0 = cases.random_state(c, seed=6)
    dt = 5 * DAY
    st, R, _ = m.assemble(y, m.accumulation(y0), dt, jacobian=False)
    pv = m.geometry()["pore_vol"]
    acc_term = pv[:, None] / dt * (m.accumulation(y) - m.accumulation(y0))
    q = m.well_rates(y)
    lhs = R.sum(axis=0)
    rhs = acc_term.sum(axis=0) + q.sum(axis=0)
    scale = np.abs(acc_term).sum(axis=0) + np.abs(q).sum(axis=0)
    assert np.all(np.abs(lhs - rhs) <= 1e-12 * scale), (lhs, rhs)


def pin_norms(lib_path=None):
    """CNV and MB are residuals in saturation units: a pure accumulation
    residual from a gas-saturation change delta in one of two cells gives
    CNV_g = delta and MB_g = delta PV_1 / (PV_0 + PV_1) (equal b)."""
    c = cases.box_case(2, 1, 1, dz=7.0, wells=[])
    c.poro = np.array([[[0.2, 0.3]]])
    m = _model(c, lib_path)
    fl = c.fluid
    y0 = np.array([[4000 * PSI, 0.3, 0.2], [4000 * PSI, 0.3, 0.2]])
    y = y0.copy()
    delta = 1.5e-3
    y[1, 2] += delta
    y[1, 1] -= delta   # keep s_o: only the gas equation is out of balance
    # zero the flux by making the states' potentials equal (same p, g acts only
    # vertically, cells side by side)
    dt = 4 * DAY
    st, R, _ = m.assemble(y, m.accumulation(y0), dt, jacobian=False)
    cnv, mb = m.norms(y, R, dt)
    pv = m.geometry()["pore_vol"]
    assert abs(cnv[2] - delta) <= 1e-12
    assert abs(mb[2] - delta * pv[1] / pv.sum()) <= 1e-12
    assert abs(cnv[0] - delta) <= 1e-12


# ---------------------------------------------------------- linear algebra
def _lu_dense(m, F):
    rp, ci = m.pattern()
    n = m.n
    L = np.eye(3 * n)
    U = np.zeros((3 * n, 3 * n))
    for i in range(n):
        for q in range(rp[i], rp[i + 1]):
            j = ci[q]
            if j < i:
                L[3 * i:3 * i + 3, 3 * j:3 * j + 3] = F[q]
            else:
                U[3 * i:3 * i + 3, 3 * j:3 * j + 3] = F[q]
    return L, U


def pin_ilu0_pattern(lib_path=None):
    """ILU(0): the product LU reproduces A on every block of A's pattern."""
    c = _wells_case(3, 3, 2, seed=9)
    m = _model(c, lib_path)
    y = cases.random_state(c, seed=2)
    st, R, J = m.assemble(y, m.accumulation(cases.random_state(c, seed=3)), DAY)
    st, F = m.ilu0(J)
    assert st == 0
    L, U = _lu_dense(m, F)
    A = _dense(m, J)
    P = L @ U
    rp, ci = m.pattern()
    for i in range(m.n):
        sc = np.abs(A[3 * i:3 * i + 3]).max()
        for q in range(rp[i], rp[i + 1]):
            j = ci[q]
            blk = P[3 * i:3 * i + 3, 3 * j:3 * j + 3] - A[3 * i:3 * i + 3, 3 * j:3 * j + 3]
            assert np.abs(blk).max() <= 1e-12 * sc


def pin_ilu0_exact_1d(lib_path=None):
    """On a 1-D chain ILU(0) has no dropped fill: it is the exact block LU,
    the preconditioner is A^{-1} and BiCGStab stops after half an iteration."""
    c = cases.box_case(7, 1, 1, seed=1, wells=[
        Well("I", cases.WELL_RATE_INJ, [(0, 0, 0)], 300 * STB / DAY),
        Well("P", cases.WELL_BHP_PROD, [(6, 0, 0)], 3000 * PSI)])
    m = _model(c, lib_path)
    y = cases.random_state(c, seed=4)
    st, R, J = m.assemble(y, m.accumulation(cases.random_state(c, seed=8)), DAY)
    st, F = m.ilu0(J)
    L, U = _lu_dense(m, F)
    A = _dense(m, J)
    assert np.abs(L @ U - A).max() <= 1e-12 * np.abs(A).max()
    st, x, its, rr = m.bicgstab(J, F, -R, rtol=1e-10)
    assert st == 0 and its <= 1.0, (st, its)
    xd = np.linalg.solve(A, -R.ravel())
    assert np.abs(x.ravel() - xd).max() <= 1e-9 * np.abs(xd).max()


def pin_bicgstab_dense(lib_path=None):
    """Preconditioned BiCGStab against numpy's dense LU on tiny grids."""
    for (nx, ny, nz), seed in [((2, 2, 2), 1), ((3, 3, 3), 2), ((4, 3, 2), 3)]:
        c = _wells_case(nx, ny, nz, seed)
        m = _model(c, lib_path)
        y = cases.random_state(c, seed=seed + 10)
        st, R, J = m.assemble(y, m.accumulation(cases.random_state(c, seed=seed + 20)), DAY)
        st, F = m.ilu0(J)
        st, x, its, rr = m.bicgstab(J, F, -R, rtol=1e-13, maxit=500)
        assert st == 0, st
        xd = np.linalg.solve(_dense(m, J), -R.ravel())
        err = np.abs(x.ravel() - xd) / (np.abs(xd.reshape(-1, 3)).max(axis=0)[None, :].repeat(m.n, 0).ravel())
        assert err.max() <= 1e-9, err.max()
        # the oracle's own dense solver agrees with numpy as well
        xo = oracle.dense_solve(_dense(m, J), -R.ravel(), lib_path=lib_path)
        assert np.allclose(xo, xd, rtol=1e-10, atol=0)


def _sub_of(case, cell_box, blk):
    """Subdomain box index of each active cell for boxes of blk cells."""
    nx, ny = case.nx, case.ny
    i, j, k = cell_box % nx, (cell_box // nx) % ny, cell_box // (nx * ny)
    return np.stack([i // blk[0], j // blk[1], k // blk[2]], axis=1)


def pin_block_ilu0_partition(lib_path=None):
    """Block ILU0 over a box partition (sec. 2.5, one block per process) is the
    ILU(0) of the matrix without its couplings between subdomains: the product
    LU reproduces A on every block of the pattern inside one subdomain, L and
    U vanish on every block between two subdomains, and the preconditioner
    solve is the exact solve with that LU (dense numpy).  Boxes of 2 x 3 x 2
    on a 5 x 4 x 3 grid leave ragged boxes on every axis."""
    c = _wells_case(5, 4, 3, seed=21)
    m = _model(c, lib_path)
    y = cases.random_state(c, seed=22)
    st, R, J = m.assemble(y, m.accumulation(cases.random_state(c, seed=23)), DAY)
    blk = (2, 3, 2)
    m.set_ilu_blocks(*blk)
    st, F = m.ilu0(J)
    assert st == 0
    sub = _sub_of(c, m.geometry()["cell_box"], blk)
    L, U = _lu_dense(m, F)
    A = _dense(m, J)
    P = L @ U
    rp, ci = m.pattern()
    n_cross = 0
    for i in range(m.n):
        sc = np.abs(A[3 * i:3 * i + 3]).max()
        for q in range(rp[i], rp[i + 1]):
            j = ci[q]
            if (sub[i] == sub[j]).all():
                blkd = P[3 * i:3 * i + 3, 3 * j:3 * j + 3] - A[3 * i:3 * i + 3, 3 * j:3 * j + 3]
                assert np.abs(blkd).max() <= 1e-12 * sc
            else:
                n_cross += 1
                assert not F[q].any(), (i, j)
    assert n_cross > 0
    r = np.random.default_rng(5).standard_normal((m.n, 3))
    x = m.ilu0_apply(F, r)
    xd = np.linalg.solve(P, r.ravel())
    assert np.abs(x.ravel() - xd).max() <= 1e-10 * np.abs(xd).max()


def pin_block_ilu0_special_cases(lib_path=None):
    """One box covering the grid is the global ILU(0) exactly; one-cell boxes
    give block Jacobi (x_i = A_ii^{-1} r_i, numpy per cell); a 1-D chain cut
    in two has no dropped fill inside either half, so the preconditioner is
    the exact inverse of the matrix without the cut coupling."""
    c = _wells_case(4, 3, 2, seed=31)
    m = _model(c, lib_path)
    y = cases.random_state(c, seed=32)
    st, R, J = m.assemble(y, m.accumulation(cases.random_state(c, seed=33)), DAY)
    st, F0 = m.ilu0(J)
    m.set_ilu_blocks(4, 3, 2)
    st, F1 = m.ilu0(J)
    assert np.array_equal(F0, F1)
    m.set_ilu_blocks(9, 9, 9)
    st, F1 = m.ilu0(J)
    assert np.array_equal(F0, F1)
    m.set_ilu_blocks(1, 1, 1)
    st, Fj = m.ilu0(J)
    r = np.random.default_rng(7).standard_normal((m.n, 3))
    x = m.ilu0_apply(Fj, r)
    rp, ci = m.pattern()
    for i in range(m.n):
        q = [q for q in range(rp[i], rp[i + 1]) if ci[q] == i][0]
        xi = np.linalg.solve(J[q], r[i])
        assert np.abs(x[i] - xi).max() <= 1e-12 * np.abs(xi).max()
    # 1-D chain of 8 cells cut between cells 2 and 3 (boxes of 3 cells)
    c = cases.box_case(8, 1, 1, seed=2, wells=[
        Well("I", cases.WELL_RATE_INJ, [(0, 0, 0)], 300 * STB / DAY),
        Well("P", cases.WELL_BHP_PROD, [(7, 0, 0)], 3000 * PSI)])
    m = _model(c, lib_path)
    y = cases.random_state(c, seed=4)
    st, R, J = m.assemble(y, m.accumulation(cases.random_state(c, seed=8)), DAY)
    m.set_ilu_blocks(3, 1, 1)
    st, F = m.ilu0(J)
    A = _dense(m, J)
    for a, b in [(2, 3), (5, 6)]:
        A[3 * a:3 * a + 3, 3 * b:3 * b + 3] = 0.0
        A[3 * b:3 * b + 3, 3 * a:3 * a + 3] = 0.0
    x = m.ilu0_apply(F, -R)
    xd = np.linalg.solve(A, -R.ravel())
    assert np.abs(x.ravel() - xd).max() <= 1e-10 * np.abs(xd).max()


def pin_block_ilu0_newton(lib_path=None):
    """The preconditioner changes the linear iterations, not the converged
    Newton state: a report step with column boxes matches the single-block
    run to the Newton tolerance, and it still conserves mass per component."""
    c = _wells_case(6, 5, 3, seed=41)
    m = _model(c, lib_path)
    opts = oracle.default_opts(c)
    dt = 10 * DAY
    st, y0, rep0 = m.advance(c.initial_state(), dt, opts)
    assert st == 0
    m.set_ilu_blocks(2, 2, 3)
    st, y1, rep1 = m.advance(c.initial_state(), dt, opts)
    assert st == 0
    assert rep1.lin_its != rep0.lin_its
    assert np.abs(y1[:, 0] - y0[:, 0]).max() <= 1e-8 * np.abs(y0[:, 0]).max()
    assert np.abs(y1[:, 1:] - y0[:, 1:]).max() <= 1e-8
    assert max(abs(e) for e in rep1.mass_err) <= 1e-10


def pin_gmres_dense(lib_path=None):
    """Restarted GMRes (sec. 2.3.1) against numpy's dense LU on tiny grids
    (restart 8, so the larger ones restart several times)."""
    for (nx, ny, nz), seed in [((2, 2, 2), 1), ((3, 3, 3), 2), ((4, 3, 2), 3)]:
        c = _wells_case(nx, ny, nz, seed)
        m = _model(c, lib_path)
        y = cases.random_state(c, seed=seed + 10)
        st, R, J = m.assemble(y, m.accumulation(cases.random_state(c, seed=seed + 20)), DAY)
        st, F = m.ilu0(J)
        st, x, its, rr = m.gmres(J, F, -R, rtol=1e-13, maxit=2000, restart=8)
        assert st == 0, st
        xd = np.linalg.solve(_dense(m, J), -R.ravel())
        err = np.abs(x.ravel() - xd) / (np.abs(xd.reshape(-1, 3)).max(axis=0)[None, :].repeat(m.n, 0).ravel())
        assert err.max() <= 1e-9, err.max()


def pin_gmres_exact_lu(lib_path=None):
    """With the exact LU of a 1-D chain as preconditioner, A M^{-1} = I and
    GMRes stops after one iteration with the solution."""
    c = cases.box_case(7, 1, 1, seed=1, wells=[
        Well("I", cases.WELL_RATE_INJ, [(0, 0, 0)], 300 * STB / DAY),
        Well("P", cases.WELL_BHP_PROD, [(6, 0, 0)], 3000 * PSI)])
    m = _model(c, lib_path)
    y = cases.random_state(c, seed=4)
    st, R, J = m.assemble(y, m.accumulation(cases.random_state(c, seed=8)), DAY)
    st, F = m.ilu0(J)
    st, x, its, rr = m.gmres(J, F, -R, rtol=1e-10)
    assert st == 0 and its == 1, (st, its)
    xd = np.linalg.solve(_dense(m, J), -R.ravel())
    assert np.abs(x.ravel() - xd).max() <= 1e-9 * np.abs(xd).max()


def pin_gmres_minimal_residual(lib_path=None):
    """Within one cycle, the k-th GMRes iterate has the smallest residual
    over x = M^{-1} u, u in span{b, (A M^{-1}) b, ..., (A M^{-1})^{k-1} b}:
    the minimum computed here by numpy least squares over that space (the
    oracle's SpMV and ILU(0) solve only build the space), and the reported
    relative residual is the true one."""
    c = _wells_case(4, 3, 3, seed=5)
    m = _model(c, lib_path)
    y = cases.random_state(c, seed=6)
    st, R, J = m.assemble(y, m.accumulation(cases.random_state(c, seed=7)), DAY)
    st, F = m.ilu0(J)
    b = -R
    bn = np.linalg.norm(b)
    U = [b.ravel()]
    for _ in range(5):
        U.append(m.spmv(J, m.ilu0_apply(F, U[-1].reshape(-1, 3))).ravel())
    for k in range(1, 6):
        st, x, its, rr = m.gmres(J, F, b, rtol=1e-14, maxit=k, restart=k)
        assert its == k
        res = np.linalg.norm(b.ravel() - m.spmv(J, x).ravel())
        AU = np.stack([m.spmv(J, m.ilu0_apply(F, u.reshape(-1, 3))).ravel() for u in U[:k]], axis=1)
        Q, _ = np.linalg.qr(AU)
        best = np.linalg.norm(b.ravel() - Q @ (Q.T @ b.ravel()))
        assert abs(res - best) <= 1e-8 * bn, (k, res, best)
        assert abs(rr - res / bn) <= 1e-8, (k, rr, res / bn)


def pin_gmres_newton(lib_path=None):
    """A report step with GMRes(30) as the linear solver converges to the
    BiCGStab run's state to the Newton tolerance and conserves mass."""
    c = _wells_case(6, 5, 3, seed=43)
    m = _model(c, lib_path)
    dt = 10 * DAY
    st, y0, rep0 = m.advance(c.initial_state(), dt, oracle.default_opts(c))
    assert st == 0
    st, y1, rep1 = m.advance(c.initial_state(), dt, oracle.default_opts(c, krylov=1, restart=30))
    assert st == 0
    assert rep1.lin_its != rep0.lin_its
    assert np.abs(y1[:, 0] - y0[:, 0]).max() <= 1e-8 * np.abs(y0[:, 0]).max()
    assert np.abs(y1[:, 1:] - y0[:, 1:]).max() <= 1e-8
    assert max(abs(e) for e in rep1.mass_err) <= 1e-10


# ------------------------------------------------------------------ Newton
def pin_one_cell_producer(lib_path=None):
    """One cell drained by a BHP producer with immobile water below connate
    saturation and no gas: water mass is conserved (s_w b_w = const) and the
    oil equation is a scalar equation in p, solved here by bisection."""
    c = cases.box_case(1, 1, 1, dx=1000 * FT, dy=1000 * FT, dz=20 * FT, sigma_ln=0.0,
                       median_md=100.0, sw_init=0.10,
                       wells=[Well("P", cases.WELL_BHP_PROD, [(0, 0, 0)], 3000 * PSI)])
    m = _model(c, lib_path)
    fl = c.fluid
    pv = m.geometry()["pore_vol"][0]
    _, wi, _ = m.conns()
    y0 = c.initial_state()
    dt = 30 * DAY
    p0, sw0 = y0[0, 0], y0[0, 1]

    def sw_of(p):
        return sw0 * _b(fl, 0, p0) / _b(fl, 0, p)

    def f(p):
        so = 1.0 - sw_of(p)
        kro = min(max(so / (1 - fl.swc), 0.0), 1.0) ** 2
        return (pv / dt * (_b(fl, 1, p) * so - _b(fl, 1, p0) * (1 - sw0))
                + _b(fl, 1, p) * kro / fl.mu[1] * wi[0] * (p - 3000 * PSI))

    lo, hi = 3000 * PSI, p0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if f(mid) > 0:
            hi = mid
        else:
            lo = mid
    p_star = 0.5 * (lo + hi)
    opts = oracle.default_opts(c, tol_cnv=1e-13, tol_mb=1e-13, lin_rtol=1e-13)
    st, y, rep = m.newton_step(y0, y0, dt, opts)
    assert st == 0
    assert abs(y[0, 0] - p_star) <= 1e-12 * p_star, (y[0, 0], p_star)
    assert abs(y[0, 1] - sw_of(p_star)) <= 1e-12
    assert y[0, 2] == 0.0


def pin_injector_mass(lib_path=None):
    """Sign convention of the well outflux density (negative for inflow): over
    one step a gas injector adds exactly Q dt of surface gas to the reservoir,
    less what the producer (last cell) takes out."""
    Q = 1e3 * cases.MSCF / DAY
    c = cases.box_case(3, 3, 1, dz=10.0, wells=[
        Well("I", cases.WELL_RATE_INJ, [(0, 0, 0)], Q, phase=cases.GAS),
        Well("P", cases.WELL_BHP_PROD, [(2, 2, 0)], 3000 * PSI)])
    m = _model(c, lib_path)
    y0 = c.initial_state()
    dt = 5 * DAY
    st, y, rep = m.advance(y0, dt, oracle.default_opts(c, lin_rtol=1e-12))
    assert st == 0, (st, rep.as_dict())
    pv = m.geometry()["pore_vol"]
    dM = (pv[:, None] * (m.accumulation(y) - m.accumulation(y0))).sum(axis=0)
    q_prod = m.well_rates(y)[-1]
    assert 0.0 <= q_prod[2] < Q
    assert abs(dM[2] - (Q - q_prod[2]) * dt) <= 1e-9 * Q * dt, (dM, Q * dt)
    assert q_prod[1] > 0.0 and abs(dM[1] + dt * q_prod[1]) <= 1e-9 * dt * q_prod[1]


def pin_quadratic_convergence(lib_path=None):
    """Newton with the exact Jacobian converges quadratically near the root:
    once CNV is small, the exponent of the next CNV at least ~doubles."""
    c = _wells_case(4, 4, 2, seed=21)
    m = _model(c, lib_path)
    y0 = c.initial_state()
    dt = 20 * DAY
    hist = []
    for k in range(0, 9):
        opts = oracle.default_opts(c, max_newton=k, lin_rtol=1e-14, tol_cnv=0.0, tol_mb=0.0)
        st, y, rep = m.newton_step(y0, y0, dt, opts)
        _, R, _ = m.assemble(y, m.accumulation(y0), dt, jacobian=False)
        cnv, mb = m.norms(y, R, dt)
        hist.append(max(cnv))
    tail = [e for e in hist if 1e-14 < e < 1e-2]
    assert len(tail) >= 2, hist
    for a, b in zip(tail[:-1], tail[1:]):
        assert math.log10(b) <= 1.6 * math.log10(a), hist


def pin_mass_balance_run(lib_path=None):
    """Per-step component mass balance of a short gas-injection run: the
    change of surface mass plus dt times the well outflux is at most 1e-10 of
    the reservoir-average measure."""
    c = cases.config1()
    m = _model(c, lib_path)
    states, reps = m.run(n_steps=3)
    for r in reps:
        assert max(r["mass_err"]) <= 1e-10, r["mass_err"]
        assert r["newton_its"] >= 1


def pin_mirror_symmetry(lib_path=None):
    """Homogeneous square box, wells on the diagonal: the solution is symmetric
    under swapping i and j."""
    nz = 2
    wells = [Well("I", cases.WELL_RATE_INJ, [(0, 0, k) for k in range(nz)], 800 * STB / DAY),
             Well("P", cases.WELL_BHP_PROD, [(4, 4, 0)], 3000 * PSI)]
    c = cases.box_case(5, 5, nz, sigma_ln=0.0, wells=wells, dz=[8.0, 12.0])
    m = _model(c, lib_path)
    opts = oracle.default_opts(c, lin_rtol=1e-11)
    y = c.initial_state()
    for dt in [10 * DAY, 10 * DAY]:
        st, y, rep = m.advance(y, dt, opts)
        assert st == 0
    Y = y.reshape(nz, 5, 5, 3)
    YT = Y.transpose(0, 2, 1, 3)
    assert np.abs(Y[..., 0] - YT[..., 0]).max() <= 1e-7 * np.abs(Y[..., 0]).max()
    assert np.abs(Y[..., 1:] - YT[..., 1:]).max() <= 1e-7
    assert Y[..., 1].max() > 0.121   # water actually moved


# ------------------------------------------------------------ live oil
# Live oil (sec. 2.1.6: gas dissolved in the oleic phase, dry gas) with the
# per-cell meaning of the third variable (eq. primaryVariableMeaning):
# x = s_g where free gas is present (the oil then saturated, r = r_s(p)),
# x = r_go where it is not (s_g = 0).
def _live_case(nx, ny, nz, seed, wells=None, g=cases.G, **kw):
    fl = cases.live_fluid()
    fl.g = g
    if wells is None:
        wells = [Well("I", cases.WELL_RATE_INJ, [(0, 0, k) for k in range(nz)], 300 * STB / DAY,
                      phase=cases.W),
                 Well("P", cases.WELL_BHP_PROD, [(nx - 1, ny - 1, nz - 1)], 2500 * PSI)]
    kw.setdefault("dz", [6.0 + 3 * k for k in range(nz)])
    return cases.box_case(nx, ny, nz, seed=seed, wells=wells, fluid=fl, **kw)


def _live_state(c, seed, mean=None):
    """A state with mixed meanings away from kinks: free-gas cells with
    s_g in [0.03, 0.2], undersaturated cells with r in [0.3, 0.9] r_s(p)."""
    rng = np.random.default_rng(seed)
    n = c.n_active
    if mean is None:
        mean = rng.integers(0, 2, n).astype(np.uint8)
    y = np.empty((n, 3))
    y[:, 0] = rng.uniform(2800, 3200, n) * PSI
    y[:, 1] = rng.uniform(0.15, 0.5, n)
    rs = c.fluid.rs_c * y[:, 0]
    y[:, 2] = np.where(mean == 0, rng.uniform(0.03, 0.2, n), rng.uniform(0.3, 0.9, n) * rs)
    return y, mean


def pin_live_dead_limit(lib_path=None):
    """Live oil with no dissolution (r_s = 0) and every cell in the s_g
    meaning is dead oil: residual and Jacobian equal the dead-oil ones
    exactly, whatever the swelling and thinning coefficients."""
    base = _wells_case(3, 3, 2, seed=7)
    live = _wells_case(3, 3, 2, seed=7)
    live.fluid = cases.Fluid(live=True, rs_c=0.0, bo_r=0.7, muo_r=0.3)
    md, ml = _model(base, lib_path), _model(live, lib_path)
    y = cases.random_state(base, seed=11)
    acc0 = md.accumulation(cases.random_state(base, seed=12))
    assert np.array_equal(ml.accumulation(y), md.accumulation(y))
    st, Rd, Jd = md.assemble(y, acc0, 2 * DAY)
    st, Rl, Jl = ml.assemble(y, acc0, 2 * DAY)
    assert np.array_equal(Rd, Rl) and np.array_equal(Jd, Jl)


def pin_live_switch_continuity(lib_path=None):
    """At the switching point (no free gas, oil exactly saturated) a cell can
    be written in either meaning: (s_g = 0) or (r = r_s(p)).  The residual
    is the same, and by the chain rule (r = r_s(p) = rs_c p in the s_g
    meaning) the Jacobian columns satisfy d/dp|_sg = d/dp|_r + rs_c d/dr and
    d/ds_w|_sg = d/ds_w|_r, for the cell's own block and its neighbours'."""
    c = _live_case(3, 3, 2, seed=4)
    m = _model(c, lib_path)
    y, mean = _live_state(c, seed=5)
    y0, mean0 = _live_state(c, seed=6)
    m.set_meaning(mean0)
    acc0 = m.accumulation(y0)
    S = np.array([1, 4, 7, 10, 16])           # cells put at the switching point
    ya, ma = y.copy(), mean.copy()
    ya[S, 2], ma[S] = 0.0, 0                  # s_g = 0
    yb, mb = y.copy(), mean.copy()
    yb[S, 2], mb[S] = c.fluid.rs_c * y[S, 0], 1   # r = r_s(p)
    m.set_meaning(ma)
    st, Ra, Ja = m.assemble(ya, acc0, 2 * DAY)
    m.set_meaning(mb)
    st, Rb, Jb = m.assemble(yb, acc0, 2 * DAY)
    scale = np.abs(Ra).max(axis=0) + 1e-300
    assert np.all(np.abs(Ra - Rb) <= 1e-13 * scale), np.abs(Ra - Rb).max(axis=0) / scale
    Da, Db = _dense(m, Ja), _dense(m, Jb)
    colscale = np.abs(Da).max(axis=0) + 1e-300
    for cidx in S:
        cp, cw, cx = 3 * cidx, 3 * cidx + 1, 3 * cidx + 2
        lhs = Da[:, cp]
        rhs = Db[:, cp] + c.fluid.rs_c * Db[:, cx]
        assert np.all(np.abs(lhs - rhs) <= 1e-11 * colscale[cp]), np.abs(lhs - rhs).max()
        assert np.all(np.abs(Da[:, cw] - Db[:, cw]) <= 1e-11 * colscale[cw])


def pin_live_jacobian_fd(lib_path=None):
    """Forward-mode AD Jacobian against central finite differences on a
    live-oil state with both meanings present (the derivative of r_s(p)
    enters through p in the s_g meaning)."""
    c = _live_case(3, 3, 2, seed=7)
    m = _model(c, lib_path)
    y0, mean0 = _live_state(c, seed=12)
    m.set_meaning(mean0)
    acc0 = m.accumulation(y0)
    y, mean = _live_state(c, seed=11)
    m.set_meaning(mean)
    dt = 2 * DAY
    st, R, J = m.assemble(y, acc0, dt)
    D = _dense(m, J)
    FD = np.zeros_like(D)
    for cidx in range(m.n):
        for v in range(3):
            h = 1e-7 * (abs(y[cidx, v]) + (1e5 if v == 0 else 0.0)) if v != 1 else 1e-7
            yp, ym = y.copy(), y.copy()
            yp[cidx, v] += h
            ym[cidx, v] -= h
            Rp = m.assemble(yp, acc0, dt, jacobian=False)[1].ravel()
            Rm = m.assemble(ym, acc0, dt, jacobian=False)[1].ravel()
            FD[:, 3 * cidx + v] = (Rp - Rm) / (2 * h)
    colscale = np.abs(D).max(axis=0) + 1e-300
    err = np.abs(D - FD) / colscale[None, :]
    assert err.max() <= 1e-6, err.max()


def pin_live_conservation(lib_path=None):
    """Flux cancellation with dissolved gas: the residuals sum to the change
    of surface volume in place (free plus dissolved gas) plus the well terms."""
    c = _live_case(4, 3, 3, seed=3)
    m = _model(c, lib_path)
    y0, mean0 = _live_state(c, seed=6)
    m.set_meaning(mean0)
    a0 = m.accumulation(y0)
    y, mean = _live_state(c, seed=5)
    m.set_meaning(mean)
    dt = 5 * DAY
    st, R, _ = m.assemble(y, a0, dt, jacobian=False)
    pv = m.geometry()["pore_vol"]
    acc_term = pv[:, None] / dt * (m.accumulation(y) - a0)
    q = m.well_rates(y)
    lhs = R.sum(axis=0)
    rhs = acc_term.sum(axis=0) + q.sum(axis=0)
    scale = np.abs(acc_term).sum(axis=0) + np.abs(q).sum(axis=0)
    assert np.all(np.abs(lhs - rhs) <= 1e-12 * scale), (lhs, rhs)


def pin_live_closed_cell(lib_path=None):
    """One closed cell without free gas that loses stock-tank oil at a fixed
    surface rate Q (a negative-rate source of the oil component only) keeps
    all its gas: the gas in place is the dissolved gas r N_o, so after a step
    r = N_g / (N_o - Q dt) with N_g = r0 N_o.  Also the definition of the
    swelling at p_ref: b_o = 1 / (1 + bo_r r)."""
    Q = 0.02 * STB / DAY
    wells = [Well("X", cases.WELL_RATE_INJ, [(0, 0, 0)], -Q, phase=cases.O)]
    c = _live_case(1, 1, 1, seed=1, wells=wells, dx=20.0, dy=20.0, dz=2.0)
    m = _model(c, lib_path)
    r0 = 4.0
    y = np.array([[3600 * PSI, c.fluid.swc, r0]])
    m.set_meaning(np.array([1], np.uint8))
    acc = m.accumulation(y)[0]
    assert abs(acc[2] - r0 * acc[1]) <= 1e-14 * acc[2]     # gas in place = r N_o
    pv = m.geometry()["pore_vol"][0]
    dt = 2 * DAY
    o = oracle.default_opts(c, tol_cnv=1e-12, tol_mb=1e-14)
    st, y1, rep = m.newton_step(y, y, dt, o)
    assert st == 0 and m.meaning()[0] == 1, (st, m.meaning())
    No = pv * acc[1]
    r1 = r0 * No / (No - Q * dt)
    assert abs(y1[0, 2] - r1) <= 1e-9 * r1, (y1[0, 2], r1)
    assert y1[0, 0] < y[0, 0]
    yr = np.array([[c.fluid.p_ref, c.fluid.swc, 2.5]])
    so = 1.0 - c.fluid.swc
    assert abs(m.accumulation(yr)[0, 1] / so - 1.0 / (1.0 + c.fluid.bo_r * 2.5)) <= 1e-15


def pin_live_dissolved_moves_with_oil(lib_path=None):
    """The dissolved gas travels with the oil phase: between two cells
    without free gas its flux is r of the oil's upwind cell times the oil
    flux, also when gas and oil potentials point opposite ways (a column
    whose pressure step lies between the oil and gas heads); a producer of
    undersaturated oil produces gas at r times its oil rate."""
    wells = [Well("P", cases.WELL_BHP_PROD, [(0, 0, 1)], 2500 * PSI)]
    c = _live_case(1, 1, 2, seed=2, wells=wells, dx=30.0, dy=30.0, dz=[10.0, 10.0])
    m = _model(c, lib_path)
    m.set_meaning(np.array([1, 1], np.uint8))
    fl = c.fluid
    p_top = 3400 * PSI
    rho_mid = 0.5 * (fl.rho_s[1] + fl.rho_s[2] * 3.0)   # between the gas and oil densities
    y = np.array([[p_top, 0.3, 3.0], [p_top + fl.g * rho_mid * 10.0, 0.3, 4.5]])
    st, R, _ = m.assemble(y, m.accumulation(y), DAY)
    q = m.well_rates(y)
    F = R - q     # the accumulation term is zero (acc0 = A(y)): fluxes only
    assert F[0, 1] > 0                          # oil flows down, from the top cell
    assert abs(F[0, 2] - 3.0 * F[0, 1]) <= 1e-12 * abs(F[0, 2]), (F[0], 3.0)
    assert q[1, 1] > 0 and abs(q[1, 2] - 4.5 * q[1, 1]) <= 1e-14 * q[1, 2]


def pin_live_hydrostatic_column(lib_path=None):
    """A column of undersaturated live oil at rest: the discrete hydrostatic
    profile uses the oil's mass per reservoir volume, which holds the
    stock-tank oil and the dissolved gas, rho_o = b_o (rho_oS + r rho_gS)
    (b_o read from the accumulation A_o = b_o s_o); no flux through any face."""
    dz = np.array([10.0, 20.0, 5.0, 15.0])
    c = _live_case(1, 1, 4, seed=3, wells=[], dx=30.0, dy=30.0, dz=dz)
    m = _model(c, lib_path)
    fl = c.fluid
    r = 4.0
    m.set_meaning(np.ones(4, np.uint8))
    so = 1.0 - fl.swc

    def rho(p):
        bo = m.accumulation(np.array([[p, fl.swc] + [r]] * 4))[0, 1] / so
        return bo * (fl.rho_s[1] + r * fl.rho_s[2])

    zc = np.cumsum(dz) - dz / 2
    p = [3500 * PSI]
    for k in range(3):
        hk = zc[k + 1] - zc[k]
        f = lambda q, pk=p[-1]: q - pk - fl.g * 0.5 * (rho(pk) + rho(q)) * hk
        p.append(brentq(f, p[-1], p[-1] + 1e7, xtol=1e-12, rtol=1e-15))
    y = np.array([[pk, fl.swc, r] for pk in p])
    st, R, _ = m.assemble(y, m.accumulation(y), DAY)
    T = m.geometry()["trans"]
    scale = T.max() * fl.g * rho(p[0]) * 20.0 / fl.mu[1]
    assert np.all(np.abs(R) <= 1e-12 * scale), (np.abs(R).max(), scale)


def pin_live_depletion_1d(lib_path=None):
    """Horizontal 1-D depletion below the bubble point (producer at one end
    at 2500 psi, bubble point 3000 psi, oil undersaturated at r_init): every
    converged state is valid (no free gas below -eps, no dissolved gas above
    r_s(p) (1 + eps)); cells without free gas keep r = r_init (the oil that
    reaches them carries r_init, no free gas reaches them upstream of the
    gas); free gas forms a contiguous zone at the producer end, only where
    the pressure is below the bubble point; each step conserves mass."""
    nx = 20
    wells = [Well("P", cases.WELL_BHP_PROD, [(nx - 1, 0, 0)], 2500 * PSI)]
    fl = cases.live_fluid()
    c = cases.box_case(nx, 1, 1, seed=8, wells=wells, fluid=fl, dz=10.0, p_init=3300 * PSI,
                       r_init=fl.rs_c * 3000 * PSI, report_dt=[5 * DAY] * 6, sigma_ln=0.0)
    m = _model(c, lib_path)
    states, reps = m.run()
    eps = fl.eps_switch
    r_init = c.r_init
    for y, mean, rep in zip(states, m.run_meanings, reps):
        assert max(rep["mass_err"]) <= 1e-10, rep["mass_err"]
        free = mean == 0
        rs = fl.rs_c * y[:, 0]
        assert np.all(y[free, 2] >= -eps)
        assert np.all(y[~free, 2] <= rs[~free] * (1 + eps))
        assert np.all(np.abs(y[~free, 2] - r_init) <= 1e-8 * r_init), np.abs(y[~free, 2] - r_init).max()
        if free.any():
            first = int(np.argmax(free))
            assert np.all(free[first:]), mean     # contiguous up to the producer
            assert np.all(y[free, 0] < 3000 * PSI * (1 + eps))
    assert (m.run_meanings[-1] == 0).sum() >= 2


# ------------------------------------------------------- standard wells
# Standard well model (sec. 2.2.1): per well x_w = (Q_t, F_w, F_g, p_bhp),
# component conservation with wellbore storage and a control equation,
# eliminated from the linear system by the Schur complement (eq.
# wellequation).
def _std_case(vol_scale=1.0):
    wells = [Well("I", cases.WELL_RATE_INJ, [(0, 0, k) for k in range(2)], 400 * STB / DAY,
                  phase=cases.W),
             Well("P", cases.WELL_BHP_PROD, [(2, 2, 0), (2, 2, 1)], 3000 * PSI)]
    c = cases.box_case(3, 3, 2, seed=7, wells=wells, dz=[6.0, 9.0])
    c.standard_wells = True
    return c


def _std_state(c, m, seed):
    """A random reservoir state and a well state with both wells flowing."""
    y = cases.random_state(c, seed=seed)
    rng = np.random.default_rng(seed)
    x = m.well_state().copy()
    x[0] = (-2e-4 * rng.uniform(0.5, 1.5), 1.0 - 0.05 * rng.uniform(), 0.01 * rng.uniform(),
            y[:, 0].mean() + 300 * PSI)
    x[1] = (3e-4 * rng.uniform(0.5, 1.5), 0.2 * rng.uniform(), 0.05 * rng.uniform(),
            y[:, 0].mean() - 300 * PSI)
    return y, x


def _full_system(m, J, B, C, D):
    """The coupled matrix [[A C] [B D]] (cells first, then 4 per well)."""
    A = _dense(m, J)
    n3, nw = 3 * m.n, m.nw
    M = np.zeros((n3 + 4 * nw, n3 + 4 * nw))
    M[:n3, :n3] = A
    cell, _, well = m.conns()
    for q in range(m.nc):
        c, w = cell[q], well[q]
        M[3 * c:3 * c + 3, n3 + 4 * w:n3 + 4 * w + 4] += C[q]
        M[n3 + 4 * w:n3 + 4 * w + 4, 3 * c:3 * c + 3] += B[q]
    for w in range(nw):
        M[n3 + 4 * w:n3 + 4 * w + 4, n3 + 4 * w:n3 + 4 * w + 4] = D[w]
    return M


def pin_std_schur_dense(lib_path=None):
    """The Schur-complement solve (eq. wellequation: Krylov on A - C D^-1 B,
    then x_w = D^-1 (R_w - B x_r)) equals numpy's dense solve of the whole
    coupled system, for BiCGStab and GMRes."""
    c = _std_case()
    m = _model(c, lib_path)
    y, x = _std_state(c, m, seed=3)
    m.set_well_state(x)
    m.well_storage_start()
    acc0 = m.accumulation(cases.random_state(c, seed=4))
    st, R, J = m.assemble(y, acc0, 2 * DAY)
    st, Rw, B, C, D = m.well_system(y, 2 * DAY)
    assert st == 0
    st, F = m.ilu0(J)
    M = _full_system(m, J, B, C, D)
    rhs = np.concatenate([R.ravel(), Rw.ravel()])
    xd = np.linalg.solve(M, rhs)
    for krylov in (0, 1):
        st, xr, xw, its = m.schur_solve(J, F, B, C, D, R, Rw, rtol=1e-13, maxit=500,
                                        krylov=krylov, restart=10)
        assert st == 0
        got = np.concatenate([xr.ravel(), xw.ravel()])
        scale = np.abs(xd).max()
        assert np.abs(got[:3 * m.n] - xd[:3 * m.n]).max() <= 1e-8 * np.abs(xd[:3 * m.n]).max()
        for k in range(4 * m.nw):   # each well unknown against its own scale
            ref = xd[3 * m.n + k]
            assert abs(got[3 * m.n + k] - ref) <= 1e-8 * (abs(ref) + 1e-12 * scale), (k, got[3 * m.n + k], ref)


def pin_std_jacobian_fd(lib_path=None):
    """The coupling blocks against central finite differences: the cell
    residual's derivatives w.r.t. the well unknowns (C), the well residual's
    w.r.t. the cell variables (B) and the well unknowns (D), and the cell
    block diagonal with the connection terms."""
    c = _std_case()
    m = _model(c, lib_path)
    y, x = _std_state(c, m, seed=5)
    m.set_well_state(x)
    m.well_storage_start()
    acc0 = m.accumulation(cases.random_state(c, seed=6))
    dt = 2 * DAY
    st, R, J = m.assemble(y, acc0, dt)
    st, Rw, B, C, D = m.well_system(y, dt)
    M = _full_system(m, J, B, C, D)

    def resid(yv, xv):
        m.set_well_state(xv)
        r = m.assemble(yv, acc0, dt, jacobian=False)[1].ravel()
        rw = m.well_system(yv, dt)[1].ravel()
        m.set_well_state(x)
        return np.concatenate([r, rw])

    n3 = 3 * m.n
    FD = np.zeros_like(M)
    for k in range(n3 + 4 * m.nw):
        yp, ym, xp, xm = y.copy(), y.copy(), x.copy(), x.copy()
        if k < n3:
            ci, v = divmod(k, 3)
            h = 1e-7 * (abs(y[ci, 0]) + 1e5) if v == 0 else 1e-7
            yp[ci, v] += h
            ym[ci, v] -= h
        else:   # well unknowns: larger steps (their columns are small next to R)
            w, e = divmod(k - n3, 4)
            h = 1e-5 * (abs(x[w, e]) + (1e5 if e == 3 else 1e-6))
            xp[w, e] += h
            xm[w, e] -= h
        FD[:, k] = (resid(yp, xp) - resid(ym, xm)) / (2 * h)
    colscale = np.abs(M).max(axis=0) + 1e-300
    err = np.abs(M - FD) / colscale[None, :]
    assert err[:, :n3].max() <= 1e-6, err[:, :n3].max()
    assert err[:, n3:].max() <= 1e-4, err[:, n3:].max()


def pin_std_simplified_limit(lib_path=None):
    """Single-connection wells with a vanishing wellbore volume reduce to
    the simplified wells: a BHP producer's connection then carries exactly
    b lambda WI (p - p_bhp)^+, a rate injector's exactly its target; the
    converged states of a 3-step run agree to the Newton tolerance.  (With
    no volume at all the wellbore composition of a well at rest is
    undetermined, one reason for the storage term.)"""
    base = cases.config1()
    ref = _model(base, lib_path)
    states_ref, _ = ref.run(n_steps=3)
    c = cases.config1()
    c.standard_wells = True
    m = _model(c, lib_path)
    vol, x0 = c.standard_well_init()
    st = m.L.ora_set_standard_wells(m.h, oracle._d(vol * 1e-9), oracle._d(x0), None)
    assert st == 0
    states, _ = m.run(n_steps=3)
    states_std = states
    for a, b in zip(states_std, states_ref):
        assert np.abs(a[:, 0] - b[:, 0]).max() <= 1e-7 * np.abs(b[:, 0]).max()
        assert np.abs(a[:, 1:] - b[:, 1:]).max() <= 1e-7


def pin_std_controls_and_storage(lib_path=None):
    """Over a run with multi-connection wells and a large wellbore: the rate
    injector's water rate Q_w = F_w Q_t (g_w = 1) equals its target, its
    wellbore holds water only (F_w = 1, F_g = 0), the producer sits at its
    BHP, and every step conserves the surface volume of each component
    counting the wellbore (storage V_w mix_a) and the surface rates Q_a."""
    c = _std_case()
    m = _model(c, lib_path)
    vol, x0 = c.standard_well_init()
    st = m.L.ora_set_standard_wells(m.h, oracle._d(vol * 2000.0), oracle._d(x0), None)
    assert st == 0
    c.report_dt = [2 * DAY] * 4
    states, reps = m.run()
    for r, x in zip(reps, m.run_well_states):
        assert max(r["mass_err"]) <= 1e-10, r["mass_err"]
        assert abs(x[0, 1] * x[0, 0] + 400 * STB / DAY) <= 1e-9 * 400 * STB / DAY
        assert x[0, 1] == 1.0 and x[0, 2] == 0.0
        assert abs(x[1, 3] - 3000 * PSI) <= 1e-6 * 3000 * PSI


def _switch_case(inj_limit_psi, prod_limit_stb):
    c = cases.config1()
    c.standard_wells = True
    c.wells[0].limit = inj_limit_psi * PSI
    c.wells[1].limit = prod_limit_stb * STB / DAY
    return c


def _oil_rate(x):
    return (1.0 - x[1] - x[2]) * x[0]   # g_o = 1


def pin_std_control_switching(lib_path=None):
    """Two-constraint wells: a limit that never binds changes nothing (the
    same bits as no limit); once a limit binds the well holds it with
    equality (the gas injector at its BHP limit, injecting less than its
    target; the producer at its oil-rate limit, above its BHP target), and at
    every report step the inactive constraint is satisfied, through a switch
    back from the rate limit to the BHP target as the reservoir depletes;
    every step conserves mass."""
    c0 = cases.config1()
    c0.standard_wells = True
    m0 = _model(c0, lib_path)
    s0, _ = m0.run(n_steps=3)
    m1 = _model(_switch_case(1e6, 1e6), lib_path)
    s1, _ = m1.run(n_steps=3)
    for a, b in zip(s0, s1):
        assert np.array_equal(a, b)
    assert all(not c.any() for c in m1.run_well_ctrls)
    # both limits bind from the first step
    c = _switch_case(7000, 1500)
    m = _model(c, lib_path)
    states, reps = m.run()
    inj_t, pmin = c.wells[0].target, c.wells[1].target
    for r, x, ctrl in zip(reps, m.run_well_states, m.run_well_ctrls):
        assert max(r["mass_err"]) <= 1e-9, r["mass_err"]
        assert list(ctrl) == [1, 1]
        assert abs(x[0, 3] - 7000 * PSI) <= 1e-7 * 7000 * PSI
        assert 0.0 < -x[0, 2] * x[0, 0] / 0.01 < inj_t
        assert abs(_oil_rate(x[1]) - 1500 * STB / DAY) <= 1e-7 * 1500 * STB / DAY
        assert x[1, 3] > pmin
    # the producer starts on its rate limit and returns to its BHP target
    c = _switch_case(4900, 2500)
    m = _model(c, lib_path)
    states, reps = m.run()
    hist = [int(ctrl[1]) for ctrl in m.run_well_ctrls]
    assert hist[0] == 1 and hist[-1] == 0 and hist == sorted(hist, reverse=True), hist
    lim = 2500 * STB / DAY
    for r, x, h in zip(reps, m.run_well_states, hist):
        assert max(r["mass_err"]) <= 1e-9, r["mass_err"]
        if h == 1:
            assert abs(_oil_rate(x[1]) - lim) <= 1e-7 * lim and x[1, 3] >= pmin
        else:
            assert abs(x[1, 3] - pmin) <= 1e-7 * pmin and _oil_rate(x[1]) <= lim


# ------------------------------------------------------------- wet gas
# Oil vaporised in the gas (sec. 2.1.6) with the third meaning x = r_og.
def _wet_fluid(rv_at_bubble=0.05):
    fl = cases.live_fluid()
    fl.rv_c = rv_at_bubble / (3000 * PSI)
    return fl


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


def pin_wet_jacobian_fd(lib_path=None):
    """With all three meanings present (s_g, r_go, r_og) and both well
    kinds, every Jacobian column matches central differences of the
    residual."""
    wells = [Well("I", cases.WELL_RATE_INJ, [(0, 0, 0)], 1e4 * 0.0283168 / DAY, phase=cases.GAS),
             Well("P", cases.WELL_BHP_PROD, [(3, 1, 0)], 2500 * PSI)]
    c = cases.box_case(4, 2, 2, seed=3, fluid=_wet_fluid(), wells=wells)
    m = _model(c, lib_path)
    y, mean = _wet_state(c, 1)
    assert set(mean) == {0, 1, 2}
    m.set_meaning(mean)
    acc0 = m.accumulation(y * 1.01)
    st, R, J = m.assemble(y, acc0, DAY)
    rp, ci = m.pattern()
    scale = np.abs(J).max()
    for c_ in range(m.n):
        for v in range(3):
            h = 1e-6 * max(abs(y[c_, v]), 1e-3)
            yp, ym = y.copy(), y.copy()
            yp[c_, v] += h
            ym[c_, v] -= h
            fd = (m.assemble(yp, acc0, DAY)[1] - m.assemble(ym, acc0, DAY)[1]) / (2 * h)
            for i in range(m.n):
                q = [q for q in range(rp[i], rp[i + 1]) if ci[q] == c_]
                an = J[q[0]][:, v] if q else np.zeros(3)
                assert np.abs(fd[i] - an).max() <= 1e-6 * np.abs(fd).max() + 1e-12 * scale


def pin_wet_dew_point_continuity(lib_path=None):
    """A cell at its dew point written either way (x = s_g = 1 - s_w with
    the gas saturated, or x = r_og = r_v(p) with no oil) gives the same
    residual."""
    c = cases.box_case(3, 2, 1, seed=4, fluid=_wet_fluid(), wells=[])
    m = _model(c, lib_path)
    y, mean = _wet_state(c, 2)
    mean[:] = 0
    y[:, 2] = 0.1
    k = 2
    ya, yb = y.copy(), y.copy()
    ya[k, 2] = 1.0 - ya[k, 1]                  # s_o = 0, meaning 0
    yb[k, 2] = c.fluid.rv_c * yb[k, 0]          # meaning 2 at saturation
    mb = mean.copy()
    mb[k] = 2
    acc = None
    m.set_meaning(mean)
    acc = m.accumulation(y)
    Ra = m.assemble(ya, acc, DAY)[1]
    m.set_meaning(mb)
    Rb = m.assemble(yb, acc, DAY)[1]
    assert np.abs(Ra - Rb).max() <= 1e-12 * np.abs(Ra).max()


def pin_wet_oil_moves_with_gas(lib_path=None):
    """Between two oil-free cells (x = r_og) the oil component moves only
    in the gas, upwinded with it: the oil flux is r_og of the upwind cell
    times the gas flux, in either direction, and the two cells' fluxes
    cancel."""
    c = cases.box_case(2, 1, 1, seed=5, fluid=_wet_fluid(), wells=[])
    m = _model(c, lib_path)
    m.set_meaning(np.array([2, 2], np.uint8))
    for hi in (0, 1):
        y = np.empty((2, 3))
        y[:, 0] = 3000 * PSI
        y[hi, 0] = 3100 * PSI
        y[:, 1] = 0.2
        y[:, 2] = [0.6 * c.fluid.rv_c * y[0, 0], 0.3 * c.fluid.rv_c * y[1, 0]]
        acc = m.accumulation(y)
        R = m.assemble(y, acc, DAY)[1]   # accumulation terms vanish: fluxes only
        assert abs(R[0, 1] + R[1, 1]) <= 1e-12 * abs(R[0, 1])
        assert abs(R[0, 2] + R[1, 2]) <= 1e-12 * abs(R[0, 2])
        assert abs(R[0, 1] - y[hi, 2] * R[0, 2]) <= 1e-12 * abs(R[0, 1])


def pin_wet_vaporisation_run(lib_path=None):
    """Dry gas injected into undersaturated oil with wet gas: every report
    step converges and conserves each component; the states stay valid (no
    negative oil in any meaning, r_og of an oil-free cell at most r_v(p),
    r_go of a gas-free cell at most r_s(p)); oil-free cells appear next to
    the injector and their number never falls."""
    c = cases.config_wet()
    m = _model(c, lib_path)
    states, reps = m.run()
    eps = c.fluid.eps_switch
    counts = []
    for y, mean, r in zip(states, m.run_meanings, reps):
        assert max(r["mass_err"]) <= 1e-10, r["mass_err"]
        sg = np.where(mean == 0, y[:, 2], np.where(mean == 2, 1.0 - y[:, 1], 0.0))
        so = 1.0 - y[:, 1] - sg
        assert so.min() >= -eps and sg.min() >= -eps
        rv, rs = c.fluid.rv_c * y[:, 0], c.fluid.rs_c * y[:, 0]
        assert np.all(y[mean == 2, 2] <= rv[mean == 2] * (1 + eps))
        assert np.all(y[mean == 1, 2] <= rs[mean == 1] * (1 + eps))
        counts.append(int((mean == 2).sum()))
    assert counts[-1] > 0 and counts == sorted(counts), counts
    inj = c.wells[0].cells[0]
    k = np.flatnonzero(m.run_meanings[-1] == 2)
    i0 = c.box_index(*inj)
    boxes = np.flatnonzero(c.mask.ravel())[k]
    ii, jj = boxes % c.nx, (boxes // c.nx) % c.ny
    assert np.hypot(ii - inj[0], jj - inj[1]).max() <= 0.5 * np.hypot(c.nx, c.ny), (ii, jj, i0)


# ---------------------------------------------------------------- CPR-AMG
# Two-stage CPR preconditioner (sec. 2.3.1) with an aggregation AMG for the
# pressure stage.
def _cpr_system(case, lib_path, seed=1):
    m = _model(case, lib_path)
    y = cases.random_state(case, seed=seed)
    st, R, J = m.assemble(y, m.accumulation(cases.random_state(case, seed=seed + 1)), 2 * DAY)
    st, F = m.ilu0(J)
    assert st == 0
    return m, R, J, F


def pin_cpr_weights_decouple(lib_path=None):
    """Quasi-IMPES weights decouple the pressure in each cell's diagonal
    block: w_i^T D_i = (1, 0, 0), and the pressure matrix holds w_i^T A_ij
    applied to the pressure unit vector."""
    c = _wells_case(3, 3, 2, seed=7)
    m = _model(c, lib_path)
    y = cases.random_state(c, seed=11)
    st, R, J = m.assemble(y, m.accumulation(cases.random_state(c, seed=12)), 2 * DAY)
    cp = m.cpr(J)
    w = cp.weights()
    rp, ci = m.pattern()
    for i in range(m.n):
        q = rp[i] + list(ci[rp[i]:rp[i + 1]]).index(i)
        row = w[i] @ J[q]
        tol = 1e-12 * 3 * np.abs(w[i]).max() * np.abs(J[q]).max()   # rounding of w^T D
        assert abs(row[0] - 1.0) <= tol and np.all(np.abs(row[1:]) <= tol), (row, tol)
    rp0, ci0, a0, _ = cp.level(0)
    Ap = np.array([w[i] @ J[q][:, 0] for i in range(m.n) for q in range(rp[i], rp[i + 1])])
    assert np.array_equal(rp0, rp) and np.array_equal(ci0, ci)
    assert np.abs(a0 - Ap).max() <= 1e-12 * np.abs(Ap).max()


def pin_cpr_galerkin_hierarchy(lib_path=None):
    """Each coarse level is the Galerkin product P^T A P with the piecewise
    constant P of geometric 2x2x2 aggregates of the level's lattice (coarse
    unknowns numbered in natural order of the occupied coarse boxes),
    rebuilt here from the cell coordinates and numpy."""
    c = cases.box_case(9, 7, 5, seed=5, mask=cases.masked_mask(
        np.random.default_rng(8), (5, 7, 9), 200), wells=[])
    m = _model(c, lib_path)
    y = cases.random_state(c, seed=3)
    st, R, J = m.assemble(y, m.accumulation(cases.random_state(c, seed=4)), 2 * DAY)
    cp = m.cpr(J)
    assert cp.nl >= 2
    boxes = m.geometry()["cell_box"]
    dims = (c.nx, c.ny, c.nz)
    for l in range(cp.nl - 1):
        rp, ci, a, agg = cp.level(l)
        n = len(rp) - 1
        A = np.zeros((n, n))
        for i in range(n):
            A[i, ci[rp[i]:rp[i + 1]]] = a[rp[i]:rp[i + 1]]
        cd = tuple((d + 1) // 2 for d in dims)
        parent = [(b % dims[0]) // 2 + cd[0] * (((b // dims[0]) % dims[1]) // 2 +
                                                 cd[1] * ((b // (dims[0] * dims[1])) // 2))
                  for b in boxes]
        occupied = sorted(set(parent))
        index = {b: k for k, b in enumerate(occupied)}
        want = np.array([index[b] for b in parent])
        assert np.array_equal(agg, want)
        P = np.zeros((n, len(occupied)))
        P[np.arange(n), want] = 1.0
        rpc, cic, ac, _ = cp.level(l + 1)
        Ac = np.zeros((len(occupied), len(occupied)))
        for I in range(len(occupied)):
            Ac[I, cic[rpc[I]:rpc[I + 1]]] = ac[rpc[I]:rpc[I + 1]]
        G = P.T @ A @ P
        assert np.abs(Ac - G).max() <= 1e-12 * np.abs(G).max()
        boxes, dims = occupied, cd
    assert len(cp.level(cp.nl - 1)[0]) - 1 <= 64 or dims == (1, 1, 1)


def pin_cpr_exact_second_stage(lib_path=None):
    """With an exact second stage (ILU(0) of a 1-D chain is its LU), CPR is
    the exact inverse whatever the pressure stage gives: z = x1 + A^{-1}(r -
    A x1) = A^{-1} r; BiCGStab with CPR stops after half an iteration."""
    c = cases.box_case(7, 1, 1, seed=3)
    m, R, J, F = _cpr_system(c, lib_path)
    cp = m.cpr(J)
    z = cp.apply(F, -R)
    xd = np.linalg.solve(_dense(m, J), -R.ravel()).reshape(-1, 3)
    assert np.abs(z - xd).max() <= 1e-9 * np.abs(xd).max()
    st, x, its, rr = cp.bicgstab(F, -R, rtol=1e-10)
    assert st == 0 and its == 0.5


def pin_cpr_vcycle_converges(lib_path=None):
    """The V(1,1) cycle as a stationary iteration on the pressure system of a
    heterogeneous 9000-cell system reduces the residual every cycle, below a
    quarter after ten."""
    c = cases.config2()
    m, R, J, F = _cpr_system(c, lib_path)
    cp = m.cpr(J)
    rp, ci, a, _ = cp.level(0)
    n = m.n

    def Ap(x):
        return np.array([a[rp[i]:rp[i + 1]] @ x[ci[rp[i]:rp[i + 1]]] for i in range(n)])

    b = np.random.default_rng(0).standard_normal(n)
    x = np.zeros(n)
    prev = 1.0
    for _ in range(10):
        x = x + cp.vcycle(b - Ap(x))
        rel = np.linalg.norm(b - Ap(x)) / np.linalg.norm(b)
        assert rel < prev
        prev = rel
    assert prev <= 0.25, prev


def pin_cpr_two_grid(lib_path=None):
    """On a two-level hierarchy (108 cells, 18 coarse unknowns solved
    exactly) the cycle is a Galerkin coarse-grid correction between two
    damped Jacobi sweeps (omega = 2/3): undoing the post-sweep gives an
    iterate x_mid whose difference from the pre-sweep omega D^-1 b lies in
    range(P) and whose residual is orthogonal to range(P), P^T (b - A x_mid)
    = 0.  Checked on a near-elliptic pressure system (a very long step)."""
    wells = [Well("P", cases.WELL_BHP_PROD, [(5, 5, 2)], 3000 * PSI)]
    c = cases.box_case(6, 6, 3, seed=4, wells=wells)
    m = _model(c, lib_path)
    y = cases.random_state(c, seed=2)
    st, R, J = m.assemble(y, m.accumulation(y), 1e5 * DAY)
    cp = m.cpr(J)
    assert cp.nl == 2
    rp, ci, a, agg = cp.level(0)
    n = m.n
    A = np.zeros((n, n))
    for i in range(n):
        A[i, ci[rp[i]:rp[i + 1]]] = a[rp[i]:rp[i + 1]]
    P = np.zeros((n, agg.max() + 1))
    P[np.arange(n), agg] = 1.0
    d = np.diag(A)
    om = 2.0 / 3.0
    b = np.random.default_rng(1).standard_normal(n)
    x = cp.vcycle(b)
    S = np.eye(n) - om * (A / d[:, None])
    x_mid = np.linalg.solve(S, x - om * b / d)
    x_pre = om * b / d
    coef = np.linalg.lstsq(P, x_mid - x_pre, rcond=None)[0]
    assert np.abs(P @ coef - (x_mid - x_pre)).max() <= 1e-9 * np.abs(x_mid).max()
    orth = P.T @ (b - A @ x_mid)
    assert np.abs(orth).max() <= 1e-9 * np.abs(P.T @ b).max(), np.abs(orth).max()


def pin_cpr_fewer_iterations(lib_path=None):
    """CPR reduces the linear iterations against the ILU(0) alone on the
    Newton system of the 9000-cell waterflood's first step, and both solve
    it to the tolerance."""
    c = cases.config2()
    m = _model(c, lib_path)
    y0 = c.initial_state()
    st, R, J = m.assemble(y0, m.accumulation(y0), c.report_dt[0])
    y1 = y0.copy()
    st, F = m.ilu0(J)
    st, x, its_ilu, _ = m.bicgstab(J, F, -R, rtol=1e-6)
    assert st == 0
    # a system off equilibrium: one Newton update in
    y1 = y0 + x
    st, R, J = m.assemble(y1, m.accumulation(y0), c.report_dt[0])
    st, F = m.ilu0(J)
    st, x, its_ilu, _ = m.bicgstab(J, F, -R, rtol=1e-6)
    cp = m.cpr(J)
    st2, x2, its_cpr, _ = cp.bicgstab(F, -R, rtol=1e-6)
    assert st == 0 and st2 == 0
    assert its_cpr < its_ilu, (its_cpr, its_ilu)
    res = -R - m.spmv(J, x2)
    assert np.linalg.norm(res) <= 1e-6 * np.linalg.norm(R) * 1.0001


def pin_cpr_newton(lib_path=None):
    """The preconditioner changes the linear iterations, not the Newton
    state: a report step with CPR matches the ILU(0) one to the Newton
    tolerance and conserves mass."""
    c = cases.config1()
    m = _model(c, lib_path)
    st, ya, ra = m.advance(c.initial_state(), c.report_dt[0])
    st2, yb, rb = m.advance(c.initial_state(), c.report_dt[0],
                            oracle.default_opts(c, precond=1))
    assert st == 0 and st2 == 0
    assert np.abs(ya[:, 0] - yb[:, 0]).max() <= 1e-8 * np.abs(ya[:, 0]).max()
    assert np.abs(ya[:, 1:] - yb[:, 1:]).max() <= 1e-8
    assert max(rb.mass_err) <= 1e-10


# ------------------------------------------------------ time-step cutting
def _held_state(m):
    """The state a model holds beside y: meanings, well state, controls."""
    if m.std_wells:
        return m.meaning().copy(), m.well_state().copy(), m.well_ctrl().copy()
    return m.meaning().copy(), None, None


def _set_held_state(m, held):
    mean, wx, ctrl = held
    m.set_meaning(mean)
    if wx is not None:
        m.set_well_state(wx)
        m.set_well_ctrl(ctrl)


def pin_time_step_cut(lib_path=None):
    """Sec. 2.3 cuts the time step when the Newton loop fails; the reading
    halves the length, keeps the shorter length for the rest of the report
    step and retries from the last accepted state (y, the variable meanings,
    the well state and the active controls, bit for bit).  A tight Newton
    cap forces cuts on dead oil (C1), on live oil whose gas comes out of
    solution (the meanings switch inside rejected attempts) and on C1 with
    standard wells whose limits bind (the controls switch inside rejected
    attempts).  Checked: every attempt's length follows the rule; each
    rejected attempt is a Newton step that really fails from the accepted
    state; and an uninterrupted sequence of Newton steps over the accepted
    lengths, on a second model, reproduces the report step's y, meanings,
    well state and controls exactly."""
    live = cases.config_live()
    runs = [(cases.config1(), [30 * DAY] * 2, 7),
            (live, list(live.report_dt[:2]), 3),
            (_switch_case(7000, 1500), [30 * DAY] * 2, 7)]
    for case, lengths, max_newton in runs:
        opts = oracle.default_opts(case, max_newton=max_newton)
        m = _model(case, lib_path)           # report steps with cuts
        u = _model(case, lib_path)           # accepted substeps only
        probe = _model(case, lib_path)       # rejected attempts, from the accepted state
        y = case.initial_state()
        yu = y.copy()
        cuts = 0
        for D in lengths:
            st, y, rep, dts, sts = m.advance_log(y, D, opts)
            assert st == 0 and len(dts) == rep.substeps + rep.cuts
            t, prev_failed, prev = 0.0, False, D
            for dt, s in zip(dts, sts):
                # exact halving after a rejection; otherwise the kept length,
                # both capped by what is left of the report step
                want = min(0.5 * prev if prev_failed else prev, D - t)
                assert dt == want, (case.name, dt, want)
                held = _held_state(u)
                if s == 0:
                    su, yu, _ = u.newton_step(yu, yu, dt, opts)
                    assert su == 0
                    t += dt
                else:
                    _set_held_state(probe, held)
                    sp, _, _ = probe.newton_step(yu, yu, dt, opts)
                    assert sp != 0
                    cuts += 1
                prev_failed, prev = s != 0, dt
            assert t == D
            assert np.array_equal(y, yu), case.name
            hm, hu = _held_state(m), _held_state(u)
            assert np.array_equal(hm[0], hu[0])
            if hm[1] is not None:
                assert np.array_equal(hm[1], hu[1]) and np.array_equal(hm[2], hu[2])
        assert cuts >= 1, case.name


ALL_PINS = [
    pin_series_transmissibility, pin_depth_pore_volume, pin_peaceman_worked_value,
    pin_compressibility, pin_darcy_flux_upwind, pin_hydrostatic_column, pin_pressure_block,
    pin_jacobian_fd, pin_conservation, pin_norms, pin_ilu0_pattern, pin_ilu0_exact_1d,
    pin_bicgstab_dense, pin_block_ilu0_partition, pin_block_ilu0_special_cases,
    pin_block_ilu0_newton, pin_gmres_dense, pin_gmres_exact_lu, pin_gmres_minimal_residual,
    pin_gmres_newton, pin_one_cell_producer, pin_injector_mass, pin_quadratic_convergence,
    pin_mass_balance_run, pin_mirror_symmetry, pin_live_dead_limit, pin_live_switch_continuity,
    pin_live_jacobian_fd, pin_live_conservation, pin_live_closed_cell,
    pin_live_dissolved_moves_with_oil, pin_live_hydrostatic_column, pin_live_depletion_1d,
    pin_std_schur_dense, pin_std_jacobian_fd, pin_std_simplified_limit,
    pin_std_controls_and_storage, pin_std_control_switching, pin_wet_jacobian_fd,
    pin_wet_dew_point_continuity, pin_wet_oil_moves_with_gas, pin_wet_vaporisation_run,
    pin_cpr_weights_decouple,
    pin_cpr_galerkin_hierarchy,
    pin_cpr_exact_second_stage, pin_cpr_vcycle_converges, pin_cpr_two_grid,
    pin_cpr_fewer_iterations,
    pin_cpr_newton, pin_time_step_cut,
]
