"""Planted mistakes in the oracle must be caught by its pins (CPU only).

Each mutant is a copy of ``oracle/oracle.c`` with one plausible slip (a
dropped term, a wrong sign, a swapped index or operand) compiled into a
temporary library; at least one pin of ``oracle_pins.py`` has to fail on it.
This shows the pins constrain every part of the oracle, not just re-run it.
"""
import os
import shutil
import subprocess

import pytest

from oracle_pins import ALL_PINS

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

MUTANTS = [
    ("gravity_sign", "dsub(dsub(Pi.p, Pj.p), dmul(dscale(rho_avg, f->g), dzij))",
     "dadd(dsub(Pi.p, Pj.p), dmul(dscale(rho_avg, f->g), dzij))"),
    ("density_not_averaged", "dscale(dadd(Pi.rho[a], Pj.rho[a]), 0.5)", "Pi.rho[a]"),
    ("upwind_reversed", "(dphi[a].v >= 0.0) ? &Pi : &Pj", "(dphi[a].v >= 0.0) ? &Pj : &Pi"),
    ("flux_not_antisymmetric", "R[3 * j + a] -= F.v;", "R[3 * j + a] += F.v;"),
    ("offdiag_block_sign", "add_block(J, bij, a, F.d + 3, 1.0);", "add_block(J, bij, a, F.d + 3, -1.0);"),
    ("neighbour_block_swapped", "add_block(J, bji, a, F.d, -1.0);", "add_block(J, bji, a, F.d + 3, -1.0);"),
    ("arithmetic_mean_trans", "tij * tji / (tij + tji)", "0.5 * (tij + tji)"),
    ("full_cell_half_trans", "return area * num / den;", "return 0.5 * area * num / den;"),
    ("linearised_b", "P->b[a] = dexp(dscale(dsub(P->p, dconst(f->p_ref)), f->c[a]));",
     "P->b[a] = dadd(dconst(1.0), dscale(dsub(P->p, dconst(f->p_ref)), f->c[a]));"),
    ("gwseg_weight_sum", "dual wsum = dadd(ww, wg);", "dual wsum = dadd(ww, ww);"),
    ("corey_linear", "dual krw = dpow(swn, f->n_corey);", "dual krw = dpow(swn, 1.0);"),
    ("gas_relperm_scaling", "dual sgn = dclamp01(ddiv(sg, dconst(den)));", "dual sgn = dclamp01(sg);"),
    ("oil_sat_sign", "dual so = dsub(dsub(dconst(1.0), sw), sg);", "dual so = dadd(dsub(dconst(1.0), sw), sg);"),
    ("quotient_rule", "(a.d[i] * b.v - a.v * b.d[i]) / (b.v * b.v)", "(a.d[i] * b.v + a.v * b.d[i]) / (b.v * b.v)"),
    ("accumulation_deriv_dropped", "      if (J) add_block(J, dblk, a, r.d, 1.0);\n    }\n  }\n  /* connection",
     "    }\n  }\n  /* connection"),
    ("ilu_transposed_operand", "mat3_mul(F + 9 * q, inv, tmp);", "mat3_mul(inv, F + 9 * q, tmp);"),
    ("ilu_update_sign", "F[9 * r + e] -= tmp[e];", "F[9 * r + e] += tmp[e];"),
    ("ilu_forward_uses_rhs", "t[a] -= F[9 * q + 3 * a + v] * w[3 * k + v];",
     "t[a] -= F[9 * q + 3 * a + v] * r[3 * k + v];"),
    ("bicgstab_direction", "p[k] = r[k] + beta * (p[k] - omega * v[k]);",
     "p[k] = r[k] + beta * (p[k] + omega * v[k]);"),
    ("producer_drawdown_sign", "dual dp = dsub(P.p, dconst(m->well_target[w]));",
     "dual dp = dsub(dconst(m->well_target[w]), P.p);"),
    ("injector_sign", "dconst(-m->well_target[w] * m->conn_wi[q] / wsum)",
     "dconst(m->well_target[w] * m->conn_wi[q] / wsum)"),
    ("cnv_without_b", "dt * fabs(R[3 * c + a]) / (P.b[a].v * m->pv[c])", "dt * fabs(R[3 * c + a]) / m->pv[c]"),
    ("depth_top_not_centre", "m->depth[c] = layer_top(m, k) + 0.5 * dz[k];", "m->depth[c] = layer_top(m, k);"),
    ("kv_not_scaled", "m->kv[c] = kv_kh * perm_h[b];", "m->kv[c] = perm_h[b];"),
    ("peaceman_radius", "double ro = 0.14 * sqrt(dx * dx + dy * dy);", "double ro = 0.2 * dx;"),
    ("chop_not_applied_to_dp", "y[3 * c] += dp;", "y[3 * c] += 0.9 * dp;"),
    ("block_couplings_kept", "if (!same_block(m, i, m->col_idx[q])) memset",
     "if (m->blk[0] < 0 && !same_block(m, i, m->col_idx[q])) memset"),
    ("block_lower_couplings_only", "if (!same_block(m, i, m->col_idx[q])) memset",
     "if (m->col_idx[q] < i && !same_block(m, i, m->col_idx[q])) memset"),
    ("block_axis_swapped", "ka / m->blk[2] == kb / m->blk[2]", "ka / m->blk[1] == kb / m->blk[1]"),
    ("gmres_gram_schmidt_sign", "for (int k = 0; k < N; ++k) w[k] -= h * vi[k];",
     "for (int k = 0; k < N; ++k) w[k] += h * vi[k];"),
    ("gmres_givens_sign", "g[j + 1] = -sn[j] * g[j];", "g[j + 1] = sn[j] * g[j];"),
    ("gmres_rotation_sign", "Hm(i + 1, j) = -sn[i] * a + cs[i] * c;", "Hm(i + 1, j) = sn[i] * a + cs[i] * c;"),
    ("gmres_update_unpreconditioned", "for (int k = 0; k < N; ++k) x[k] += z[k];",
     "for (int k = 0; k < N; ++k) x[k] += w[k];"),
    # live oil
    ("live_dissolved_gas_not_stored", "if (a == 2) A = dadd(A, dmul(P->r, dmul(P->b[1], P->s[1])));",
     "if (a == 2) A = dadd(A, dconst(0.0));"),
    ("live_dissolved_gas_gas_upwind",
     "F = dadd(F, dmul(dmul(U[1]->r, dmul(U[1]->b[1], U[1]->lam[1])), dscale(dphi[1], T)));",
     "F = dadd(F, dmul(dmul(U[2]->r, dmul(U[2]->b[1], U[2]->lam[1])), dscale(dphi[1], T)));"),
    ("live_rs_derivative_dropped", "(mean == 1 ? x : dscale(P->p, f->rs_c))",
     "(mean == 1 ? x : dconst(P->p.v * f->rs_c))"),
    ("live_oil_density_without_gas",
     "P->rho[1] = dmul(P->b[1], dadd(dconst(f->rho_s[1]), dscale(P->r, f->rho_s[2])));",
     "P->rho[1] = dscale(P->b[1], f->rho_s[1]);"),
    ("live_swelling_inverted", "P->b[1] = ddiv(P->b[1], dadd(dconst(1.0), dscale(P->r, f->bo_r)));",
     "P->b[1] = dmul(P->b[1], dadd(dconst(1.0), dscale(P->r, f->bo_r)));"),
    ("live_producer_without_dissolved_gas", "      if (m->fl.live)\n        out[2] = dadd(out[2],",
     "      if (0)\n        out[2] = dadd(out[2],"),
    ("live_gas_never_appears", "if (yc[2] > rs * (1.0 + f->eps_switch)) {", "if (0) {"),
    ("live_free_gas_in_undersaturated_cell", "dual sg = (f->live && mean == 1) ? dconst(0.0)",
     "dual sg = (f->live && mean == 1) ? x"),
    # standard wells and the Schur complement
    ("std_schur_operator_sign", "y[3 * c + a] -= op->C[12 * q + 4 * a + k] * u[k];",
     "y[3 * c + a] += op->C[12 * q + 4 * a + k] * u[k];"),
    ("std_schur_rhs_missing", "b[3 * c + a] -= C[12 * q + 4 * a + k] * u[k];",
     "b[3 * c + a] -= 0.0 * C[12 * q + 4 * a + k] * u[k];"),
    ("std_well_recovery_sign", "t[e] -= B[12 * q + 3 * e + v] * xr[3 * c + v];",
     "t[e] += B[12 * q + 3 * e + v] * xr[3 * c + v];"),
    ("std_injection_uses_cell_phases",
     "    for (int a = 0; a < 3; ++a) out[a] = dmul(dmul(dscale(lt, wi), dp), W.mix[a]);",
     "    for (int a = 0; a < 3; ++a) out[a] = dmul(dscale(dmul(P.b[a], P.lam[a]), wi), dp);"),
    ("std_storage_dropped", "R[a] = dadd(st, dscale(dmul(W.F[a], W.Qt), 1.0 / kWellG[a]));",
     "R[a] = dadd(dscale(st, 0.0), dscale(dmul(W.F[a], W.Qt), 1.0 / kWellG[a]));"),
    ("std_B_sign", "B[12 * q + 3 * a + v] = -qr[a].d[v];", "B[12 * q + 3 * a + v] = qr[a].d[v];"),
    ("std_C_wrong_slots", "C[12 * q + 4 * a + k] = qr[a].d[3 + k];",
     "C[12 * q + 4 * a + k] = qr[a].d[k];"),
    ("std_bhp_control_sign", "R[3] = dsub(W.pb, dconst(m->well_target[w]));",
     "R[3] = dadd(W.pb, dconst(m->well_target[w]));"),
    # CPR-AMG
    ("cpr_weights_not_transposed",
     "double T[9] = {Dg[0], Dg[3], Dg[6], Dg[1], Dg[4], Dg[7], Dg[2], Dg[5], Dg[8]};",
     "double T[9] = {Dg[0], Dg[1], Dg[2], Dg[3], Dg[4], Dg[5], Dg[6], Dg[7], Dg[8]};"),
    ("cpr_pressure_column_wrong", "for (int a = 0; a < 3; ++a) v += c->w[3 * i + a] * J[9 * q + 3 * a];",
     "for (int a = 0; a < 3; ++a) v += c->w[3 * i + a] * J[9 * q + 3 * a + 1];"),
    ("cpr_restrict_rhs_not_residual", "bc[c->agg[l][i]] += b[i] - r[i];",
     "bc[c->agg[l][i]] += b[i];"),
    ("cpr_prolongation_dropped", "x[i] += xc[c->agg[l][i]];   /* prolong */",
     "x[i] += 0.0 * xc[c->agg[l][i]];   /* prolong */"),
    ("cpr_post_smooth_sign", "x[i] += kJacobiOmega * (b[i] - r[i]) / csr_diag(c, l, i);",
     "x[i] -= kJacobiOmega * (b[i] - r[i]) / csr_diag(c, l, i);"),
    ("cpr_second_stage_on_r", "for (int k = 0; k < 3 * n; ++k) r2[k] = r[k] - r2[k];",
     "for (int k = 0; k < 3 * n; ++k) r2[k] = r[k];"),
    ("cpr_galerkin_drops_entries", "acc[J] += c->a[l][q];", "acc[J] = c->a[l][q];"),
    ("std_rate_control_sign",
     "R[3] = dadd(dscale(dmul(W.F[ph], W.Qt), 1.0 / kWellG[ph]), dconst(m->well_target[w]));",
     "R[3] = dsub(dscale(dmul(W.F[ph], W.Qt), 1.0 / kWellG[ph]), dconst(m->well_target[w]));"),
    ("std_switch_rate_compare", "if (*c == 0 && qo > m->well_limit[w]) *c = 1;",
     "if (*c == 0 && qo < m->well_limit[w]) *c = 1;"),
    ("std_switch_back_reversed", "else if (*c == 1 && x[3] < m->well_target[w]) *c = 0;",
     "else if (*c == 1 && x[3] > m->well_target[w]) *c = 0;"),
    ("std_rate_limit_wrong_phase",
     "R[3] = dsub(dscale(dmul(W.F[1], W.Qt), 1.0 / kWellG[1]), dconst(m->well_limit[w]));",
     "R[3] = dsub(dscale(dmul(W.F[0], W.Qt), 1.0 / kWellG[0]), dconst(m->well_limit[w]));"),
    ("std_injector_limit_uses_target", "R[3] = dsub(W.pb, dconst(m->well_limit[w]));",
     "R[3] = dsub(W.pb, dconst(m->well_target[w]));"),
    ("wet_vaporised_oil_not_upwinded",
     "F = dadd(F, dmul(dmul(U[2]->rv, dmul(U[2]->b[2], U[2]->lam[2])), dscale(dphi[2], T)));",
     "F = dadd(F, dmul(dmul(Pi.rv, dmul(U[2]->b[2], U[2]->lam[2])), dscale(dphi[2], T)));"),
    ("wet_oil_free_gas_saturation", "            : (wet && mean == 2)    ? dsub(dconst(1.0), sw)",
     "            : (wet && mean == 2)    ? x"),
    # time-step cutting
    ("cut_quarter_length", "dt_try = 0.5 * dt;", "dt_try = 0.25 * dt;"),
    ("cut_state_not_restored", "      memcpy(y, yn, sizeof(double) * N);\n      memcpy(m->mean, mn",
     "      memcpy(m->mean, mn"),
    ("cut_meanings_not_restored", "      memcpy(m->mean, mn, (size_t)m->n);\n      if (wbytes)",
     "      if (wbytes)"),
    ("cut_well_state_not_restored", "if (wbytes) memcpy(m->wx, wn, wbytes);", ""),
    ("cut_controls_not_restored", "if (cbytes) memcpy(m->wctrl, cn, cbytes);", ""),
    ("cut_length_not_kept", "      t += dt;\n", "      t += dt;\n      dt_try = dt_report;\n"),
]


@pytest.fixture(scope="module")
def mutant_dir(tmp_path_factory):
    return tmp_path_factory.mktemp("oracle_mutants")


def _build(mdir, name, old, new):
    src = open(os.path.join(ROOT, "oracle", "oracle.c")).read()
    assert src.count(old) == 1, f"mutation anchor for {name} must occur exactly once"
    d = os.path.join(str(mdir), name)
    os.makedirs(d, exist_ok=True)
    shutil.copy(os.path.join(ROOT, "oracle", "oracle.h"), d)
    with open(os.path.join(d, "oracle.c"), "w") as fh:
        fh.write(src.replace(old, new))
    so = os.path.join(d, "liboracle_mut.so")
    subprocess.run(["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fPIC", "-shared", "-o", so,
                    os.path.join(d, "oracle.c"), "-lm"], check=True)
    return so


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(mutant_dir, name, old, new):
    so = _build(mutant_dir, name, old, new)
    caught = None
    for pin in ALL_PINS:   # the first pin that fails is enough
        try:
            pin(lib_path=so)
        except Exception as e:   # an assertion, a solver failure or a NaN all count
            caught = f"{pin.__name__}: {type(e).__name__}"
            break
    assert caught, f"planted mistake '{name}' passed every pin"
