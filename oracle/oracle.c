/*
 * oracle.c -- plain FP64 CPU reference of the TPFA black-oil Newton path.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h).  Written for readability, not
 * speed: one generic dual-number type, faces visited once, block entries
 * located by searching the row, generic IKJ ILU(0), textbook BiCGStab.
 *
 * What pins each part (tests/test_oracle_*.py):
 *   geometry        series-resistance and equal-permeability closed forms,
 *                   the layered-depth definition, Peaceman worked value
 *   properties      defining ODE of constant compressibility (b'/b = c),
 *                   Corey worked values, gwseg two-phase reductions
 *   residual        hydrostatic column (R = 0 to round-off), 1-D Darcy flux
 *                   against the series-resistance formula, upwind selection,
 *                   single-phase pressure block closed form, exact flux
 *                   cancellation (sum of residuals = accumulation + wells)
 *   Jacobian        central finite differences of the residual
 *   ILU(0)          (LU)_ij = A_ij on every pattern entry; exact LU on 1-D
 *   block ILU0      LU = A inside subdomains and 0 between them; one box =
 *                   ILU(0); one-cell boxes = block Jacobi; cut 1-D chain
 *   BiCGStab        dense direct solve (numpy) on tiny grids
 *   GMRes           dense direct solve with restarts; one iteration with an
 *                   exact LU; least-squares minimum over the Krylov space
 *   Newton          one-cell producer root by bisection, quadratic
 *                   convergence, mass balance per step, mirror symmetry
 * Full multi-step runs are not pinned against the paper (it prints no
 * states); they are pinned only through the properties above.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* Threads of the OpenMP build (the CPU baseline); the plain build used by
 * the tests is single-threaded and ignores this. */
void ora_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

int ora_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* ------------------------------------------------------------------ timing */
static double now_s(void) {
  struct timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

/* ------------------------------------------- forward-mode AD (sec. 2.4.1)
 * A value paired with a fixed number of partial derivatives; every operation
 * applies the chain rule.  Slots 0-2 are d/d(p, s_w, x) of the first cell
 * of a connection, slots 3-5 those of the second cell; for a standard-well
 * connection slots 3-6 are d/d(Q_t, F_w, F_g, p_bhp) of the well. */
#define ND 7
typedef struct {
  double v;
  double d[ND];
} dual;

static dual dconst(double v) {
  dual r;
  r.v = v;
  for (int i = 0; i < ND; ++i) r.d[i] = 0.0;
  return r;
}
static dual dvar(double v, int slot) {
  dual r = dconst(v);
  r.d[slot] = 1.0;
  return r;
}
static dual dadd(dual a, dual b) {
  dual r;
  r.v = a.v + b.v;
  for (int i = 0; i < ND; ++i) r.d[i] = a.d[i] + b.d[i];
  return r;
}
static dual dsub(dual a, dual b) {
  dual r;
  r.v = a.v - b.v;
  for (int i = 0; i < ND; ++i) r.d[i] = a.d[i] - b.d[i];
  return r;
}
static dual dmul(dual a, dual b) {   /* (uv)' = u'v + uv' */
  dual r;
  r.v = a.v * b.v;
  for (int i = 0; i < ND; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i];
  return r;
}
static dual ddiv(dual a, dual b) {   /* (u/v)' = (u'v - uv')/v^2 */
  dual r;
  r.v = a.v / b.v;
  for (int i = 0; i < ND; ++i) r.d[i] = (a.d[i] * b.v - a.v * b.d[i]) / (b.v * b.v);
  return r;
}
static dual dscale(dual a, double s) {
  dual r;
  r.v = a.v * s;
  for (int i = 0; i < ND; ++i) r.d[i] = a.d[i] * s;
  return r;
}
static dual dexp(dual a) {
  dual r;
  r.v = exp(a.v);
  for (int i = 0; i < ND; ++i) r.d[i] = r.v * a.d[i];
  return r;
}
static dual dpow(dual a, double n) {   /* a >= 0, n >= 1 */
  dual r;
  r.v = pow(a.v, n);
  double dv = n * pow(a.v, n - 1.0);
  for (int i = 0; i < ND; ++i) r.d[i] = dv * a.d[i];
  return r;
}
/* clamp to [0,1]; on the bounds themselves the argument passes through */
static dual dclamp01(dual a) {
  if (a.v < 0.0) return dconst(0.0);
  if (a.v > 1.0) return dconst(1.0);
  return a;
}
/* max(a, 0); at a == 0 the constant branch is taken */
static dual dmax0(dual a) {
  if (a.v > 0.0) return a;
  return dconst(0.0);
}

/* ------------------------------------------------------------------ model */
struct ora_model {
  int nx, ny, nz, n, nf, nnzb, nw, nc;
  double dx, dy;
  ora_fluid fl;
  double* dz;      /* [nz] */
  int* cell_box;   /* [n]  */
  int* box_cell;   /* [nx*ny*nz], -1 if inactive */
  double* kh;      /* [n] horizontal permeability */
  double* kv;      /* [n] vertical permeability   */
  double* pv;      /* [n] phi_ref V                */
  double* depth;   /* [n] cell-centre depth, positive down */
  int* face;       /* [nf][2], face[f][0] < face[f][1] */
  double* trans;   /* [nf] */
  int* row_ptr;    /* [n+1] */
  int* col_idx;    /* [nnzb] */
  int* well_kind;  /* [nw] */
  int* well_phase; /* [nw] */
  double* well_target;
  int* well_beg;   /* [nw+1] connection ranges */
  int* conn_cell;  /* [nc] */
  double* conn_wi; /* [nc] */
  int* conn_well;  /* [nc] */
  int blk[3];      /* ILU(0) subdomain box (cells per axis); 0: one block */
  unsigned char* mean;   /* [n] meaning of the third variable: 0 s_g, 1 r_go */
  int std_wells;         /* 1: standard well model with well unknowns */
  double* well_vol;      /* [nw] wellbore volume V_w */
  double* wx;            /* [nw][4] well state (Q_t, F_w, F_g, p_bhp) */
  double* well_limit;    /* [nw] limit of the other control, 0 = none */
  int* wctrl;            /* [nw] active control: 0 the well's own, 1 its limit */
  double* wA0;           /* [nw][3] wellbore storage at the start of the step */
};

int ora_n_cells(const ora_model* m) { return m->n; }
int ora_n_faces(const ora_model* m) { return m->nf; }
int ora_nnzb(const ora_model* m) { return m->nnzb; }
int ora_n_conns(const ora_model* m) { return m->nc; }

void ora_destroy(ora_model* m) {
  if (!m) return;
  free(m->dz); free(m->cell_box); free(m->box_cell); free(m->kh); free(m->kv);
  free(m->pv); free(m->depth); free(m->face); free(m->trans); free(m->row_ptr);
  free(m->col_idx); free(m->well_kind); free(m->well_phase); free(m->well_target);
  free(m->well_beg); free(m->conn_cell); free(m->conn_wi); free(m->conn_well);
  free(m->mean);
  free(m->well_vol); free(m->wx); free(m->wA0); free(m->well_limit); free(m->wctrl);
  free(m);
}

/* Cell centre of box cell (i, j, k); z is depth measured down from the top. */
static double layer_top(const ora_model* m, int k) {
  double z = 0.0;
  for (int q = 0; q < k; ++q) z += m->dz[q];
  return z;
}

/* Half-transmissibility of appendix B:
 * t = |F| (K (c_f - c) . n) / |c_f - c|^2 for a diagonal K. */
static double half_trans(double area, const double K[3], const double c[3], const double cf[3],
                         const double nrm[3]) {
  double d[3] = {cf[0] - c[0], cf[1] - c[1], cf[2] - c[2]};
  double Kd[3] = {K[0] * d[0], K[1] * d[1], K[2] * d[2]};
  double num = Kd[0] * nrm[0] + Kd[1] * nrm[1] + Kd[2] * nrm[2];
  double den = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
  return area * num / den;
}

static int find_block(const ora_model* m, int i, int j) {
  for (int q = m->row_ptr[i]; q < m->row_ptr[i + 1]; ++q)
    if (m->col_idx[q] == j) return q;
  return -1;
}

ora_model* ora_create(int nx, int ny, int nz, double dx, double dy, const double* dz,
                      const double* perm_h, double kv_kh, const double* poro,
                      const unsigned char* mask, const ora_fluid* fluid, int n_wells,
                      const int* well_kind, const int* well_phase, const double* well_target,
                      const double* well_rw, const int* well_nconn, const int* conn_ijk) {
  if (nx <= 0 || ny <= 0 || nz <= 0 || n_wells < 0) return NULL;
  ora_model* m = (ora_model*)calloc(1, sizeof(ora_model));
  const int nb = nx * ny * nz;
  m->nx = nx; m->ny = ny; m->nz = nz; m->dx = dx; m->dy = dy; m->fl = *fluid;
  m->dz = (double*)malloc(sizeof(double) * nz);
  memcpy(m->dz, dz, sizeof(double) * nz);
  m->box_cell = (int*)malloc(sizeof(int) * nb);
  int n = 0;
  for (int b = 0; b < nb; ++b) m->box_cell[b] = (mask == NULL || mask[b]) ? n++ : -1;
  m->n = n;
  m->cell_box = (int*)malloc(sizeof(int) * (n > 0 ? n : 1));
  m->mean = (unsigned char*)calloc((size_t)n + 1, 1);
  for (int b = 0; b < nb; ++b)
    if (m->box_cell[b] >= 0) m->cell_box[m->box_cell[b]] = b;

  /* rock: porosity, permeability tensor diag(kh, kh, kv), pore volume, depth */
  m->kh = (double*)malloc(sizeof(double) * (n + 1));
  m->kv = (double*)malloc(sizeof(double) * (n + 1));
  m->pv = (double*)malloc(sizeof(double) * (n + 1));
  m->depth = (double*)malloc(sizeof(double) * (n + 1));
  for (int c = 0; c < n; ++c) {
    int b = m->cell_box[c];
    int k = b / (nx * ny);
    m->kh[c] = perm_h[b];
    m->kv[c] = kv_kh * perm_h[b];
    m->pv[c] = poro[b] * (dx * dy * dz[k]);
    m->depth[c] = layer_top(m, k) + 0.5 * dz[k];
  }

  /* faces: the +x, +y, +z neighbours of each active cell (so i < j) */
  m->face = (int*)malloc(sizeof(int) * 2 * (3 * n + 1));
  m->trans = (double*)malloc(sizeof(double) * (3 * n + 1));
  int nf = 0;
  for (int c = 0; c < n; ++c) {
    int b = m->cell_box[c];
    int i = b % nx, j = (b / nx) % ny, k = b / (nx * ny);
    double ci[3] = {(i + 0.5) * dx, (j + 0.5) * dy, m->depth[c]};
    double Ki[3] = {m->kh[c], m->kh[c], m->kv[c]};
    for (int dir = 0; dir < 3; ++dir) {
      int ii = i + (dir == 0), jj = j + (dir == 1), kk = k + (dir == 2);
      if (ii >= nx || jj >= ny || kk >= nz) continue;
      int nbx = ii + nx * (jj + ny * kk);
      int cn = m->box_cell[nbx];
      if (cn < 0) continue;
      double cj[3] = {(ii + 0.5) * dx, (jj + 0.5) * dy, m->depth[cn]};
      double Kj[3] = {m->kh[cn], m->kh[cn], m->kv[cn]};
      double cf[3] = {ci[0], ci[1], ci[2]};
      double nrm[3] = {0.0, 0.0, 0.0};
      double area;
      if (dir == 0) { cf[0] = (i + 1) * dx; area = dy * dz[k]; }
      else if (dir == 1) { cf[1] = (j + 1) * dy; area = dx * dz[k]; }
      else { cf[2] = layer_top(m, k + 1); area = dx * dy; }
      nrm[dir] = 1.0;
      double mnrm[3] = {-nrm[0], -nrm[1], -nrm[2]};
      double tij = half_trans(area, Ki, ci, cf, nrm);
      double tji = half_trans(area, Kj, cj, cf, mnrm);
      m->face[2 * nf] = c;
      m->face[2 * nf + 1] = cn;
      m->trans[nf] = (tij + tji > 0.0) ? tij * tji / (tij + tji) : 0.0;
      ++nf;
    }
  }
  m->nf = nf;

  /* block-CSR pattern: diagonal plus both cells of every face, columns sorted */
  m->row_ptr = (int*)calloc((size_t)n + 1, sizeof(int));
  for (int c = 0; c < n; ++c) m->row_ptr[c + 1] = 1;
  for (int f = 0; f < nf; ++f) {
    m->row_ptr[m->face[2 * f] + 1]++;
    m->row_ptr[m->face[2 * f + 1] + 1]++;
  }
  for (int c = 0; c < n; ++c) m->row_ptr[c + 1] += m->row_ptr[c];
  m->nnzb = m->row_ptr[n];
  m->col_idx = (int*)malloc(sizeof(int) * (m->nnzb + 1));
  int* fill = (int*)malloc(sizeof(int) * (n + 1));
  for (int c = 0; c < n; ++c) {
    fill[c] = m->row_ptr[c];
    m->col_idx[fill[c]++] = c;
  }
  for (int f = 0; f < nf; ++f) {
    int a = m->face[2 * f], b = m->face[2 * f + 1];
    m->col_idx[fill[a]++] = b;
    m->col_idx[fill[b]++] = a;
  }
  free(fill);
  for (int c = 0; c < n; ++c) {   /* insertion sort of each row */
    for (int q = m->row_ptr[c] + 1; q < m->row_ptr[c + 1]; ++q) {
      int v = m->col_idx[q], r = q - 1;
      while (r >= m->row_ptr[c] && m->col_idx[r] > v) {
        m->col_idx[r + 1] = m->col_idx[r];
        --r;
      }
      m->col_idx[r + 1] = v;
    }
  }

  /* wells and their connections; Peaceman well index (skin 0) */
  m->nw = n_wells;
  m->well_kind = (int*)malloc(sizeof(int) * (n_wells + 1));
  m->well_phase = (int*)malloc(sizeof(int) * (n_wells + 1));
  m->well_target = (double*)malloc(sizeof(double) * (n_wells + 1));
  m->well_beg = (int*)malloc(sizeof(int) * (n_wells + 1));
  int nc = 0;
  for (int w = 0; w < n_wells; ++w) nc += well_nconn[w];
  m->nc = nc;
  m->conn_cell = (int*)malloc(sizeof(int) * (nc + 1));
  m->conn_wi = (double*)malloc(sizeof(double) * (nc + 1));
  m->conn_well = (int*)malloc(sizeof(int) * (nc + 1));
  int q = 0;
  for (int w = 0; w < n_wells; ++w) {
    m->well_kind[w] = well_kind[w];
    m->well_phase[w] = well_phase[w];
    m->well_target[w] = well_target[w];
    m->well_beg[w] = q;
    for (int t = 0; t < well_nconn[w]; ++t, ++q) {
      int i = conn_ijk[3 * q], j = conn_ijk[3 * q + 1], k = conn_ijk[3 * q + 2];
      if (i < 0 || i >= nx || j < 0 || j >= ny || k < 0 || k >= nz ||
          m->box_cell[i + nx * (j + ny * k)] < 0) {
        ora_destroy(m);
        return NULL;
      }
      int c = m->box_cell[i + nx * (j + ny * k)];
      double ro = 0.14 * sqrt(dx * dx + dy * dy);
      m->conn_cell[q] = c;
      m->conn_wi[q] = 2.0 * M_PI * m->kh[c] * dz[k] / log(ro / well_rw[w]);
      m->conn_well[q] = w;
    }
  }
  m->well_beg[n_wells] = q;
  return m;
}

void ora_geometry(const ora_model* m, int* face_cells, double* trans, double* pv, double* depth,
                  int* cell_box) {
  if (face_cells) memcpy(face_cells, m->face, sizeof(int) * 2 * m->nf);
  if (trans) memcpy(trans, m->trans, sizeof(double) * m->nf);
  if (pv) memcpy(pv, m->pv, sizeof(double) * m->n);
  if (depth) memcpy(depth, m->depth, sizeof(double) * m->n);
  if (cell_box) memcpy(cell_box, m->cell_box, sizeof(int) * m->n);
}

void ora_pattern(const ora_model* m, int* row_ptr, int* col_idx) {
  memcpy(row_ptr, m->row_ptr, sizeof(int) * (m->n + 1));
  memcpy(col_idx, m->col_idx, sizeof(int) * m->nnzb);
}

void ora_conns(const ora_model* m, int* cell, double* wi, int* well) {
  if (cell) memcpy(cell, m->conn_cell, sizeof(int) * m->nc);
  if (wi) memcpy(wi, m->conn_wi, sizeof(double) * m->nc);
  if (well) memcpy(well, m->conn_well, sizeof(int) * m->nc);
}

/* ------------------------------------------- cell properties (sec. 2.1.4-6) */
typedef struct {
  dual p;
  dual s[3];    /* s_w, s_o, s_g */
  dual b[3];    /* shrinkage / expansion factors */
  dual rho[3];  /* reservoir densities */
  dual lam[3];  /* mobilities k_r / mu */
  dual r;       /* dissolved gas-oil ratio r_go (0 for dead oil) */
  dual rv;      /* vaporised oil-gas ratio r_og (0 without wet gas) */
  int wet;      /* wet gas: the oil component includes r_og b_g s_g */
} props;

/* Properties of one cell from its (p, s_w, x) and the meaning of x (sec.
 * 2.1.1, eq. primaryVariableMeaning): x = s_g (free gas present; for live
 * oil the oil is then saturated, r_go = r_s(p)) or x = r_go (no free gas,
 * s_g = 0) or, with wet gas, x = r_og (no oil, s_g = 1 - s_w).  Wet gas
 * (sec. 2.1.6): r_v(p) = rv_c p, saturated where gas and oil coexist; the
 * vaporised oil adds to the gas density, rho_g = b_g (rho_gS + r_og rho_oS)
 * (b_g and mu_g unchanged).  Live oil (sec. 2.1.6): r_s(p) = rs_c p; dissolved gas swells
 * the oil, b_o = exp(c_o (p - p_ref)) / (1 + bo_r r), thins it,
 * mu_o = mu_o / (1 + muo_r r), and adds its surface mass to the oil
 * density, rho_o = b_o (rho_oS + r rho_gS). */
static void cell_props(const ora_fluid* f, const double* y, int off, int mean, props* P) {
  P->p = dvar(y[0], off + 0);
  dual sw = dvar(y[1], off + 1);
  dual x = dvar(y[2], off + 2);
  const int wet = f->live && f->rv_c > 0.0;
  /* meaning 2 (wet gas): no oil, s_g = 1 - s_w, x = r_og */
  dual sg = (f->live && mean == 1) ? dconst(0.0)
            : (wet && mean == 2)    ? dsub(dconst(1.0), sw)
                                    : x;
  P->r = !f->live ? dconst(0.0) : (mean == 1 ? x : dscale(P->p, f->rs_c));
  P->rv = !wet ? dconst(0.0) : (mean == 2 ? x : dscale(P->p, f->rv_c));
  P->wet = wet;
  dual so = dsub(dsub(dconst(1.0), sw), sg);   /* s_w + s_o + s_g = 1 */
  P->s[0] = sw; P->s[1] = so; P->s[2] = sg;
  for (int a = 0; a < 3; ++a) {
    /* constant compressibility: (1/b) db/dp = c with b(p_ref) = 1 */
    P->b[a] = dexp(dscale(dsub(P->p, dconst(f->p_ref)), f->c[a]));
    P->rho[a] = dscale(P->b[a], f->rho_s[a]);   /* rho = b rho_S */
  }
  if (f->live) {
    P->b[1] = ddiv(P->b[1], dadd(dconst(1.0), dscale(P->r, f->bo_r)));
    P->rho[1] = dmul(P->b[1], dadd(dconst(f->rho_s[1]), dscale(P->r, f->rho_s[2])));
  }
  /* wet gas: the gas density holds the vaporised oil */
  if (wet) P->rho[2] = dmul(P->b[2], dadd(dconst(f->rho_s[2]), dscale(P->rv, f->rho_s[1])));
  /* Corey two-phase curves with residuals 0 except connate water */
  double den = 1.0 - f->swc;
  dual swn = dclamp01(ddiv(dsub(sw, dconst(f->swc)), dconst(den)));
  dual sgn = dclamp01(ddiv(sg, dconst(den)));
  dual son = dclamp01(ddiv(so, dconst(den)));
  dual krw = dpow(swn, f->n_corey);
  dual krg = dpow(sgn, f->n_corey);
  dual krow = dpow(son, f->n_corey);
  dual krog = dpow(son, f->n_corey);
  /* three-phase oil by the segregation model, eq. (gwseg) */
  dual ww = dmax0(dsub(sw, dconst(f->swc)));
  dual wg = dmax0(sg);
  dual wsum = dadd(ww, wg);
  dual kro;
  if (wsum.v > 1e-14)
    kro = ddiv(dadd(dmul(ww, krow), dmul(wg, krog)), wsum);
  else
    kro = krow;
  P->lam[0] = ddiv(krw, dconst(f->mu[0]));
  P->lam[1] = f->live
                  ? ddiv(kro, ddiv(dconst(f->mu[1]), dadd(dconst(1.0), dscale(P->r, f->muo_r))))
                  : ddiv(kro, dconst(f->mu[1]));
  P->lam[2] = ddiv(krg, dconst(f->mu[2]));
}

/* Surface volume per pore volume of component a: b_a s_a, plus the gas
 * dissolved in the oil, r b_o s_o, for the gas component and the oil
 * vaporised in the gas, r_v b_g s_g, for the oil component (wet gas). */
static dual component_acc(const props* P, int a) {
  dual A = dmul(P->b[a], P->s[a]);
  if (a == 2) A = dadd(A, dmul(P->r, dmul(P->b[1], P->s[1])));
  if (a == 1 && P->wet) A = dadd(A, dmul(P->rv, dmul(P->b[2], P->s[2])));
  return A;
}

int ora_set_meaning(ora_model* m, const unsigned char* mean) {
  for (int c = 0; c < m->n; ++c) {
    const unsigned char v = mean ? mean[c] : 0;
    if (v > 2 || (v >= 1 && !m->fl.live) || (v == 2 && !(m->fl.rv_c > 0.0))) return ORA_EINVAL;
  }
  for (int c = 0; c < m->n; ++c) m->mean[c] = mean ? mean[c] : 0;
  return ORA_OK;
}

void ora_get_meaning(const ora_model* m, unsigned char* mean) {
  memcpy(mean, m->mean, (size_t)m->n);
}

static void accumulation_of(const ora_model* m, const unsigned char* mean, const double* y,
                            double* acc) {
  for (int c = 0; c < m->n; ++c) {
    props P;
    cell_props(&m->fl, y + 3 * c, 0, mean[c], &P);
    for (int a = 0; a < 3; ++a) acc[3 * c + a] = component_acc(&P, a).v;
  }
}

void ora_accumulation(const ora_model* m, const double* y, double* acc) {
  accumulation_of(m, m->mean, y, acc);
}

static void std_conn_rate(const ora_model* m, int q, const double* y, const double* wx,
                          dual out[3]);

/* Well term of one connection as duals in slots 0-2 (sec. 2.2.1):
 * rate injector: fixed surface rate split over connections by WI share;
 * BHP producer: q_alpha = b_alpha lambda_alpha WI (p - p_bhp)^+, and for
 * live oil the gas dissolved in the produced oil, r b_o lambda_o WI (.)^+ . */
static void conn_rates(const ora_model* m, int q, const double* y, dual out[3]) {
  int w = m->conn_well[q];
  int c = m->conn_cell[q];
  for (int a = 0; a < 3; ++a) out[a] = dconst(0.0);
  if (m->well_kind[w] == ORA_WELL_RATE_INJ) {
    double wsum = 0.0;
    for (int t = m->well_beg[w]; t < m->well_beg[w + 1]; ++t) wsum += m->conn_wi[t];
    out[m->well_phase[w]] = dconst(-m->well_target[w] * m->conn_wi[q] / wsum);
  } else {
    props P;
    cell_props(&m->fl, y + 3 * c, 0, m->mean[c], &P);
    dual dp = dsub(P.p, dconst(m->well_target[w]));
    if (dp.v > 0.0) {
      for (int a = 0; a < 3; ++a)
        out[a] = dmul(dscale(dmul(P.b[a], P.lam[a]), m->conn_wi[q]), dp);
      if (m->fl.live)
        out[2] = dadd(out[2], dmul(dscale(dmul(P.r, dmul(P.b[1], P.lam[1])), m->conn_wi[q]), dp));
      if (m->fl.live && m->fl.rv_c > 0.0)
        out[1] = dadd(out[1], dmul(dscale(dmul(P.rv, dmul(P.b[2], P.lam[2])), m->conn_wi[q]), dp));
    }
  }
}

void ora_well_rates(const ora_model* m, const double* y, double* qout) {
  memset(qout, 0, sizeof(double) * 3 * m->n);
  for (int q = 0; q < m->nc; ++q) {
    dual r[3];
    if (m->std_wells)
      std_conn_rate(m, q, y, m->wx, r);
    else
      conn_rates(m, q, y, r);
    for (int a = 0; a < 3; ++a) qout[3 * m->conn_cell[q] + a] += r[a].v;
  }
}

/* --------------------------------------- residual + Jacobian (sec. 2.1.1) */
static void add_block(double* J, int blk, int a, const double* d, double sign) {
  for (int v = 0; v < 3; ++v) J[9 * blk + 3 * a + v] += sign * d[v];
}

int ora_assemble(const ora_model* m, const double* y, const double* acc0, double dt, double* R,
                 double* J) {
  const ora_fluid* f = &m->fl;
  memset(R, 0, sizeof(double) * 3 * m->n);
  if (J) memset(J, 0, sizeof(double) * 9 * m->nnzb);
  /* accumulation: PV/dt (A - A0); cells are independent (the OpenMP build
   * of the CPU baseline runs them in parallel, same arithmetic) */
#pragma omp parallel for schedule(static)
  for (int c = 0; c < m->n; ++c) {
    props P;
    cell_props(f, y + 3 * c, 0, m->mean[c], &P);
    int dblk = J ? find_block(m, c, c) : -1;
    for (int a = 0; a < 3; ++a) {
      dual A = component_acc(&P, a);
      dual r = dscale(dsub(A, dconst(acc0[3 * c + a])), m->pv[c] / dt);
      R[3 * c + a] += r.v;
      if (J) add_block(J, dblk, a, r.d, 1.0);
    }
  }
  /* connection fluxes, each face once; u_ij = -u_ji exactly.  The fluxes
   * of all faces are evaluated first (faces are independent: the OpenMP
   * build runs them in parallel) and then added in face order, so the sums
   * are the same with any number of threads. */
  dual* flux = (dual*)malloc(sizeof(dual) * 3 * (size_t)(m->nf > 0 ? m->nf : 1));
  if (!flux) return ORA_EINVAL;
#pragma omp parallel for schedule(static)
  for (int fc = 0; fc < m->nf; ++fc) {
    int i = m->face[2 * fc], j = m->face[2 * fc + 1];
    props Pi, Pj;
    cell_props(f, y + 3 * i, 0, m->mean[i], &Pi);
    cell_props(f, y + 3 * j, 3, m->mean[j], &Pj);
    double T = m->trans[fc];
    dual dzij = dconst(m->depth[i] - m->depth[j]);
    /* phase potentials and upwind cells; component a = phase a, plus for
     * gas the gas dissolved in the oil phase, carried with the oil */
    dual dphi[3];
    const props* U[3];
    for (int a = 0; a < 3; ++a) {
      dual rho_avg = dscale(dadd(Pi.rho[a], Pj.rho[a]), 0.5);
      dphi[a] = dsub(dsub(Pi.p, Pj.p), dmul(dscale(rho_avg, f->g), dzij));
      U[a] = (dphi[a].v >= 0.0) ? &Pi : &Pj;
    }
    for (int a = 0; a < 3; ++a) {
      dual F = dmul(dmul(U[a]->b[a], U[a]->lam[a]), dscale(dphi[a], T));
      if (a == 2 && f->live)
        F = dadd(F, dmul(dmul(U[1]->r, dmul(U[1]->b[1], U[1]->lam[1])), dscale(dphi[1], T)));
      /* wet gas: the oil vaporised in the gas moves with the gas phase */
      if (a == 1 && f->live && f->rv_c > 0.0)
        F = dadd(F, dmul(dmul(U[2]->rv, dmul(U[2]->b[2], U[2]->lam[2])), dscale(dphi[2], T)));
      flux[3 * fc + a] = F;
    }
  }
  for (int fc = 0; fc < m->nf; ++fc) {
    int i = m->face[2 * fc], j = m->face[2 * fc + 1];
    int bii = -1, bij = -1, bjj = -1, bji = -1;
    if (J) {
      bii = find_block(m, i, i); bij = find_block(m, i, j);
      bjj = find_block(m, j, j); bji = find_block(m, j, i);
    }
    for (int a = 0; a < 3; ++a) {
      dual F = flux[3 * fc + a];
      R[3 * i + a] += F.v;
      R[3 * j + a] -= F.v;
      if (J) {
        add_block(J, bii, a, F.d, 1.0);
        add_block(J, bij, a, F.d + 3, 1.0);
        add_block(J, bjj, a, F.d + 3, -1.0);
        add_block(J, bji, a, F.d, -1.0);
      }
    }
  }
  free(flux);
  /* wells: q_alpha (outflux positive) */
  for (int q = 0; q < m->nc; ++q) {
    int c = m->conn_cell[q];
    dual r[3];
    if (m->std_wells)
      std_conn_rate(m, q, y, m->wx, r);
    else
      conn_rates(m, q, y, r);
    int dblk = J ? find_block(m, c, c) : -1;
    for (int a = 0; a < 3; ++a) {
      R[3 * c + a] += r[a].v;
      if (J) add_block(J, dblk, a, r[a].d, 1.0);
    }
  }
  for (int k = 0; k < 3 * m->n; ++k)
    if (!isfinite(R[k])) return ORA_ENONFINITE;
  return ORA_OK;
}

/* CNV: max local residual in saturation units; MB: reservoir average. */
void ora_norms(const ora_model* m, const double* y, const double* R, double dt, double cnv[3],
               double mb[3]) {
  double sumR[3] = {0, 0, 0}, sumb[3] = {0, 0, 0}, pvsum = 0.0;
  for (int a = 0; a < 3; ++a) cnv[a] = 0.0;
  for (int c = 0; c < m->n; ++c) {
    props P;
    cell_props(&m->fl, y + 3 * c, 0, m->mean[c], &P);
    pvsum += m->pv[c];
    for (int a = 0; a < 3; ++a) {
      double v = dt * fabs(R[3 * c + a]) / (P.b[a].v * m->pv[c]);
      if (v > cnv[a]) cnv[a] = v;
      sumR[a] += R[3 * c + a];
      sumb[a] += P.b[a].v;
    }
  }
  for (int a = 0; a < 3; ++a) mb[a] = dt * fabs(sumR[a]) / ((sumb[a] / m->n) * pvsum);
}

/* ------------------------------------------------------- small dense algebra */
/* Gauss-Jordan inverse with partial pivoting; -1 on an exactly zero pivot. */
static int inv3(const double* A, double* X) {
  double a[3][6];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 6; ++c) a[r][c] = (c < 3) ? A[3 * r + c] : (c - 3 == r ? 1.0 : 0.0);
  for (int col = 0; col < 3; ++col) {
    int piv = col;
    for (int r = col + 1; r < 3; ++r)
      if (fabs(a[r][col]) > fabs(a[piv][col])) piv = r;
    if (a[piv][col] == 0.0 || !isfinite(a[piv][col])) return -1;
    if (piv != col)
      for (int c = 0; c < 6; ++c) {
        double t = a[col][c]; a[col][c] = a[piv][c]; a[piv][c] = t;
      }
    for (int r = 0; r < 3; ++r) {
      if (r == col) continue;
      double fct = a[r][col] / a[col][col];
      for (int c = 0; c < 6; ++c) a[r][c] -= fct * a[col][c];
    }
  }
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) X[3 * r + c] = a[r][3 + c] / a[r][r];
  return 0;
}

static void mat3_mul(const double* A, const double* B, double* C) {
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      double s = 0.0;
      for (int k = 0; k < 3; ++k) s += A[3 * r + k] * B[3 * k + c];
      C[3 * r + c] = s;
    }
}

int ora_dense_solve(int n, double* A, double* b) {
  for (int col = 0; col < n; ++col) {
    int piv = col;
    for (int r = col + 1; r < n; ++r)
      if (fabs(A[(size_t)r * n + col]) > fabs(A[(size_t)piv * n + col])) piv = r;
    if (A[(size_t)piv * n + col] == 0.0) return ORA_ESINGULAR;
    if (piv != col) {
      for (int c = 0; c < n; ++c) {
        double t = A[(size_t)col * n + c];
        A[(size_t)col * n + c] = A[(size_t)piv * n + c];
        A[(size_t)piv * n + c] = t;
      }
      double t = b[col]; b[col] = b[piv]; b[piv] = t;
    }
    for (int r = col + 1; r < n; ++r) {
      double fct = A[(size_t)r * n + col] / A[(size_t)col * n + col];
      if (fct == 0.0) continue;
      for (int c = col; c < n; ++c) A[(size_t)r * n + c] -= fct * A[(size_t)col * n + c];
      b[r] -= fct * b[col];
    }
  }
  for (int r = n - 1; r >= 0; --r) {
    double s = b[r];
    for (int c = r + 1; c < n; ++c) s -= A[(size_t)r * n + c] * b[c];
    b[r] = s / A[(size_t)r * n + r];
  }
  return ORA_OK;
}

/* -------------------------------------------------- block ILU(0) (sec. 2.3.1)
 * Generic IKJ elimination restricted to the sparsity pattern of A: for each
 * row i and each k < i in the row, L_ik = A_ik U_kk^{-1}; then every entry
 * (i, j) with j > k that is also in row k's pattern is updated by -L_ik U_kj. */
int ora_set_ilu_blocks(ora_model* m, int bx, int by, int bz) {
  if (!(bx == 0 && by == 0 && bz == 0) && (bx <= 0 || by <= 0 || bz <= 0)) return ORA_EINVAL;
  m->blk[0] = bx;
  m->blk[1] = by;
  m->blk[2] = bz;
  return ORA_OK;
}

/* Subdomain of a cell: the box (i / bx, j / by, k / bz) of the lattice. */
static int same_block(const ora_model* m, int a, int b) {
  if (m->blk[0] == 0) return 1;
  const int ba = m->cell_box[a], bb = m->cell_box[b];
  const int ia = ba % m->nx, ja = (ba / m->nx) % m->ny, ka = ba / (m->nx * m->ny);
  const int ib = bb % m->nx, jb = (bb / m->nx) % m->ny, kb = bb / (m->nx * m->ny);
  return ia / m->blk[0] == ib / m->blk[0] && ja / m->blk[1] == jb / m->blk[1] &&
         ka / m->blk[2] == kb / m->blk[2];
}

int ora_ilu0(const ora_model* m, const double* J, double* F) {
  memcpy(F, J, sizeof(double) * 9 * m->nnzb);
  /* block ILU0 of a partitioned grid (sec. 2.5, one block per process):
   * the factorisation sees the matrix without its couplings between
   * different subdomains, i.e. the ILU(0) of each subdomain's own matrix */
  for (int i = 0; i < m->n; ++i)
    for (int q = m->row_ptr[i]; q < m->row_ptr[i + 1]; ++q)
      if (!same_block(m, i, m->col_idx[q])) memset(F + 9 * q, 0, sizeof(double) * 9);
  double inv[9], tmp[9];
  for (int i = 0; i < m->n; ++i) {
    for (int q = m->row_ptr[i]; q < m->row_ptr[i + 1]; ++q) {
      int k = m->col_idx[q];
      if (k >= i) break;
      int dk = find_block(m, k, k);
      if (inv3(F + 9 * dk, inv)) return ORA_ESINGULAR;
      mat3_mul(F + 9 * q, inv, tmp);
      memcpy(F + 9 * q, tmp, sizeof(tmp));
      for (int r = q + 1; r < m->row_ptr[i + 1]; ++r) {
        int j = m->col_idx[r];
        int kj = find_block(m, k, j);
        if (kj < 0) continue;
        mat3_mul(F + 9 * q, F + 9 * kj, tmp);
        for (int e = 0; e < 9; ++e) F[9 * r + e] -= tmp[e];
      }
    }
  }
  for (int i = 0; i < m->n; ++i)
    if (inv3(F + 9 * find_block(m, i, i), inv)) return ORA_ESINGULAR;
  return ORA_OK;
}

/* x = (LU)^{-1} r: forward substitution with unit L, then backward with U. */
void ora_ilu0_apply(const ora_model* m, const double* F, const double* r, double* x) {
  double* w = (double*)malloc(sizeof(double) * 3 * m->n);
  for (int i = 0; i < m->n; ++i) {
    double t[3] = {r[3 * i], r[3 * i + 1], r[3 * i + 2]};
    for (int q = m->row_ptr[i]; q < m->row_ptr[i + 1]; ++q) {
      int k = m->col_idx[q];
      if (k >= i) break;
      for (int a = 0; a < 3; ++a)
        for (int v = 0; v < 3; ++v) t[a] -= F[9 * q + 3 * a + v] * w[3 * k + v];
    }
    for (int a = 0; a < 3; ++a) w[3 * i + a] = t[a];
  }
  for (int i = m->n - 1; i >= 0; --i) {
    double t[3] = {w[3 * i], w[3 * i + 1], w[3 * i + 2]};
    int dq = -1;
    for (int q = m->row_ptr[i]; q < m->row_ptr[i + 1]; ++q) {
      int j = m->col_idx[q];
      if (j == i) dq = q;
      if (j <= i) continue;
      for (int a = 0; a < 3; ++a)
        for (int v = 0; v < 3; ++v) t[a] -= F[9 * q + 3 * a + v] * x[3 * j + v];
    }
    double D[9];
    memcpy(D, F + 9 * dq, sizeof(D));
    ora_dense_solve(3, D, t);
    for (int a = 0; a < 3; ++a) x[3 * i + a] = t[a];
  }
  free(w);
}

void ora_spmv(const ora_model* m, const double* J, const double* x, double* y) {
#pragma omp parallel for schedule(static)
  for (int i = 0; i < m->n; ++i) {
    double t[3] = {0, 0, 0};
    for (int q = m->row_ptr[i]; q < m->row_ptr[i + 1]; ++q) {
      int j = m->col_idx[q];
      for (int a = 0; a < 3; ++a)
        for (int v = 0; v < 3; ++v) t[a] += J[9 * q + 3 * a + v] * x[3 * j + v];
    }
    for (int a = 0; a < 3; ++a) y[3 * i + a] = t[a];
  }
}



/* -------------------------------------------------- CPR-AMG (sec. 2.3.1)
 * Two-stage constrained-pressure-residual preconditioner.  Stage 1: the
 * quasi-IMPES weights w_i solve D_i^T w_i = e_p (D_i the diagonal block of
 * row i), the pressure system is (A_p)_ij = w_i^T A_ij e_p, and one V(1,1)
 * cycle of an aggregation AMG approximates A_p^{-1} (w^T r).  Stage 2: the
 * (block-)ILU(0) of the whole system on the remaining residual,
 * z = x1 + M_ILU^{-1} (r - A x1), x1 = e_p (pressure correction).
 * AMG: unsmoothed aggregation with geometric 2x2x2 aggregates of the
 * level's lattice (coarse unknown = a coarse box holding at least one
 * unknown, natural order), Galerkin coarse matrices A_c = P^T A P with the
 * piecewise-constant P, damped Jacobi (omega = 2/3) before and after the
 * coarse correction, dense LU on the coarsest level (<= 64 unknowns or
 * no further coarsening). */
#define ORA_AMG_MAX 12
#define ORA_AMG_COARSE 64
static const double kJacobiOmega = 2.0 / 3.0;

struct ora_cpr {
  int nl;
  int n[ORA_AMG_MAX];
  int dims[ORA_AMG_MAX][3];
  int* box[ORA_AMG_MAX];    /* lattice box of each unknown */
  int* rp[ORA_AMG_MAX];
  int* ci[ORA_AMG_MAX];
  double* a[ORA_AMG_MAX];
  int* agg[ORA_AMG_MAX];    /* unknown of level l -> unknown of level l + 1 */
  double* w;                /* [n][3] */
};

static void cpr_free(ora_cpr* c);
void ora_cpr_destroy(ora_cpr* c) {
  if (c) cpr_free(c);
}

static void cpr_free(ora_cpr* c) {
  for (int l = 0; l < ORA_AMG_MAX; ++l) {
    free(c->box[l]); free(c->rp[l]); free(c->ci[l]); free(c->a[l]); free(c->agg[l]);
  }
  free(c->w);
  free(c);
}

/* Coarse matrix of level l + 1: sum of the level-l entries between the
 * aggregates (sparse accumulation row by row, columns ascending). */
static void galerkin(ora_cpr* c, int l) {
  const int nf = c->n[l], nc = c->n[l + 1];
  int* cnt = (int*)calloc((size_t)nc + 1, sizeof(int));
  int* mark = (int*)malloc(sizeof(int) * nc);
  double* acc = (double*)calloc((size_t)nc, sizeof(double));
  for (int J = 0; J < nc; ++J) mark[J] = -1;
  /* children of each coarse unknown */
  int* chp = (int*)calloc((size_t)nc + 1, sizeof(int));
  int* ch = (int*)malloc(sizeof(int) * (nf + 1));
  for (int i = 0; i < nf; ++i) chp[c->agg[l][i] + 1]++;
  for (int I = 0; I < nc; ++I) chp[I + 1] += chp[I];
  int* fill = (int*)malloc(sizeof(int) * (nc + 1));
  memcpy(fill, chp, sizeof(int) * nc);
  for (int i = 0; i < nf; ++i) ch[fill[c->agg[l][i]]++] = i;
  /* pass 1: row lengths */
  for (int I = 0; I < nc; ++I) {
    for (int t = chp[I]; t < chp[I + 1]; ++t) {
      const int i = ch[t];
      for (int q = c->rp[l][i]; q < c->rp[l][i + 1]; ++q) {
        const int J = c->agg[l][c->ci[l][q]];
        if (mark[J] != I) { mark[J] = I; cnt[I + 1]++; }
      }
    }
  }
  for (int I = 0; I < nc; ++I) cnt[I + 1] += cnt[I];
  c->rp[l + 1] = cnt;
  c->ci[l + 1] = (int*)malloc(sizeof(int) * (cnt[nc] + 1));
  c->a[l + 1] = (double*)malloc(sizeof(double) * (cnt[nc] + 1));
  for (int J = 0; J < nc; ++J) mark[J] = -1;
  for (int I = 0; I < nc; ++I) {
    int len = 0;
    int* cols = c->ci[l + 1] + cnt[I];
    for (int t = chp[I]; t < chp[I + 1]; ++t) {
      const int i = ch[t];
      for (int q = c->rp[l][i]; q < c->rp[l][i + 1]; ++q) {
        const int J = c->agg[l][c->ci[l][q]];
        if (mark[J] != I) { mark[J] = I; cols[len++] = J; acc[J] = 0.0; }
        acc[J] += c->a[l][q];
      }
    }
    for (int u = 1; u < len; ++u) {   /* columns ascending */
      int v = cols[u], r = u - 1;
      while (r >= 0 && cols[r] > v) { cols[r + 1] = cols[r]; --r; }
      cols[r + 1] = v;
    }
    for (int u = 0; u < len; ++u) c->a[l + 1][cnt[I] + u] = acc[cols[u]];
  }
  free(mark); free(acc); free(chp); free(ch); free(fill);
}

/* Build the hierarchy for the Jacobian J (weights, A_p and coarse levels). */
int ora_cpr_setup(const ora_model* m, const double* J, ora_cpr** out) {
  ora_cpr* c = (ora_cpr*)calloc(1, sizeof(ora_cpr));
  const int n = m->n;
  c->w = (double*)malloc(sizeof(double) * 3 * (n + 1));
  /* quasi-IMPES weights: D_i^T w_i = e_p */
  for (int i = 0; i < n; ++i) {
    const double* Dg = J + 9 * find_block(m, i, i);
    double T[9] = {Dg[0], Dg[3], Dg[6], Dg[1], Dg[4], Dg[7], Dg[2], Dg[5], Dg[8]};
    double e[3] = {1.0, 0.0, 0.0};
    if (ora_dense_solve(3, T, e) != ORA_OK) { cpr_free(c); return ORA_ESINGULAR; }
    for (int a = 0; a < 3; ++a) c->w[3 * i + a] = e[a];
  }
  /* level 0: the pressure system on the block pattern */
  c->n[0] = n;
  c->dims[0][0] = m->nx; c->dims[0][1] = m->ny; c->dims[0][2] = m->nz;
  c->rp[0] = (int*)malloc(sizeof(int) * (n + 1));
  memcpy(c->rp[0], m->row_ptr, sizeof(int) * (n + 1));
  c->ci[0] = (int*)malloc(sizeof(int) * (m->nnzb + 1));
  memcpy(c->ci[0], m->col_idx, sizeof(int) * m->nnzb);
  c->a[0] = (double*)malloc(sizeof(double) * (m->nnzb + 1));
  c->box[0] = (int*)malloc(sizeof(int) * (n + 1));
  memcpy(c->box[0], m->cell_box, sizeof(int) * n);
  for (int i = 0; i < n; ++i)
    for (int q = m->row_ptr[i]; q < m->row_ptr[i + 1]; ++q) {
      double v = 0.0;
      for (int a = 0; a < 3; ++a) v += c->w[3 * i + a] * J[9 * q + 3 * a];
      c->a[0][q] = v;
    }
  /* coarse levels: 2x2x2 boxes of the level's lattice */
  int l = 0;
  while (c->n[l] > ORA_AMG_COARSE && l + 1 < ORA_AMG_MAX) {
    const int* d = c->dims[l];
    if (d[0] == 1 && d[1] == 1 && d[2] == 1) break;
    int cd[3] = {(d[0] + 1) / 2, (d[1] + 1) / 2, (d[2] + 1) / 2};
    const int nb = cd[0] * cd[1] * cd[2];
    int* idx = (int*)malloc(sizeof(int) * nb);
    for (int b = 0; b < nb; ++b) idx[b] = -1;
    int* parent = (int*)malloc(sizeof(int) * (c->n[l] + 1));
    for (int i = 0; i < c->n[l]; ++i) {
      const int b = c->box[l][i];
      const int x = b % d[0], y = (b / d[0]) % d[1], z = b / (d[0] * d[1]);
      parent[i] = x / 2 + cd[0] * (y / 2 + cd[1] * (z / 2));
      idx[parent[i]] = 0;
    }
    int nc = 0;
    for (int b = 0; b < nb; ++b)
      if (idx[b] >= 0) idx[b] = nc++;
    c->agg[l] = (int*)malloc(sizeof(int) * (c->n[l] + 1));
    for (int i = 0; i < c->n[l]; ++i) c->agg[l][i] = idx[parent[i]];
    c->box[l + 1] = (int*)malloc(sizeof(int) * (nc + 1));
    for (int b = 0; b < nb; ++b)
      if (idx[b] >= 0) c->box[l + 1][idx[b]] = b;
    c->n[l + 1] = nc;
    memcpy(c->dims[l + 1], cd, sizeof(cd));
    free(idx); free(parent);
    galerkin(c, l);
    ++l;
  }
  c->nl = l + 1;
  *out = c;
  return ORA_OK;
}

static void csr_mv(const ora_cpr* c, int l, const double* x, double* y) {
  for (int i = 0; i < c->n[l]; ++i) {
    double s = 0.0;
    for (int q = c->rp[l][i]; q < c->rp[l][i + 1]; ++q) s += c->a[l][q] * x[c->ci[l][q]];
    y[i] = s;
  }
}

static double csr_diag(const ora_cpr* c, int l, int i) {
  for (int q = c->rp[l][i]; q < c->rp[l][i + 1]; ++q)
    if (c->ci[l][q] == i) return c->a[l][q];
  return 0.0;
}

/* x = V(1,1)-cycle approximation of A_l^{-1} b (x starts at zero). */
static void vcycle(const ora_cpr* c, int l, const double* b, double* x) {
  const int n = c->n[l];
  if (l == c->nl - 1) {   /* coarsest: dense LU */
    double* A = (double*)calloc((size_t)n * n + 1, sizeof(double));
    for (int i = 0; i < n; ++i) {
      for (int q = c->rp[l][i]; q < c->rp[l][i + 1]; ++q) A[(size_t)i * n + c->ci[l][q]] = c->a[l][q];
      x[i] = b[i];
    }
    ora_dense_solve(n, A, x);
    free(A);
    return;
  }
  const int nc = c->n[l + 1];
  double* r = (double*)malloc(sizeof(double) * (n + 1));
  double* bc = (double*)calloc((size_t)nc + 1, sizeof(double));
  double* xc = (double*)calloc((size_t)nc + 1, sizeof(double));
  for (int i = 0; i < n; ++i) x[i] = kJacobiOmega * b[i] / csr_diag(c, l, i);   /* pre-smooth */
  csr_mv(c, l, x, r);
  for (int i = 0; i < n; ++i) bc[c->agg[l][i]] += b[i] - r[i];   /* restrict the residual */
  vcycle(c, l + 1, bc, xc);
  for (int i = 0; i < n; ++i) x[i] += xc[c->agg[l][i]];   /* prolong */
  csr_mv(c, l, x, r);
  for (int i = 0; i < n; ++i) x[i] += kJacobiOmega * (b[i] - r[i]) / csr_diag(c, l, i);   /* post-smooth */
  free(r); free(bc); free(xc);
}

int ora_cpr_levels(const ora_cpr* c) { return c->nl; }

void ora_cpr_level_size(const ora_cpr* c, int l, int* n, int* nnz) {
  *n = c->n[l];
  *nnz = c->rp[l][c->n[l]];
}

void ora_cpr_level(const ora_cpr* c, int l, int* rp, int* ci, double* a, int* agg) {
  memcpy(rp, c->rp[l], sizeof(int) * (c->n[l] + 1));
  memcpy(ci, c->ci[l], sizeof(int) * c->rp[l][c->n[l]]);
  memcpy(a, c->a[l], sizeof(double) * c->rp[l][c->n[l]]);
  if (agg && l + 1 < c->nl) memcpy(agg, c->agg[l], sizeof(int) * c->n[l]);
}

void ora_cpr_weights(const ora_cpr* c, double* w) { memcpy(w, c->w, sizeof(double) * 3 * c->n[0]); }

void ora_cpr_vcycle(const ora_cpr* c, const double* b, double* x) { vcycle(c, 0, b, x); }

/* z = CPR(r): pressure stage then (block-)ILU(0) stage on the rest. */
static void cpr_apply(const ora_model* m, const ora_cpr* c, const double* J, const double* F,
                      const double* r, double* z) {
  const int n = m->n;
  double* bp = (double*)malloc(sizeof(double) * (n + 1));
  double* xp = (double*)malloc(sizeof(double) * (n + 1));
  double* x1 = (double*)calloc(3 * (size_t)n + 1, sizeof(double));
  double* r2 = (double*)malloc(sizeof(double) * (3 * n + 1));
  double* z2 = (double*)malloc(sizeof(double) * (3 * n + 1));
  for (int i = 0; i < n; ++i)
    bp[i] = c->w[3 * i] * r[3 * i] + c->w[3 * i + 1] * r[3 * i + 1] + c->w[3 * i + 2] * r[3 * i + 2];
  vcycle(c, 0, bp, xp);
  for (int i = 0; i < n; ++i) x1[3 * i] = xp[i];
  ora_spmv(m, J, x1, r2);
  for (int k = 0; k < 3 * n; ++k) r2[k] = r[k] - r2[k];
  ora_ilu0_apply(m, F, r2, z2);
  for (int k = 0; k < 3 * n; ++k) z[k] = x1[k] + z2[k];
  free(bp); free(xp); free(x1); free(r2); free(z2);
}

/* ---------------------------------------------- standard wells (sec. 2.2.1)
 * Each well has the unknowns x_w = (Q_t, F_w, F_g, p_bhp) (eq.
 * weighted_total_rate): the weighted total surface rate (production
 * positive), the weighted water and gas fractions of the wellbore fluid and
 * the bottom-hole pressure, with weights g = (1, 1, 0.01); the component
 * surface rates are Q_a = F_a Q_t / g_a with F_o = 1 - F_w - F_g.  The
 * wellbore fluid holds mix_a = (F_a / g_a) / sum_b F_b / (g_b b_b(p_bhp))
 * surface volume of component a per reservoir volume (b at p_bhp, no gas
 * dissolved in the wellbore). */
static const double kWellG[3] = {1.0, 1.0, 0.01};

typedef struct {
  dual Qt, F[3], pb;
  dual mix[3];
} wellvars;

static void well_vars(const ora_fluid* f, const double* xw, wellvars* W) {
  W->Qt = dvar(xw[0], 3);
  W->F[0] = dvar(xw[1], 4);
  W->F[2] = dvar(xw[2], 5);
  W->F[1] = dsub(dsub(dconst(1.0), W->F[0]), W->F[2]);
  W->pb = dvar(xw[3], 6);
  dual S = dconst(0.0);
  for (int a = 0; a < 3; ++a) {
    dual b = dexp(dscale(dsub(W->pb, dconst(f->p_ref)), f->c[a]));
    S = dadd(S, ddiv(dscale(W->F[a], 1.0 / kWellG[a]), b));
  }
  for (int a = 0; a < 3; ++a) W->mix[a] = ddiv(dscale(W->F[a], 1.0 / kWellG[a]), S);
}

/* Surface rate of each component through connection q (production
 * positive; eq. wellinflow with h_w,j = 0): a producing connection
 * (p_j > p_bhp) carries the cell's phases, q_a = WI b_a lambda_a (p_j -
 * p_bhp) (live oil: plus r b_o lambda_o for gas); an injecting one carries
 * the wellbore fluid at the cell's total mobility, q_a = WI lambda_t (p_j -
 * p_bhp) mix_a.  Slots 0-2: the cell's variables; 3-6: the well's. */
static void std_conn_rate(const ora_model* m, int q, const double* y, const double* wx,
                          dual out[3]) {
  const int c = m->conn_cell[q], w = m->conn_well[q];
  props P;
  cell_props(&m->fl, y + 3 * c, 0, m->mean[c], &P);
  wellvars W;
  well_vars(&m->fl, wx + 4 * w, &W);
  dual dp = dsub(P.p, W.pb);
  const double wi = m->conn_wi[q];
  if (dp.v > 0.0) {
    for (int a = 0; a < 3; ++a) out[a] = dmul(dscale(dmul(P.b[a], P.lam[a]), wi), dp);
    if (m->fl.live)
      out[2] = dadd(out[2], dmul(dscale(dmul(P.r, dmul(P.b[1], P.lam[1])), wi), dp));
    if (m->fl.live && m->fl.rv_c > 0.0)
      out[1] = dadd(out[1], dmul(dscale(dmul(P.rv, dmul(P.b[2], P.lam[2])), wi), dp));
  } else {
    dual lt = dadd(dadd(P.lam[0], P.lam[1]), P.lam[2]);
    for (int a = 0; a < 3; ++a) out[a] = dmul(dmul(dscale(lt, wi), dp), W.mix[a]);
  }
}

int ora_set_standard_wells(ora_model* m, const double* well_vol, const double* x0,
                           const double* limits) {
  if (m->nw == 0) return ORA_EINVAL;
  for (int w = 0; w < m->nw; ++w)
    if (!(well_vol[w] >= 0.0) || (limits && !(limits[w] >= 0.0))) return ORA_EINVAL;
  free(m->well_vol); free(m->wx); free(m->wA0); free(m->well_limit); free(m->wctrl);
  m->well_vol = (double*)malloc(sizeof(double) * m->nw);
  m->wx = (double*)malloc(sizeof(double) * 4 * m->nw);
  m->wA0 = (double*)calloc(3 * (size_t)m->nw, sizeof(double));
  m->well_limit = (double*)calloc((size_t)m->nw, sizeof(double));
  m->wctrl = (int*)calloc((size_t)m->nw, sizeof(int));
  memcpy(m->well_vol, well_vol, sizeof(double) * m->nw);
  memcpy(m->wx, x0, sizeof(double) * 4 * m->nw);
  if (limits) memcpy(m->well_limit, limits, sizeof(double) * m->nw);
  m->std_wells = 1;
  return ORA_OK;
}

void ora_get_well_ctrl(const ora_model* m, int* ctrl) {
  if (m->std_wells) memcpy(ctrl, m->wctrl, sizeof(int) * m->nw);
}

void ora_set_well_ctrl(ora_model* m, const int* ctrl) {
  if (m->std_wells)
    for (int w = 0; w < m->nw; ++w) m->wctrl[w] = ctrl[w] != 0 && m->well_limit[w] > 0.0;
}

/* Control switching (sec. 2.2.1 names BHP and rate controls; the rule is a
 * reading): a well with a limit runs on its own control (BHP for a
 * producer, the surface rate of one component for an injector) until the
 * limit is exceeded (a producer's oil surface rate above it, an injector's
 * BHP above it), then on the limit (Q_o = limit, p_bhp = limit) until its
 * own control binds again (the producer's BHP below its target, the
 * injector's rate above its target).  Checked on the well state after
 * every Newton update. */
static double well_frac(const double* x, int a) {
  return a == 0 ? x[1] : a == 2 ? x[2] : 1.0 - x[1] - x[2];
}

static void well_switch(const ora_model* m) {
  for (int w = 0; w < m->nw; ++w) {
    if (!(m->well_limit[w] > 0.0)) continue;
    const double* x = m->wx + 4 * w;
    int* c = m->wctrl + w;
    if (m->well_kind[w] == ORA_WELL_BHP_PROD) {
      const double qo = well_frac(x, 1) * x[0] / kWellG[1];
      if (*c == 0 && qo > m->well_limit[w]) *c = 1;
      else if (*c == 1 && x[3] < m->well_target[w]) *c = 0;
    } else {
      const int ph = m->well_phase[w];
      const double inj = -well_frac(x, ph) * x[0] / kWellG[ph];
      if (*c == 0 && x[3] > m->well_limit[w]) *c = 1;
      else if (*c == 1 && inj > m->well_target[w]) *c = 0;
    }
  }
}

/* The target of the active control. */
static double active_target(const ora_model* m, int w) {
  return m->wctrl[w] ? m->well_limit[w] : m->well_target[w];
}

void ora_get_well_state(const ora_model* m, double* x) {
  if (m->std_wells) memcpy(x, m->wx, sizeof(double) * 4 * m->nw);
}

void ora_set_well_state(ora_model* m, const double* x) {
  if (m->std_wells) memcpy(m->wx, x, sizeof(double) * 4 * m->nw);
}

/* Wellbore storage A_a,w = V_w mix_a of a well state: A [nw][3]. */
static void well_storage(const ora_model* m, const double* wx, double* A) {
  for (int w = 0; w < m->nw; ++w) {
    wellvars W;
    well_vars(&m->fl, wx + 4 * w, &W);
    for (int a = 0; a < 3; ++a) A[3 * w + a] = m->well_vol[w] * W.mix[a].v;
  }
}

void ora_well_storage_start(ora_model* m) {
  if (m->std_wells) well_storage(m, m->wx, m->wA0);
}

/* Well equations at (y, model well state) and their coupling blocks:
 * component conservation with wellbore storage (eq. conseq-swell),
 * R_a,w = V_w (mix_a - mix_a^0)/dt + Q_a - sum_j q_a,j, and the control
 * (eq. well-control-bhp / -rate): p_bhp - target for a BHP producer,
 * Q_a + target for an injector of component a at the surface rate target.
 * Rw [nw][4]; B [nc][4][3] = dRw/dx_cell; C [nc][3][4] = d(cell residual
 * (+q))/dx_w; D [nw][4][4] = dRw/dx_w. */
int ora_well_system(const ora_model* m, const double* y, double dt, double* Rw, double* B,
                    double* C, double* D) {
  if (!m->std_wells) return ORA_EINVAL;
  memset(B, 0, sizeof(double) * 12 * m->nc);
  memset(C, 0, sizeof(double) * 12 * m->nc);
  for (int w = 0; w < m->nw; ++w) {
    wellvars W;
    well_vars(&m->fl, m->wx + 4 * w, &W);
    dual R[4];
    for (int a = 0; a < 3; ++a) {
      dual st = dscale(dsub(W.mix[a], dconst(m->wA0[3 * w + a] /
                                             (m->well_vol[w] > 0.0 ? m->well_vol[w] : 1.0))),
                       m->well_vol[w] / dt);
      R[a] = dadd(st, dscale(dmul(W.F[a], W.Qt), 1.0 / kWellG[a]));
    }
    for (int q = m->well_beg[w]; q < m->well_beg[w + 1]; ++q) {
      dual qr[3];
      std_conn_rate(m, q, y, m->wx, qr);
      for (int a = 0; a < 3; ++a) {
        R[a] = dsub(R[a], qr[a]);
        for (int v = 0; v < 3; ++v) B[12 * q + 3 * a + v] = -qr[a].d[v];
        for (int k = 0; k < 4; ++k) C[12 * q + 4 * a + k] = qr[a].d[3 + k];
      }
    }
    if (m->well_kind[w] == ORA_WELL_BHP_PROD && m->wctrl[w] == 0) {
      R[3] = dsub(W.pb, dconst(m->well_target[w]));
    } else if (m->well_kind[w] == ORA_WELL_BHP_PROD) {   /* oil surface rate at the limit */
      R[3] = dsub(dscale(dmul(W.F[1], W.Qt), 1.0 / kWellG[1]), dconst(m->well_limit[w]));
    } else if (m->wctrl[w] == 0) {
      const int ph = m->well_phase[w];
      R[3] = dadd(dscale(dmul(W.F[ph], W.Qt), 1.0 / kWellG[ph]), dconst(m->well_target[w]));
    } else {   /* injector at its BHP limit */
      R[3] = dsub(W.pb, dconst(m->well_limit[w]));
    }
    for (int e = 0; e < 4; ++e) {
      Rw[4 * w + e] = R[e].v;
      for (int k = 0; k < 4; ++k) D[16 * w + 4 * e + k] = R[e].d[3 + k];
    }
  }
  return ORA_OK;
}

/* The Krylov operator: the reservoir matrix, with standard wells their
 * Schur complement (eq. wellequation), y = A x - sum_w C_w D_w^{-1} B_w x. */
typedef struct {
  const ora_model* m;
  const double* J;
  const double* B;      /* NULL without standard wells */
  const double* C;
  const double* Dinv;   /* [nw][4][4] */
  const ora_cpr* cpr;   /* NULL: the (block-)ILU(0) preconditioner alone */
} oper;

/* The preconditioner: (block-)ILU(0), or CPR with it as second stage. */
static void prec_apply(const oper* op, const double* F, const double* r, double* z) {
  if (op->cpr)
    cpr_apply(op->m, op->cpr, op->J, F, r, z);
  else
    ora_ilu0_apply(op->m, F, r, z);
}

static void op_apply(const oper* op, const double* x, double* y) {
  const ora_model* m = op->m;
  ora_spmv(m, op->J, x, y);
  if (!op->B) return;
  for (int w = 0; w < m->nw; ++w) {
    double t[4] = {0, 0, 0, 0}, u[4] = {0, 0, 0, 0};
    for (int q = m->well_beg[w]; q < m->well_beg[w + 1]; ++q) {
      const int c = m->conn_cell[q];
      for (int e = 0; e < 4; ++e)
        for (int v = 0; v < 3; ++v) t[e] += op->B[12 * q + 3 * e + v] * x[3 * c + v];
    }
    for (int e = 0; e < 4; ++e)
      for (int k = 0; k < 4; ++k) u[e] += op->Dinv[16 * w + 4 * e + k] * t[k];
    for (int q = m->well_beg[w]; q < m->well_beg[w + 1]; ++q) {
      const int c = m->conn_cell[q];
      for (int a = 0; a < 3; ++a)
        for (int k = 0; k < 4; ++k) y[3 * c + a] -= op->C[12 * q + 4 * a + k] * u[k];
    }
  }
}

static int inv4(const double* A, double* X) {
  for (int k = 0; k < 4; ++k) {
    double M[16], e[4] = {0, 0, 0, 0};
    memcpy(M, A, sizeof(M));
    e[k] = 1.0;
    if (ora_dense_solve(4, M, e) != ORA_OK) return ORA_ESINGULAR;
    for (int r = 0; r < 4; ++r) X[4 * r + k] = e[r];
  }
  return ORA_OK;
}

static int bicgstab_op(const oper* op, const double* F, const double* b, double* x, double rtol,
                       int maxit, double* its_out, double* relres_out);

void ora_cpr_apply(const ora_model* m, const ora_cpr* c, const double* J, const double* F,
                   const double* r, double* z) {
  cpr_apply(m, c, J, F, r, z);
}

int ora_bicgstab_cpr(const ora_model* m, const double* J, const double* F, const ora_cpr* c,
                     const double* b, double* x, double rtol, int maxit, double* its,
                     double* relres) {
  oper op = {m, J, NULL, NULL, NULL, c};
  return bicgstab_op(&op, F, b, x, rtol, maxit, its, relres);
}

static int gmres_op(const oper* op, const double* F, const double* b, double* x, double rtol,
                    int maxit, int restart, double* its_out, double* relres_out);

static int schur_solve(const ora_model* m, const double* J, const double* F, const double* B,
                       const double* C, const double* D, const double* Rr, const double* Rw,
                       double* xr, double* xw, double rtol, int maxit, int krylov, int restart,
                       double* its, double* relres, const ora_cpr* cpr);

int ora_schur_solve(const ora_model* m, const double* J, const double* F, const double* B,
                    const double* C, const double* D, const double* Rr, const double* Rw,
                    double* xr, double* xw, double rtol, int maxit, int krylov, int restart,
                    double* its, double* relres) {
  return schur_solve(m, J, F, B, C, D, Rr, Rw, xr, xw, rtol, maxit, krylov, restart, its, relres,
                     NULL);
}

static int schur_solve(const ora_model* m, const double* J, const double* F, const double* B,
                       const double* C, const double* D, const double* Rr, const double* Rw,
                       double* xr, double* xw, double rtol, int maxit, int krylov, int restart,
                       double* its, double* relres, const ora_cpr* cpr) {
  const int N = 3 * m->n;
  double* Dinv = (double*)malloc(sizeof(double) * 16 * (m->nw + 1));
  double* b = (double*)malloc(sizeof(double) * N);
  int st = ORA_OK;
  for (int w = 0; w < m->nw && st == ORA_OK; ++w) st = inv4(D + 16 * w, Dinv + 16 * w);
  if (st != ORA_OK) goto out;
  /* b = R_r - sum_w C_w D_w^{-1} R_w */
  memcpy(b, Rr, sizeof(double) * N);
  for (int w = 0; w < m->nw; ++w) {
    double u[4] = {0, 0, 0, 0};
    for (int e = 0; e < 4; ++e)
      for (int k = 0; k < 4; ++k) u[e] += Dinv[16 * w + 4 * e + k] * Rw[4 * w + k];
    for (int q = m->well_beg[w]; q < m->well_beg[w + 1]; ++q) {
      const int c = m->conn_cell[q];
      for (int a = 0; a < 3; ++a)
        for (int k = 0; k < 4; ++k) b[3 * c + a] -= C[12 * q + 4 * a + k] * u[k];
    }
  }
  {
    oper op = {m, J, B, C, Dinv, cpr};
    st = krylov == 1 ? gmres_op(&op, F, b, xr, rtol, maxit, restart, its, relres)
                     : bicgstab_op(&op, F, b, xr, rtol, maxit, its, relres);
  }
  /* x_w = D_w^{-1} (R_w - B_w x_r) */
  for (int w = 0; w < m->nw; ++w) {
    double t[4];
    for (int e = 0; e < 4; ++e) t[e] = Rw[4 * w + e];
    for (int q = m->well_beg[w]; q < m->well_beg[w + 1]; ++q) {
      const int c = m->conn_cell[q];
      for (int e = 0; e < 4; ++e)
        for (int v = 0; v < 3; ++v) t[e] -= B[12 * q + 3 * e + v] * xr[3 * c + v];
    }
    for (int e = 0; e < 4; ++e) {
      xw[4 * w + e] = 0.0;
      for (int k = 0; k < 4; ++k) xw[4 * w + e] += Dinv[16 * w + 4 * e + k] * t[k];
    }
  }
out:
  free(Dinv);
  free(b);
  return st;
}

/* ----------------------------------------------- BiCGStab (sec. 2.3.1)
 * van der Vorst's stabilised BiCG with right preconditioning M = LU,
 * x0 = 0, stopping on the 2-norm of the residual relative to ||b||. */
static double dot(int n, const double* a, const double* b) {
  double s = 0.0;
  for (int k = 0; k < n; ++k) s += a[k] * b[k];
  return s;
}

int ora_bicgstab(const ora_model* m, const double* J, const double* F, const double* b, double* x,
                 double rtol, int maxit, double* its_out, double* relres_out) {
  oper op = {m, J, NULL, NULL, NULL, NULL};
  return bicgstab_op(&op, F, b, x, rtol, maxit, its_out, relres_out);
}

static int bicgstab_op(const oper* op, const double* F, const double* b, double* x, double rtol,
                       int maxit, double* its_out, double* relres_out) {
  const ora_model* m = op->m;
  const int N = 3 * m->n;
  double* r = (double*)malloc(sizeof(double) * N);
  double* rh = (double*)malloc(sizeof(double) * N);
  double* p = (double*)calloc(N, sizeof(double));
  double* v = (double*)calloc(N, sizeof(double));
  double* ph = (double*)malloc(sizeof(double) * N);
  double* s = (double*)malloc(sizeof(double) * N);
  double* sh = (double*)malloc(sizeof(double) * N);
  double* t = (double*)malloc(sizeof(double) * N);
  for (int k = 0; k < N; ++k) { x[k] = 0.0; r[k] = b[k]; rh[k] = b[k]; }
  double bnorm = sqrt(dot(N, b, b));
  double rho0 = 1.0, alpha = 1.0, omega = 1.0;
  int status = ORA_ENOTCONV;
  double its = 0.0, relres = 1.0;
  if (bnorm == 0.0) { status = ORA_OK; relres = 0.0; goto done; }
  for (int it = 1; it <= maxit; ++it) {
    double rho = dot(N, rh, r);
    if (fabs(rho) < 1e-300) { status = ORA_EBREAKDOWN; break; }
    double beta = (rho / rho0) * (alpha / omega);
    for (int k = 0; k < N; ++k) p[k] = r[k] + beta * (p[k] - omega * v[k]);
    prec_apply(op, F, p, ph);
    op_apply(op, ph, v);
    double rv = dot(N, rh, v);
    if (rv == 0.0) { status = ORA_EBREAKDOWN; break; }
    alpha = rho / rv;
    for (int k = 0; k < N; ++k) s[k] = r[k] - alpha * v[k];
    double snorm = sqrt(dot(N, s, s));
    if (snorm <= rtol * bnorm) {
      for (int k = 0; k < N; ++k) x[k] += alpha * ph[k];
      its = it - 0.5; relres = snorm / bnorm; status = ORA_OK;
      break;
    }
    prec_apply(op, F, s, sh);
    op_apply(op, sh, t);
    double tt = dot(N, t, t);
    if (tt == 0.0) { status = ORA_EBREAKDOWN; break; }
    omega = dot(N, t, s) / tt;
    for (int k = 0; k < N; ++k) {
      x[k] += alpha * ph[k] + omega * sh[k];
      r[k] = s[k] - omega * t[k];
    }
    double rnorm = sqrt(dot(N, r, r));
    its = it; relres = rnorm / bnorm;
    if (rnorm <= rtol * bnorm) { status = ORA_OK; break; }
    if (omega == 0.0) { status = ORA_EBREAKDOWN; break; }
    rho0 = rho;
  }
done:
  if (its_out) *its_out = its;
  if (relres_out) *relres_out = relres;
  free(r); free(rh); free(p); free(v); free(ph); free(s); free(sh); free(t);
  return status;
}

/* ------------------------------------ restarted GMRes (sec. 2.3.1, GMRes(m))
 * Saad and Schultz's minimal-residual method, right preconditioned:
 * x = M^{-1} u with u from the Krylov space of A M^{-1} built from the
 * residual r0 = b - A x0, each space of at most m vectors (restart length),
 * orthonormalised by modified Gram-Schmidt; the least-squares problem is
 * reduced by Givens rotations, whose last entry |g_{j+1}| is the residual
 * norm of the current iterate.  x0 = 0, stop on |g_{j+1}| <= rtol ||b||,
 * at the iteration cap, or on an exact (happy) breakdown h_{j+1,j} = 0. */
int ora_gmres(const ora_model* m, const double* J, const double* F, const double* b, double* x,
              double rtol, int maxit, int restart, double* its_out, double* relres_out) {
  oper op = {m, J, NULL, NULL, NULL, NULL};
  return gmres_op(&op, F, b, x, rtol, maxit, restart, its_out, relres_out);
}

static int gmres_op(const oper* op, const double* F, const double* b, double* x, double rtol,
                    int maxit, int restart, double* its_out, double* relres_out) {
  const ora_model* m = op->m;
  const int N = 3 * m->n;
  if (restart < 1) return ORA_EINVAL;
  double* V = (double*)malloc(sizeof(double) * (size_t)N * (restart + 1));
  double* H = (double*)calloc((size_t)(restart + 1) * restart, sizeof(double));
  double* cs = (double*)malloc(sizeof(double) * restart);
  double* sn = (double*)malloc(sizeof(double) * restart);
  double* g = (double*)malloc(sizeof(double) * (restart + 1));
  double* y = (double*)malloc(sizeof(double) * restart);
  double* w = (double*)malloc(sizeof(double) * N);
  double* z = (double*)malloc(sizeof(double) * N);
  for (int k = 0; k < N; ++k) x[k] = 0.0;
  const double bnorm = sqrt(dot(N, b, b)), tol = rtol * bnorm;
  int status = ORA_ENOTCONV, its = 0;
  double relres = bnorm > 0.0 ? 1.0 : 0.0;
  if (bnorm == 0.0) { status = ORA_OK; goto done; }
#define Hm(i, j) H[(size_t)(i) * restart + (j)]
  while (its < maxit) {
    /* residual of the current iterate starts the space */
    op_apply(op, x, w);
    for (int k = 0; k < N; ++k) V[k] = b[k] - w[k];
    const double beta = sqrt(dot(N, V, V));
    relres = beta / bnorm;
    if (beta <= tol) { status = ORA_OK; break; }
    for (int k = 0; k < N; ++k) V[k] /= beta;
    for (int i = 0; i <= restart; ++i) g[i] = 0.0;
    g[0] = beta;
    int k_used = 0, done_cycle = 0;
    for (int j = 0; j < restart && its < maxit; ++j) {
      double* vj = V + (size_t)j * N;
      prec_apply(op, F, vj, z);
      op_apply(op, z, w);
      for (int i = 0; i <= j; ++i) {
        const double* vi = V + (size_t)i * N;
        const double h = dot(N, w, vi);
        Hm(i, j) = h;
        for (int k = 0; k < N; ++k) w[k] -= h * vi[k];
      }
      const double hn = sqrt(dot(N, w, w));
      Hm(j + 1, j) = hn;
      /* earlier rotations on the new column, then the one that zeroes it */
      for (int i = 0; i < j; ++i) {
        const double a = Hm(i, j), c = Hm(i + 1, j);
        Hm(i, j) = cs[i] * a + sn[i] * c;
        Hm(i + 1, j) = -sn[i] * a + cs[i] * c;
      }
      const double d = hypot(Hm(j, j), Hm(j + 1, j));
      cs[j] = d > 0.0 ? Hm(j, j) / d : 1.0;
      sn[j] = d > 0.0 ? Hm(j + 1, j) / d : 0.0;
      Hm(j, j) = d;
      Hm(j + 1, j) = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      ++its;
      k_used = j + 1;
      relres = fabs(g[j + 1]) / bnorm;
      if (fabs(g[j + 1]) <= tol || hn == 0.0) { done_cycle = 1; break; }
      double* vn = V + (size_t)(j + 1) * N;
      for (int k = 0; k < N; ++k) vn[k] = w[k] / hn;
    }
    /* y = R^{-1} g over the columns used, x += M^{-1} V y */
    for (int i = k_used - 1; i >= 0; --i) {
      double t = g[i];
      for (int c = i + 1; c < k_used; ++c) t -= Hm(i, c) * y[c];
      if (Hm(i, i) == 0.0) { status = ORA_EBREAKDOWN; goto done; }
      y[i] = t / Hm(i, i);
    }
    for (int k = 0; k < N; ++k) w[k] = 0.0;
    for (int i = 0; i < k_used; ++i) {
      const double* vi = V + (size_t)i * N;
      for (int k = 0; k < N; ++k) w[k] += y[i] * vi[k];
    }
    prec_apply(op, F, w, z);
    for (int k = 0; k < N; ++k) x[k] += z[k];
    if (done_cycle) { status = ORA_OK; break; }
  }
#undef Hm
done:
  if (its_out) *its_out = its;
  if (relres_out) *relres_out = relres;
  free(V); free(H); free(cs); free(sn); free(g); free(y); free(w); free(z);
  return status;
}

/* ------------------------------------------------ Newton (sec. 2.3, eq. linsystem) */
static int all_finite(int n, const double* a) {
  for (int k = 0; k < n; ++k)
    if (!isfinite(a[k])) return 0;
  return 1;
}

/* Variable switch of one cell after an update (eq. primaryVariableMeaning,
 * with a threshold against oscillation): free gas gone (s_g < -eps) ->
 * x = r_go = r_s(p), the oil saturated at the switch; dissolved gas above
 * saturation (r_go > r_s(p) (1 + eps)) -> x = s_g = 0, free gas appears from
 * the next iteration on; a negative r_go is set to 0.  Wet gas: oil gone
 * (s_o < -eps) -> x = r_og = r_v(p); vaporised oil above saturation
 * (r_og > r_v(p) (1 + eps)) -> x = s_g = 1 - s_w (oil appears from the
 * next iteration on); a negative r_og is set to 0. */
static void switch_variable(const ora_fluid* f, double* yc, unsigned char* mean) {
  const double rs = f->rs_c * yc[0];
  const double rv = f->rv_c * yc[0];
  if (*mean == 0) {
    if (yc[2] < -f->eps_switch) {
      *mean = 1;
      yc[2] = rs;
    } else if (f->rv_c > 0.0 && 1.0 - yc[1] - yc[2] < -f->eps_switch) {
      /* wet gas: the oil is gone (s_o < -eps) -> x = r_og = r_v(p) */
      *mean = 2;
      yc[2] = rv;
    }
  } else if (*mean == 1) {
    if (yc[2] > rs * (1.0 + f->eps_switch)) {
      *mean = 0;
      yc[2] = 0.0;
    } else if (yc[2] < 0.0) {
      yc[2] = 0.0;
    }
  } else {
    /* vaporised oil above saturation -> oil appears: x = s_g = 1 - s_w */
    if (yc[2] > rv * (1.0 + f->eps_switch)) {
      *mean = 0;
      yc[2] = 1.0 - yc[1];
    } else if (yc[2] < 0.0) {
      yc[2] = 0.0;
    }
  }
}

int ora_newton_step(const ora_model* m, double* y, const double* y_prev, double dt,
                    const ora_opts* o, ora_report* rep) {
  const int n = m->n, N = 3 * n;
  double* acc0 = (double*)malloc(sizeof(double) * N);
  double* R = (double*)malloc(sizeof(double) * N);
  double* J = (double*)malloc(sizeof(double) * 9 * m->nnzb);
  double* F = (double*)malloc(sizeof(double) * 9 * m->nnzb);
  double* b = (double*)malloc(sizeof(double) * N);
  double* dx = (double*)malloc(sizeof(double) * N);
  const int nw = m->std_wells ? m->nw : 0, nc = m->std_wells ? m->nc : 0;
  double* Rw = (double*)malloc(sizeof(double) * (4 * nw + 1));
  double* bw = (double*)malloc(sizeof(double) * (4 * nw + 1));
  double* dxw = (double*)malloc(sizeof(double) * (4 * nw + 1));
  double* Bw = (double*)malloc(sizeof(double) * (12 * nc + 1));
  double* Cw = (double*)malloc(sizeof(double) * (12 * nc + 1));
  double* Dw = (double*)malloc(sizeof(double) * (16 * nw + 1));
  memset(rep, 0, sizeof(*rep));
  ora_accumulation(m, y_prev, acc0);
  if (m->std_wells) well_storage(m, m->wx, m->wA0);   /* the well state at entry is the old one */
  int status = ORA_ENOTCONV;
  for (int it = 0;; ++it) {
    double t0 = now_s();
    int st = ora_assemble(m, y, acc0, dt, R, J);
    if (st == ORA_OK && m->std_wells) st = ora_well_system(m, y, dt, Rw, Bw, Cw, Dw);
    rep->t_assemble += now_s() - t0;
    if (st != ORA_OK) { status = st; break; }
    ora_norms(m, y, R, dt, rep->cnv, rep->mb);
    double cmax = fmax(rep->cnv[0], fmax(rep->cnv[1], rep->cnv[2]));
    double mmax = fmax(rep->mb[0], fmax(rep->mb[1], rep->mb[2]));
    /* wells: component residuals in saturation units of the perforated pore
     * volume, the control relative to its target */
    for (int w = 0; w < nw; ++w) {
      double vref = 0.0;
      for (int q = m->well_beg[w]; q < m->well_beg[w + 1]; ++q) vref += m->pv[m->conn_cell[q]];
      for (int a = 0; a < 3; ++a) {
        const double bw_a = exp(m->fl.c[a] * (m->wx[4 * w + 3] - m->fl.p_ref));
        cmax = fmax(cmax, dt * fabs(Rw[4 * w + a]) / (bw_a * vref));
      }
      cmax = fmax(cmax, fabs(Rw[4 * w + 3]) / fabs(active_target(m, w)));
    }
    if (cmax <= o->tol_cnv && mmax <= o->tol_mb) { status = ORA_OK; break; }
    if (it >= o->max_newton) { status = ORA_ENOTCONV; break; }
    t0 = now_s();
    st = ora_ilu0(m, J, F);
    rep->t_factor += now_s() - t0;
    if (st != ORA_OK) { status = st; break; }
    for (int k = 0; k < N; ++k) b[k] = -R[k];
    for (int k = 0; k < 4 * nw; ++k) bw[k] = -Rw[k];
    double its = 0.0, rr = 0.0;
    ora_cpr* cpr = NULL;
    if (o->precond == 1 && (st = ora_cpr_setup(m, J, &cpr)) != ORA_OK) { status = st; break; }
    t0 = now_s();
    if (m->std_wells) {
      st = schur_solve(m, J, F, Bw, Cw, Dw, b, bw, dx, dxw, o->lin_rtol, o->lin_maxit, o->krylov,
                       o->restart, &its, &rr, cpr);
    } else {
      oper op = {m, J, NULL, NULL, NULL, cpr};
      st = o->krylov == 1
               ? gmres_op(&op, F, b, dx, o->lin_rtol, o->lin_maxit, o->restart, &its, &rr)
               : bicgstab_op(&op, F, b, dx, o->lin_rtol, o->lin_maxit, &its, &rr);
    }
    ora_cpr_destroy(cpr);
    rep->t_krylov += now_s() - t0;
    rep->lin_its += its;
    if (st != ORA_OK) { status = st; break; }
    t0 = now_s();
    /* Appleyard-type chop: bound |dp| by dp_max_rel |p|, scale the saturation
     * update of a cell so that its largest component is at most ds_max (the
     * third variable counts only where it is s_g; a change of r_go is not
     * chopped).  Then, for live oil, the variable switch. */
    for (int c = 0; c < n; ++c) {
      double dp = dx[3 * c], lim = o->dp_max_rel * fabs(y[3 * c]);
      if (dp > lim) dp = lim;
      if (dp < -lim) dp = -lim;
      const int is_sg = !m->fl.live || m->mean[c] == 0;
      double dsw = dx[3 * c + 1], dx3 = dx[3 * c + 2];
      double mx = is_sg ? fmax(fabs(dsw), fabs(dx3)) : fabs(dsw);
      if (mx > o->ds_max) {
        double sc = o->ds_max / mx;
        dsw *= sc;
        if (is_sg) dx3 *= sc;
      }
      y[3 * c] += dp;
      y[3 * c + 1] += dsw;
      y[3 * c + 2] += dx3;
      if (m->fl.live) switch_variable(&m->fl, y + 3 * c, &m->mean[c]);
    }
    /* well unknowns: |dp_bhp| <= dp_max_rel p_bhp, the fraction pair scaled
     * to at most ds_max, fractions kept in [0, 1] with F_w + F_g <= 1 */
    for (int w = 0; w < nw; ++w) {
      double* x = m->wx + 4 * w;
      double dpb = dxw[4 * w + 3], lim = o->dp_max_rel * fabs(x[3]);
      if (dpb > lim) dpb = lim;
      if (dpb < -lim) dpb = -lim;
      double dfw = dxw[4 * w + 1], dfg = dxw[4 * w + 2];
      double mx = fmax(fabs(dfw), fabs(dfg));
      if (mx > o->ds_max) {
        dfw *= o->ds_max / mx;
        dfg *= o->ds_max / mx;
      }
      x[0] += dxw[4 * w];
      x[1] = fmin(fmax(x[1] + dfw, 0.0), 1.0);
      x[2] = fmin(fmax(x[2] + dfg, 0.0), 1.0);
      if (x[1] + x[2] > 1.0) {
        const double sc = 1.0 / (x[1] + x[2]);
        x[1] *= sc;
        x[2] *= sc;
      }
      x[3] += dpb;
    }
    if (nw > 0) well_switch(m);
    rep->t_update += now_s() - t0;
    rep->newton_its++;
    rep->cell_newton_its += (double)n;
    if (!all_finite(N, y)) { status = ORA_ENONFINITE; break; }
  }
  rep->status = status;
  free(acc0); free(R); free(J); free(F); free(b); free(dx);
  free(Rw); free(bw); free(dxw); free(Bw); free(Cw); free(Dw);
  return status;
}

/* y_old with its meaning mean_old (and well state wx_old); y_new with the
 * model's current ones.  With standard wells the surface volume in place
 * includes the wellbore and the outflow is the wells' surface rates. */
static void mass_error(const ora_model* m, const double* y_old, const unsigned char* mean_old,
                       const double* wx_old, const double* y_new, double dt, double err[3]) {
  const int n = m->n;
  double* a0 = (double*)malloc(sizeof(double) * 3 * n);
  double* a1 = (double*)malloc(sizeof(double) * 3 * n);
  double* q = (double*)malloc(sizeof(double) * 3 * n);
  double* w0 = (double*)calloc(3 * (size_t)m->nw + 3, sizeof(double));
  double* w1 = (double*)calloc(3 * (size_t)m->nw + 3, sizeof(double));
  accumulation_of(m, mean_old, y_old, a0);
  ora_accumulation(m, y_new, a1);
  ora_well_rates(m, y_new, q);
  if (m->std_wells) {
    well_storage(m, wx_old, w0);
    well_storage(m, m->wx, w1);
  }
  for (int a = 0; a < 3; ++a) {
    double M0 = 0.0, M1 = 0.0, Q = 0.0, bsum = 0.0, pvs = 0.0;
    if (m->std_wells) {
      for (int w = 0; w < m->nw; ++w) {
        M0 += w0[3 * w + a];
        M1 += w1[3 * w + a];
        const double* x = m->wx + 4 * w;
        const double Fa = a == 0 ? x[1] : (a == 2 ? x[2] : 1.0 - x[1] - x[2]);
        Q += Fa * x[0] / kWellG[a];   /* Q_a = F_a Q_t / g_a */
      }
    }
    for (int c = 0; c < n; ++c) {
      M0 += m->pv[c] * a0[3 * c + a];
      M1 += m->pv[c] * a1[3 * c + a];
      if (!m->std_wells) Q += q[3 * c + a];
      props P;
      cell_props(&m->fl, y_new + 3 * c, 0, m->mean[c], &P);
      bsum += P.b[a].v;
      pvs += m->pv[c];
    }
    err[a] = fabs(M1 - M0 + dt * Q) / ((bsum / n) * pvs);
  }
  free(a0); free(a1); free(q); free(w0); free(w1);
}

int ora_advance(const ora_model* m, double* y, double dt_report, const ora_opts* o,
                ora_report* rep) {
  return ora_advance_log(m, y, dt_report, o, rep, NULL, NULL, 0, NULL);
}

/* Time-step cutting (sec. 2.3): a step whose Newton loop fails is retried
 * from the last accepted state (y, meanings, well state, controls) with half
 * the length, and the shorter length is kept for the rest of the report
 * step.  Each attempt's length and status go to dt_log / st_log (up to
 * log_cap entries; n_log receives the number of attempts). */
int ora_advance_log(const ora_model* m, double* y, double dt_report, const ora_opts* o,
                    ora_report* rep, double* dt_log, int* st_log, int log_cap, int* n_log) {
  const int N = 3 * m->n;
  double* yn = (double*)malloc(sizeof(double) * N);
  unsigned char* mn = (unsigned char*)malloc((size_t)m->n + 1);
  const size_t wbytes = m->std_wells ? sizeof(double) * 4 * m->nw : 0;
  double* wn = (double*)malloc(wbytes + sizeof(double));
  const size_t cbytes = m->std_wells ? sizeof(int) * m->nw : 0;
  int* cn = (int*)malloc(cbytes + sizeof(int));
  memcpy(yn, y, sizeof(double) * N);
  memcpy(mn, m->mean, (size_t)m->n);
  if (wbytes) memcpy(wn, m->wx, wbytes);
  if (cbytes) memcpy(cn, m->wctrl, cbytes);
  memset(rep, 0, sizeof(*rep));
  double t = 0.0, dt_try = dt_report;
  int status = ORA_OK, attempts = 0;
  while (dt_report - t > 1e-9 * dt_report) {
    double dt = fmin(dt_try, dt_report - t);
    ora_report r1;
    int st = ora_newton_step(m, y, yn, dt, o, &r1);
    if (dt_log && attempts < log_cap) {
      dt_log[attempts] = dt;
      st_log[attempts] = st;
    }
    attempts++;
    rep->newton_its += r1.newton_its;
    rep->lin_its += r1.lin_its;
    rep->cell_newton_its += r1.cell_newton_its;
    rep->t_assemble += r1.t_assemble;
    rep->t_factor += r1.t_factor;
    rep->t_krylov += r1.t_krylov;
    rep->t_update += r1.t_update;
    if (st == ORA_OK) {
      double e[3];
      mass_error(m, yn, mn, wn, y, dt, e);
      for (int a = 0; a < 3; ++a) {
        if (e[a] > rep->mass_err[a]) rep->mass_err[a] = e[a];
        rep->cnv[a] = r1.cnv[a];
        rep->mb[a] = r1.mb[a];
      }
      memcpy(yn, y, sizeof(double) * N);
      memcpy(mn, m->mean, (size_t)m->n);
      if (wbytes) memcpy(wn, m->wx, wbytes);
      if (cbytes) memcpy(cn, m->wctrl, cbytes);
      t += dt;
      rep->substeps++;
    } else {
      memcpy(y, yn, sizeof(double) * N);
      memcpy(m->mean, mn, (size_t)m->n);
      if (wbytes) memcpy(m->wx, wn, wbytes);
      if (cbytes) memcpy(m->wctrl, cn, cbytes);
      dt_try = 0.5 * dt;
      rep->cuts++;
      if (rep->cuts > o->max_cuts) { status = st; break; }
    }
  }
  rep->status = status;
  if (n_log) *n_log = attempts;
  free(yn);
  free(mn);
  free(wn);
  free(cn);
  return status;
}
