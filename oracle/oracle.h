/*
 * oracle.h -- plain, slow, FP64 CPU reference for the fully implicit
 * three-phase TPFA Newton path of the Open Porous Media Flow paper
 * (arXiv 1910.06059).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the GPU library includes, links or
 * calls this code; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no source with the GPU path: its own
 * grid and transmissibility code, its own forward-mode AD type, a generic
 * IKJ block ILU(0), a textbook BiCGStab and its own Newton loop.
 *
 * Paper references (section / equation labels of the paper):
 *   residual            sec. 2.1.1 "Discrete equations", eq. (materialbalance)
 *   fluxes, upwinding   sec. 2.1.1, eqs. (flux1), (head) and the upwind rule
 *   relative perm.      sec. 2.1.5, eq. (gwseg)
 *   PVT                 sec. 2.1.6 (constant compressibility)
 *   wells               sec. 2.2.1, eq. (wellinflow)
 *   Newton / chop       sec. 2.3, eq. (linsystem)
 *   CNV / MB criteria   sec. 2.3 (tolerance-cnv / tolerance-mb)
 *   ILU0 + BiCGStab     sec. 2.3.1
 *   forward-mode AD     sec. 2.4.1
 *   transmissibility    appendix B
 *
 * Units are SI throughout.  Phase / component order is (water, oil, gas);
 * the primary variables per cell are (p_o, s_w, x) with x = s_g, or, for live
 * oil in a cell without free gas, x = r_go (the meaning of x is a per-cell
 * state held by the model, eq. primaryVariableMeaning).  Cell numbering is the
 * natural order of active cells, c = i + nx*(j + ny*k) restricted to the mask.
 *
 * Parity status of each function (what pins it) is listed in the header of
 * oracle.c.
 */
#ifndef ORACLE_H
#define ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

#define ORA_OK 0
#define ORA_EINVAL (-1)
#define ORA_ESINGULAR (-2)
#define ORA_ENOTCONV (-3)
#define ORA_EBREAKDOWN (-4)
#define ORA_ENONFINITE (-5)

#define ORA_WELL_RATE_INJ 0
#define ORA_WELL_BHP_PROD 1

typedef struct ora_fluid {
  double rho_s[3];   /* surface densities (w, o, g) [kg/m^3]              */
  double c[3];       /* compressibilities [1/Pa]                           */
  double p_ref;      /* reference pressure of b = exp(c (p - p_ref)) [Pa]  */
  double mu[3];      /* viscosities [Pa s]                                 */
  double swc;        /* connate water saturation                           */
  double n_corey;    /* Corey exponent of every two-phase curve            */
  double g;          /* gravitational acceleration [m/s^2]                 */
  /* live oil (sec. 2.1.6: gas dissolved in the oleic phase; dry gas) */
  double rs_c;       /* saturated gas-oil ratio r_s(p) = rs_c p [1/Pa]      */
  double bo_r;       /* swelling: b_o = exp(c_o (p - p_ref)) / (1 + bo_r r) */
  double muo_r;      /* thinning: mu_o = mu_o / (1 + muo_r r)               */
  double eps_switch; /* threshold of the variable switch (s_g, relative r)  */
  int live;          /* 0 dead oil (x = s_g everywhere), 1 live oil         */
  int pad;
  /* wet gas (sec. 2.1.6: oil vaporised in the gaseous phase; live oil
   * only): saturated oil-gas ratio r_v(p) = rv_c p [1/Pa], 0 = dry gas */
  double rv_c;
} ora_fluid;

typedef struct ora_opts {
  double tol_cnv;     /* max local scaled residual                          */
  double tol_mb;      /* reservoir-average scaled residual                  */
  double ds_max;      /* Appleyard chop: max saturation change / iteration  */
  double dp_max_rel;  /* Appleyard chop: max |dp| / |p| per iteration       */
  double lin_rtol;    /* BiCGStab relative residual tolerance               */
  int max_newton;     /* max linear solves per time step                    */
  int lin_maxit;      /* BiCGStab iteration cap                             */
  int max_cuts;       /* time-step halvings allowed per report step         */
  int krylov;         /* 0 BiCGStab, 1 restarted GMRes                      */
  int restart;        /* GMRes restart length                               */
  int precond;        /* 0 (block-)ILU(0), 1 CPR-AMG with it as stage two   */
  int pad;
} ora_opts;

typedef struct ora_report {
  int status;           /* ORA_OK or an error code                          */
  int newton_its;       /* linear solves (summed over substeps in advance)  */
  int substeps;         /* accepted substeps                                */
  int cuts;             /* time-step halvings                               */
  double lin_its;       /* BiCGStab iterations (half iterations count 0.5)  */
  double cnv[3], mb[3]; /* final norms of the last accepted substep         */
  double mass_err[3];   /* max over substeps of the mass-balance error      */
  double t_assemble, t_factor, t_krylov, t_update;   /* seconds              */
  double cell_newton_its;   /* sum over Newton iterations of active cells   */
} ora_report;

typedef struct ora_model ora_model;

/* Build the discrete model of a (masked) Cartesian box.  All arrays are host
 * memory and are copied.  3-D fields are [nz][ny][nx] in C order.  Wells:
 * conn_ijk holds (i, j, k) triples of all wells' connections in well order. */
ora_model* ora_create(int nx, int ny, int nz, double dx, double dy, const double* dz,
                      const double* perm_h, double kv_kh, const double* poro,
                      const unsigned char* mask, const ora_fluid* fluid, int n_wells,
                      const int* well_kind, const int* well_phase, const double* well_target,
                      const double* well_rw, const int* well_nconn, const int* conn_ijk);
void ora_destroy(ora_model* m);

int ora_n_cells(const ora_model* m);
int ora_n_faces(const ora_model* m);
int ora_nnzb(const ora_model* m);
int ora_n_conns(const ora_model* m);

/* Geometry (appendix B): face_cells [nf][2] (i<j), trans [nf], pore volume and
 * cell-centre depth [n], box index of each active cell [n]. */
void ora_geometry(const ora_model* m, int* face_cells, double* trans, double* pv,
                  double* depth, int* cell_box);
/* Block-CSR pattern of the Jacobian: row_ptr [n+1], col_idx [nnzb], sorted. */
void ora_pattern(const ora_model* m, int* row_ptr, int* col_idx);
/* Well connections: active cell, well index, owning well [n_conns]. */
void ora_conns(const ora_model* m, int* cell, double* wi, int* well);

/* The per-cell meaning of the third variable (0: s_g, 1: r_go, 2: r_og
 * with wet gas), the state that goes with y: every function below reads
 * the model's current meaning; ora_newton_step / ora_advance update it with
 * y.  Set from `mean` [n] (NULL: every cell 0); dead oil requires all 0.
 * ORA_EINVAL for a value above 2, 1 or 2 with a dead-oil fluid, or 2
 * without wet gas (rv_c = 0). */
int ora_set_meaning(ora_model* m, const unsigned char* mean);
void ora_get_meaning(const ora_model* m, unsigned char* mean);

/* A_alpha = b_alpha s_alpha per cell (m_phi = 1), plus r_go b_o s_o in the
 * gas component for live oil: acc [n][3]. */
void ora_accumulation(const ora_model* m, const double* y, double* acc);
/* Surface well rates q [n][3] (outflux positive) at state y. */
void ora_well_rates(const ora_model* m, const double* y, double* q);
/* Residual R [n][3] and, if J != NULL, Jacobian blocks J [nnzb][3][3]
 * (row = equation w,o,g; column = variable p,s_w,s_g). */
int ora_assemble(const ora_model* m, const double* y, const double* acc0, double dt,
                 double* R, double* J);
/* CNV_alpha and MB_alpha of a residual. */
void ora_norms(const ora_model* m, const double* y, const double* R, double dt,
               double cnv[3], double mb[3]);

/* Block ILU(0), generic IKJ form: F [nnzb][3][3] holds L (unit diagonal
 * implied) below and U (with diagonal) on/above the block diagonal. */
int ora_ilu0(const ora_model* m, const double* J, double* F);
/* Block ILU0 over a partition of the grid into boxes of bx x by x bz cells
 * (sec. 2.5: one block per process): ora_ilu0 then factors the matrix
 * with every block coupling two different subdomains removed (those blocks
 * of F are zero).  All three 0 restores the single block.  ORA_EINVAL for
 * other non-positive sizes. */
int ora_set_ilu_blocks(ora_model* m, int bx, int by, int bz);
void ora_ilu0_apply(const ora_model* m, const double* F, const double* r, double* x);
void ora_spmv(const ora_model* m, const double* J, const double* x, double* y);
/* Right-preconditioned BiCGStab, x0 = 0.  its counts half iterations as 0.5. */
/* Right-preconditioned restarted GMRes(restart), x0 = 0, modified
 * Gram-Schmidt, Givens rotations; its counts inner iterations.
 * ORA_EINVAL for restart < 1. */
int ora_gmres(const ora_model* m, const double* J, const double* F, const double* b, double* x,
              double rtol, int maxit, int restart, double* its, double* relres);
int ora_bicgstab(const ora_model* m, const double* J, const double* F, const double* b,
                 double* x, double rtol, int maxit, double* its, double* relres);

/* One implicit Euler step of length dt: Newton from the guess in y (in/out),
 * y_prev is the state at the start of the step.  No time-step cutting. */
int ora_newton_step(const ora_model* m, double* y, const double* y_prev, double dt,
                    const ora_opts* o, ora_report* rep);
/* Advance y over one report step of length dt with halving on failure. */
int ora_advance(const ora_model* m, double* y, double dt, const ora_opts* o, ora_report* rep);
/* Threads of the OpenMP build of these sources (the CPU baseline: cells of
 * the accumulation, faces of the flux evaluation and rows of the product
 * with J in parallel, every sum in the serial order, so the results are the
 * serial build's bits); the plain build is single-threaded. */
void ora_set_threads(int n);
int ora_threads(void);
/* The same, recording every attempted substep: its length dt_log[k] and the
 * Newton step's status st_log[k] for k < min(*n_log, log_cap). */
int ora_advance_log(const ora_model* m, double* y, double dt, const ora_opts* o, ora_report* rep,
                    double* dt_log, int* st_log, int log_cap, int* n_log);

/* Standard well model (sec. 2.2.1): every well of the model gets the
 * unknowns x_w = (Q_t, F_w, F_g, p_bhp) (weighted total surface rate,
 * production positive; weighted water and gas fractions of the wellbore
 * fluid; bottom-hole pressure) with weights g = (1, 1, 0.01), component
 * conservation with wellbore storage (volume well_vol [nw]) and its control
 * (BHP producer: p_bhp = target; rate injector of component a:
 * Q_a = -target); connection rates by eq. wellinflow with h_w,j = 0.  x0:
 * [nw][4] initial well state.  The well state is held by the model like the
 * variable meaning; ora_newton_step / ora_advance solve the coupled system
 * by the Schur complement (eq. wellequation). */
int ora_set_standard_wells(ora_model* m, const double* well_vol, const double* x0,
                           const double* limits);
/* limits [nw] (may be NULL = none): the other control of each well, 0 =
 * none: an injector's maximum BHP, a BHP producer's maximum oil surface
 * rate.  The active control (0 the well's own, 1 its limit) switches after
 * each Newton update when the inactive constraint is violated, and is held
 * by the model with the well state (restored on a time-step cut). */
void ora_get_well_ctrl(const ora_model* m, int* ctrl);
void ora_set_well_ctrl(ora_model* m, const int* ctrl);
void ora_get_well_state(const ora_model* m, double* x);
void ora_set_well_state(ora_model* m, const double* x);
/* Record the wellbore storage of the current well state as the storage at
 * the start of a step (ora_newton_step does it at entry). */
void ora_well_storage_start(ora_model* m);
/* Well equations at y and the model's well state: Rw [nw][4] (water, oil,
 * gas conservation, control), B [nc][4][3] = dRw/d(cell variables of the
 * connection), C [nc][3][4] = d(cell residual)/dx_w, D [nw][4][4] =
 * dRw/dx_w.  ORA_EINVAL without standard wells. */
int ora_well_system(const ora_model* m, const double* y, double dt, double* Rw, double* B,
                    double* C, double* D);
/* Solve [[A C] [B D]] [x_r; x_w] = [Rr; Rw] by the Schur complement: the
 * Krylov method (0 BiCGStab, 1 GMRes(restart)) on (A - sum C D^-1 B) x_r =
 * Rr - sum C D^-1 Rw with the ILU(0) factors F of A as preconditioner, then
 * x_w = D^-1 (Rw - B x_r). */
int ora_schur_solve(const ora_model* m, const double* J, const double* F, const double* B,
                    const double* C, const double* D, const double* Rr, const double* Rw,
                    double* xr, double* xw, double rtol, int maxit, int krylov, int restart,
                    double* its, double* relres);

/* CPR-AMG (sec. 2.3.1): the two-stage constrained-pressure-residual
 * preconditioner with an aggregation AMG for the pressure stage.  Setup for
 * a Jacobian J: quasi-IMPES weights (D_i^T w_i = e_p, D_i the diagonal
 * block), pressure matrix (A_p)_ij = w_i^T A_ij e_p on the block pattern,
 * coarse levels by geometric 2x2x2 aggregation of each level's lattice with
 * Galerkin matrices P^T A P (P piecewise constant) down to <= 64 unknowns.
 * Application: one V(1,1) cycle (damped Jacobi, omega = 2/3; dense LU on the
 * coarsest level) on w^T r, x1 = e_p x_p, then z = x1 + M_ILU^{-1}(r - A x1)
 * with the (block-)ILU(0) factors F of A. */
typedef struct ora_cpr ora_cpr;
int ora_cpr_setup(const ora_model* m, const double* J, ora_cpr** out);
void ora_cpr_destroy(ora_cpr* c);
int ora_cpr_levels(const ora_cpr* c);
void ora_cpr_level_size(const ora_cpr* c, int l, int* n, int* nnz);
/* Level l's CSR matrix (rp [n+1], ci / a [nnz]) and, for l < levels - 1,
 * its aggregation map agg [n] (may be NULL). */
void ora_cpr_level(const ora_cpr* c, int l, int* rp, int* ci, double* a, int* agg);
void ora_cpr_weights(const ora_cpr* c, double* w);
/* x = one V(1,1) cycle on A_p x = b (x starts at zero). */
void ora_cpr_vcycle(const ora_cpr* c, const double* b, double* x);
void ora_cpr_apply(const ora_model* m, const ora_cpr* c, const double* J, const double* F,
                   const double* r, double* z);
/* Right-preconditioned BiCGStab with CPR (second stage: the factors F). */
int ora_bicgstab_cpr(const ora_model* m, const double* J, const double* F, const ora_cpr* c,
                     const double* b, double* x, double rtol, int maxit, double* its,
                     double* relres);

/* Dense LU with partial pivoting: solves A x = b in place (A [n][n] row-major
 * is overwritten).  Returns ORA_ESINGULAR on a zero pivot. */
int ora_dense_solve(int n, double* A, double* b);

#ifdef __cplusplus
}
#endif
#endif
