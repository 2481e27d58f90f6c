/*
 * opm_gpu.h -- C ABI of the MI355X (gfx950) Newton linearisation and solve
 * of the fully implicit three-phase black-oil equations of the Open Porous
 * Media Flow paper (arXiv 1910.06059), immiscible subset.
 *
 * The discrete problem (paper sec. 2.1.1, eq. materialbalance) is, per cell
 * i and component alpha in (water, oil, gas):
 *
 *   R_alpha,i = PV_i/dt (A_alpha,i - A0_alpha,i) + sum_{j in C(i)} u_alpha,ij + q_alpha,i = 0
 *
 * with A_alpha = b_alpha s_alpha (m_phi = 1), TPFA fluxes
 * u_alpha,ij = (b_alpha lambda_alpha)_U T_ij dPhi_alpha,ij (eqs. flux1, head;
 * U the upwind cell of dPhi), primary variables y_i = (p_o, s_w, s_g)
 * (sec. 2.1.2), capillary pressure zero, constant-compressibility PVT
 * b = exp(c (p - p_ref)) (sec. 2.1.6), Corey two-phase curves combined by the
 * segregation model for oil (eq. gwseg), and wells as cell source terms
 * (eq. wellinflow with fixed BHP, or a fixed surface-rate injector).
 * Newton (sec. 2.3, eq. linsystem) solves J dy = -R with block-ILU(0)
 * preconditioned BiCGStab (sec. 2.3.1) on a 3x3-block CSR Jacobian.
 *
 * Conventions shared by every entry point:
 *  - Units are SI.  Vectors indexed by cell are [n_cells][3] row-major:
 *    state (p [Pa], s_w, s_g), residual (water, oil, gas) [surface m^3/s].
 *  - Jacobian blocks J[nnzb][3][3]: row = equation (w, o, g), column =
 *    variable (p, s_w, s_g), row-major; block q of row i sits at column
 *    col_idx[q], with row_ptr/col_idx the block-CSR pattern of opm_topology.
 *  - "device" pointers are HIP device memory owned by the caller (the Python
 *    binding passes torch CUDA tensors); "host" pointers are host memory.
 *    Every buffer, workspaces included, comes from the caller: the library
 *    never allocates device memory for data.  It keeps no pointer to caller
 *    memory after a call returns, with one exception: opm_bicgstab (and the
 *    Newton entry points that call it) caches up to 16 instantiated HIP
 *    graphs of a chunk of its iterations, keyed by every launch argument
 *    (the opm_problem by value, the buffers' device addresses, the stream,
 *    the precision, the launch options, the device) and a hash of the host
 *    arrays whose contents shape the launches (level_ptr_h and the CPR
 *    hierarchy's sizes); a graph is replayed only for a call with the same
 *    key, evicted oldest first, and released at process exit.  Capturing
 *    needs a non-null stream, so the library creates one capture stream per
 *    device (default priority) on first use.  A mutex serialises the cache
 *    and the capture streams between host threads; OPM_OPT_KRYLOV_GRAPH = 0
 *    turns the cache off.  Besides the cache and the graph runtime's own
 *    objects, what persists between calls is: the process-wide values of
 *    opm_set_option, the kernels' LDS attributes, per-host-thread HIP events
 *    of the Newton step's phase timers and 48 bytes of pinned host memory
 *    for its status reads, per host thread and device two events, 192
 *    bytes of pinned host memory for opm_bicgstab's reads of its iteration
 *    state and the iteration count of its last solve (the host polls these
 *    events rather than sleeping in a blocking wait),
 *    and per device the static 5 MiB scratch array of opm_assemble_noalloc
 *    (see there).
 *  - stream is a hipStream_t (NULL = default stream).  Calls are asynchronous
 *    on that stream unless their comment says that they synchronise.
 *  - Every entry point returns an int status: OPM_OK (0) or a negative code;
 *    opm_strerror names it.  No exception crosses the ABI.  Invalid arguments
 *    are reported as OPM_EINVAL before any device work is queued.
 */
#ifndef OPM_GPU_H
#define OPM_GPU_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define OPM_OK 0
#define OPM_EINVAL (-1)        /* bad argument or unsupported pattern        */
#define OPM_ESINGULAR (-2)     /* zero / non-finite 3x3 pivot in ILU(0)       */
#define OPM_ENOTCONV (-3)      /* Newton or a Krylov solver did not converge */
#define OPM_EBREAKDOWN (-4)    /* Krylov breakdown (BiCGStab: rho, <r^,v>, omega,
                                  * <t,t>; GMRes: singular triangular factor) */
#define OPM_ENONFINITE (-5)    /* NaN or Inf in residual or state            */
#define OPM_EHIP (-6)          /* a HIP runtime call failed                   */

#define OPM_WELL_RATE_INJ 0    /* fixed surface rate of one component          */
#define OPM_WELL_BHP_PROD 1    /* bottom-hole pressure producer                */

#define OPM_PREC_FP64 0        /* ILU(0) factors and sweeps in FP64            */
#define OPM_PREC_MIXED 1       /* ILU(0) factors stored and swept in FP32      */

#define OPM_KRYLOV_BICGSTAB 0  /* Newton's linear solver: BiCGStab (default)     */
#define OPM_KRYLOV_GMRES 1     /* Newton's linear solver: restarted GMRes        */
#define OPM_GMRES_MAX_RESTART 32
#define OPM_PRECOND_ILU0 0     /* the (block-)ILU(0) preconditioner            */
#define OPM_PRECOND_CPR 1      /* CPR-AMG, the (block-)ILU(0) as second stage */

/* Fluid and rock-fluid constants (phase order water, oil, gas). */
typedef struct opm_fluid {
  double rho_s[3];   /* surface densities [kg/m^3]                          */
  double c[3];       /* compressibilities [1/Pa]: b = exp(c (p - p_ref))   */
  double p_ref;      /* reference pressure [Pa]                             */
  double mu[3];      /* viscosities [Pa s]                                  */
  double swc;        /* connate water saturation of the Corey curves        */
  double n_corey;    /* Corey exponent of every two-phase curve (>= 1)      */
  double g;          /* gravitational acceleration [m/s^2], depth positive down */
  /* Live oil (sec. 2.1.6: gas dissolved in the oleic phase; dry gas).  With
   * live = 0 the oil is dead and the fields below are unused. */
  double rs_c;       /* saturated gas-oil ratio r_s(p) = rs_c p [1/Pa]      */
  double bo_r;       /* swelling: b_o = exp(c_o (p - p_ref)) / (1 + bo_r r) */
  double muo_r;      /* thinning: mu_o = mu_o / (1 + muo_r r); the oil
                        density is rho_o = b_o (rho_oS + r rho_gS)          */
  double eps_switch; /* threshold of the variable switch: free gas below
                        -eps_switch, dissolved gas above r_s (1 + eps_switch) */
  int32_t live;      /* 0 dead oil, 1 live oil                               */
  int32_t pad;
  /* wet gas (sec. 2.1.6: oil vaporised in the gas; live oil only): the
   * saturated oil-gas ratio r_v(p) = rv_c p [1/Pa]; 0 = dry gas.  With
   * rv_c > 0 a cell's meaning may also be 2: no oil, s_g = 1 - s_w and
   * x = r_og (switched to when s_o < -eps_switch, back to x = s_g when
   * r_og > r_v(p) (1 + eps_switch)). */
  double rv_c;
} opm_fluid;

/* Connectivity of a masked nx*ny*nz Cartesian box (host arrays, filled by
 * opm_topology_build, sized from opm_topology_count).  Active cells are
 * numbered in natural order c = i + nx (j + ny k) restricted to the mask;
 * faces are the (+x, +y, +z) neighbours of each active cell, so
 * face_cells[f][0] < face_cells[f][1].  The level schedule lists rows by
 * level: the levels are the hyperplanes i + j + k = const that hold active
 * cells, in increasing order, rows of one level in ascending order.  Every
 * lower neighbour of a row lies on the previous level, so this is an order
 * in which ILU(0) factorisation and triangular sweeps may proceed in
 * parallel (any such order gives the same factors). */
typedef struct opm_topology {
  int32_t* cell_box;    /* [n_cells]  box index of each active cell            */
  int32_t* face_cells;  /* [n_faces][2] lower and upper cell                   */
  int32_t* face_dir;    /* [n_faces]  0 = x, 1 = y, 2 = z                      */
  int32_t* row_ptr;     /* [n_cells+1]                                          */
  int32_t* col_idx;     /* [nnzb], nnzb = n_cells + 2 n_faces, sorted per row   */
  int32_t* blk_face;    /* [nnzb] face of an off-diagonal block, -1 on diagonal */
  int32_t* diag_pos;    /* [n_cells] position of the diagonal block            */
  int32_t* level_ptr;   /* [n_cells+1] level l holds positions level_ptr[l..l+1) */
  int32_t* perm;        /* [n_cells] level-order position -> cell               */
  int32_t* iperm;       /* [n_cells] cell -> level-order position               */
  int32_t* lo_blk;      /* [n_cells][3] by position: block (i,k) of each lower
                           neighbour k (-1 if absent)                           */
  int32_t* lo_tblk;     /* [n_cells][3] the transposed block (k,i)              */
  int32_t* lo_pos;      /* [n_cells][3] level-order position of k               */
  int32_t* up_blk;      /* [n_cells][3] block (i,j) of each upper neighbour j   */
  int32_t* up_pos;      /* [n_cells][3] level-order position of j               */
  int32_t n_levels;     /* out                                                  */
  int32_t max_level;    /* out: largest number of rows in one level             */
  int32_t sweep_span;   /* out: largest |position(i) - position(j)| over the
                           connections (i,j) in the level order                 */
} opm_topology;

/* Count active cells and faces (host, synchronous).  mask may be NULL (all
 * cells active).  Returns OPM_EINVAL for non-positive sizes. */
int opm_topology_count(int32_t nx, int32_t ny, int32_t nz, const uint8_t* mask,
                       int32_t* n_cells, int32_t* n_faces);
/* Fill an opm_topology whose arrays the caller sized from opm_topology_count
 * (host, synchronous; paper sec. 2.1.1 connection set C(i), sec. 2.3.1 block
 * matrix storage, ILU(0) dependency levels). */
int opm_topology_build(int32_t nx, int32_t ny, int32_t nz, const uint8_t* mask,
                       opm_topology* topo);

/* Block ILU0 over a partition of the grid into subdomain boxes (paper
 * sec. 2.5: a block ILU0 with one block per process; sec. 3.7.2 observes
 * that the linear iterations barely grow with the number of blocks).  The
 * box of cell (i, j, k) is (i / bx, j / by, k / bz); boxes without active
 * cells are dropped and the rest numbered densely in box order.  The
 * preconditioner is the ILU(0) of the matrix with every block that couples
 * two different subdomains removed, i.e. each subdomain's own ILU(0); the
 * matrix products of the solver still use the whole matrix.  The paper keeps
 * strongly coupled cells in one subdomain: boxes spanning whole columns
 * (bz = nz) suit layered models, whose vertical transmissibilities are the
 * largest.  Host arrays, filled by opm_topology_build_blocks. */
typedef struct opm_ilu_blocks {
  int32_t bx, by, bz;       /* in: subdomain box, cells per axis (each >= 1; a box
                               longer than the grid spans the whole axis)        */
  int32_t* sub_level_ptr;   /* out [n_levels * (n_sub + 1)]: the rows of subdomain
                               s on level l are the positions
                               [sub_level_ptr[l (n_sub+1) + s], ... + s + 1)     */
  int32_t* slot;            /* out [n_cells] by position: index of the row inside
                               its subdomain, counting the subdomain's rows level
                               by level                                          */
  int32_t n_sub;            /* out: subdomains holding active cells              */
  int32_t max_sub;          /* out: most rows of one subdomain                   */
  int32_t max_width;        /* out: most rows of one subdomain on one level      */
} opm_ilu_blocks;

/* Number of nonempty subdomains and of levels of a partition (host): size
 * sub_level_ptr as n_levels * (n_sub + 1).  OPM_EINVAL for non-positive
 * sizes. */
int opm_ilu_blocks_count(int32_t nx, int32_t ny, int32_t nz, const uint8_t* mask, int32_t bx,
                         int32_t by, int32_t bz, int32_t* n_sub, int32_t* n_levels);
/* opm_topology_build for the block ILU0 of a partition (host, synchronous).
 * Connectivity and block-CSR pattern are those of opm_topology_build.  The
 * levels are the local hyperplanes (i mod bx) + (j mod by) + (k mod bz) that
 * hold active cells; inside a level the rows are grouped by subdomain
 * (positions ordered by level, subdomain, cell).  The ILU neighbour lists
 * (lo_*, up_*) hold only neighbours in the same subdomain, so every ILU(0)
 * factorisation and sweep of the library computes the block ILU0 on such a
 * topology.  OPM_EINVAL on a NULL array or non-positive box size. */
int opm_topology_build_blocks(int32_t nx, int32_t ny, int32_t nz, const uint8_t* mask,
                              opm_ilu_blocks* blocks, opm_topology* topo);

/* Transmissibility, pore volume and depth (appendix B; sec. 2.1.4), device:
 * T_ij = t_ij t_ji / (t_ij + t_ji) with half-transmissibilities
 * t = |F| k / (d/2) of the axis-aligned cells, k = perm_h for x/y faces and
 * kv_kh * perm_h for z faces; PV = poro dx dy dz_k; depth = cell centre.
 * perm_h, poro: [n_cells] (active-cell order); dz: [nz]; cell_box,
 * face_cells, face_dir from opm_topology (device copies).  Outputs trans
 * [n_faces], pore_vol [n_cells], depth [n_cells]. */
int opm_geometry(int32_t nx, int32_t ny, int32_t nz, double dx, double dy, const double* dz,
                 const double* perm_h, double kv_kh, const double* poro, int32_t n_cells,
                 int32_t n_faces, const int32_t* cell_box, const int32_t* face_cells,
                 const int32_t* face_dir, double* trans, double* pore_vol, double* depth,
                 void* stream);

/* Well connections (sec. 2.2.1, eq. wellinflow), device.  Inputs per well
 * [n_wells]: kind, injected phase, target (surface rate [m^3/s] for
 * OPM_WELL_RATE_INJ, BHP [Pa] for OPM_WELL_BHP_PROD) and wellbore radius rw;
 * per connection [n_conns]: active cell and owning well.  Outputs per
 * connection: the Peaceman index wi = 2 pi k_h dz / ln(0.14 sqrt(dx^2+dy^2)
 * / rw) (skin 0), the fixed injection source rate = -target wi / sum(wi of
 * the well) (0 for producers), and the well's kind, phase and BHP target
 * (0 for injectors).  perm_h [n_cells], dz [nz], cell_box as above. */
int opm_well_index(int32_t nx, int32_t ny, double dx, double dy, const double* dz,
                   const double* perm_h, const int32_t* cell_box, int32_t n_wells,
                   const int32_t* well_kind, const int32_t* well_phase,
                   const double* well_target, const double* well_rw, int32_t n_conns,
                   const int32_t* conn_cell, const int32_t* conn_well, double* conn_wi,
                   double* conn_rate, int32_t* conn_kind, int32_t* conn_phase,
                   double* conn_bhp, void* stream);

/* Group well connections by cell (host, synchronous): cell_conn_ptr
 * [n_cells+1] and cell_conn [n_conns] list the connections of each cell in
 * ascending connection order.  conn_cell [n_conns] (host).  OPM_EINVAL if a
 * cell index is out of range. */
int opm_well_groups(int32_t n_cells, int32_t n_conns, const int32_t* conn_cell,
                    int32_t* cell_conn_ptr, int32_t* cell_conn);

/* CPR-AMG hierarchy (sec. 2.3.1: the two-stage CPR preconditioner with an
 * AMG for the pressure system).  Level 0 is the pressure system on the
 * cells (the block pattern, row_ptr / col_idx / diag_pos of the problem);
 * level l + 1 aggregates the unknowns of level l in geometric 2x2x2 boxes of
 * level l's lattice (its coarse unknowns: the occupied coarse boxes in
 * natural order), down to at most OPM_AMG_COARSE unknowns (OPM_EINVAL if
 * OPM_AMG_MAX_LEVELS levels do not get there).  Filled on the
 * host by opm_amg_build (host arrays), then the same struct with device
 * copies is referenced from opm_problem.amg.  Arrays of level l (l >= 1
 * for row_ptr / col / dpos; l < n_levels - 1 for agg / child_ptr / child;
 * l >= 1 for gmap_ptr / gmap):
 *   row_ptr [n+1], col [nnz]: CSR pattern, columns ascending;
 *   dpos [n]: position of each row's diagonal entry;
 *   agg [n_l]: the unknown of level l + 1 that holds each unknown;
 *   child_ptr [n_{l+1}+1], child [n_l]: the unknowns of each aggregate,
 *     ascending;
 *   gmap_ptr [nnz_l + 1], gmap [nnz_{l-1}]: the level l-1 entries whose sum
 *     is each entry of level l (the Galerkin product P^T A P with the
 *     piecewise-constant P), in the order children, then row entries. */
#define OPM_AMG_MAX_LEVELS 12
#define OPM_AMG_COARSE 64
typedef struct opm_amg {
  int32_t n_levels;
  int32_t n[OPM_AMG_MAX_LEVELS];
  int32_t nnz[OPM_AMG_MAX_LEVELS];
  int32_t* row_ptr[OPM_AMG_MAX_LEVELS];
  int32_t* col[OPM_AMG_MAX_LEVELS];
  int32_t* dpos[OPM_AMG_MAX_LEVELS];
  int32_t* agg[OPM_AMG_MAX_LEVELS];
  int32_t* child_ptr[OPM_AMG_MAX_LEVELS];
  int32_t* child[OPM_AMG_MAX_LEVELS];
  int32_t* gmap_ptr[OPM_AMG_MAX_LEVELS];
  int32_t* gmap[OPM_AMG_MAX_LEVELS];
} opm_amg;

/* Sizes of the hierarchy of a topology (n_levels, n[], nnz[] of out; the
 * pointers untouched).  row_ptr / col_idx: the block pattern of
 * opm_topology_build (host). */
int opm_amg_count(int32_t nx, int32_t ny, int32_t nz, const uint8_t* mask, int32_t n_cells,
                  const int32_t* row_ptr, const int32_t* col_idx, opm_amg* out);
/* Fill the arrays of out (host, sized from opm_amg_count; level 0's
 * row_ptr / col / dpos pointers are not used). */
int opm_amg_build(int32_t nx, int32_t ny, int32_t nz, const uint8_t* mask, int32_t n_cells,
                  const int32_t* row_ptr, const int32_t* col_idx, opm_amg* out);

/* The discrete problem handed to the path (device pointers unless noted).
 * Well connections must be grouped by cell: cell_conn_ptr[n_cells+1] gives
 * the connections of cell i as conn ids cell_conn[cell_conn_ptr[i] ..]. */
typedef struct opm_problem {
  int32_t n_cells, n_faces, nnzb, n_levels, max_level;
  int32_t n_conns;
  const double* trans;          /* [n_faces]                                  */
  const double* pore_vol;       /* [n_cells]                                  */
  const double* depth;          /* [n_cells]                                  */
  const int32_t* row_ptr;       /* [n_cells+1]                                */
  const int32_t* col_idx;       /* [nnzb]                                     */
  const int32_t* blk_face;      /* [nnzb]                                     */
  const int32_t* face_cells;    /* [n_faces][2]                               */
  const int32_t* diag_pos;      /* [n_cells]                                  */
  const int32_t* level_ptr;     /* [n_levels+1] device copy                   */
  const int32_t* level_ptr_h;   /* [n_levels+1] HOST copy (launch schedule)   */
  const int32_t* perm;          /* [n_cells]                                  */
  const int32_t* iperm;         /* [n_cells]                                  */
  const int32_t* lo_blk;        /* [n_cells][3]                               */
  const int32_t* lo_tblk;       /* [n_cells][3]                               */
  const int32_t* lo_pos;        /* [n_cells][3]                               */
  const int32_t* up_blk;        /* [n_cells][3]                               */
  const int32_t* up_pos;        /* [n_cells][3]                               */
  const int32_t* cell_conn_ptr; /* [n_cells+1]                                */
  const int32_t* cell_conn;     /* [n_conns]                                  */
  const int32_t* conn_kind;     /* [n_conns] OPM_WELL_* of the owning well    */
  const int32_t* conn_phase;    /* [n_conns] injected component               */
  const double* conn_wi;        /* [n_conns]                                  */
  const double* conn_rate;      /* [n_conns] fixed source (injectors)         */
  const double* conn_bhp;       /* [n_conns] BHP target (producers)           */
  opm_fluid fluid;
  int32_t sweep_span;           /* opm_topology.sweep_span                    */
  /* block ILU0 (topology from opm_topology_build_blocks); n_sub = 0 for the
   * single-block ILU(0) of opm_topology_build, the rest then unused */
  int32_t n_sub;                /* opm_ilu_blocks.n_sub                       */
  int32_t max_sub;              /* opm_ilu_blocks.max_sub                     */
  int32_t max_width;            /* opm_ilu_blocks.max_width                   */
  const int32_t* sub_level_ptr; /* [n_levels*(n_sub+1)] device copy          */
  const int32_t* slot;          /* [n_cells] device copy                      */
  /* Meaning of the third primary variable per cell (sec. 2.1.1, eq.
   * primaryVariableMeaning): 0 x = s_g (free gas present; live oil then
   * saturated, r_go = r_s(p)), 1 x = r_go (live oil without free gas,
   * s_g = 0), 2 x = r_og (wet gas, opm_fluid.rv_c > 0: no oil,
   * s_g = 1 - s_w).  Device [n_cells], part of the state that goes with y:
   * opm_newton_step / opm_advance update it in place.  NULL for dead oil
   * (every cell 0); required (non-NULL) for live oil. */
  uint8_t* meaning;
  /* Standard well model (sec. 2.2.1), enabled by n_wells > 0: each well has
   * the unknowns x_w = (Q_t, F_w, F_g, p_bhp) -- weighted total surface
   * rate (production positive), weighted water and gas fractions of the
   * wellbore fluid (weights g = (1, 1, 0.01), Q_a = F_a Q_t / g_a,
   * F_o = 1 - F_w - F_g) and bottom-hole pressure -- with component
   * conservation including wellbore storage V_w mix_a (eq. conseq-swell;
   * mix_a = (F_a / g_a) / sum_b F_b / (g_b b_b(p_bhp))) and its control
   * (eq. well-control-bhp: p_bhp = target; eq. well-control-rate: Q_a =
   * -target for an injector of component a).  A producing connection
   * carries the cell's phases, q_a = WI b_a lambda_a (p - p_bhp) (plus
   * r b_o lambda_o for gas with live oil), an injecting one the wellbore
   * fluid at the cell's total mobility, q_a = WI lambda_t (p - p_bhp) mix_a
   * (eq. wellinflow, h_w,j = 0).  The Newton step eliminates the well
   * unknowns by the Schur complement (eq. wellequation).  With n_wells = 0
   * the wells are the fixed sources / BHP sinks described by conn_kind.
   * Connections are numbered well by well. */
  int32_t n_wells;
  int32_t pad_w;
  const int32_t* well_conn_ptr; /* [n_wells+1] connections of each well      */
  const int32_t* conn_cell;     /* [n_conns] cell of each connection          */
  const int32_t* conn_well;     /* [n_conns] well of each connection          */
  const int32_t* well_kind;     /* [n_wells] OPM_WELL_*                       */
  const int32_t* well_phase;    /* [n_wells] controlled component (injectors) */
  const double* well_target;    /* [n_wells] BHP [Pa] or surface rate [m3/s]  */
  const double* well_vol;       /* [n_wells] wellbore volume V_w [m3]         */
  double* well_state;           /* [n_wells][4] device, in/out: the state of
                                   the well unknowns that goes with y         */
  /* CPR-AMG hierarchy (host struct holding device arrays), or NULL: needed
   * for opm_newton_opts.precond = OPM_PRECOND_CPR and opm_cpr_*. */
  const opm_amg* amg;
  /* Control limits of standard wells (sec. 2.2.1 BHP and rate controls),
   * or NULL for none.  well_limit [n_wells] (device): the other control of
   * each well, 0 = none: an injector's maximum BHP [Pa], a BHP producer's
   * maximum oil surface rate [m3/s].  well_ctrl [n_wells] (device, in/out,
   * part of the state with well_state; required with well_limit): the
   * active control, 0 the well's own, 1 its limit (control equation
   * p_bhp - limit, resp. Q_o - limit).  After each Newton update a well on
   * its own control moves to its limit when the limit is exceeded, and one
   * on its limit moves back when its own control binds again (a producer's
   * BHP below its target, an injector's rate above its target);
   * opm_advance restores the controls with the well state on a cut. */
  const double* well_limit;
  int32_t* well_ctrl;
  /* The lattice of the cells (sec. 2.4.2 localisation): box dims and
   * box_cell [nx*ny*nz] (device), the active-cell index of each box cell in
   * natural order i + nx (j + ny k), -1 for an inactive one.  With box_cell
   * set, the dead-oil assembly with fixed-source wells runs on lattice
   * tiles whose cell properties and face fluxes are staged in LDS; NULL
   * (or live oil, or standard wells) selects the row-per-lane assembly.
   * Both give the same residual and Jacobian up to rounding. */
  int32_t nx, ny, nz, pad_l;
  const int32_t* box_cell;
  /* cell_box [n_cells] (device): the box index of each active cell (the
   * inverse of box_cell).  With both maps, the ILU(0) sweeps of a system
   * too large for one workgroup run plane by plane in one launch each: one
   * workgroup per z-plane walks the plane's diagonals i + j, and a row waits
   * only for the value of its neighbour in the plane below (forward) or
   * above (backward).  NULL: one launch per level. */
  const int32_t* cell_box;
} opm_problem;

/* Library set-up: checks that the current device is a gfx950 (MI355X) and
 * that its kernels load.  Call once per process and device before any other
 * device entry point (synchronous); returns OPM_EHIP otherwise. */
int opm_init(void);

/* ---------------------------------------------------------- hot path ---- */

/* A0 = b(p) s per cell at the start of a time step (eq. acc): y [n][3] ->
 * acc0 [n][3] (device). */
int opm_accumulation(const opm_problem* pb, const double* y, double* acc0, void* stream);

/* Size in bytes of the device buffer `norms` of opm_assemble. */
size_t opm_norms_bytes(const opm_problem* pb);

/* Residual and Jacobian by forward-mode AD (sec. 2.4.1-2.4.2; eqs.
 * materialbalance, flux1, head, gwseg, wellinflow).  With live oil the gas
 * component also holds the gas dissolved in the oil (r b_o s_o in the
 * accumulation, r (b_o lambda_o) T dPhi_o upwinded with the oil phase in the
 * flux, r times the oil rate in a producer), and the third Jacobian column
 * of a cell is d/ds_g, d/dr_go or d/dr_og by its meaning (wet gas adds
 * r_og b_g s_g to the oil accumulation and r_og (b_g lambda_g) T dPhi_g,
 * upwinded with the gas phase, to the oil flux).  y, acc0: [n][3]; R:
 * [n][3] out; J: [nnzb][3][3] out (may be NULL for the residual only).
 * norms (may be NULL): device buffer of opm_norms_bytes; its first 8
 * doubles receive CNV_w, CNV_o, CNV_g, MB_w, MB_o, MB_g, max CNV, max MB,
 * where CNV_a = dt max_i |R_a,i| / (b_a(p_i) PV_i) and
 * MB_a = dt |sum_i R_a,i| / (mean_i b_a(p_i) sum_i PV_i) (sec. 2.3,
 * tolerance-cnv / tolerance-mb); the rest holds per-workgroup partials.
 * All device pointers. */
int opm_assemble(const opm_problem* pb, const double* y, const double* acc0, double dt,
                 double* R, double* J, double* norms, void* stream);

/* opm_assemble for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same kernels and results, with the per-workgroup partials of the
 * norms kept in a static device array of the library (5 MiB per GPU, held
 * until the process ends) instead of the caller's buffer.  norms (may be
 * NULL): device, 8 doubles, the same values as opm_assemble's first 8.
 * Supports at most 16,777,216 cells: larger problems return OPM_EINVAL
 * before any device work.  The call allocates nothing (the array's address
 * is resolved by opm_init, or by the first call on a device).  Every call on
 * a GPU shares that GPU's array, so calls that overlap on one GPU (several
 * streams or host threads) race and must be serialised by the caller. */
int opm_assemble_noalloc(const opm_problem* pb, const double* y, const double* acc0, double dt,
                         double* R, double* J, double* norms, void* stream);

/* Size in bytes of the ILU(0) factor storage for a precision
 * (OPM_PREC_FP64 or OPM_PREC_MIXED). */
size_t opm_ilu0_bytes(const opm_problem* pb, int precision);

/* Block ILU(0) of J (sec. 2.3.1) into ilu (device, opm_ilu0_bytes): the
 * inverse pivot blocks D_i^{-1} with D_i = A_ii - sum_{k<i} A_ik D_k^{-1} A_ki
 * (exact ILU(0) for a pattern without triangles, which the 7-point TPFA
 * stencil is) and level-ordered copies of the off-diagonal blocks, in FP64 or
 * FP32.  status (device int, may be NULL) receives OPM_ESINGULAR on a zero or
 * non-finite pivot, and OPM_EHIP if the plane-pipelined factorisation of a
 * lattice system (OPM_OPT_PLANE_SWEEP) gave up waiting for a neighbouring
 * plane (OPM_OPT_PLANE_SPIN). */
int opm_ilu0_factor(const opm_problem* pb, const double* J, void* ilu, int precision,
                    int32_t* status, void* stream);

/* x = (LU)^{-1} r with the factors of opm_ilu0_factor (device [n][3]). */
int opm_ilu0_apply(const opm_problem* pb, const void* ilu, int precision, const double* r,
                   double* x, void* stream);

/* y = J x (device [n][3]). */
int opm_spmv(const opm_problem* pb, const double* J, const double* x, double* y, void* stream);

/* Report of one linear solve. */
typedef struct opm_solve_report {
  int32_t status;     /* OPM_OK, OPM_ENOTCONV or OPM_EBREAKDOWN             */
  int32_t half;       /* 1 if it stopped after the first half of an iteration */
  int32_t its;        /* iterations started                                  */
  int32_t pad;
  double rel_res;     /* ||r|| / ||b|| at exit                               */
} opm_solve_report;

/* Size in bytes of the Krylov workspace (device). */
size_t opm_krylov_bytes(const opm_problem* pb);

/* Right-preconditioned BiCGStab (sec. 2.3.1), x0 = 0, stops when
 * ||r||_2 <= rtol ||b||_2 or after maxit iterations.  b, x: device [n][3];
 * work: device, opm_krylov_bytes; report: HOST struct.  The call returns
 * once x and the report are final: the host reads the iteration state after
 * each chunk of iterations, and where the last solve's iteration count says
 * that the next chunk will be needed it is queued before that read.  A chunk
 * so queued may still be on the stream when the call returns (its kernels
 * find the solve done and change neither x nor work, which must stay
 * allocated until the stream has passed it, as for any queued work). */
int opm_bicgstab(const opm_problem* pb, const double* J, const void* ilu, int precision,
                 const double* b, double* x, double rtol, int32_t maxit, void* work,
                 opm_solve_report* report, void* stream);

/* Size in bytes of the GMRes workspace (device) for a restart length in
 * 1..OPM_GMRES_MAX_RESTART (0 for an invalid one): restart + 1 basis
 * vectors, their restart preconditioned images, one more vector and the
 * reduction partials. */
size_t opm_gmres_bytes(const opm_problem* pb, int32_t restart);

/* Restarted GMRes(restart), right preconditioned by the ILU(0) (or block
 * ILU0) factors in ilu (sec. 2.3.1 names GMRes as the alternative to
 * BiCGStab).  x0 = 0; every cycle restarts from the true residual
 * b - A x; orthogonalisation is classical Gram-Schmidt applied twice; the
 * Hessenberg least-squares problem is reduced with Givens rotations; the
 * update of a cycle is Z y with z_j = M^{-1} v_j kept from the iterations
 * (for a linear M equal to M^{-1} V y; with FP32 factors it keeps the
 * iterate consistent with the minimised residual).  Stops
 * when the residual norm of the iterate (the rotated right-hand side, or the
 * true residual at a cycle start) is <= rtol ||b||_2, after maxit
 * iterations (OPM_ENOTCONV in the report), or on an exact breakdown (a
 * singular triangular factor: OPM_EBREAKDOWN, x keeps the previous cycles).
 * b, x: device [n][3] (x is overwritten); work: device, opm_gmres_bytes;
 * report: HOST (its = inner iterations, rel_res = the residual estimate
 * above / ||b||); the call synchronises the stream a few times per cycle.
 * Returns OPM_EINVAL for a bad argument or restart outside
 * 1..OPM_GMRES_MAX_RESTART, OPM_EHIP on a runtime failure, else OPM_OK
 * (the solver's own outcome is report->status). */
int opm_gmres(const opm_problem* pb, const double* J, const void* ilu, int precision,
              const double* b, double* x, double rtol, int32_t maxit, int32_t restart, void* work,
              opm_solve_report* report, void* stream);

/* Newton options (sec. 2.3). */
typedef struct opm_newton_opts {
  double tol_cnv;      /* converged when max CNV <= tol_cnv ...             */
  double tol_mb;       /* ... and max MB <= tol_mb                          */
  double ds_max;       /* Appleyard chop: largest saturation change         */
  double dp_max_rel;   /* Appleyard chop: largest |dp| / |p|                */
  double lin_rtol;     /* Krylov relative tolerance                         */
  int32_t max_newton;  /* linear solves allowed per time step               */
  int32_t lin_maxit;   /* Krylov iteration cap                              */
  int32_t precision;   /* OPM_PREC_FP64 or OPM_PREC_MIXED                   */
  int32_t max_cuts;    /* time-step halvings per report step (opm_advance)  */
  int32_t krylov;      /* OPM_KRYLOV_BICGSTAB or OPM_KRYLOV_GMRES           */
  int32_t restart;     /* GMRes restart length (1..OPM_GMRES_MAX_RESTART)   */
  int32_t precond;     /* OPM_PRECOND_ILU0 or OPM_PRECOND_CPR (BiCGStab)    */
  int32_t pad;
} opm_newton_opts;

/* CPR-AMG preconditioner (sec. 2.3.1, the two-stage CPR preconditioner):
 * stage 1 solves the quasi-IMPES pressure system approximately by one
 * V(1,1) cycle of the aggregation AMG of opm_problem.amg (damped Jacobi,
 * omega = 2/3; the coarsest level by its inverse), stage 2 applies the
 * (block-)ILU(0) of the whole system to what is left:
 *   w_i: D_i^T w_i = e_p (D_i the diagonal block of row i);
 *   (A_p)_ij = w_i^T A_ij e_p; coarse levels A_{l+1} = P_l^T A_l P_l;
 *   z = x1 + M_ILU^{-1} (r - A x1), x1 = e_p V(A_p, w^T r).
 * All buffers are device memory; the workspace cpr holds opm_cpr_bytes
 * bytes and is owned by the caller.  Every call needs pb->amg (OPM_EINVAL
 * without); nothing is allocated. */
size_t opm_cpr_bytes(const opm_problem* pb);
/* Weights, pressure matrices and coarsest inverse for the Jacobian J
 * ([nnzb][3][3]); *status (device) is set to OPM_ESINGULAR on a singular
 * diagonal block or coarsest matrix and left alone otherwise. */
int opm_cpr_setup(const opm_problem* pb, const double* J, void* cpr, int32_t* status,
                  void* stream);
/* x = V(1,1)-cycle approximation of A_p^{-1} b (b, x: [n_cells]). */
int opm_cpr_vcycle(const opm_problem* pb, const void* cpr, const double* b, double* x,
                   void* stream);
/* z = CPR(r) (r, z: [n_cells][3], distinct) with the ILU(0) factors ilu of
 * the same J in the given precision. */
int opm_cpr_apply(const opm_problem* pb, const double* J, const void* ilu, int precision,
                  const void* cpr, const double* r, double* z, void* stream);
/* Copies out level `level`'s matrix values (a: [amg->nnz[level]], the
 * level's CSR order; level 0 on the block pattern) and the weights (w:
 * [n_cells][3]); either may be NULL. */
int opm_cpr_values(const opm_problem* pb, const void* cpr, int32_t level, double* a,
                   double* w, void* stream);
/* opm_bicgstab with CPR (set up for J) as the preconditioner. */
int opm_bicgstab_cpr(const opm_problem* pb, const double* J, const void* ilu, int precision,
                     const void* cpr, const double* b, double* x, double rtol, int32_t maxit,
                     void* work, opm_solve_report* report, void* stream);

/* Report of one time step (or of one report step for opm_advance). */
typedef struct opm_newton_report {
  int32_t status;
  int32_t newton_its;  /* linear solves                                     */
  int32_t lin_its;     /* Krylov iterations (BiCGStab half ones round up)   */
  int32_t substeps;    /* accepted substeps (opm_advance)                   */
  int32_t cuts;        /* time-step halvings (opm_advance)                  */
  int32_t pad;
  double cnv[3], mb[3];
  double cell_newton_its;   /* sum over Newton iterations of n_cells        */
  double t_assemble, t_factor, t_krylov, t_update;   /* s, HIP events     */
} opm_newton_report;

/* Size in bytes of the device workspace of opm_assemble_wells (0 without
 * standard wells). */
size_t opm_wells_bytes(const opm_problem* pb);

/* The coupled linearization with standard wells (sec. 2.2.1, eq.
 * wellequation): the reservoir residual R [n][3] and Jacobian J
 * [nnzb][3][3] as opm_assemble (the connection terms now from the well
 * unknowns in pb->well_state), the well residuals Rw [n_wells][4] (water,
 * oil, gas conservation with wellbore storage relative to the well state
 * well_state0 at the start of the step, then the control), and the coupling
 * blocks B [n_conns][4][3] = dRw/d(cell variables of the connection), C
 * [n_conns][3][4] = d(cell residual)/d(well unknowns), D [n_wells][4][4] =
 * dRw/d(well unknowns).  All device; work: opm_wells_bytes.  Synchronises;
 * OPM_ESINGULAR when a D is singular, OPM_EINVAL without standard wells. */
int opm_assemble_wells(const opm_problem* pb, const double* y, const double* acc0,
                       const double* well_state0, double dt, double* R, double* J, double* Rw,
                       double* B, double* C, double* D, void* work, void* stream);

/* Size in bytes of the Newton workspace (device) for a precision, with
 * BiCGStab as the linear solver. */
size_t opm_newton_bytes(const opm_problem* pb, int precision);

/* Size in bytes of the Newton workspace (device) for these options (their
 * precision, Krylov method and restart length); 0 for invalid options.
 * Equal to opm_newton_bytes for BiCGStab. */
size_t opm_newton_work_bytes(const opm_problem* pb, const opm_newton_opts* opts);

/* One implicit Euler step of length dt (sec. 2.3): Newton iterations from
 * the guess in y (device [n][3], in/out) with y_prev the state at the start
 * of the step (with live oil, pb->meaning at entry describes both y_prev
 * and y, and is updated by the variable switch after each Newton update),
 * each one assemble -> convergence test -> ILU(0) ->
 * BiCGStab (or GMRes) -> Appleyard-chopped update, at most max_newton
 * linear solves.
 * No time-step cutting (opm_advance does that).  work: device,
 * opm_newton_bytes.  report: HOST; the call synchronises the stream once per
 * Newton iteration (convergence test) and a few times per linear solve.
 * With opts->krylov = OPM_KRYLOV_GMRES, work must hold
 * opm_newton_work_bytes.  With standard wells (pb->n_wells > 0) each
 * iteration also assembles the well equations, solves the reservoir system
 * with the chosen Krylov method on the Schur complement (A - sum C D^-1 B)
 * (the preconditioner built from A alone), recovers the well update and
 * updates pb->well_state (|dp_bhp| <= dp_max_rel p_bhp, the fraction pair
 * scaled to ds_max and kept in [0, 1]) and, with limits, pb->well_ctrl;
 * convergence also requires every well's component residuals
 * (dt |R_a,w| / (b_a(p_bhp) PV_perforated)) and its control residual
 * relative to its active target to be below tol_cnv.  pb->well_state at entry is the state at the start of the
 * step (its wellbore storage). */
int opm_newton_step(const opm_problem* pb, double* y, const double* y_prev, double dt,
                    const opm_newton_opts* opts, void* work, opm_newton_report* report,
                    void* stream);

/* Advance y (device, in/out) over a report step of length dt: substeps with
 * halving on failure (sec. 2.3 time-step cutting), at most max_cuts halvings;
 * after a cut the shorter substep length is kept for the rest of the report
 * step.  y_save: device [n][3] scratch for the last accepted state; with
 * live oil the variable meanings (pb->meaning), with standard wells the well
 * state (pb->well_state), are saved and restored with it, in the Newton
 * workspace. */
int opm_advance(const opm_problem* pb, double* y, double dt, const opm_newton_opts* opts,
                void* work, double* y_save, opm_newton_report* report, void* stream);

/* ------------------------------------------------------ batched ensemble --
 * Many independent members (each a complete opm_problem of its own grid,
 * rock and wells) advanced over n_steps report steps of length dt_report in
 * one launch of a persistent kernel: one workgroup per member runs that
 * member's time loop (substeps halved on failure, at most max_cuts
 * halvings per report step), Newton iterations (sec. 2.3), assembly
 * (sec. 2.1.1, 2.4), block ILU(0) and BiCGStab (sec. 2.3.1) entirely on the
 * device.  Members never wait for each other.  The launch reads only device
 * memory prepared by opm_ensemble_prepare, so it can be captured in a graph. */
typedef struct opm_ensemble_report {
  int32_t status;      /* OPM_OK, or the code of the step that failed      */
  int32_t newton_its;  /* linear solves over all substeps                  */
  int32_t lin_its;     /* BiCGStab iterations                              */
  int32_t substeps;    /* accepted substeps                                */
  int32_t cuts;        /* time-step halvings                               */
  int32_t steps_done;  /* report steps completed                           */
  double cell_newton_its;
  double cnv[3], mb[3];   /* norms of the last Newton iteration           */
} opm_ensemble_report;

/* Device workspace of an ensemble (bytes); members: host array [n_members]
 * of problems whose pointers are device memory. */
size_t opm_ensemble_bytes(const opm_problem* members, int32_t n_members, int precision);

/* Lay out the workspace (device, opm_ensemble_bytes) for the members and
 * their states y[m] (host array of device pointers [n_cells_m][3], updated in
 * place by the launches).  Host, synchronous (copies a member table to the
 * device).  OPM_EINVAL if the widest ILU(0) level of a member does not fit
 * the kernel's LDS window, or if a member's fluid is live oil (the ensemble
 * kernel is dead oil only). */
int opm_ensemble_prepare(const opm_problem* members, double* const* y, int32_t n_members,
                         int precision, void* work, size_t work_bytes);

/* One asynchronous launch advancing every member by n_steps report steps.
 * max_level: the largest max_level of the members; reports: device
 * [n_members].  opts->precision is ignored (the workspace's precision is
 * passed explicitly); opts->krylov must be OPM_KRYLOV_BICGSTAB (else
 * OPM_EINVAL): the members' solver is BiCGStab. */
int opm_ensemble_launch(const void* work, int32_t n_members, int precision, int32_t max_level,
                        double dt_report, int32_t n_steps, const opm_newton_opts* opts,
                        opm_ensemble_report* reports, void* stream);

/* ------------------------------------------- learned Newton initial guess --
 * Newton starts each time step from the previous state (sec. 2.3).  These
 * calls add a learned start: a three-layer 3-D convolutional network
 * (3x3x3 kernels, 16 channels, zero padding at the box faces, ReLU after
 * layers 1 and 2) on the nx*ny*nz box of the grid predicts the change of
 * (p, s_w, s_g) over one report step from the two last states, the
 * log-permeability and the well terms of each cell: the last change
 * y_n - y_{n-1} (linear extrapolation, a skip connection kept in FP64) plus a
 * learned correction, applied away from wells: in cells whose 3x3x3 box
 * neighbourhood has no non-zero well channel in the features (equal report
 * steps are assumed).  The prediction is used
 * only when its max CNV (sec. 2.3) is below that of the previous state, and
 * the convergence test is unchanged, so a converged step meets the same
 * tolerances whichever start it took.
 *
 * Tensors of the network (device, caller-owned):
 *  - master: FP32 parameters, OPM_GUESS_PARAMS floats: for layer l = 0, 1, 2
 *    the weights W_l[27][16 out][16 in] followed by the bias b_l[16]; tap
 *    t = 9 (dz+1) + 3 (dy+1) + (dx+1) reads box cell (x+dx, y+dy, z+dz).
 *  - wbf16: BF16 copies of the weights (2 * 3 * 27*16*16 uint16; the forward
 *    layout [l][t][out][in], then the backward layout [l][t][in][out]),
 *    written by opm_guess_pack_weights.
 *  - activations: BF16 (uint16, round to nearest even) channels-last
 *    [box cell][16], box cell = x + nx (y + ny z), padded to a multiple of
 *    16 box cells; products accumulate in FP32.
 *  - features (layer-0 input) of an active cell: (p_n - 4800 psi)/1000 psi,
 *    s_w,n, s_g,n, the last change (p_n - p_{n-1})/100 psi,
 *    (s_w,n - s_w,n-1)/0.1, (s_g,n - s_g,n-1)/0.1, log10(k_h / 1 mD) - 2, the fixed
 *    injection rates of water, oil and gas per 10 m^3/day, and
 *    ln(1 + sum WI (p_n - p_bhp)^+ / 1 cP per 10 m^3/day) of producers;
 *    channels 11-15 and inactive box cells are zero.
 *  - output (layer 2, FP32): channels 0-2 correct the extrapolated step
 *    y_n - y_{n-1}, as dp / 100 psi, ds_w / 0.1 and ds_g / 0.1. */
#define OPM_GUESS_CHANNELS 16
#define OPM_GUESS_PARAMS (3 * (27 * 16 * 16 + 16))

typedef struct opm_guess_net {
  int32_t nx, ny, nz, pad;
  const int32_t* cell_box;   /* device [n_cells] (opm_topology.cell_box)      */
  const double* perm_h;      /* device [n_cells] horizontal permeability [m^2] */
  float* master;             /* device [OPM_GUESS_PARAMS]                      */
  void* wbf16;               /* device, see above                             */
} opm_guess_net;

/* BF16 operand copies of the master weights (device in, device out). */
int opm_guess_pack_weights(const float* master, void* wbf16, void* stream);

/* One convolution layer: out = conv(in, W) + b over the box; relu != 0
 * gives max(out, 0) in BF16 into out_bf16, else FP32 into out_f32.  in:
 * BF16 [box][16]; w_fwd: BF16 [27][16 out][16 in] of that layer. */
int opm_guess_conv(int32_t nx, int32_t ny, int32_t nz, const void* in, const void* w_fwd,
                   const float* bias, int32_t relu, void* out_bf16, float* out_f32,
                   void* stream);

/* Workspace (bytes) of opm_guess_conv_backward. */
size_t opm_guess_conv_backward_bytes(int32_t nx, int32_t ny, int32_t nz);

/* Backward of one layer: grad (device FP32 [27*16*16 + 16], overwritten) =
 * dL/dW in [t][out][in] order then dL/db, from the layer input `in` and
 * dout = dL/d(pre-activation output) (both BF16 [box][16]).  If din is not
 * NULL it receives dL/d(pre-activation input) in BF16: the transposed
 * convolution of dout with w_bwd (BF16 [27][16 in][16 out]) where
 * act_in > 0, else 0.  The sums over cells run in a fixed order. */
int opm_guess_conv_backward(int32_t nx, int32_t ny, int32_t nz, const void* in, const void* dout,
                            const void* w_bwd, const void* act_in, void* din, float* grad,
                            void* work, size_t work_bytes, void* stream);

/* Layer-0 input (BF16 [box][16], all of it written) from y_n and y_{n-1}. */
int opm_guess_features(const opm_problem* pb, const opm_guess_net* net, const double* y_n,
                       const double* y_nm1, void* feats, void* stream);

/* Workspace (bytes) of opm_guess_infer / opm_guess_train_step; 0 if the
 * problem or the network is invalid. */
size_t opm_guess_work_bytes(const opm_problem* pb, const opm_guess_net* net);

/* y_guess (device [n][3]) = y_n + (y_n - y_{n-1}) + the network's
 * correction (output channels 0-2 scaled back: dp = 100 psi * out_0,
 * ds = 0.1 * out_1,2), the correction used only away from wells (see above)
 * and only where finite; s_w and s_g clamped to [0, 1] and s_g
 * lowered so that s_w + s_g <= 1. */
int opm_guess_infer(const opm_problem* pb, const opm_guess_net* net, const double* y_n,
                    const double* y_nm1, double* y_guess, void* work, void* stream);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8; step >= 1) on
 * loss = sum over active cells away from wells and the three outputs of
 * (output - target)^2, divided by 3 n_cells, where target is the
 * scaled correction of the step to the extrapolated one:
 * d = (y_next - y_n) - (y_n - y_{n-1}), target = (d_p / 100 psi,
 * d_sw / 0.1, d_sg / 0.1).  Updates master, adam_m, adam_v (device FP32
 * [OPM_GUESS_PARAMS]) and wbf16; loss: device double, the loss before the
 * step. */
int opm_guess_train_step(const opm_problem* pb, const opm_guess_net* net, const double* y_n,
                         const double* y_nm1, const double* y_next, float* adam_m, float* adam_v,
                         int32_t step, float lr, double* loss, void* work, void* stream);

/* Choice of the Newton start: assembles at y_prev and at y_guess (both
 * against the accumulation of y_prev over dt) and copies into y the one
 * with the lower max CNV (y_prev on ties; a guess with a non-finite norm is
 * never taken).  work: the
 * Newton workspace (opm_newton_bytes, any precision).  chosen (host): 1 if
 * y_guess was taken; cnv (host [2]): max CNV at y_prev and at y_guess.
 * Synchronises the stream.  Dead oil only (OPM_EINVAL for live oil). */
int opm_guess_select(const opm_problem* pb, double* y, const double* y_prev,
                     const double* y_guess, double dt, void* work, int32_t* chosen, double* cnv,
                     void* stream);

/* opm_advance whose first attempt at the full report step starts from the
 * best of three (lowest max CNV against the accumulation of the previous
 * state, earlier ones winning ties): the previous state, the learned guess
 * (opm_guess_infer from y and y_nm1), the extrapolation y_n + (y_n - y_{n-1})
 * alone (the guess without its learned correction); every substep after a
 * cut starts from the previous state.  net may be NULL (then it is
 * opm_advance).  guess_work: opm_guess_work_bytes; y_guess: device [n][3]
 * scratch; guess_used (host): 0 previous state, 1 learned guess,
 * 2 extrapolation.  With a net, dead oil only (OPM_EINVAL for live oil). */
int opm_advance_guess(const opm_problem* pb, double* y, const double* y_nm1, double dt,
                      const opm_newton_opts* opts, const opm_guess_net* net, void* guess_work,
                      double* y_guess, void* work, double* y_save, opm_newton_report* report,
                      int32_t* guess_used, void* stream);

/* Launch shape of the ensemble kernel: the schedule knobs that the
 * autotuner chooses.  threads: workgroup size (128 or 256);
 * fac_window: keep the previous level's ILU(0) pivots in LDS during the
 * factorisation (allowed when every member has at most 640 rows per level);
 * ring: members whose LDS ring (the values of the last sweep_span +
 * max_level + 1 rows, rounded up to a power of two) fits sweep through the
 * ring, the others through the two-level LDS window; sweep_bytes: out, the
 * sweep storage of a launch (set by opm_ensemble_default_config and
 * opm_ensemble_configure); wgs: 0 one workgroup per member, else (in) the
 * workgroups of the launch (at least n_members, at most 2048, ring 0):
 * members built with a block-ILU0 topology (opm_topology_build_blocks) get
 * workgroups in proportion to their rows, at most one per subdomain, each
 * owning a contiguous range of the member's subdomains (its rows in
 * assembly, vector operations and SpMV, its subdomains in the factorisation
 * and sweeps), the member's workgroups meeting at device-memory barriers
 * for halo reads and reductions; out, the workgroups configured.  Every
 * workgroup of such a launch must be resident at once (checked against the
 * device's occupancy: OPM_EINVAL otherwise); a barrier that waits too long
 * fails the member with OPM_EHIP instead of hanging. */
typedef struct opm_ensemble_config {
  int32_t threads, fac_window, ring, sweep_bytes, wgs;
} opm_ensemble_config;

/* The shape opm_ensemble_launch uses (256 threads, factor window when
 * allowed, window sweeps); host. */
int opm_ensemble_default_config(const opm_problem* members, int32_t n_members, int precision,
                                opm_ensemble_config* cfg);

/* Apply a shape to a prepared workspace: writes each member's sweep choice
 * into the device table and fills cfg->sweep_bytes.  Host, synchronous.
 * OPM_EINVAL if the shape is invalid or does not fit in LDS. */
int opm_ensemble_configure(const opm_problem* members, int32_t n_members, int precision,
                           void* work, opm_ensemble_config* cfg);

/* opm_ensemble_launch with the shape last passed to opm_ensemble_configure
 * (asynchronous, capturable like opm_ensemble_launch). */
int opm_ensemble_launch_config(const void* work, int32_t n_members, int precision,
                               int32_t max_level, const opm_ensemble_config* cfg,
                               double dt_report, int32_t n_steps, const opm_newton_opts* opts,
                               opm_ensemble_report* reports, void* stream);

/* Autotuner: times one report step of length dt_report of the whole
 * ensemble for every valid shape (threads 256/128 x ring off/on x factor
 * window on/off, and with members that have subdomains also as many
 * workgroups as the device has compute units), restoring the members' states before each trial and at
 * the end, then configures the workspace with the fastest shape among the
 * trials in which every member completed the step (status OPM_OK) and
 * returns it in best; OPM_ENOTCONV (the workspace keeps the last trial's shape) if no trial
 * completed.  seconds (host, optional, >= 16 entries) receives the trial
 * times in trial order, n_tried (host, optional) their number.  Host,
 * synchronous; results of later launches do not depend on the shape beyond
 * the order of summation in reductions. */
int opm_ensemble_autotune(const opm_problem* members, int32_t n_members, int precision,
                          void* work, double dt_report, const opm_newton_opts* opts,
                          opm_ensemble_config* best, double* seconds, int32_t* n_tried,
                          void* stream);

/* Process-wide tuning knobs (host, synchronous); they change speed, never
 * results beyond round-off.  Returns OPM_OK, or OPM_EINVAL for an unknown
 * option or value.
 *   OPM_OPT_SWEEP_MODE: ILU(0) factor/sweep launch shape: -1 automatic,
 *     0 one workgroup walks all levels, 1 one launch per level, 2 (block
 *     ILU0 topologies; else automatic) one workgroup per subdomain, also
 *     for a single subdomain.  Automatic picks 2 for a block ILU0 topology
 *     of two or more subdomains whose subdomain vector fits in LDS.
 *   OPM_OPT_KRYLOV_CHUNK: BiCGStab iterations enqueued between reads of the
 *     convergence state (0 automatic, else >= 1).
 *   OPM_OPT_SWEEP_KERNEL: the one-workgroup LDS-ring sweep: 0 automatic,
 *     1 right-hand side gathered inside the sweep, 2-6 right-hand side
 *     gathered into level order first and branch-free prefetch with 512,
 *     256 or 128 threads (2, 3, 4) or with wavefronts that have no row in a
 *     level skipping their loads (5: 512, 6: 256 threads).
 *   OPM_OPT_BLOCK_DEPTH: block-ILU0 sweeps, levels whose data is loaded
 *     while a level is computed: 0 automatic (2 for the sweeps fused with
 *     BiCGStab, and for the others on a system of 256 or more subdomains;
 *     else 1), 1 or 2.
 *   OPM_OPT_KRYLOV_GRAPH: 1 (default) replays each chunk of BiCGStab
 *     iterations after the first chunk of a solve as a HIP graph captured
 *     once per set of arguments (kept until the process ends, at most 16),
 *     0 enqueues the kernels one by one.
 *   OPM_OPT_ASSEMBLY: 1 (default) the LDS-tiled assembly where the problem
 *     allows it (box_cell set, dead oil, fixed-source wells), 0 always the
 *     row-per-lane assembly.
 *   OPM_OPT_PLANE_SWEEP: factorisation and sweeps of the ILU(0) of a large
 *     system (sweep mode 1): 1 (default) plane-pipelined where box_cell and
 *     cell_box are set (one workgroup per z-plane), 0 one launch per level.
 *   OPM_OPT_PLANE_SPIN: re-reads a plane sweep makes of a value of the
 *     neighbouring plane that is not yet written before it gives up
 *     (default 262144; 0 gives up at once, to exercise the failure path): a
 *     sweep that gives up returns NaN, so the Krylov solver reports
 *     non-finite values instead of hanging.
 *   OPM_OPT_ENSEMBLE_SPIN: polls a member barrier of an ensemble launch
 *     with several workgroups per member makes before it gives up (default
 *     4194304; 0 gives up at once, to exercise the failure path): the
 *     member then reports OPM_EHIP. */
#define OPM_OPT_SWEEP_MODE 1
#define OPM_OPT_KRYLOV_CHUNK 2
#define OPM_OPT_SWEEP_KERNEL 3
#define OPM_OPT_BLOCK_DEPTH 4
#define OPM_OPT_KRYLOV_GRAPH 5
#define OPM_OPT_ASSEMBLY 6
#define OPM_OPT_PLANE_SWEEP 7
#define OPM_OPT_PLANE_SPIN 8
#define OPM_OPT_ENSEMBLE_SPIN 9
int opm_set_option(int option, int value);

const char* opm_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif
