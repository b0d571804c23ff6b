/*
 * htr.h -- C interface of the MI355X (gfx950) library for the explicit
 * right-hand side of the compressible multicomponent reacting Navier-Stokes
 * equations on structured periodic grids, and its SSP-RK3 time step.
 *
 * Paper: Maeda et al., "An integrated heterogeneous computing framework for
 * ensemble simulations of laser-induced ignition", arXiv 2202.02319.
 *   - conserved state, fluxes, sources: Methods › Solver, eqs. (1)-(3); closure eq. (4)
 *   - transport: Wilke viscosity, heat flux eq. (5), diffusion velocity
 *     eq. (6) with mixture-averaged (Bird) and binary (Hirschfelder) D
 *   - chemistry: finite-rate reversible Arrhenius reactions (Methods › Solver)
 *   - discretisation: conservative finite differences with TENO6 / central
 *     convective fluxes, second-order central diffusive fluxes, SSP-RK3
 *     (Methods › Numerical method); grid metrics of the mapped equations
 *     (Methods › Numerical method) in their rectilinear form
 *   - laser energy source q_L: Methods › Diffusion flame › Physical model and numerical setup, eq. (laser-qs)
 *
 * Conventions shared by every entry point
 *   - Units are SI.  All floating-point data are IEEE double.
 *   - A state U is stored variable-major: U[v][k][j][i] with i fastest,
 *     v = 0..ns-1 the partial densities rho*Y_s, then rho*u, rho*v, rho*w,
 *     then the total energy E (which includes the species enthalpies of
 *     formation).  nv = ns + 4.  N = nx*ny*nz cells.
 *   - Every pointer named *_dev, and every state / field pointer of the
 *     compute calls (U, T_io, dUdt, work, ...), is DEVICE memory on the
 *     device current at htr_create; descriptor pointers of htr_create are
 *     HOST memory and are copied.
 *   - `stream` is a hipStream_t passed as void*; NULL means the default
 *     stream.  Compute calls are asynchronous: they validate their
 *     arguments synchronously (returning HTR_EINVAL before any launch) and
 *     then only enqueue work.  They never allocate device memory.
 *   - Device-side numerical failures (non-finite state, rho <= 0, Newton
 *     not converged, T outside [Tmin, Tmax]) are latched in a status word
 *     owned by the context and reported by htr_check.
 *   - The library never throws across this interface and never exits.
 *   - Boundaries are periodic in every direction; an axis with n = 1 is
 *     inactive (no flux), which gives 1-D and 2-D problems.
 *   - Calls on one context that overlap in time (different streams without
 *     ordering) race on the context's internal buffers.
 */
#ifndef HTR_H
#define HTR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HTR_OK = 0,
  HTR_EINVAL = 1,        /* bad argument (null, size, range)                 */
  HTR_ENOMEM = 2,        /* device allocation failed (htr_create only)       */
  HTR_EDEVICE = 3,       /* HIP runtime error                                */
  HTR_ENONFINITE = 4,    /* non-finite state or rho <= 0 met on the device   */
  HTR_ENEWTON = 5,       /* temperature Newton iteration did not converge    */
  HTR_ETRANGE = 6,       /* temperature left [Tmin, Tmax]                    */
  HTR_EUNSUPPORTED = 7   /* valid but not supported (e.g. ns > HTR_MAX_NS)   */
} htr_status;

#define HTR_MAX_NS 12          /* species per mechanism                      */
#define HTR_MAX_NR 64          /* reactions per mechanism                    */
#define HTR_MAX_SIDE 3         /* distinct species on one side of a reaction */

/* scheme flags */
#define HTR_CHEM_OFF      1u   /* no chemical source (the paper's inert stage, Methods › Model rocket combustor › Physical model) */
#define HTR_VISC_OFF      2u   /* no diffusive fluxes                                      */
#define HTR_FORCE_CENTRAL 4u   /* central flux on every face                               */
#define HTR_FORCE_TENO    8u   /* TENO6 on every face                                      */
#define HTR_WENO3Z       16u   /* WENO3-Z instead of TENO6 where the scheme captures shocks
                                  (Methods › Numerical method's alternative; no adjoint: HTR_EUNSUPPORTED)    */

/* boundary types of a non-periodic axis side (htr_set_boundaries) */
#define HTR_BC_PERIODIC 0
#define HTR_BC_WALL     1      /* no-slip, isothermal: u and T held at the node's values */
#define HTR_BC_INFLOW   2      /* velocity, temperature and composition held             */
#define HTR_BC_OUTFLOW  3      /* characteristic outflow relaxing p to p_inf             */

typedef struct htr_ctx htr_ctx;
typedef struct htr_batch htr_batch;

/* Mechanism tables (HOST pointers, copied by htr_create).  Methods › Solver. */
typedef struct {
  int32_t ns, nr;
  const double* W;          /* [ns] molar masses, kg/mol                           */
  const double* nasa7;      /* [ns][7] NASA 7-coefficient polynomial, one range    */
  const double* lj_sigma;   /* [ns] Lennard-Jones diameter, m                       */
  const double* lj_epsk;    /* [ns] Lennard-Jones well depth over k_B, K            */
  const double* lnA;        /* [nr] ln of the SI pre-exponential factor             */
  const double* beta;       /* [nr] temperature exponent                            */
  const double* Ea;         /* [nr] activation energy, J/mol                        */
  const int32_t* nu_f;      /* [nr][ns] reactant stoichiometric coefficients        */
  const int32_t* nu_r;      /* [nr][ns] product stoichiometric coefficients         */
  double Tmin, Tmax;        /* validity range of the polynomials, K                 */
} htr_mech_desc;

/* Rectilinear periodic grid (HOST pointers, copied).  For axis a:
 * xnode[a][i] node coordinate, xi_node[a][i] = d(xi)/dx at node i,
 * xi_face[a][i] = d(xi)/dx at face i+1/2, L[a] the period.  A uniform grid
 * has xi_node = xi_face = 1/dx.  For an inactive axis (n = 1) xi_node[0] is
 * 1/width (it enters the cell volume only). */
typedef struct {
  int32_t n[3];
  const double* xnode[3];
  const double* xi_node[3];
  const double* xi_face[3];
  double L[3];
} htr_grid_desc;

/* Gaussian laser kernel, eq. (laser-qs), generalised to d active axes:
 * q_L = E / ((2 pi)^((d+1)/2) sigma_r^d sigma_t) * prod_a G_a(x_a)
 *       * exp(-(t - t0)^2 / (2 sigma_t^2)),
 * G_a the Gaussian of width sigma_r wrapped over the periodic images. */
typedef struct {
  double E;
  double center[3];
  double sigma_r;
  double t0;
  double sigma_t;
  int32_t on;
} htr_laser;

typedef struct {
  double cfl;        /* CFL number of htr_stable_dt                       */
  double theta_c;    /* dilatation sensor threshold of the hybrid switch  */
  double psi_c;      /* relative pressure-jump threshold                  */
  double teno_CT;    /* TENO cut-off C_T                                  */
  uint32_t flags;    /* HTR_* scheme flags                                */
} htr_scheme;

/* Create a context for one mechanism, one grid and one scheme on the current
 * device; allocates the context's device tables and scratch.  *out is NULL on
 * failure.  Errors: HTR_EINVAL (null pointer, n < 1, ns < 1, metric <= 0,
 * bad stoichiometry), HTR_EUNSUPPORTED (ns > HTR_MAX_NS, nr > HTR_MAX_NR,
 * more than HTR_MAX_SIDE species or total order > 3 on a reaction side),
 * HTR_ENOMEM, HTR_EDEVICE. */
htr_status htr_create(const htr_mech_desc* mech, const htr_grid_desc* grid, const htr_scheme* scheme,
                      htr_ctx** out);

/* General curvilinear periodic grid (HOST pointers, copied), Methods › Numerical method: the
 * equations mapped to a uniform index space (spacing 1) with U~ = U/J and
 * F~_d = (d xi_d / d x) . (F, G, H) / J, J = det(d xi / d x).
 * xyz[3][N]: node coordinates x, y, z, node (i, j, k) at i + n0 (j + n1 k).
 * period[a][c]: displacement of the node lattice when index a advances by
 * n[a] (the image of node (i, j, k) n[a] cells further along a is at
 * xyz + period[a]).  An inactive axis (n = 1) must have its period along its
 * own coordinate, and the other periods no component along it. */
typedef struct {
  int32_t n[3];
  const double* xyz;
  double period[3][3];
} htr_curv_grid_desc;

/* Context on a curvilinear grid.  Metric terms are computed on the device
 * in the conservative (Thomas-Lombard) form with sixth-order central
 * differences, face values by the matching six-point interpolation, so a
 * uniform flow is preserved to rounding.  Every single-grid entry point
 * works on it (htr_rhs, htr_cells, htr_stable_dt, htr_rk3_step); the tape,
 * the adjoint and the tiling/autotune calls return HTR_EUNSUPPORTED.
 * The host arrays are copied; the context owns, besides the rectilinear
 * context's scratch, 22 N doubles of geometry (metric terms, face metric
 * terms, coordinates) and (10 ns + 36) N doubles of per-stage scratch.
 * Creation blocks: it runs the metric kernels and checks J on the host.
 * On such a grid the laser centre is a physical position, the Gaussian is
 * summed over the lattice images, and cell volumes (J objective) are 1/J.
 * Errors: HTR_EINVAL for NULL arguments, non-finite coordinates or periods,
 * an invalid lattice (see the descriptor) or a node where det(d x / d xi)
 * is not positive; these checks other than the last precede any device
 * work. */
htr_status htr_create_curvilinear(const htr_mech_desc* mech, const htr_curv_grid_desc* grid,
                                  const htr_scheme* scheme, htr_ctx** out);

/* Copies a curvilinear context's metric terms into caller DEVICE buffers:
 * mt[10][N] ((d xi_d / d x_c) / J at row 3d + c, J at row 9) and mf[9][N]
 * (the same at face i+1/2 along d).  Asynchronous on stream.  HTR_EINVAL on
 * a rectilinear context. */
htr_status htr_grid_metrics(htr_ctx* ctx, double* mt, double* mf, void* stream);
/* Waits for the work this context enqueued (an event recorded on every
 * stream an entry point was given; not the whole device) and frees it.
 * Work enqueued while the caller captured a stream into a graph is not
 * tracked: the caller synchronises its graph launches first.  NULL is
 * HTR_EINVAL. */
htr_status htr_destroy(htr_ctx* ctx);
/* Non-periodic boundaries of a rectilinear single-grid context (Methods ›
 * Diffusion flame › Physical model and numerical setup: characteristic
 * in/outflow boundaries after Poinsot & Lele and no-slip walls; Methods ›
 * Model rocket combustor › Numerical setup: isothermal walls).
 *   bc[a][side]     HOST, per axis a and side (0 low, 1 high): HTR_BC_*; an
 *                   axis is periodic on both sides or bounded on both
 *   pinf[a][side]   HOST, far-field pressure of an outflow side (Pa, > 0)
 *   relax[a][side]  HOST, relaxation coefficient sigma of an outflow side
 *                   (>= 0; K = sigma c (1 - M^2) / L_axis)
 * On a bounded axis the first and last nodes lie on the boundary (their
 * xnode are the boundary positions).  Faces whose six-point stencil does not
 * fit take the widest centred interpolation that does, or the local
 * Lax-Friedrichs (Rusanov) flux where the hybrid switch marks them; the
 * sensor and tangential derivatives are one-sided at boundary nodes.
 * Boundary nodes take the locally one-dimensional characteristic treatment:
 * an outflow's entering acoustic wave relaxes p to p_inf (entering entropy,
 * shear and species waves of a backflow are zero; zero normal gradient of
 * the diffusive fluxes); walls hold the node's velocity and temperature
 * (set them to the wall's in the state), its density following continuity
 * and its species diffusing with zero flux through the wall; inflows hold
 * velocity, temperature and composition.  A bounded axis needs n >= 8; the
 * laser sums no images across it.  Errors (before any device work):
 * HTR_EINVAL for NULL, mismatched sides, n < 8, bad types or outflow
 * parameters; HTR_EUNSUPPORTED on a curvilinear context.  Ensembles built
 * from the context, the tape and the adjoint calls return HTR_EUNSUPPORTED
 * once any axis is bounded.  All-periodic bc restores the periodic grid. */
htr_status htr_set_boundaries(htr_ctx* ctx, const int32_t bc[3][2], const double pinf[3][2],
                              const double relax[3][2]);

/* Replace the scheme flags of an existing context. */
htr_status htr_set_flags(htr_ctx* ctx, uint32_t flags);
/* Number of cells of the context's grid (0 for NULL). */
int64_t htr_num_cells(const htr_ctx* ctx);

/* Conserved state from primitive fields (eq. 4 for rho; E includes the
 * formation enthalpies): Y[ns][N], T[N], p[N], vel[3][N] -> U[nv][N]. */
htr_status htr_prim_to_cons(htr_ctx* ctx, const double* Y, const double* T, const double* p,
                            const double* vel, double* U, void* stream);

/* One right-hand side evaluation dUdt = L(U, t) (eqs. 1-3 in the mapped
 * conservative form of Methods › Numerical method): hybrid TENO6/central convective fluxes,
 * second-order diffusive fluxes, chemistry and laser sources.
 *   U      [nv][N] in
 *   T_io   [N] in/out: Newton starting guess in, converged T out
 *   dUdt   [nv][N] out
 *   hrr    [N] out, nullable: heat-release rate -sum_s h_s wdot_s (W/m^3)
 *   laser  HOST pointer, nullable (no laser) */
htr_status htr_rhs(htr_ctx* ctx, const double* U, double* T_io, double t, const htr_laser* laser, double* dUdt,
                   double* hrr, void* stream);

/* Per-cell derived quantities of the right-hand side, for inspection:
 * out[nq][N] with rows T, p, c, mu, lambda, D_s (ns rows), wdot_s (ns rows),
 * hrr, q_L, theta (the dilatation sensor); nq = 5 + 2 ns + 3. */
htr_status htr_cells(htr_ctx* ctx, const double* U, double* T_io, double t, const htr_laser* laser,
                     double* out, void* stream);

/* Stable step: dt = cfl * min over cells of the convective limit
 * 1 / sum_d (|u_d| + c) xi_d and, unless HTR_VISC_OFF, the diffusive limit
 * 1 / (2 sum_d xi_d^2 max(mu/rho, lambda/(rho c_p), max_s D_s)).
 * Writes one double to dt_dev (device). */
htr_status htr_stable_dt(htr_ctx* ctx, const double* U, double* T_io, double* dt_dev, void* stream);

/* Bytes of caller-owned work memory htr_rk3_step needs (two stage states). */
size_t htr_work_bytes(const htr_ctx* ctx);

/* One SSP-RK3 step in Shu-Osher form (Gottlieb et al. 2001, Methods › Numerical method):
 *   U1 = U + dt L(U, t); U2 = 3/4 U + 1/4 (U1 + dt L(U1, t+dt));
 *   U <- 1/3 U + 2/3 (U2 + dt L(U2, t+dt/2)).
 *   U          [nv][N] in/out (device)
 *   T_io       [N] in/out Newton guess cache (holds T of the last stage)
 *   t_dev      device double in/out: the time, advanced by dt at the end
 *   dt_dev     device double: the step; read, or, when compute_dt != 0,
 *              written first with the htr_stable_dt value of U (computed in
 *              the first stage's per-cell kernel, no extra pass)
 *   dlnA_dev   nullable device [nr]: offsets added to ln A for this call
 *   work       device, >= htr_work_bytes(ctx)
 *   J_dev      nullable device double: J += dt sum_k b_k sum_cells dV hrr(U^(k), t_k)
 *              with b = (1/6, 1/6, 2/3): the time-integrated heat release.
 * The host never waits inside a step. */
htr_status htr_rk3_step(htr_ctx* ctx, double* U, double* T_io, double* t_dev, double* dt_dev, int compute_dt,
                        const htr_laser* laser, const double* dlnA_dev, double* work, double* J_dev,
                        void* stream);

/* The step of htr_rk3_step without any allocation, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Arguments and results are those of
 * htr_rk3_step without `work`: the two stage states and the step's per-cell
 * scratch (derived fields, sources, sensor flags, velocity gradients,
 * partial right-hand side, block partials) live in one fixed device array
 * of HTR_NOALLOC_MAX_BYTES per GPU, held until the process ends.  The
 * context still owns its tables and status word (htr_check).  The call makes
 * no hipMalloc/hipFree and no allocating library call; it returns
 * HTR_EINVAL, before any device work, when the grid needs more than the
 * array holds: 8 N (3 (ns + 4) + (7 + ns) + (ns + 1) + 9) + N bytes plus
 * block partials and 256-byte alignment: about 113,000 cells at ns = 9 (48^3).
 * Every call on one GPU shares that GPU's array (also across contexts), so
 * calls that overlap on one GPU (different streams or threads) race; the
 * array keeps the last call's contents, and nothing in it needs clearing
 * (each step writes every region before reading it).  HTR_EINVAL also when
 * the current device is not the context's. */
#define HTR_NOALLOC_MAX_BYTES (64u << 20)
htr_status htr_rk3_step_noalloc(htr_ctx* ctx, double* U, double* T_io, double* t_dev, double* dt_dev,
                                int compute_dt, const htr_laser* laser, const double* dlnA_dev, double* J_dev,
                                void* stream);

/* Kernel timing for diagnostics: while enabled, every kernel the context
 * launches is bracketed by HIP events on its stream.  htr_timing_read
 * synchronises and returns, per kernel class (0 per-cell point kernel,
 * 1 sensor (on curvilinear grids with the mole fractions and index-space
 * differences), 2 convective flux sweep (curvilinear: face kernel),
 * 3 diffusive flux sweep with the stage update (curvilinear: face kernel),
 * 4 reductions and small kernels, 5 the curvilinear stage update), the
 * summed milliseconds and launch counts since htr_timing(ctx, 1).  ms and
 * launches are HOST arrays of HTR_TIMING_CLASSES entries. */
#define HTR_TIMING_CLASSES 6
htr_status htr_timing(htr_ctx* ctx, int enable);
htr_status htr_timing_read(htr_ctx* ctx, double* ms, int64_t* launches);

/* ------------------------------------------------------------------------
 * Discrete adjoint (reverse mode), for the time-integrated heat release
 * J = sum_steps dt sum_k b_k sum_cells dV HRR(U^(k), t_k) and the parameters
 * theta = (E, centre x, centre y, centre z, ln A_1 .. ln A_nr) of the laser
 * kernel (Methods › Diffusion flame › Physical model and numerical setup) and of the Arrhenius rates (Methods › Solver).  The paper
 * obtains sensitivities from ensembles of forward runs (Results › Ensemble simulation); this is the
 * reverse-mode alternative.  Discrete switches (hybrid sensor, TENO
 * cut-offs, argmax of the Lax-Friedrichs speed, Newton iteration count) are
 * frozen: the derivative is that of the scheme with those switches fixed,
 * which is the exact derivative wherever no switch flips.  The Newton
 * temperature is differentiated through its implicit definition.
 * ------------------------------------------------------------------------ */

/* Bytes of caller-owned scratch the adjoint calls need. */
size_t htr_adjoint_work_bytes(const htr_ctx* ctx);

/* Vector-Jacobian product of one right-hand side and of its heat release
 * H = sum_cells dV HRR, at state U and time t:
 *   Ubar_acc[nv][N] += s (dL/dU)^T lam + h dH/dU
 *   pbar_acc[4+nr]  += s (dL/dtheta)^T lam + h dH/dtheta
 * lam [nv][N] is a cotangent of dU/dt.  T_io is the Newton guess cache
 * (updated).  dlnA_dev (nullable) are the ln A offsets the forward used.
 * All arrays are device memory; adj_work >= htr_adjoint_work_bytes. */
htr_status htr_rhs_adjoint(htr_ctx* ctx, const double* U, double* T_io, double t, const htr_laser* laser,
                           const double* dlnA_dev, const double* lam, double s, double h, double* Ubar_acc,
                           double* pbar_acc, double* adj_work, void* stream);

/* Bytes of a forward tape of one step: per stage the per-cell fields
 * [7 + ns][N] and the temperature [N] (doubles), then per stage the sensor
 * flags [N], then per stage the TENO cut-off patterns [3][nv][N] (bytes: per
 * axis, variable and face, indexed by the face's upper cell). */
size_t htr_tape_bytes(const htr_ctx* ctx);
/* htr_rk3_step that also records its tape (device, >= htr_tape_bytes).
 * Rectilinear periodic grids of fewer than 2^31 cells; otherwise
 * HTR_EUNSUPPORTED. */
htr_status htr_rk3_step_taped(htr_ctx* ctx, double* U, double* T_io, double* t_dev, double* dt_dev, int compute_dt,
                              const htr_laser* laser, const double* dlnA_dev, double* work, double* J_dev,
                              void* tape, void* stream);

/* Adjoint of one htr_rk3_step taken with the fixed step dt from U^n at time
 * t (and contributing Jbar * its J increment).  Un is U^n; stages is the work
 * buffer as that htr_rk3_step left it (U1 then U2).  Ubar [nv][N] holds the
 * cotangent of U^{n+1} on entry and that of U^n on return; pbar_acc[4+nr]
 * accumulates the parameter cotangent.  tape (nullable) is the step's tape
 * from htr_rk3_step_taped: the stages' per-cell fields, temperatures, sensor
 * flags and TENO cut-off patterns are then taken from it instead of being
 * recomputed (T_io is then not used). */
htr_status htr_rk3_step_adjoint(htr_ctx* ctx, const double* Un, const double* stages, double* T_io, double t,
                                double dt, const htr_laser* laser, const double* dlnA_dev, double Jbar,
                                double* Ubar, double* pbar_acc, double* adj_work, const void* tape, void* stream);

/* ------------------------------------------------------------------------
 * Ensembles: many independent grids (members) sharing the context's
 * mechanism and scheme, advanced together (the paper's ensemble workflow,
 * Results › Ensemble simulation, and Application examples: samples with perturbed laser energy, position and
 * rates).  Member m owns cells [off_m, off_m + N_m) of packed arrays: a
 * [rows][N] field of the member starts at base + rows * off_m.  Each member
 * has its own uniform periodic grid, laser kernel, ln A offsets, time, step
 * and heat-release accumulator.  Every kernel of a batched call is ONE launch
 * covering the tiles of all members.
 * ------------------------------------------------------------------------ */
typedef struct {
  int32_t n[3];          /* member grid                                        */
  double dx[3];          /* uniform spacing (for an inactive axis: its width)  */
  htr_laser laser;       /* member's deposition kernel                         */
  const double* dlnA;    /* HOST [nr] ln A offsets of the member, nullable     */
} htr_member_desc;

/* Create an ensemble of nmem members on the context's mechanism and scheme.
 * Descriptors are HOST memory, copied.  Errors: HTR_EINVAL (nmem < 1, bad
 * member), HTR_ENOMEM, HTR_EDEVICE. */
htr_status htr_batch_create(htr_ctx* ctx, int32_t nmem, const htr_member_desc* members, htr_batch** out);
/* Waits for the ensemble's own work (as htr_destroy) and its graph replays,
 * then frees it.  The context must outlive its ensembles. */
htr_status htr_batch_destroy(htr_batch* b);
/* Total packed cells; if offsets (HOST, nmem + 1 entries) is non-NULL it
 * receives the member cell offsets (offsets[nmem] = total). */
int64_t htr_batch_cells(const htr_batch* b, int64_t* offsets);
/* Packed primitive fields Y[ns], T, p, vel[3] -> packed U (as htr_prim_to_cons). */
htr_status htr_batch_prim_to_cons(htr_batch* b, const double* Y, const double* T, const double* p,
                                  const double* vel, double* U, void* stream);
/* One right-hand side of every member at its own time t_dev[m] (device
 * [nmem]); packed U in, packed dUdt out, packed T_io in/out, hrr nullable. */
htr_status htr_rhs_batched(htr_batch* b, const double* U, double* T_io, const double* t_dev, double* dUdt,
                           double* hrr, void* stream);
size_t htr_batch_work_bytes(const htr_batch* b);
/* nsteps SSP-RK3 steps of every member (each with its own dt; with
 * compute_dt each member's dt is its own stable step, as htr_rk3_step).
 * t_dev, dt_dev, J_dev (nullable) are device [nmem].  With use_graph != 0
 * the nsteps steps are captured once into a HIP graph (re-captured when any
 * pointer argument, nsteps, compute_dt or the context's scheme (flags,
 * thresholds, CFL) changes) and replayed with one graph launch per call. */
htr_status htr_rk3_steps_batched(htr_batch* b, double* U, double* T_io, double* t_dev, double* dt_dev,
                                 int compute_dt, int nsteps, double* work, double* J_dev, int use_graph,
                                 void* stream);
/* As htr_check, for the ensemble's status word. */
htr_status htr_batch_check(htr_batch* b, void* stream);
/* Per member, the largest value of a packed per-cell field (device [Ntot],
 * member-major as the batch packs T_io) into max_dev[m] (device [nmem],
 * caller-owned); with accumulate != 0, max_dev[m] = max(max_dev[m], that),
 * so repeated calls track a running peak.  NaN entries are ignored by the
 * maximum (htr_batch_check reports non-finite states).  Asynchronous on
 * stream; HTR_EINVAL for NULL pointers.  For ensemble workflows such as the
 * ignition-energy search (Application examples › Ignition of a diffusion flame › Ensemble and data analysis: the minimum laser energy for ignition,
 * judged here by the peak temperature). */
htr_status htr_batch_member_max(htr_batch* b, const double* field, double* max_dev, int accumulate,
                                void* stream);

/* ------------------------------------------------------------------------
 * Tiles, persistent launches, autotuning.  The convective sweep works on
 * 256-cell tiles; any shape with extent 1 along inactive axes that its
 * staging buffers hold is accepted (16x4x4, 8x8x4, 8x4x8, 4x8x8 in 3-D;
 * 16x16, 32x8, 8x32, 64x4 in 2-D; 256 in 1-D).  The diffusive sweep works
 * on 192-cell tiles of a fixed shape (16x4x3 in 3-D, 16x12 in 2-D, 192 in
 * 1-D).  grid > 0 launches the forward
 * kernels (per-cell, sensor, both sweeps) as grid persistent blocks that
 * stride over their logical blocks; grid = 0 launches one block per
 * logical block.  Results are bitwise independent of both choices (every
 * face is evaluated once with the same arithmetic).  Changing the tiling
 * synchronises the device, and it discards an ensemble's captured graph.
 * ------------------------------------------------------------------------ */
/* HTR_OK if shape[3] is a valid tile for a grid of n[3] cells, else
 * HTR_EINVAL with the reason in htr_last_error.  Host only. */
htr_status htr_tile_shape_check(const int32_t n[3], const int32_t shape[3]);
/* Sets the tile shape (HOST [3]; NULL: the default) and persistent grid. */
htr_status htr_set_tiling(htr_ctx* ctx, const int32_t shape[3], int32_t grid);
htr_status htr_get_tiling(const htr_ctx* ctx, int32_t shape[3], int32_t* grid);
/* Times one RK3 stage (right-hand side and stage update, written to work,
 * >= htr_work_bytes) for every candidate shape and persistent grid (and, at
 * grid 0, convective split; see htr_set_conv_split), twice, and keeps the
 * fastest; writes the choice to shape_out[3] and grid_out
 * (both nullable).  U and T_io as for htr_rhs (T_io is refreshed); U is not
 * modified. */
htr_status htr_autotune(htr_ctx* ctx, const double* U, double* T_io, double* work, void* stream,
                        int32_t shape_out[3], int32_t* grid_out);
/* Ensemble: the shape of member m (m = -1: all members; shape NULL: their
 * defaults) and the batch's persistent grid. */
htr_status htr_batch_set_tiling(htr_batch* b, int32_t member, const int32_t shape[3], int32_t grid);
htr_status htr_batch_get_tiling(const htr_batch* b, int32_t member, int32_t shape[3], int32_t* grid);
/* Tunes the shape of each class of equal-size members (timed on a member
 * table holding only that class), then the batch's persistent grid and
 * convective split; work >= htr_batch_work_bytes.  Allocates and frees one
 * small device table. */
htr_status htr_batch_autotune(htr_batch* b, const double* U, double* T_io, double* work, void* stream);
/* The convective sweep at grid = 0 runs, by default (split = 1), as two
 * launches: a lean variant, with fewer registers and more waves per SIMD,
 * does the tiles none of whose faces takes the TENO path and marks the
 * others, which the full sweep then does; split = 0 runs every tile in the
 * full sweep.  Results are bitwise the same; htr_autotune and
 * htr_batch_autotune time both.  HTR_EINVAL for split outside {0, 1};
 * curvilinear contexts: HTR_EUNSUPPORTED.  Changing it discards an
 * ensemble's captured graph. */
htr_status htr_set_conv_split(htr_ctx* ctx, int32_t split);
htr_status htr_get_conv_split(const htr_ctx* ctx, int32_t* split);
htr_status htr_batch_set_conv_split(htr_batch* b, int32_t split);
htr_status htr_batch_get_conv_split(const htr_batch* b, int32_t* split);

/* Synchronises `stream`, returns the first device-side error latched since
 * the last htr_check (and clears it), or HTR_EDEVICE for a HIP error. */
htr_status htr_check(htr_ctx* ctx, void* stream);

/* Message of the last error returned on the calling thread. */
const char* htr_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* HTR_H */
