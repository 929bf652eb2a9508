/* csi.h -- C-ABI of the MI355X (gfx950) component-splitting implicit solver.
 *
 * The library computes one pseudo-time iteration of the implicit scheme of
 * the paper (Section 2.2, Eq. (linearizedimplicit), Eq. (implicitscheme),
 * Eq. (ijkiterate) and the LU-SGS forward/backward sweeps; Section 2.3, the
 * component-splitting method and its consistence corrections) for the 2D
 * multicomponent reacting Navier-Stokes equations (Section 2.1, Eq. (govern),
 * Eq. (flux)) on a structured grid, with hand-written HIP kernels.
 *
 * Conventions
 *  - Every call returns an int status: CSI_OK (0) or a negative CSI_ERR_*.
 *    csi_last_error() gives the text of the last error on that context.
 *  - Host pointers are owned by the caller and copied on entry.  Device
 *    pointers (workspace, state with on_device=1, surrogate buffers) are owned
 *    by the caller; the library never allocates device memory.
 *  - All work is enqueued on the HIP stream given to csi_create; calls that
 *    return host data synchronise that stream.
 *  - Stored state q is FP64 structure-of-arrays [nv][nj][ni] (i fastest),
 *    q = (rho_1..rho_ns, rho u, rho v, rho E, [rho e_ve]),
 *    nv = ns + 3 (one temperature) or ns + 4 (two temperatures).
 *  - Increments: coupled [nb][N] in z = (rho, rho u, rho v, rho E, [rho e_ve],
 *    rho_1..rho_{ns-1}), nb = nf + ns - 1; split [nf + ns][N] =
 *    (rho, rho u, rho v, rho E, [rho e_ve] | rho_1..rho_ns); nf = 4 or 5.
 *  - Call order: create -> set_grid -> set_mechanism -> set_freestream ->
 *    workspace_bytes -> bind_workspace -> set_state -> residual /
 *    implicit_op / consistency_correct / step.  set_grid or set_mechanism
 *    after binding invalidates the binding (CSI_ERR_STATE until rebound).
 */
#ifndef CSI_H
#define CSI_H
#include <stddef.h>
#ifdef __cplusplus
extern "C" {
#endif

enum {
  CSI_OK = 0,
  CSI_ERR_ARG = -1,       /* invalid argument or size */
  CSI_ERR_STATE = -2,     /* call out of order / workspace not bound */
  CSI_ERR_HIP = -3,       /* HIP runtime error */
  CSI_ERR_NONFINITE = -4, /* non-physical or non-finite state; cell index in stats / csi_bad_cell */
  CSI_ERR_SINGULAR = -5,  /* zero pivot in a diagonal block */
  CSI_ERR_UNSUPPORTED = -6 /* species count / temperature model / feature without kernels for it */
};
enum { CSI_COUPLED = 0, CSI_SPLIT = 1 };
enum { CSI_FP64 = 0, CSI_MIXED = 1 }; /* MIXED: FP32 blocks and sweeps; FP64 residual, chemistry, corrections */
enum { CSI_CLOSURE = 0, CSI_CC1 = 1, CSI_CC2 = 2 };
enum { CSI_JAC_EXACT = 0, CSI_JAC_SURROGATE = 1 };

typedef struct csi_ctx csi_ctx;

/* Mechanism tables (host, copied).  Species kinds: 0 atom / atomic ion,
 * 1 linear molecule / molecular ion, 2 electron.  Arrhenius A in SI units,
 * k_f = A Tf^b exp(-theta/Tf) with Tf = T, sqrt(T Tv) or Tv (tctl 0/1/2);
 * backward rates from equilibrium constants of the species' Gibbs energies.
 * Limits: ns <= 32, nr <= 64, at most three reactant and three product
 * molecules per reaction. */
typedef struct {
  int ns, nr, two_temp;
  const double *M, *theta_v, *theta_r, *sigma, *g_el, *h_form, *sc, *lt_a, *lt_b; /* [ns] */
  const int *kind;                                                              /* [ns] */
  const double *A, *b, *theta;                                                  /* [nr] */
  const int *tctl, *third;                                                      /* [nr] */
  const int *nu_f, *nu_b;                                                       /* [nr*ns] */
  const double *eff;                                                            /* [nr*ns] */
  double mu_ref, T_ref, mu_exp;
} csi_mechanism;

typedef struct {
  int mode;        /* CSI_COUPLED or CSI_SPLIT */
  int precision;   /* CSI_FP64 or CSI_MIXED */
  int kind;        /* CSI_CLOSURE (coupled), CSI_CC1 or CSI_CC2 (split) */
  int jac;         /* CSI_JAC_EXACT or CSI_JAC_SURROGATE */
  double cfl;      /* target CFL */
  int cfl_ramp;    /* geometric ramp from 1 to cfl over this many iterations (0: none) */
  int max_iter;    /* iterations to run */
  double tol;      /* stop once r_rho / r_rho(iteration 0) <= tol (<= 0: run max_iter) */
  int check_every; /* iterations between host checks of the stop / error flags */
} csi_step_params;

typedef struct {
  int iters;       /* iterations run by this call */
  int converged;   /* 1 if the tolerance was reached (iteration index in it_conv) */
  int it_conv;
  int n_clipped;   /* cells with a clipped partial density */
  int bad_cell;    /* first non-physical cell, or -1 */
  double r0, r_last;
  long long n_dd_fallback; /* cell-iterations whose surrogate block failed the dominance check (exact used) */
  int surrogate_off_at;    /* iteration from which the surrogate was switched off (stall policy or
                              divergence fallback), or -1 */
  int surrogate_diverged;  /* 1 if iterations with the surrogate ended in a non-physical state or a zero
                              pivot and the call restarted from its first state with the exact block */
} csi_step_stats;

int csi_create(csi_ctx **ctx, int device, void *hip_stream);
int csi_destroy(csi_ctx *ctx);
const char *csi_last_error(const csi_ctx *ctx);

/* Structured grid of the finite-volume form of Eq. (iterate) (Section 2.2:
 * the generalised-coordinate fluxes become face fluxes F.n S_f, 1/J becomes the
 * cell area V_P).  Grid nodes x_nodes, y_nodes: host [(nj+1)][(ni+1)], i
 * fastest, copied; cell (i, j) has nodes (i..i+1, j..j+1).  Cell areas
 * (shoelace) and face vectors (one per face, shared by its two cells) are
 * derived here.  bc_mode 0: isothermal no-slip non-catalytic wall at j = 0
 * (T_wall; the isothermal wall of the paper's cylinder case, Section 3.2),
 * free-stream far field at j = nj, zero-gradient outflow at i = 0 and i = ni;
 * bc_mode 1: free stream on all four sides (the far-field box of Section 3.1).
 * Errors: CSI_ERR_ARG for ni, nj < 1, more than 2e9 cells, null arrays,
 * T_wall <= 0 or another bc_mode. */
int csi_set_grid(csi_ctx *ctx, int ni, int nj, const double *x_nodes, const double *y_nodes, double T_wall,
                 int bc_mode);
/* Thermochemical model of the governing equations (Section 2.1, Eq. (govern)
 * and Eq. (flux): ns species continuity equations with source omega_s, the
 * mixture momentum and total energy, and in two temperatures the vibrational-
 * electronic energy with its source omega_ve; the thermodynamic, kinetic and
 * transport laws the paper defers to its references are fixed by the tables of
 * csi_mechanism).  The host tables are copied.  Compiled species counts: 2, 3,
 * 5 and 11 (one and two temperatures), 16, 20 and 32 (one temperature).  Any
 * other count up to CSI_WIDE_MAX_SPECIES runs on the species-generic kernels,
 * which take one temperature and no reactions (nr = 0: the non-reacting flow
 * of the species-count study, Section 3.1); there the coupled form inverts
 * its dense block by blocked Gauss-Jordan elimination, sweeps and block
 * solves run in FP64 with per-hyperplane launches, and the surrogate,
 * physical time and flux differences are not available (CSI_ERR_UNSUPPORTED).
 * Errors: CSI_ERR_UNSUPPORTED for a species count with neither (two
 * temperatures or reactions above 32 species); CSI_ERR_ARG for ns < 2, ns >
 * CSI_WIDE_MAX_SPECIES, nr > 64 or bad tables. */
#define CSI_WIDE_MAX_SPECIES 4096
int csi_set_mechanism(csi_ctx *ctx, const csi_mechanism *m);
/* Residual scheme: 0 (default) first-order HLLE mixture flux with upwinded
 * species and e_ve fluxes; 1 the second-order scheme of the paper's cylinder
 * case (Section 3.2): MUSCL reconstruction of (rho_s, u, v, T, Tv) with the
 * minmod limiter at interior faces (boundary faces first order) and Roe's
 * flux for the mixture (Roe-averaged u, v, H and dp/d(rho E); the waves at
 * u.n carry the rest of the rho E jump, which keeps Roe's property for a
 * real-gas mixture; Harten's entropy fix on the acoustic waves; Sanders,
 * Morano and Druguet's H-correction against the carbuncle), the species and
 * e_ve carried by the mixture mass flux at the upwind mass fraction / e_ve.
 * Only the residual changes: the implicit operator keeps its first-order
 * spectral-radius form.  A non-physical reconstructed state is reported as
 * CSI_ERR_NONFINITE by the residual or step.  Errors: CSI_ERR_ARG for another
 * value; CSI_ERR_UNSUPPORTED for 1 on the species-generic kernels (and
 * csi_set_mechanism refuses those kernels while the scheme is 1). */
int csi_set_residual_scheme(csi_ctx *ctx, int scheme);
/* on = 1: the next csi_set_mechanism takes the species-generic kernels for
 * every species count (so that they can be compared with the compiled ones on
 * the same case); on = 0 (the default): only above 32 species.  Errors:
 * CSI_ERR_ARG for another value. */
int csi_set_species_generic(csi_ctx *ctx, int on);
/* In-place inverse of `count` dense n x n FP64 matrices at a (device,
 * row-major, contiguous; caller-owned): blocked Gauss-Jordan elimination with
 * partial pivoting (largest magnitude in the pivot column among the rows not
 * yet used, lowest row on ties), the coupled form's block solve of Section
 * 2.2 (the diagonal point blocks of Eq. (ijkiterate)) on the species-generic
 * path.  work: device scratch of at least csi_block_inverse_work(n, count)
 * bytes, 256-byte aligned, caller-owned (row interchanges [count][n], pivot
 * rows [count][64][n], a flag).  Runs on ctx's stream and synchronises it.
 * *singular (optional) receives -1, or the lowest index of a matrix with a
 * zero pivot (then CSI_ERR_SINGULAR; that matrix's contents are undefined, the
 * others are inverted).  Errors: CSI_ERR_ARG for n < 1, n >
 * CSI_WIDE_MAX_SPECIES + 3, count < 0, a null a with count > 0, or a missing,
 * misaligned or short work buffer. */
int csi_block_inverse_work(int n, int count, size_t *bytes);
int csi_block_inverse(csi_ctx *ctx, int n, int count, double *a, void *work, size_t work_bytes, int *singular);
/* Free-stream state of the far-field boundary (the Dirichlet far field of
 * Section 3; also the uniform flow of the Section 3.1 box) from primitives:
 * partial densities rho_s [ns] (host, copied), velocity (u, v), temperatures
 * T and Tv (Tv ignored in one temperature).  Errors: CSI_ERR_ARG for a
 * non-positive temperature; CSI_ERR_STATE before set_mechanism. */
int csi_set_freestream(csi_ctx *ctx, const double *rho_s, double u, double v, double T, double Tv);
int csi_workspace_bytes(const csi_ctx *ctx, size_t *bytes);
/* dev_ptr: device memory of at least csi_workspace_bytes, 256-byte aligned; caller owns it */
int csi_bind_workspace(csi_ctx *ctx, void *dev_ptr, size_t bytes);
int csi_set_state(csi_ctx *ctx, const double *q, int on_device);
int csi_get_state(csi_ctx *ctx, double *q, int on_device);

/* Residual R = sum_f F_f S_f - V S(Q) (Section 2.2, Eq. (iterate) in finite-
 * volume form) with local time steps at this CFL (Eq. for Delta tau), face
 * spectral radii and the chemical source.  norms (host, nullable):
 * [r_rho, r_E] = L2 norms over cells of sum_s R_rho_s / V and R_E / V. */
int csi_residual(csi_ctx *ctx, double cfl, double *norms);
/* Diagonal blocks of `mode` in `precision` (Section 2.2: I_m = V/dtau I - V A_S
 * plus the spectral and viscous radii; Section 2.3: flow radius |U|+c and
 * species radius |U| for the split parts), their inverses, then the LU-SGS
 * forward and backward sweeps on the last residual.  dQ stays in the
 * workspace.  jac: CSI_JAC_EXACT (analytic source Jacobian) or
 * CSI_JAC_SURROGATE (split species block from the installed network, exact
 * fallback per cell when the diagonal-dominance check fails). */
int csi_implicit_op(csi_ctx *ctx, int mode, int precision, int jac);
/* Dual time stepping for unsteady flows (Section 2.2, Eq. (dualimplicit) and
 * Eq. (linearizedimplicit)): with dt > 0 every later residual is the unsteady
 * residual R(Q) + V [(1 + theta)(Q - Q^n) - theta (Q^n - Q^{n-1})] / dt (its
 * norms included) and every diagonal block gains (1 + theta) V / dt next to
 * V / dtau, so that the pseudo-time iterations of csi_step converge to the
 * implicit physical time step.  theta = 0: first-order backward Euler;
 * theta = 1/2: the second-order backward difference (the paper's text gives
 * theta = 2 for second order, which makes the scheme first order; 1/2 is the
 * value for which the discretisation is second order).  dt = 0 (default):
 * steady.  Errors: CSI_ERR_ARG for a negative or non-finite dt or theta. */
int csi_set_physical_time(csi_ctx *ctx, double dt, double theta);
/* Start a physical time step: Q^{n-1} <- Q^n, Q^n <- Q (csi_set_state sets
 * both levels to the state), and the next csi_step starts its residual drop
 * and CFL ramp afresh.  Errors: CSI_ERR_STATE without a bound state. */
int csi_advance_time(csi_ctx *ctx);
/* Set the time levels Q^n and Q^{n-1} directly (restart of an unsteady run):
 * FP64 [nv][nj][ni] each, host (on_device = 0) or device memory, copied.
 * Errors: CSI_ERR_STATE without a bound state. */
int csi_set_time_levels(csi_ctx *ctx, const double *qn, const double *qnm1, int on_device);

/* closure (coupled) or CC1 / CC2 (split) and the FP64 update of Q (paper Section 2.3) */
int csi_consistency_correct(csi_ctx *ctx, int kind);
/* iterate: residual -> implicit_op -> consistency_correct, with a CFL ramp and stop test.
 * With CSI_JAC_SURROGATE the state at the start of the call is kept in the
 * workspace: if iterations with the surrogate on end in a non-physical state or
 * a zero pivot, the call restarts from it with the exact block (surrogate
 * switched off from the call's first iteration; stats surrogate_diverged), once
 * per call.  Without the surrogate, or after that, such iterations return
 * CSI_ERR_NONFINITE / CSI_ERR_SINGULAR. */
int csi_step(csi_ctx *ctx, const csi_step_params *p, csi_step_stats *s);
/* Which source Jacobian the split species block carries (Section 2.3, the
 * component operator solves Q_C with the flow variables unchanged; the paper
 * does not say which variables the chemical source is differentiated at).
 * reading 0 (the default in two temperatures): J_C = d omega_s / d rho_r at
 * fixed T, Tv.  reading 1 (the default in one temperature):
 * at fixed velocities and fixed internal (and vibrational) energy densities,
 * so that the temperatures follow the composition (the Jacobian of an
 * adiabatic constant-volume reactor): J_C + d omega_s/dT dT/d rho_r
 * (+ the Tv term).  reading 2: as 1, with Tv held as well in two
 * temperatures (rho e_ve takes the added mass's e_ve,r(Tv) out of the same
 * internal energy, so T alone follows; the same as 1 in one temperature).  The reading also sets the targets of
 * csi_sample_jacobians, so that a network trained on them learns the same
 * block (its inputs T, Tv, rho, Y determine either reading).  Errors:
 * CSI_ERR_ARG for another value, CSI_ERR_STATE before set_mechanism.
 * set_mechanism restores the default of its temperature model. */
int csi_set_species_jacobian(csi_ctx *ctx, int reading);

/* Wall heat flux, the quantity whose convergence the paper tracks beside the
 * residual (Section 3.2 and later cases; conduction only: the wall is
 * non-catalytic, so no diffusive enthalpy flux): per wall cell i
 * q_w = k (T_i0 - T_w) / d_i + k_ve (Tv_i0 - T_w) / d_i with the wall-face
 * conductivities and d_i the cell-centre-to-wall distance, from the last
 * csi_residual; host [ni], nullable.  q_stag (host, nullable): mean of the two
 * cells beside the stagnation line (ni even) or the middle cell.  Synchronises
 * with the device.  Errors: CSI_ERR_STATE without a bound state or on a grid
 * without a wall (bc_mode 1). */
int csi_wall_heat_flux(csi_ctx *ctx, double *qw, double *q_stag);
/* residual-norm history of csi_step calls: host [2*n] (r_rho, r_E per iteration) */
int csi_norm_history(csi_ctx *ctx, int n, double *hist);

/* Conservative state from primitives with the library's thermodynamics (host
 * arrays): rho_s [ns][n], u, v, T, Tv [n] -> q [nv][n] */
int csi_prim_to_cons(csi_ctx *ctx, int n, const double *rho_s, const double *u, const double *v, const double *T,
                     const double *Tv, double *q);
/* Sweep schedule (Section 2.2 sweeps in i+j order).  schedule 0 launches one
 * kernel per i+j hyperplane with cell-major records.  schedule 1 (default)
 * runs each sweep as one persistent kernel: every cell of a strip is owned by
 * a group of G lanes of one wavefront (G = unknowns of the swept part: nb
 * coupled, nf flow, ns species) and a wavefront holds C = 64 / G columns.
 * Errors: CSI_ERR_ARG for any other value.  Changing the schedule invalidates
 * the records of the last implicit operator (csi_get_array). */
int csi_set_sweep(csi_ctx *ctx, int schedule);
/* Off-diagonal operator of the sweeps (Section 2.2: the neighbour terms are
 * applied without storing their Jacobians).  op 0 (default): the linear
 * Jacobian-vector product A_N(n) x of the spectral splitting.  op 1: the flux
 * difference F(Q_N + x).n - F(Q_N).n in its place (coupled and flow parts;
 * the species part is the same either way), which needs the neighbour's
 * temperatures at Q_N + x inside the sweep: it runs in the per-hyperplane
 * schedule (op 1 sets schedule 0) with FP64 sweeps only (CSI_ERR_UNSUPPORTED
 * for CSI_MIXED).  A neighbour state Q_N + x that is not physical makes
 * csi_implicit_op / csi_step return CSI_ERR_NONFINITE.  Errors: CSI_ERR_ARG
 * for another value. */
int csi_set_offdiag(csi_ctx *ctx, int op);
/* Phase timing of csi_step with HIP events on the context's stream (on = 1 to
 * enable; on = 2 also records a per-strip trace of the group-schedule sweeps,
 * read with csi_get_array(ctx, "sweep_trace"); 0 disables both).
 * csi_phase_times returns the accumulated milliseconds of the
 * phases [prim, faces, cell, block, norms, sweep_fwd, sweep_bwd, update]
 * (ms[0..7]; cell: the cell kernel, block: the diagonal-block kernel of
 * ns >= 5, zero below) and the number of timed iterations in ms[8];
 * reset = 1 clears the accumulators.  ms must hold 9 doubles. */
int csi_set_timing(csi_ctx *ctx, int on);
int csi_phase_times(csi_ctx *ctx, double *ms, int reset);

/* Debug / parity access to named workspace arrays, copied to host as FP64:
 * "R" [nv][N], "dtau" [N], "src" [nv][N], "b" "dqs" "dq" [nsol][N], "T" "Tv" "p" "c" [N],
 * "qw" [ni], "Dinv" (coupled [nb*nb][N] row-major D^-1; split [nf*nf + ns*ns][N]: the
 * flow block's inverse as a dense matrix, then the species inverse), "Jsur" [ns*ns][N]
 * (surrogate species block of the last surrogate iteration), "sweep_trace"
 * [2 sweeps (fwd, bwd)][2 parts][ni strips][8] of the last sweep pair with the
 * trace on: wall clock (100 MHz ticks) at the compute wave's start and end,
 * its spins on step records and on boundary pushes, the copy wave's spins on
 * free ring slots and the boundary wave's spins on pushes (unused entries are
 * stale). */
int csi_get_array(csi_ctx *ctx, const char *name, double *out, size_t count);
/* The arrays "R", "b", "dqs", "dq" and "Dinv" of csi_get_array at the listed
 * cells only (cells[k] = j * ni + i, 0 <= cells[k] < N): out [F][n_cells]
 * (host), F as in csi_get_array, element (f, k) at out[f * n_cells + k].  For
 * checks of full-size runs at sampled cells.  Errors: CSI_ERR_ARG for an unknown
 * name or a cell out of range; CSI_ERR_STATE before an implicit operator for
 * the records. */
int csi_get_cells(csi_ctx *ctx, const char *name, const long long *cells, int n_cells, double *out);

/* ------------------------------------------------------------------------
 * Surrogate of the split species block J_C = d omega_s / d rho_r at fixed T,
 * Tv (the chemical source Jacobian that the species diagonal block of Section
 * 2.3 carries).  Network: x -> tanh(W1 x + b1) -> tanh(W2 h1 + b2) -> W3 h2 + b3,
 * hidden width 64, n_in <= 64 inputs, n_out <= 1024 outputs; BF16 operands,
 * FP32 accumulation on the matrix cores, FP32 master parameters
 * [W1 (64 x n_in) | b1 | W2 (64 x 64) | b2 | W3 (n_out x 64) | b3] (row-major).
 * Features x_raw = (ln T, ln Tv, ln rho, Y_1..Y_ns) (n_in = ns + 3), standardised
 * x = (x_raw - mu) / sigma; targets t = asinh(tau0 J_C) with J_C row-major
 * (s, r) (n_out = ns^2) and tau0 = 1 / the geometric mean of the non-zero
 * |J_C| of the training set; the network's J_C is sinh(y) / tau0.
 * All pointers below not marked host are device pointers owned by the caller;
 * `work` is caller-owned device scratch of at least the size csi_mlp_sizes
 * reports, 256-byte aligned.  Errors: CSI_ERR_ARG for sizes out of range or a
 * short work buffer; CSI_ERR_HIP for launch failures. */

/* number of FP32 master parameters and the work bytes the calls below need
 * for up to `batch` samples per call (host outputs) */
int csi_mlp_sizes(int n_in, int n_out, int batch, int *n_params, size_t *work_bytes);
/* Training-set statistics and transforms: scales_host[2 n_in + 1] =
 * (mu, sigma, tau0) from x_raw [n][n_in] and jc [n][n_out] (sigma = 1 for a
 * feature with standard deviation < 1e-12); x [n][n_in] and t [n][n_out]
 * receive the standardised features and targets. */
int csi_mlp_prepare(csi_ctx *ctx, int n, int n_in, int n_out, const float *x_raw, const float *jc, float *x,
                    float *t, double *scales_host, void *work, size_t work_bytes);
/* y [n][n_out] = network(x [n][n_in]) with the BF16 path above */
int csi_mlp_forward(csi_ctx *ctx, int n_in, int n_out, int n, const float *params, const float *x, float *y,
                    void *work, size_t work_bytes);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation):
 * csi_mlp_forward without the work argument.  The packed BF16 operands go to
 * a library-owned device array of CSI_MLP_NOALLOC_SCRATCH_BYTES, one per GPU,
 * held until the process ends; its address is taken at csi_create on that
 * context's device.  The call allocates nothing and launches the same kernels
 * as csi_mlp_forward on the context's stream (asynchronous).  Every call on
 * one GPU shares that GPU's array: calls that overlap on one GPU (other
 * streams, other contexts, other host threads) race and must be serialised
 * by the caller.  Every network within the limits above (n_in <= 64,
 * n_out <= 1024: at most 286 720 bytes of packed operands) fits; a larger
 * packed size returns CSI_ERR_ARG.  Other errors as csi_mlp_forward. */
#define CSI_MLP_NOALLOC_SCRATCH_BYTES 327680
int csi_mlp_forward_noalloc(csi_ctx *ctx, int n_in, int n_out, int n, const float *params, const float *x,
                            float *y);

typedef struct {
  int n_in, n_out;
  int n_data;        /* rows of x and t */
  int batch;         /* samples in this call, >= 1 */
  const float *x;    /* [n_data][n_in] standardised features */
  const float *t;    /* [n_data][n_out] targets */
  const int *idx;    /* [batch] rows of this batch (entries outside [0, n_data) are skipped) */
  float *params;     /* [n_params] FP32 master parameters */
  void *work;
  size_t work_bytes;
} csi_mlp_batch;
typedef struct { double lr, beta1, beta2, eps; } csi_adam;

/* Mean squared error over the batch's samples and outputs (loss, host,
 * nullable) and its gradient (grad [n_params], FP32) with respect to params. */
int csi_mlp_grad(csi_ctx *ctx, const csi_mlp_batch *b, float *grad, double *loss);
/* One training step: the gradient as above, then a bias-corrected Adam update
 * of params and of the moments m, v [n_params] (step counts from 1). */
int csi_mlp_train_step(csi_ctx *ctx, const csi_mlp_batch *b, float *m, float *v, int step, const csi_adam *h,
                       double *loss);

/* One epoch: Adam steps (as csi_mlp_train_step) over the rows order[0..n_rows)
 * (device int array, each a row of b->x / b->t) taken b->batch at a time, the
 * last batch possibly shorter; steps are numbered step0 + 1, step0 + 2, ...
 * (b->idx is not used).  Launches only, except that the host waits for loss
 * (host, nullable): the mean squared error of the last batch before its
 * update.  Errors: CSI_ERR_ARG for bad sizes, pointers or Adam arguments. */
int csi_mlp_train_epoch(csi_ctx *ctx, const csi_mlp_batch *b, const int *order, int n_rows, float *m, float *v,
                        int step0, const csi_adam *h, double *loss);

/* Training samples for the surrogate of the species block's source Jacobian
 * J_C (the component operator of Section 2.3), taken from Jacobians the
 * solver itself generates, from the bound state: n = min(N,
 * max_samples) rows, returned in *n_written, of raw features x_raw [n][ns + 3]
 * (ln T, ln Tv, ln rho, Y) and the exact J_C [n][ns * ns] (FP32) of the
 * species block's reading (csi_set_species_jacobian); host-visible or device
 * pointers the device can write.  n = N: row r is cell r (the seed is
 * unused).  n < N: a seeded subset of distinct cells, row r being cell
 * (b + r a) mod N with b = splitmix64(seed) mod N and a the first value
 * coprime with N from 1 + splitmix64(seed + 1) mod (N - 1) upwards, wrapping
 * within [1, N - 1] (splitmix64: one step of Vigna's SplitMix64).  Overwrites
 * the diagonal-block hand-off of the last implicit operator (ns >= 5).
 * Errors: CSI_ERR_ARG (max_samples < 1, null buffers), CSI_ERR_STATE (no
 * state), CSI_ERR_UNSUPPORTED (species-generic kernels), CSI_ERR_NONFINITE. */
int csi_sample_jacobians(csi_ctx *ctx, int max_samples, unsigned long long seed, float *x_raw, float *jc,
                         int *n_written);
/* Install a trained network for CSI_JAC_SURROGATE (split form only):
 * params [n_params] (device, copied into the workspace), scales (host,
 * [2 n_in + 1] as from csi_mlp_prepare), n_in = ns + 3, n_out = ns^2.  Per
 * cell and iteration the surrogate block is used when D_C = dC I - V J_C is
 * strictly row diagonally dominant with a positive diagonal in molar units
 * (D_rr M_r > sum_{c != r} |D_rc| M_c), else the exact J_C; and in
 * csi_step, once stall_window iterations have run with it, the
 * first iteration whose density residual exceeds stall_ratio times the one
 * stall_window iterations earlier switches it off for the rest of the call. */
int csi_set_surrogate(csi_ctx *ctx, const float *params, const double *scales, int n_in, int n_out,
                      double stall_ratio, int stall_window);

#ifdef __cplusplus
}
#endif
#endif
