/* Oracle C-ABI: TEST INFRASTRUCTURE ONLY (tests/, smoke(), bench.py cpu_baseline).
 *
 * Plain FP64 CPU reference of one pseudo-time iteration of the implicit solver
 * described in the paper, Section 2.2 (implicit time integration, LU-SGS
 * forward/backward sweeps) and Section 2.3 (component-splitting method: flow
 * part, component part, consistence corrections).  Host memory only; every
 * array argument is owned by the caller and copied on entry.
 *
 * Layouts: state q is SoA [nv][nj][ni] (i fastest) with
 *   nv = ns + 3 (one temperature) or ns + 4 (two temperatures),
 *   q = (rho_1..rho_ns, rho u, rho v, rho E, [rho e_ve]).
 * Increment vectors ("dq", "dqs") are SoA [nsol][nj][ni]:
 *   coupled: nsol = nb = nf + ns - 1, z = (rho, rho u, rho v, rho E, [rho e_ve], rho_1..rho_{ns-1})
 *   split:   nsol = nf + ns, (rho, rho u, rho v, rho E, [rho e_ve] | rho_1..rho_ns)
 * Return codes: 0 ok, negative on error (text via orc_last_error).
 */
#ifndef ORC_H
#define ORC_H
#ifdef __cplusplus
extern "C" {
#endif

typedef struct orc_ctx orc_ctx;

typedef struct {
  int ns, nr, two_temp;
  const double *M;        /* [ns] molar mass, kg/mol */
  const int *kind;        /* [ns] 0 atom or atomic ion, 1 linear molecule or ion, 2 electron */
  const double *theta_v;  /* [ns] vibrational characteristic temperature, K */
  const double *theta_r;  /* [ns] rotational characteristic temperature, K */
  const double *sigma;    /* [ns] rotational symmetry number */
  const double *g_el;     /* [ns] electronic ground-state degeneracy */
  const double *h_form;   /* [ns] formation enthalpy at 0 K, J/mol */
  const double *sc;       /* [ns] Schmidt number */
  const double *lt_a;     /* [ns] Landau-Teller exponent constant a_s */
  const double *lt_b;     /* [ns] Landau-Teller constant b_s */
  const double *A;        /* [nr] pre-exponential, SI (m^3/mol)^(order-1)/s */
  const double *b;        /* [nr] temperature exponent */
  const double *theta;    /* [nr] activation temperature, K */
  const int *tctl;        /* [nr] controlling temperature 0:T 1:sqrt(T Tv) 2:Tv */
  const int *third;       /* [nr] 1 if a third body [M] multiplies the rate */
  const int *nu_f;        /* [nr*ns] reactant stoichiometry */
  const int *nu_b;        /* [nr*ns] product stoichiometry */
  const double *eff;      /* [nr*ns] third-body efficiencies */
  double mu_ref, T_ref, mu_exp; /* mu = mu_ref (T/T_ref)^mu_exp */
} orc_mechanism;

enum { ORC_COUPLED = 0, ORC_SPLIT = 1 };
enum { ORC_CLOSURE = 0, ORC_CC1 = 1, ORC_CC2 = 2 };
enum { ORC_HYPERPLANE = 0, ORC_LEXICOGRAPHIC = 1 };

int orc_create(orc_ctx **ctx);
void orc_destroy(orc_ctx *ctx);
const char *orc_last_error(const orc_ctx *ctx);
int orc_set_threads(orc_ctx *ctx, int n);
/* named options: "residual_scheme" (0: first-order HLLE; 1: MUSCL with the
 * minmod limiter on (rho_s, u, v, T, Tv) at interior faces and the Roe flux);
 * "jc_fixed_qf" (0: split species block at fixed T, Tv;
 * 1: at fixed momenta and energies; 2: at fixed velocities and internal
 * energy densities, the temperatures following; 3: as 2 with Tv held; the
 * default after orc_set_mechanism is 2 in one temperature and 0 in two);
 * "flux_diff" (0: linear
 * Jacobian-vector products off the diagonal; 1: flux differences
 * F(Q_N + x) - F(Q_N)) */
int orc_set_option(orc_ctx *ctx, const char *name, double value);
/* dual time stepping (paper Section 2.2, Eq. (linearizedimplicit)): physical
 * step dt (0: steady) and theta; orc_advance_time: Q^{n-1} <- Q^n <- Q
 * (orc_set_state sets both levels to the state) */
int orc_set_physical_time(orc_ctx *ctx, double dt, double theta);
int orc_advance_time(orc_ctx *ctx);
int orc_set_time_levels(orc_ctx *ctx, const double *qn, const double *qnm1);

/* nodes [(nj+1)][(ni+1)]; bc_mode 0: wall at j=0, far field at j=nj, outflow at i=0,ni;
 * bc_mode 1: free-stream Dirichlet on all four sides (free-stream preservation test). */
int orc_set_grid(orc_ctx *ctx, int ni, int nj, const double *xn, const double *yn, double T_wall,
                 int bc_mode);
int orc_set_mechanism(orc_ctx *ctx, const orc_mechanism *m);
int orc_set_freestream(orc_ctx *ctx, const double *rho_s, double u, double v, double T, double Tv);
int orc_prim_to_cons(orc_ctx *ctx, int n, const double *rho_s, const double *u, const double *v,
                     const double *T, const double *Tv, double *q);
int orc_set_state(orc_ctx *ctx, const double *q);
int orc_get_state(orc_ctx *ctx, double *q);

/* R, local time step, face spectral radii, source terms, source Jacobians
 * and diagonal blocks at the current state; norms[0..1] = (r_rho, r_E). */
int orc_residual(orc_ctx *ctx, double cfl, double *norms);
/* LU-SGS forward+backward sweeps with b = -R (mode coupled/split, order hyperplane/lexicographic) */
int orc_implicit_op(orc_ctx *ctx, int mode, int order);
/* One cell (i, j) of the sweeps of the last residual's operator, every other
 * cell's values given ([nsol][N] arrays): fwd = 1 solves the cell's row of
 * (D+L) dQ* = b (b formed from the residual as orc_implicit_op forms it) with
 * the lower neighbours' dQ* from xs; fwd = 0 the row of (D+U) dQ = D dQ* with
 * the upper neighbours' dQ from x and the cell's dQ* from xs.  out [nsol].
 * For checks of a full-size run at sampled cells (on a patch of the grid). */
int orc_sweep_cell(orc_ctx *ctx, int mode, int fwd, int i, int j, const double *xs, const double *x, double *out);
/* the sweeps of orc_implicit_op with a caller RHS b [nsol][N]; result x [nsol][N] */
int orc_sweep_rhs(orc_ctx *ctx, int mode, int order, const double *b, double *x);
/* closure (coupled) or CC1/CC2 (split) and the update of q */
int orc_consistency_correct(orc_ctx *ctx, int mode, int kind, int *n_clipped);
/* n_iter iterations; cfl(m) = cfl^(min(m, ramp)/ramp) for iteration m = it0 + k (ramp 0: fixed) */
int orc_step(orc_ctx *ctx, int mode, int kind, double cfl, int ramp, int it0, int n_iter,
             double *norm_hist);
int orc_wall_heat_flux(orc_ctx *ctx, double *qw, double *q_stag);

/* named arrays for tests: "R" [nv][N], "dtau" [N], "omega" [nv][N], "dqs" "dq" [nsol][N],
 * "T" "Tv" "p" "c" [N], "qw" [ni], "dK" "dF" "dC" [N], "JK" [nb*nb][N], "JC" [ns*ns][N],
 * "Jve" [nf][N], "DK" [nb*nb][N], "DF" [nf*nf][N], "DC" [ns*ns][N] (row-major blocks),
 * "FvI" [nv][(ni+1)*nj], "FvJ" [nv][ni*(nj+1)] (viscous part of the face fluxes F.n, per unit length) */
int orc_get(orc_ctx *ctx, const char *name, double *out);

/* dense global operator on small grids: unknown index = cell * nsol + k;
 * D, L, U each [(N*nsol)^2] row-major. */
int orc_dense_operator(orc_ctx *ctx, int mode, double *D, double *L, double *U);

/* point evaluations for pins */
int orc_point_thermo(orc_ctx *ctx, double T, double Tv, double *e, double *h, double *cv_total,
                     double *g_RT);
int orc_point_production(orc_ctx *ctx, const double *rho_s, double T, double Tv, double *omega,
                         double *omega_ve);
int orc_point_prim(orc_ctx *ctx, const double *q, double *T, double *Tv, double *p, double *c);
int orc_point_flux_jacobian(orc_ctx *ctx, const double *q, double nx, double ny, double *A);
int orc_point_flux(orc_ctx *ctx, const double *q, double nx, double ny, double *F);
/* HLLE face flux between left state qL and right state qR, unit normal (nx, ny) from L to R */
int orc_point_hlle(orc_ctx *ctx, const double *qL, const double *qR, double nx, double ny, double *F);
/* Roe face flux (MUSCL + Roe residual scheme) between states qL and qR; eta
 * >= 0: the H-correction's floor on the wave speeds (0 for none) */
int orc_point_roe(orc_ctx *ctx, const double *qL, const double *qR, double nx, double ny, double eta, double *F);
/* MUSCL (minmod) face state on the side of cell B: A beyond B, C across the face */
int orc_point_muscl(orc_ctx *ctx, const double *qA, const double *qB, const double *qC, double *qf);
/* off-diagonal neighbour term at state q: mode 0 coupled (x in z), 1 flow part
 * (x in Q_F at frozen Y); fd 0: A(n) x, fd 1: F(q + x).n - F(q).n */
int orc_point_offdiag(orc_ctx *ctx, const double *q, double nx, double ny, int mode, int fd, const double *x,
                      double *out);
int orc_point_source_jacobian(orc_ctx *ctx, const double *q, int which, double *J);

#ifdef __cplusplus
}
#endif
#endif
