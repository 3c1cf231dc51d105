/*
 * oracle.h -- plain FP64 CPU reference of the multi-scale semi-Lagrangian
 * lattice Boltzmann step (Kallikounis, Dorschner & Karlin, arXiv 2102.12559).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or calls
 * this library: only the test suite, the smoke check and the CPU leg of the
 * benchmark do.  It shares no source with the GPU library.
 *
 * The oracle follows the paper's definitions literally:
 *   - Gauss-Hermite rules by Newton iteration on He_n (Sec. II.A, Tab. I);
 *   - tensor-product velocity sets, W_i = w_ix w_iy (w_iz) (eqs. ci, wi);
 *   - moment matrix M[(m,n),i] = c_ix^m c_iy^n, m,n < sqrt(Q) (eq. momf), inverted
 *     in long double;
 *   - lattice equilibrium f^L = M_L^{-1} M_{u,T} f^eq with f^eq = rho W
 *     (Sec. II.C.2, eqs. feqL, geqL, feqL0);
 *   - lifting m_q (+) M^eq_{Q-q} and projection M_q (Sec. III.B, III.C, App. C);
 *   - semi-Lagrangian propagation with lifting / projection applied to each
 *     collocation point of the other order (Sec. III.D), then the collision of
 *     eqs. Pond_f, Pond_g: BGK (omega1 = omega2), or the two-relaxation model
 *     with the quasi-equilibria of eqs. fqeq, gqeq.
 *
 * Pins (tests/test_oracle_*.py): Table I nodes and weights, Gauss-Hermite
 * exactness, the printed diagonal moments (eqs. QxxxL, RxxL, QxxxPonD, RxxPond)
 * and Fig. 1's 3 %, the closed Hermite product form of f^L, lifting/projection
 * moment properties and round trips, exact equality with a textbook D2Q9 LBM
 * at CFL 1 (also in a frame moving by one cell per step, as a Galilean shift),
 * conservation, fixed points, the shear-wave viscosity, vortex translation,
 * Couette symmetry, the second-order Taylor-Green convergence of App. A, the
 * |Pi_neq|/p criterion on a hand-set stress, the closure's per-tile error
 * check against hand-computed errors, finite-difference gradients of the MLP.
 *
 * The run may use a global constant reference frame {u_ref, T_ref} (eq. veli):
 * particle velocities, moments, equilibria, lifting and projection are then
 * taken in that frame's velocities v_i = sqrt(T_ref) c_i + u_ref.
 *
 * Conventions: cell index = x + nx*(y + ny*z); population index
 * i = a + n*b (+ n*n*c) with a, b, c the ascending 1D node indices along x, y, z;
 * population arrays are [Q][ncell].  All functions return 0 on success and a
 * negative value on invalid input.
 */
#ifndef MSL_ORACLE_H
#define MSL_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct or_config {
  int dim, nx, ny, nz;
  int n_low, n_high;          /* 1D Gauss-Hermite orders; n_high = 0: one lattice */
  int thermal;                /* 0: T = T_L, f only; 1: f and g, ideal gas with cv */
  double tau, cv, cfl;
  int tau_mode;               /* 0: constant tau; 1: mu = mu_ref (T/T_ref)^mu_exp */
  double mu_exp, tau_ref_rho, tau_ref_T;
  double rho0, T0;            /* reference state of the reduced-precision storage */
  int store;                  /* 0 fp64, 1 fp32, 2 fp16 deviation, 3 bf16 deviation */
  int lift_mode;              /* 0 raw moments (App. C), 1 Hermite coefficients, 2 MLP */
  int bc[6];                  /* face = 2*axis + side: 0 periodic, 1 fixed eq, 2 zero gradient, 3 diffuse wall */
  double bc_state[6][5];      /* rho, ux, uy, uz, T (walls: u_w, T_w) */
  double slot_state[6][5];
  int slot[6][4];             /* [lo0,hi0) [lo1,hi1) on the tangential axes; lo>=hi: none */
  double slot_edge[6];        /* > 0: tanh edges of this width blend slot and face states */
  int crit_kind;              /* 0 none, 1 Mach, 2 |Pi_neq|/p, 3 Knudsen number lambda |grad rho| / rho */
  double crit_thr;
  int crit_every;
  double u_ref[3], T_ref;     /* global constant reference frame (eq. veli): particle
                                 velocities v_i = sqrt(T_ref) c_i + u_ref; T_ref <= 0: 1 */
  double store_u[3];          /* velocity of the reduced-precision storage reference state
                                 (rho0, store_u, T0): the deviation scale of population i
                                 is rho0 prod_a w_a r(c_a), r the density ratio of
                                 N(s, T0/T_ref) to N(0, 1), s = (store_u - u_ref)/sqrt(T_ref) */
  double tau2;                /* > 0 and != tau: two-relaxation quasi-equilibrium model
                                 (eqs. Pond_f/g with omega2 = 1/tau2 at the reference state;
                                 Pr = (tau - 1/2)/(tau2 - 1/2) kept where tau varies with T);
                                 otherwise BGK */
  int crit_margin;            /* > 0: the high-order set also takes every cell within this
                                 many cells (per axis) of a cell the criterion selects */
} or_config;

typedef struct or_ctx or_ctx;

/* ---- lattice-level routines (for pins) ---- */
int or_gh_rule(int n, double *x, double *w);
int or_lattice_feq(int dim, int n, double rho, const double *u, double theta, double *out);
int or_moment_matrix(int dim, int n, double *M, double *Minv);
/* lifting / projection of one cell's populations; g may be NULL when thermal=0 */
int or_lift(int dim, int nq, int nQ, int thermal, double cv, int mode,
            const double *fq, const double *gq, double *fQ, double *gQ);
int or_project(int dim, int nQ, int nq, const double *fQ, const double *gQ,
               double *fq, double *gq);
/* Lagrange weights of the 3-point stencil through -1, 0, 1 at xi */
int or_lagrange3(double xi, double *a);
/* round-to-nearest-even conversions used by the deviation-storage emulation */
double or_round_fp16(double v);
double or_round_bf16(double v);

/* quasi-equilibria f*, g* (eqs. fqeq, gqeq, in the run's frame) of one cell's
 * populations f (and g when thermal) of lattice `which` */
int or_qeq(const or_ctx *ctx, int which, const double *f, const double *g, double *fstar,
           double *gstar);
/* OpenMP threads of the stepper (n >= 1); returns the previous count */
int or_set_threads(int n);

/* ---- stepper ---- */
int or_create(const or_config *cfg, or_ctx **out);
void or_destroy(or_ctx *ctx);
double or_dt(const or_ctx *ctx);
int or_reach(const or_ctx *ctx);
/* per population of lattice `which`: base offsets n0[Q][D] and weights a[Q][D][3] */
int or_stencil(const or_ctx *ctx, int which, int *n0, double *a);
int or_set_mask_raw(or_ctx *ctx, const uint8_t *mask);   /* no conversion */
int or_set_mask(or_ctx *ctx, const uint8_t *mask);       /* lift/project switched cells */
int or_get_mask(const or_ctx *ctx, uint8_t *mask);
int or_eval_criterion(const or_ctx *ctx, uint8_t *newmask, double *value);
int or_init(or_ctx *ctx, const double *rho, const double *u, const double *T);
int or_step(or_ctx *ctx, int nsteps);
long or_step_count(const or_ctx *ctx);
int or_get_pops(const or_ctx *ctx, int which, int fg, double *out);
int or_set_pops(or_ctx *ctx, int which, int fg, const double *in);
int or_macros(const or_ctx *ctx, double *rho, double *u, double *T);
int or_conservation(const or_ctx *ctx, double *out);     /* sum rho, sum j (3), sum rhoE */
/* next-step populations (native lattice) of selected cells, state untouched */
int or_step_cells(const or_ctx *ctx, int ncells, const int64_t *cells,
                  double *fout, double *gout);

/* out[k] = max of in over the cells within `margin` cells of k along each axis
 * (a box; periodic faces wrap, other faces end the box): the criterion's margin */
int or_dilate_mask(const or_config *cfg, const uint8_t *in, uint8_t *out);

/* ---- co-moving reference frames (PonD, Sec. II.C.1), one or two sets ----
 * Each cell keeps its populations, of its own velocity set, in its own frame
 * {u, T}; a step runs the predictor-corrector to convergence and collides in
 * the converged frame.  With two sets (n_high > n_low), a collocation point of
 * the other set is lifted or projected into the cell's set in its own frame
 * (lift_mode 0 or 1); crit_kind 0 keeps the sets of or_pond_set_mask, 3
 * re-selects them every crit_every steps by the Knudsen number.  Needs FP64
 * storage (store 0) and periodic, fixed-equilibrium, zero-gradient or (not on
 * x faces) diffuse-wall faces.
 * or_pond_step returns -4 when a departure point leaves the two-cell reach or
 * a state turns non-finite. */
typedef struct or_pond or_pond;
int or_pond_create(const or_config *cfg, or_pond **out);
void or_pond_destroy(or_pond *ctx);
double or_pond_dt(const or_pond *ctx);
int or_pond_init(or_pond *ctx, const double *rho, const double *u, const double *T);
int or_pond_step(or_pond *ctx, int nsteps);
int or_pond_macros(const or_pond *ctx, double *rho, double *u, double *T);
/* set `which` at every cell ([Q][ncell], own frames): native values at cells of
 * that set, the converted state elsewhere */
int or_pond_get_pops(const or_pond *ctx, int which, int fg, double *out);
/* sets of the cells (0/1); convert: cells whose set changes convert their state */
int or_pond_set_mask(or_pond *ctx, const uint8_t *mask, int convert);
int or_pond_get_mask(const or_pond *ctx, uint8_t *out);
int or_pond_get_frames(const or_pond *ctx, double *out);         /* [4][ncell]: u_x,u_y,u_z,T */
int or_pond_iterations(const or_pond *ctx, double *mean, int *max);   /* of the last step */
/* G_src^dst f (eq. fll) for one population vector, frames as {u_x, u_y, u_z, T} */
int or_pond_transfer(int dim, int n, const double *src, const double *dst, const double *f,
                     double *out);

/* ---- learned lifting closure (MLP) ---- */
/* MLP F -> H -> H -> O, SiLU hidden activations; flat parameter layout
 * W1[F][H], b1[H], W2[H][H], b2[H], W3[H][O], b3[O]. */
int or_mlp_nparams(int F, int H, int O);
int or_mlp_forward(const double *p, int F, int H, int O, int n, const double *X,
                   double *Y, int bf16_inputs);
int or_mlp_loss_grad(const double *p, int F, int H, int O, int n, const double *X,
                     const double *T, double *loss, double *grad);
int or_adam(double *p, double *m, double *v, const double *g, int np, int t,
            double lr, double b1, double b2, double eps);
/* features / targets of the closure */
int or_mlp_dims(int dim, int nq, int nQ, int *F, int *O);
int or_mlp_features(int dim, int nq, int thermal, double cv, const double *fq,
                    const double *gq, double *feat);
int or_mlp_targets(int dim, int nq, int nQ, int thermal, double cv, const double *fQ,
                   const double *gQ, double *targ);
/* install a network for lift_mode 2: params, input mean/std [F], target mean/std [O] */
int or_set_mlp(or_ctx *ctx, int H, const double *params, const double *xmean,
               const double *xstd, const double *tmean, const double *tstd, int bf16);
/* per check tile (64 x 64 (x 64) cells) flag: 1 = use the network, 0 = Grad */
int or_set_mlp_flags(or_ctx *ctx, const uint8_t *flags);
int or_get_mlp_flags(const or_ctx *ctx, uint8_t *flags, double *emlp, double *egrad);
int or_mlp_check(or_ctx *ctx);   /* recompute the flags from the high-order band cells */
int or_lift_cell(const or_ctx *ctx, const double *fq, const double *gq, int tile,
                 double *fQ, double *gQ);

#ifdef __cplusplus
}
#endif
#endif
