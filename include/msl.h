/*
 * msl.h -- C-ABI of the MI355X multi-scale semi-Lagrangian lattice Boltzmann
 * step (Kallikounis, Dorschner & Karlin, "Multi-scale semi-Lagrangian lattice
 * Boltzmann method", arXiv 2102.12559).
 *
 * The state is a set of post-collision populations per cell; each cell uses
 * either the low-order or the high-order Gauss-Hermite tensor velocity set
 * (Sec. II.A, Tab. I; Sec. III.A).  One step streams every population from its
 * departure point x - c_i dt with a 3-point-per-axis Lagrange stencil
 * (eqs. reconstructionPond, advectionPond in the lattice frame), lifts or
 * projects collocation points of the other order (Sec. III.B-D), and relaxes
 * each cell by BGK towards the lattice equilibrium (eqs. Pond_f/g with
 * omega1 = omega2, eqs. feqL, geqL).
 *
 * Conventions for every entry point:
 *  - all functions return an int status: MSL_OK (0) or a negative MSL_E* code;
 *    no C++ exception crosses the boundary; msl_last_error() describes the
 *    last failure of a context;
 *  - device pointers are plain HIP device addresses; host pointers are marked;
 *  - the caller owns every buffer it passes (workspace, inputs, outputs); the
 *    library allocates no device memory and never frees caller memory;
 *  - all work is enqueued on the HIP stream given to msl_create, in order;
 *    only msl_conservation, msl_get_state/msl_set_state, msl_mlp_train, a
 *    msl_step with check_every > 0, and on grids with more tiles than four
 *    times what the GPU holds at once the first step after each change of the
 *    velocity-set mask (it reads back the number of live tiles), synchronise
 *    that stream;
 *  - a context is not thread-safe; use one context per stream;
 *  - cell index = x + nx*(y + ny*z); population index i = a + n*b (+ n*n*c),
 *    a, b, c the ascending 1D node indices along x, y, z; population arrays
 *    are [Q][ncell] doubles, velocity arrays [dim][ncell].
 */
#ifndef MSL_H
#define MSL_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  MSL_OK = 0,
  MSL_EINVAL = -1,     /* invalid argument or configuration */
  MSL_ENOMEM = -2,     /* workspace too small */
  MSL_EHIP = -3,       /* a HIP runtime call failed */
  MSL_EUNSTABLE = -4,  /* the conservation sentinel saw NaN/Inf or rho <= 0 */
  MSL_ESTATE = -5      /* call out of order (e.g. step before init) */
};

/* storage precision of the population planes */
enum { MSL_FP64 = 0, MSL_FP32 = 1, MSL_FP16_DEV = 2, MSL_BF16_DEV = 3 };
/* lifting: paper's raw-moment completion (App. C), Hermite-coefficient
 * completion, raw completion plus the learned non-equilibrium closure */
enum { MSL_LIFT_GRAD = 0, MSL_LIFT_GRAD_HERMITE = 1, MSL_LIFT_MLP = 2 };
/* boundary rule of a face (face = 2*axis + side) */
enum { MSL_BC_PERIODIC = 0, MSL_BC_FIXED_EQ = 1, MSL_BC_OUTFLOW_ZG = 2, MSL_BC_DIFFUSE_WALL = 3 };
/* refinement criterion (Sec. III.A): local Mach number; |Pi_neq|_F / p; local
 * Knudsen number Kn = lambda / L, L = rho / |grad rho| (Sec. IV.A.3), with
 * the hard-sphere mean free path lambda = 16/(5 sqrt(2 pi gamma)) mu a / p of
 * the cell's own state (a = sqrt(gamma T), p = rho T, mu = (tau - 1/2) rho T dt
 * of the collision) and central differences of the cell densities (one-sided
 * over one cell across a face that is not periodic).  MSL_CRIT_KN takes
 * 16 bytes of workspace per cell. */
enum { MSL_CRIT_NONE = 0, MSL_CRIT_MA = 1, MSL_CRIT_PINEQ = 2, MSL_CRIT_KN = 3 };

typedef struct msl_config {
  int dim, nx, ny, nz;        /* nz ignored (1) when dim == 2 */
  int n_low, n_high;          /* 1D Gauss-Hermite orders (Tab. I): 3 D2Q9/D3Q27, 4 D2Q16/D3Q64,
                                 5 D2Q25, 6 D2Q36; n_high = 0 runs one velocity set */
  int thermal;                /* 0: athermal (T = T_L = 1), f only; 1: f and g populations,
                                 ideal gas with specific heat cv (Sec. II.B) */
  double tau, cv, cfl;        /* BGK relaxation time; cv; CFL = max|c_i| dt/dx (Sec. IV) */
  int tau_mode;               /* 0 constant tau; 1 mu = mu_ref (T/tau_ref_T)^mu_exp with
                                 mu_ref = (tau - 1/2) tau_ref_rho tau_ref_T dt */
  double mu_exp, tau_ref_rho, tau_ref_T;
  double rho0, T0;            /* reference state of the 16-bit deviation storage */
  int store;                  /* MSL_FP64 .. MSL_BF16_DEV */
  int lift_mode;              /* MSL_LIFT_* */
  int bc[6];                  /* MSL_BC_* per face: x-, x+, y-, y+, z-, z+ */
  double bc_state[6][5];      /* fixed-equilibrium state rho, ux, uy, uz, T; walls: u_w, T_w */
  double slot_state[6][5];    /* state inside the face's slot */
  int slot[6][4];             /* slot [lo0,hi0) x [lo1,hi1) on the face's tangential axes
                                 (ascending axis order); lo0 >= hi0: no slot */
  double slot_edge[6];        /* > 0: the face state blends from bc_state to slot_state with
                                 weight 1/2[tanh((t-lo+1/2)/w) - tanh((t-hi+1/2)/w)] per
                                 restricted tangential axis; 0: sharp slot */
  int crit_kind;              /* MSL_CRIT_* */
  double crit_thr;
  int crit_every;             /* evaluate the criterion every k steps (from step 0); 0: never */
  int check_every;            /* conservation sentinel every k steps (synchronises); 0: never */
  int mlp_hidden;             /* hidden width of the closure (lift_mode MLP); 0 -> 64 */
  int mlp_check_every;        /* closure error check every k steps; 0 -> 20 */
  double u_ref[3], T_ref;     /* global constant reference frame (eq. veli, Sec. II.A): every
                                 population moves with v_i = sqrt(T_ref) c_i + u_ref, and
                                 moments, equilibria (eqs. feqL, geqL with this frame as the
                                 target of eq. fll), lifting and projection are taken in these
                                 velocities; u_ref = 0, T_ref = 1 is the lattice frame of
                                 Sec. II.C.2.  T_ref <= 0 stands for 1.  The learned closure
                                 needs the lattice frame. */
  double store_u[3];          /* velocity of the 16-bit storage reference state
                                 (rho0, store_u, T0): population f_i is stored as
                                 h = f_i / s_i - 1 (g_i: scale (cv - D/2) T0 s_i) with
                                 s_i = rho0 prod_a w_a r(c_a), r the density ratio of the
                                 Gaussian N(z_a, T0/T_ref) to N(0, 1) at the node and
                                 z = (store_u - u_ref) / sqrt(T_ref); s_i = rho0 W_i when
                                 the storage reference is the frame's rest state */
  double tau2;                /* > 0 and != tau: the two-relaxation quasi-equilibrium model of
                                 eqs. Pond_f/g (Sec. II.B, eqs. fqeq, gqeq): stress relaxes at
                                 1/tau, the non-equilibrium third moment and heat flux at
                                 omega2 = 1/tau2, Pr = (tau - 1/2)/(tau2 - 1/2) (kept where tau
                                 follows mu(T)); 2D only.  Otherwise BGK (omega1 = omega2). */
  int pond;                   /* 1: co-moving reference frames (PonD, Sec. II.C.1): every cell
                                 keeps its populations in its own frame {u, T}, a step runs the
                                 predictor-corrector (eqs. correctorfields) to convergence and
                                 collides in the converged frame (eqs. feqPond, geqPond).  With
                                 two velocity sets, a collocation point of the other set is
                                 lifted or projected into the cell's set in its own frame
                                 (lift_mode Grad or Hermite), and the sets are those of
                                 msl_set_mask or, with crit_kind MSL_CRIT_KN, re-selected every
                                 crit_every steps from each cell's own state.  Needs dim 2, FP64
                                 storage, no other criterion and the lattice frame; faces
                                 periodic, fixed-equilibrium, zero-gradient or diffuse walls
                                 (y faces; the wall's co-moving equilibrium in the wall's frame
                                 at the density balancing the wall-normal flux of the adjacent
                                 cell, both counted in the wall's frame); dt = cfl / max|c| of
                                 the sets, and a step whose departure point leaves the two-cell
                                 reach in some frame returns MSL_EUNSTABLE (lower cfl).
                                 Populations out (msl_get_populations) are given in each cell's
                                 own frame (msl_pond_frames); populations in, conservation sums,
                                 error norms and checkpoints are not offered.  0: one global
                                 frame. */
  int crit_margin;            /* >= 0: the high-order set also takes every cell within this many
                                 cells (per axis, a box; periodic faces wrap) of a cell the
                                 criterion selects; 0: the criterion's cells only (the paper's
                                 rule).  At most 1024. */
} msl_config;

typedef struct msl_ctx msl_ctx;

/* Device workspace size (bytes) that msl_create needs for `cfg`.  MSL_EINVAL
 * for an invalid configuration, including a grid of 2^31 cells or more, or one
 * whose padded population plane (ghosts included) takes 2^31 bytes or more in
 * the storage precision: the kernels address a plane with 32-bit byte offsets
 * and drop the stores of foreign cells at offset 2^31, which must lie beyond
 * the plane. */
int msl_workspace_bytes(const msl_config *cfg, size_t *bytes);

/* Validates `cfg`, builds the velocity-set tables (Gauss-Hermite rules,
 * dt = cfl / max|c|, stencil offsets and Lagrange weights, lifting and
 * projection matrices) and lays the state out inside `workspace` (device, at
 * least msl_workspace_bytes; caller-owned, must outlive the context).
 * `hip_stream` is a hipStream_t (NULL: the null stream).  The mask starts all
 * low order; the state is undefined until msl_init.  Errors: MSL_EINVAL
 * (n_low >= n_high, tau <= 1/2, unsupported order/dim, stencil reach beyond
 * the ghost layers, diffuse walls on non-y/z faces, grid smaller than the
 * stencil, grid of 2^31 cells or more, padded plane of 2^31 bytes or more,
 * learned lifting outside the lattice frame), MSL_ENOMEM (bytes too small),
 * MSL_EHIP. */
int msl_create(const msl_config *cfg, void *workspace, size_t bytes, void *hip_stream,
               msl_ctx **out);
void msl_destroy(msl_ctx *ctx);   /* frees the host-side context only */
const char *msl_last_error(const msl_ctx *ctx);
int msl_get_dt(const msl_ctx *ctx, double *dt);   /* host out */

/* Populations from macroscopic fields (device FP64 arrays rho[ncell],
 * u[dim][ncell], T[ncell]; T may be NULL when athermal): every cell gets the
 * lattice equilibrium of its current order (eqs. feqL, geqL); cells next to the
 * other order also get their converted state. */
int msl_init(msl_ctx *ctx, const double *rho, const double *u, const double *T);

/* Velocity-set switching (Sec. III.A): `mask` (device uint8[ncell], 0 low /
 * 1 high order).  After msl_init, every cell whose order changes lifts or
 * projects its own state; the band of cells bordering the other order is
 * rebuilt.  Errors: MSL_EINVAL for a value other than 0/1 or 1 without a high
 * order (checked on the device; this call synchronises only then). */
int msl_set_mask(msl_ctx *ctx, const uint8_t *mask);
int msl_get_mask(msl_ctx *ctx, uint8_t *mask);      /* device out */

/* `nsteps` time steps (Sec. III.D): [criterion + switching every crit_every
 * steps], ghost fill, stream-and-collide of each order, band conversion.
 * Asynchronous unless check_every > 0; then MSL_EUNSTABLE reports a failed
 * sentinel (the state is left as is). */
int msl_step(msl_ctx *ctx, int nsteps);
/* How msl_step issues its launches (an execution choice; every mode gives the
 * same bits).  mode 0 (the default): launch by launch.  mode 1: 2D contexts
 * without the learned closure and without a conservation check run blocks of
 * steps between criterion passes (crit_every steps when that is at most 64,
 * else 16) as HIP graphs: the first block that starts from each of the two
 * population buffers is captured (host and device memory for the instantiated
 * graph, held until msl_destroy or a mode change) and replayed on the
 * context's stream.  mode 2: as 1, with the two sets' stream-collide launches
 * on parallel branches of the graph; in contexts that run no graphs (3D, the
 * learned closure, a conservation check) the two launches of each step still
 * run on two streams, forked and joined by events (a second stream and two
 * events, created once, held until msl_destroy).  Criterion passes, steps that
 * msl_profile times and the rest of a call shorter than a block run launch by
 * launch.  A context whose high-order set runs over a compact tile list (large
 * grids, where the host reads the list length) turns to mode 0 at its first
 * capture.  Under a stream capture of the caller's own, use mode 0.  EINVAL
 * for other modes. */
int msl_set_graph(msl_ctx *ctx, int mode);
int msl_get_step(const msl_ctx *ctx, long *step);   /* host out */

/* rho, u[dim], T per cell from each cell's own populations (Sec. II.B
 * conservation laws, eq. E); device FP64 outputs, any may be NULL. */
int msl_macros(msl_ctx *ctx, double *rho, double *u, double *T);

/* Populations of order `which` (0 low, 1 high), f (fg = 0) or g (fg = 1), as
 * device FP64 [Q][ncell].  Values are meaningful at cells of that order and at
 * band cells of the other order; elsewhere they are stale. */
int msl_get_populations(msl_ctx *ctx, int which, int fg, double *out);
/* Overwrite the stored populations of order `which` at the cells of that order
 * (device FP64 [Q][ncell]); the band is re-converted. */
int msl_set_populations(msl_ctx *ctx, int which, int fg, const double *in);

/* Global sums over each cell's own populations: rho, rho u_x, rho u_y, rho u_z,
 * rho E (host out[5], FP64, deterministic order).  Synchronises. */
int msl_conservation(msl_ctx *ctx, double *out);

/* Co-moving frames (pond = 1): each cell's frame as device FP64
 * out[4][cells] = u_x, u_y, u_z (0), T.  MSL_EINVAL for other contexts. */
int msl_pond_frames(msl_ctx *ctx, double *out);
/* Co-moving frames: predictor-corrector passes of the last msl_step call,
 * mean per cell and step and maximum (host).  Synchronises. */
int msl_pond_iterations(msl_ctx *ctx, double *mean, int *max);

/* Error norms of the macroscopic fields (Sec. II.B moments of each cell's own
 * populations, as msl_macros) against caller reference fields: rho_ref
 * [cells], u_ref [dim][cells], T_ref [cells], device FP64 in msl_macros'
 * layout; a NULL reference skips that field.  out (host, 6 doubles): for rho,
 * u, T in turn the relative L2 norm sqrt(sum |x - x_ref|^2 / sum |x_ref|^2)
 * (u: Euclidean norm over the components; the root mean square of the
 * difference where the reference is zero everywhere) and the maximum of
 * |x - x_ref| over the cells; 0 for skipped fields.  FP64 sums: wave
 * shuffles, LDS, then a second pass over the per-block partials (fixed order,
 * deterministic).  Synchronises the stream. */
int msl_error_norms(msl_ctx *ctx, const double *rho_ref, const double *u_ref, const double *T_ref,
                    double *out);

/* Checkpoint: the raw planes, mask, step counter and closure weights to a host
 * buffer; *bytes in: capacity, out: size used (buf NULL: size query).
 * Synchronises.  Restoring on a context of the same config resumes bit-exactly. */
int msl_get_state(msl_ctx *ctx, void *host_buf, size_t *bytes);
int msl_set_state(msl_ctx *ctx, const void *host_buf, size_t bytes);

/* ---- learned lifting closure (not in the paper; replaces the equilibrium
 * completion M^eq_{Q-q} of Sec. III.B by M^eq_{Q-q} + rho T^{|p|/2} t_p) ---- */

/* Sizes of the closure: F inputs, O outputs, H hidden, P parameters. */
int msl_mlp_dims(const msl_ctx *ctx, int *F, int *O, int *H, int *P);
/* From a run on the high-order set: for each high-order cell, the features of
 * its projected low-order state and the normalised non-equilibrium parts of the
 * missing raw moments.  Device float outputs feats[max][F], targets[max][O];
 * *n (host) receives the number written.  Synchronises. */
int msl_collect_snapshots(msl_ctx *ctx, float *feats, float *targets, int max, int *n);
/* Install / read the closure: params[P] (layout W1[F][H] b1[H] W2[H][H] b2[H]
 * W3[H][O] b3[O]), feature mean/std [F], target mean/std [O]; host float. */
int msl_mlp_set_weights(msl_ctx *ctx, const float *params, const float *xmean,
                        const float *xstd, const float *tmean, const float *tstd);
int msl_mlp_get_weights(msl_ctx *ctx, float *params);
/* Adam training on the GPU with the BF16 MFMA kernels: device float
 * X[n][F] (standardised features), Y[n][O] (standardised targets); batches of
 * `batch` rows in order, `epochs` passes; loss per step written to host
 * loss_log[steps] when not NULL.  Weights start from the installed ones.
 * Synchronises. */
int msl_mlp_train(msl_ctx *ctx, const float *X, const float *Y, int n, int batch, int epochs,
                  float lr, float *loss_log);
/* One forward and backward pass over device X[n][F], Y[n][O]: loss (host) and
 * gradient (device float[P]).  For gradient checks.  Synchronises. */
int msl_mlp_grad(msl_ctx *ctx, const float *X, const float *Y, int n, float *loss, float *grad);
/* msl_mlp_grad for callers that cannot allocate device memory or touch a
 * workspace beyond their inputs and outputs (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation): the same loss
 * (host) and gradient (device float[P]) from the same kernels, with the
 * per-workgroup gradient and loss partials kept in a static device array of
 * the library (4 MiB = 2^20 floats per GPU, held until the process ends)
 * instead of the context's workspace.  Calls no hipMalloc / hipFree.  The
 * scratch needs ceil(n/64) * (P + 1) + 1 floats; larger requests (and n <= 0
 * or n > 16384) return MSL_EINVAL with msl_last_error saying why.  Every call
 * on one GPU shares that GPU's array: calls that overlap in time on the same
 * GPU (other streams or threads) race.  Synchronises the context's stream. */
int msl_mlp_grad_noalloc(msl_ctx *ctx, const float *X, const float *Y, int n, float *loss,
                         float *grad);
/* Forward pass only: device Yout[n][O]. */
int msl_mlp_forward(msl_ctx *ctx, const float *X, int n, float *Yout);
/* Per check tile (64 x 64 (x 64) cells): 1 if the closure passed its error
 * check (used), 0 if that tile falls back to Grad lifting; device uint8 out /
 * in.  Setting flags disables the automatic check. */
int msl_mlp_get_flags(msl_ctx *ctx, uint8_t *flags);
int msl_mlp_set_flags(msl_ctx *ctx, const uint8_t *flags);
int msl_num_check_tiles(const msl_ctx *ctx, int *n);

/* ---- measurement ---- */

/* Per-kernel timing of msl_step with HIP events recorded on the context's
 * stream around the launches of every `every`-th step (every >= 1; 0
 * disables; a second call changes the period).  Each event record costs the
 * stream a few microseconds, so sampling keeps the timed run close to an
 * untimed one.  The events form a ring of 2048 launches; when it is
 * three-quarters full the host waits for the oldest half, which completed long
 * before, so the stream never drains.  The number of high-order cells in force
 * (which sets the bytes of a stream-collide launch) is written by the GPU into
 * a small pinned host buffer that the first enable allocates (hipHostMalloc)
 * and msl_destroy frees.  EINVAL for every < 0. */
int msl_profile(msl_ctx *ctx, int every);
/* stats[k][0..3] for launch class k = 0 ghost fill, 1 stream-collide of the
 * low-order set, 2 stream-collide of the high-order set, 3 band conversion,
 * 4 criterion and switching, 5 learned closure: number of launches, total
 * milliseconds, algorithmic bytes (classes 1, 2: read and write of every
 * population of each cell of that order), cells updated.  Host out, 24
 * doubles; the counters restart.  Synchronises. */
int msl_profile_read(msl_ctx *ctx, double *stats);
/* Plain device-to-device copy of `bytes` (a multiple of 16) on `hip_stream`:
 * the bandwidth reference for roofline figures.  Device pointers. */
int msl_device_copy(void *dst, const void *src, size_t bytes, void *hip_stream);

#ifdef __cplusplus
}
#endif
#endif
