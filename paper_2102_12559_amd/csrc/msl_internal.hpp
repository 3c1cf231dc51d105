// msl_internal.hpp -- shared declarations of the MI355X library: device-side
// tables, grid geometry, storage codecs and the host context.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/msl.h"

#define MSL_MAXN 8
#define MSL_MAXQ 64   // largest velocity set (D3Q64)
#define MSL_G 2            // ghost layers (stencil reach of a 3-point stencil at CFL <= 1)
#define MSL_TX 64          // tile width in x (one wavefront)
#define MSL_MTY 4          // micro-tile height (rows) of the per-tile class flags
#define MSL_CHECK_TILE 64  // check tiles of the learned closure
#define MSL_PROF_REC 2048  // ring of timed launches (the oldest half is read while the rest run)
#define MSL_PROF_K 6       // launch classes of msl_profile_read
#define MSL_MLP_MAXBLK 256       // workgroups of one training step (64 rows each)
#define MSL_MLP_LOSS_RING 65536  // device loss history of the training steps

// Per velocity set: 1D Gauss-Hermite nodes c_a (in the units of the run's
// reference frame) and weights, the Hermite-weighted basis of the
// equilibrium, the particle velocity of every node along each axis
// (v = sqrt(T_ref) c + u_ref, eq. veli), the 1D stencil (base offset and 3
// Lagrange weights) of each node's departure point along each axis, the
// frame's map of (u, T) to the equilibrium arguments, and the storage scale of
// every f population.
struct LatTab {
  int n, Q;
  double cr[MSL_MAXN], w[MSL_MAXN];
  double hw[MSL_MAXN][MSL_MAXN];   // w_a He_j(c_a) / j!
  double v[3][MSL_MAXN];           // particle velocity of node a along axis
  int n0[3][MSL_MAXN];
  double a[3][MSL_MAXN][3];
  // equilibrium in the frame: per-axis factors at (u - ur) isq with reduced
  // temperature T iTr (isq = 1/sqrt(T_ref), iTr = 1/T_ref)
  double ur[3], isq, iTr;
  double sc[MSL_MAXQ];             // 16-bit storage scale of f_i (g_i: gfac T0 sc[i])
  double isc[MSL_MAXQ];            // 1 / sc[i]
  float vf[3][MSL_MAXN], wf[MSL_MAXN];
  float hwf[MSL_MAXN][MSL_MAXN];
  float af[3][MSL_MAXN][3];
  float scf[MSL_MAXQ], iscf[MSL_MAXQ];
};

struct Tab {
  LatTab lat[2];
  // lift, raw completion in the frame's velocities, per axis: K[ax][a][a']
  // (high node a, low node a')
  double K[3][MSL_MAXN][MSL_MAXN];
  double KH[MSL_MAXN][MSL_MAXN];   // lift, Hermite completion
  double P[MSL_MAXN][MSL_MAXN];    // project: P[a'][a] = l^low_{a'}(C_a)
  double Vi[MSL_MAXN][MSL_MAXN];   // inverse Vandermonde of the high nodes: Vi[a][m]
  double dt, cv, gfac, tau, omega, mu_ref, mu_exp, tau_ref_T, rho0, T0;
  // two-relaxation model: 1/omega2 - 1/2 = qe_ratio (1/omega1 - 1/2), with
  // qe_ratio = (tau2 - 1/2)/(tau - 1/2) = 1/Pr; qe = 0: BGK
  double qe_ratio;
  int qe;
  double igsc;    // 1 / (gfac T0): the g scale is gfac T0 sc[i] (0 when athermal)
  float igscf;
  double mu_T1;   // mu_ref (1 / tau_ref_T)^mu_exp: the viscosity at T = 1
  float omegaf;
  int tau_mode, thermal, dim, nlat, lift_mode;
  // diffuse walls, per face and velocity set: the equilibrium at the wall state
  // with unit density, and its flux of particles leaving the wall
  double wall_eq[6][2][MSL_MAXQ];
  double wall_out[6][2];
};

struct Geo {
  int nx, ny, nz, dim;
  int xo;                 // column of interior x = 0 inside a row
  int pitch;              // elements per row
  int rows;               // ny + 2G
  int slabs;              // nz + 2G (3D) or 1
  long long plane;        // elements per population plane
  long long ncell;
  int ntx, nty, ntz;      // micro-tiles (64 x 4 (x 1))
  // element offset of interior cell (x, y, z) inside a plane (planes are
  // padded so that every staged window of a tile stays inside the plane)
  __host__ __device__ int idx(int x, int y, int z) const {
    int zz = dim == 3 ? z + MSL_G : 0;
    return (zz * rows + (y + MSL_G)) * pitch + xo + x;
  }
};

// ---------------------------------------------------------------------------
// storage codecs: FP64 / FP32 populations, or 16-bit deviations
// h = f / (rho0 W_i) - 1 (g: scale (cv - D/2) rho0 T0 W_i) in FP16 or BF16,
// rounded to nearest even.
// ---------------------------------------------------------------------------
struct bf16_t { uint16_t u; };

template <typename S> struct StoreTraits;
template <> struct StoreTraits<double> {
  using C = double;
  static constexpr bool dev = false;
  __device__ static double load(double v) { return v; }
  __device__ static double store(double v) { return v; }
};
template <> struct StoreTraits<float> {
  using C = float;
  static constexpr bool dev = false;
  __device__ static float load(float v) { return v; }
  __device__ static float store(float v) { return v; }
};
template <> struct StoreTraits<_Float16> {
  using C = float;
  static constexpr bool dev = true;
  __device__ static float load(_Float16 v) { return (float)v; }
  __device__ static _Float16 store(float v) { return (_Float16)v; }
};
template <> struct StoreTraits<bf16_t> {
  using C = float;
  static constexpr bool dev = true;
  __device__ static float load(bf16_t v) { return __uint_as_float(((uint32_t)v.u) << 16); }
  __device__ static bf16_t store(float v) {
    uint32_t b = __float_as_uint(v);
    bf16_t r;
    if ((b & 0x7fffffffu) > 0x7f800000u) { r.u = (uint16_t)((b >> 16) | 0x40u); return r; }
    b += 0x7fffu + ((b >> 16) & 1u);
    r.u = (uint16_t)(b >> 16);
    return r;
  }
};

// ---------------------------------------------------------------------------
// host context
// ---------------------------------------------------------------------------
struct msl_ctx {
  msl_config cfg;
  hipStream_t stream;
  int device;             // the device current at msl_create
  char err[256];
  Geo geo;
  int D, nlat, Q[2];
  long long ncell;
  Tab htab;
  Tab *dtab;
  size_t esz;
  char *planes[2][2];     // [lattice][buffer]: f planes then g planes
  int cur;
  uint8_t *cls;           // bit0 order (0 low, 1 high), bit1 band
  uint8_t *newmask;
  double *kn_rho, *kn_lam;   // Knudsen-number criterion: density and mean free path per cell
  // co-moving frames: populations [NP][ncell] of each velocity set and
  // buffer ([set][buffer]) and frames [4][ncell] of each buffer; stats:
  // iteration sum (u64), then maximum (int)
  double *pond_f[2][2], *pond_fr[2];
  double *pond_wall;      // diffuse y walls: wall density per column [2][nx] (low, high face)
  unsigned long long *pond_stats;
  long long pond_cells_steps;
  uint8_t *tflag;         // per micro-tile: bit0 has low cells, bit1 has high cells
  int *blist[2];          // band cells of each order, ascending cell index
  int *bcount;            // device: [0] low band, [1] high band counts
  int *blk;               // compaction scratch: per-block counts / offsets (2 lists)
  int nblk;
  double *red;            // reduction partials
  int nred;
  int *flag;              // device error flag (mask values)
  double *wall_rho;       // diffuse wall densities
  long step;
  int initialized;
  // 3D, x periodic: the step's stream-collide and band conversion also write
  // the x ghost columns of the new buffer (xmir), so the next ghost fill
  // leaves out the x faces while xg_ok says they hold the current values
  int xmir, xg_ok;
  // live tiles of the high-order set, ascending (sparse stream-collide
  // launches walk this list instead of the whole tile grid); tl_ok: the list
  // matches the current tile flags
  int *tlist, *tcount;
  int tl_ok, tl_n;        // tl_n: host copy of the count, read when the list is built
  // learned closure
  int mlpF, mlpO, mlpH, mlpP, mlp_on, mlp_manual;
  float *mlp_w;           // fp32 master parameters [P]
  float *mlp_stats;       // xmean[F], xstd[F], tmean[O], tstd[O]
  float *mlp_feat;        // [ncell cap][F] features of band cells
  float *mlp_out;         // [ncell cap][O]
  float *mlp_m, *mlp_v, *mlp_g;  // Adam moments, gradient
  float *mlp_loss;        // device scalars
  uint8_t *mlp_flag;      // per check tile
  double *mlp_err;        // per check tile: E_mlp, E_grad
  float *mlp_gpart;       // per-block gradient partials [MSL_MLP_MAXBLK][P], then loss partials
  float *mlp_tgt;         // check: true normalised targets of the high-order band cells
  double *mlp_cerr;       // check: per-cell E_mlp, E_grad
  long mlp_steps;         // Adam steps taken
  int nctile, nct[3];
  // per-kernel timing with HIP events (msl_profile)
  int prof;
  hipEvent_t ev[2 * MSL_PROF_REC];
  long long nrec, ndone;  // records issued / read
  int rec_cls[MSL_PROF_REC];
  int rec_lat[MSL_PROF_REC];      // stream-collide: velocity set; else -1
  int rec_slot[MSL_PROF_REC];     // high-order cell count snapshot in force
  double rec_bpc[MSL_PROF_REC];   // algorithmic bytes per cell update
  double rec_cells[MSL_PROF_REC];
  double pstat[MSL_PROF_K][4];
  int *prof_nh;           // pinned host ring of high-order cell counts, written by the GPU
  long long nsnap;
  // step graphs (2D): blocks of gB steps without a criterion pass, captured
  // once per parity of the current buffer at the block's start and replayed.
  // gmode 0: launches one by one; 1: one graph of the launches in stream
  // order; 2: the same with the two sets' stream-collide launches on
  // parallel branches.  capturing: a capture of this context is under way
  // (paths that need the host inside a step refuse it).
  int gmode, gB, capturing;
  // the stream-collide launches convert the band cells themselves (no band
  // conversion launch in a step)
  int fuse;
  // 2D zero-gradient faces applied by the stream-collide launches to their
  // staged windows (bits: x low, x high, y low, y high); set when every face
  // is zero-gradient or fixed, and then no ghost fill runs per step
  int zgm;
  hipStream_t gs[2];
  hipEvent_t gev[2];
  hipGraphExec_t gx[2];
};

// launch helpers implemented in the .hip files
// oth: the other set's new planes, written at this set's band cells (2D
// two-set contexts where msl_stream_sc2_all holds); nullptr: no conversion
int msl_launch_stream_collide(msl_ctx *c, int lat, const char *in, char *out, char *oth);
// every set of a 2D context runs the stream-collide kernel with all planes
// resident in LDS
int msl_stream_sc2_all(const msl_ctx *c);
int msl_launch_tile_list(msl_ctx *c, int lat, int rows_per_tile, int planes_per_tile);
int msl_launch_bc(msl_ctx *c, char *buf_low, char *buf_high);
int msl_launch_bc_fixed(msl_ctx *c);
int msl_launch_band_convert(msl_ctx *c, char *buf_low, char *buf_high);
int msl_launch_init_eq(msl_ctx *c, const double *rho, const double *u, const double *T);
int msl_launch_criterion(msl_ctx *c);
int msl_launch_switch(msl_ctx *c, const uint8_t *newmask);
int msl_launch_classify(msl_ctx *c);
int msl_launch_macros(msl_ctx *c, double *rho, double *u, double *T);
int msl_launch_pops(msl_ctx *c, int which, int fg, double *out, const double *in);
int msl_launch_conservation(msl_ctx *c, double *dev_out5);
int msl_pond_launch_init(msl_ctx *c, const double *rho, const double *u, const double *T);
int msl_pond_launch_macros(msl_ctx *c, double *rho, double *u, double *T);
int msl_pond_launch_step(msl_ctx *c);
// co-moving frames, two sets: cells whose set differs from `mask` convert their
// own state in their own frame (convert = 0: only the sets change), then the
// band is rebuilt and converted
int msl_pond_launch_set_mask(msl_ctx *c, const uint8_t *mask, int convert);
int msl_launch_kn_mask(msl_ctx *c);
// the criterion's margin (crit_margin > 0): newmask dilated by a box per axis
int msl_launch_dilate(msl_ctx *c);
int msl_launch_error_norms(msl_ctx *c, const double *rref, const double *uref, const double *Tref,
                           double *dev_out6);
int msl_launch_check_mask(msl_ctx *c, const uint8_t *mask);
int msl_launch_get_mask(msl_ctx *c, uint8_t *mask);
// closure
int msl_mlp_band_lift(msl_ctx *c, char *buf_low, char *buf_high);
int msl_mlp_check_launch(msl_ctx *c);
int msl_mlp_snapshots_launch(msl_ctx *c, float *feats, float *targets, int max, int *count_dev);
int msl_mlp_forward_launch(msl_ctx *c, const float *X, int n, float *Y);
int msl_mlp_grad_launch(msl_ctx *c, const float *X, const float *Y, int n, float *grad,
                        float *loss_dev);
int msl_mlp_adam_launch(msl_ctx *c, int t, float lr);
int msl_noalloc_setup(int device);

#define MSL_HIP(call)                                                       \
  do {                                                                      \
    hipError_t e_ = (call);                                                 \
    if (e_ != hipSuccess) return MSL_EHIP;                                  \
  } while (0)
