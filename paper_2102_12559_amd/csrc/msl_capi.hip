// msl_capi.hip -- the C-ABI entry points: configuration checks, velocity-set
// tables, workspace layout and the time-step driver.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <new>

#include "msl_device.hpp"

typedef long double ld;

// ---------------------------------------------------------------------------
// host tables
// ---------------------------------------------------------------------------

// Gauss-Hermite rule for the weight exp(-c^2/2)/sqrt(2 pi) by the Golub-Welsch
// method: the nodes are the eigenvalues of the Jacobi matrix of the orthonormal
// Hermite recurrence x p_k = sqrt(k+1) p_{k+1} + sqrt(k) p_{k-1}, the weights
// the squared first components of its unit eigenvectors.  Cyclic Jacobi
// rotations in long double.
static int gauss_hermite(int n, ld *x, ld *w) {
  if (n < 1 || n > MSL_MAXN) return -1;
  ld A[MSL_MAXN][MSL_MAXN] = {{0}}, V[MSL_MAXN][MSL_MAXN] = {{0}};
  for (int k = 0; k < n; ++k) V[k][k] = 1.0L;
  for (int k = 0; k + 1 < n; ++k) A[k][k + 1] = A[k + 1][k] = sqrtl((ld)(k + 1));
  for (int sweep = 0; sweep < 100; ++sweep) {
    ld off = 0;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) off += A[p][q] * A[p][q];
    if (off < 1e-60L) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        if (A[p][q] == 0.0L) continue;
        const ld th = (A[q][q] - A[p][p]) / (2.0L * A[p][q]);
        const ld t = (th >= 0 ? 1.0L : -1.0L) / (fabsl(th) + sqrtl(th * th + 1.0L));
        const ld cs = 1.0L / sqrtl(t * t + 1.0L), sn = t * cs;
        for (int k = 0; k < n; ++k) {
          const ld akp = A[k][p], akq = A[k][q];
          A[k][p] = cs * akp - sn * akq;
          A[k][q] = sn * akp + cs * akq;
        }
        for (int k = 0; k < n; ++k) {
          const ld apk = A[p][k], aqk = A[q][k];
          A[p][k] = cs * apk - sn * aqk;
          A[q][k] = sn * apk + cs * aqk;
        }
        for (int k = 0; k < n; ++k) {
          const ld vkp = V[k][p], vkq = V[k][q];
          V[k][p] = cs * vkp - sn * vkq;
          V[k][q] = sn * vkp + cs * vkq;
        }
      }
  }
  // sort ascending
  int idx[MSL_MAXN];
  for (int k = 0; k < n; ++k) idx[k] = k;
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j)
      if (A[idx[j]][idx[j]] < A[idx[i]][idx[i]]) { int t = idx[i]; idx[i] = idx[j]; idx[j] = t; }
  for (int k = 0; k < n; ++k) {
    x[k] = A[idx[k]][idx[k]];
    w[k] = V[0][idx[k]] * V[0][idx[k]];
  }
  // symmetrise (the rule is symmetric about 0)
  for (int k = 0; k < n / 2; ++k) {
    const ld xs = 0.5L * (x[n - 1 - k] - x[k]), ws = 0.5L * (w[k] + w[n - 1 - k]);
    x[k] = -xs; x[n - 1 - k] = xs;
    w[k] = ws; w[n - 1 - k] = ws;
  }
  if (n % 2) x[n / 2] = 0.0L;
  return 0;
}

static ld hermite_he(int j, ld x) {
  ld h0 = 1.0L, h1 = x;
  if (j == 0) return h0;
  for (int k = 1; k < j; ++k) {
    const ld h2 = x * h1 - (ld)k * h0;
    h0 = h1;
    h1 = h2;
  }
  return h1;
}

// coefficients (ascending powers) of the Lagrange basis polynomial l_a of `nodes`
static void lagrange_coeffs(int n, const ld *nodes, int a, ld *coef) {
  ld p[MSL_MAXN + 1] = {0};
  p[0] = 1.0L;
  int deg = 0;
  ld den = 1.0L;
  for (int b = 0; b < n; ++b) {
    if (b == a) continue;
    for (int k = deg + 1; k >= 1; --k) p[k] = p[k - 1] - nodes[b] * p[k];
    p[0] = -nodes[b] * p[0];
    ++deg;
    den *= nodes[a] - nodes[b];
  }
  for (int k = 0; k < n; ++k) coef[k] = p[k] / den;
}

static ld lagrange_eval(int n, const ld *nodes, int a, ld x) {
  ld v = 1.0L;
  for (int b = 0; b < n; ++b)
    if (b != a) v *= (x - nodes[b]) / (nodes[a] - nodes[b]);
  return v;
}

// One velocity set of 1D order n in the run's frame {u_ref, T_ref} (eq. veli):
// Gauss-Hermite nodes c_a and weights (Tab. I), the Hermite-weighted basis of
// the equilibrium, the particle velocity v = sqrt(T_ref) c_a + u_ref of every
// node along each axis with the 3-point stencil of its departure point
// x - v dt, and the 16-bit storage scale of every population: the weight
// rho0 W_i carried over to the storage reference state (rho0, store_u, T0),
// rho0 prod_a w_a r(c_a) with r the density ratio of the Gaussian N(z_a, th)
// to N(0, 1), z = (store_u - u_ref)/sqrt(T_ref), th = T0/T_ref.
static void build_lat(LatTab &L, int n, int dim, const ld *x, const ld *w, double dt,
                      const double *ur, double Tr, const double *su, double rho0, double T0) {
  memset(&L, 0, sizeof(L));
  L.n = n;
  L.Q = dim == 2 ? n * n : n * n * n;
  const ld sq = sqrtl((ld)Tr);
  for (int a = 0; a < n; ++a) {
    L.cr[a] = (double)x[a];
    L.w[a] = (double)w[a];
    L.wf[a] = (float)w[a];
    ld fact = 1.0L;
    for (int j = 0; j < n; ++j) {
      if (j > 0) fact *= (ld)j;
      const ld v = w[a] * hermite_he(j, x[a]) / fact;
      L.hw[a][j] = (double)v;
      L.hwf[a][j] = (float)v;
    }
  }
  for (int ax = 0; ax < 3; ++ax) {
    const ld u = ax < dim ? (ld)ur[ax] : 0.0L;
    L.ur[ax] = (double)u;
    for (int a = 0; a < n; ++a) {
      const ld v = sq * x[a] + u;
      L.v[ax][a] = (double)v;
      L.vf[ax][a] = (float)v;
      // departure point x - v dt: base node n0 = nearest integer offset, xi in [-1/2, 1/2)
      const ld d = -v * (ld)dt;
      const int n0 = (int)floorl(d + 0.5L);
      const ld xi = d - (ld)n0;
      const ld wts[3] = {0.5L * xi * (xi - 1.0L), 1.0L - xi * xi, 0.5L * xi * (xi + 1.0L)};
      L.n0[ax][a] = n0;
      for (int s = 0; s < 3; ++s) {
        L.a[ax][a][s] = (double)wts[s];
        L.af[ax][a][s] = (float)wts[s];
      }
    }
  }
  L.isq = (double)(1.0L / sq);
  L.iTr = (double)(1.0L / (ld)Tr);
  const ld th = (ld)T0 / (ld)Tr;
  for (int i = 0; i < L.Q; ++i) {
    ld s = (ld)rho0;
    for (int ax = 0, r = i; ax < dim; ++ax, r /= n) {
      const ld z = ((ld)su[ax] - (ld)ur[ax]) / sq, c = x[r % n];
      s *= w[r % n] * expl(0.5L * c * c - 0.5L * (c - z) * (c - z) / th) / sqrtl(th);
    }
    L.sc[i] = (double)s;
    L.scf[i] = (float)s;
    L.isc[i] = (double)(1.0L / s);
    L.iscf[i] = (float)(1.0L / s);
  }
}

static void set_err(msl_ctx *c, const char *m) {
  if (c) snprintf(c->err, sizeof(c->err), "%s", m);
}

// ---------------------------------------------------------------------------
// configuration checks and workspace layout
// ---------------------------------------------------------------------------

static size_t store_size(int s) {
  switch (s) {
    case MSL_FP64: return 8;
    case MSL_FP32: return 4;
    case MSL_FP16_DEV:
    case MSL_BF16_DEV: return 2;
  }
  return 0;
}

static const char *check_config(const msl_config *cfg) {
  if (!cfg) return "null config";
  if (cfg->dim != 2 && cfg->dim != 3) return "dim must be 2 or 3";
  if (cfg->nx < 4 || cfg->ny < 4 || (cfg->dim == 3 && cfg->nz < 4)) return "grid smaller than the stencil";
  const int maxn = cfg->dim == 2 ? 6 : 4;
  if (cfg->n_low < 3 || cfg->n_low > maxn) return "unsupported low order";
  if (cfg->n_high && (cfg->n_high <= cfg->n_low || cfg->n_high > maxn)) return "need n_low < n_high <= 6 (2D) / 4 (3D)";
  if (!(cfg->tau > 0.5)) return "tau must exceed 1/2";
  if (!(cfg->cfl > 0.0) || cfg->cfl > 1.0) return "cfl must be in (0, 1] for the 3-point stencil";
  if (store_size(cfg->store) == 0) return "unknown storage precision";
  if (cfg->thermal && !(cfg->cv > 0.5 * cfg->dim)) return "thermal model needs cv > D/2";
  if (cfg->lift_mode < 0 || cfg->lift_mode > 2) return "unknown lift mode";
  if (cfg->lift_mode == MSL_LIFT_MLP && !cfg->n_high) return "learned lifting needs two velocity sets";
  if (cfg->crit_kind < 0 || cfg->crit_kind > 3) return "unknown criterion";
  if (cfg->store >= MSL_FP16_DEV && !(cfg->rho0 > 0.0 && cfg->T0 > 0.0)) return "deviation storage needs rho0, T0 > 0";
  for (int a = 0; a < 3; ++a)
    if (!isfinite(cfg->u_ref[a]) || !isfinite(cfg->store_u[a])) return "frame and storage velocities must be finite";
  if (isnan(cfg->T_ref) || isinf(cfg->T_ref)) return "T_ref must be finite";
  const bool trivial_frame = cfg->u_ref[0] == 0.0 && cfg->u_ref[1] == 0.0 &&
                             (cfg->dim == 2 || cfg->u_ref[2] == 0.0) && (cfg->T_ref <= 0.0 || cfg->T_ref == 1.0);
  if (cfg->lift_mode == MSL_LIFT_MLP && !trivial_frame) return "learned lifting needs the lattice frame";
  if (isnan(cfg->tau2) || (cfg->tau2 > 0.0 && !(cfg->tau2 > 0.5))) return "tau2 must exceed 1/2 (or be <= 0 for BGK)";
  if (cfg->tau2 > 0.0 && cfg->tau2 != cfg->tau && cfg->dim != 2) return "the two-relaxation model is built for 2D";
  const long long cells = (long long)cfg->nx * cfg->ny * (cfg->dim == 3 ? cfg->nz : 1);
  if (cells >= (1ll << 31)) return "grid too large";
  if (cfg->pond != 0 && cfg->pond != 1) return "pond must be 0 or 1";
  if (cfg->crit_margin < 0 || cfg->crit_margin > 1024) return "crit_margin must lie in [0, 1024]";
  if (cfg->pond) {
    if (cfg->dim != 2) return "co-moving frames are built for 2D";
    if (cfg->n_high && cfg->lift_mode == MSL_LIFT_MLP) return "co-moving frames: Grad or Hermite lifting";
    if (cfg->store != MSL_FP64) return "co-moving frames keep FP64 populations";
    if (cfg->crit_kind != MSL_CRIT_NONE && cfg->crit_kind != MSL_CRIT_KN)
      return "co-moving frames: fixed sets or the Knudsen-number criterion";
    if (!trivial_frame) return "co-moving frames replace the global frame";
  }
  for (int f = 0; f < 2 * cfg->dim; ++f) {
    if (cfg->bc[f] < 0 || cfg->bc[f] > 3) return "unknown boundary rule";
    if ((cfg->bc[f] == MSL_BC_PERIODIC) != (cfg->bc[f ^ 1] == MSL_BC_PERIODIC)) return "periodic faces must come in pairs";
    if (cfg->bc[f] == MSL_BC_DIFFUSE_WALL) {
      if (f / 2 == 0) return "diffuse walls only on y or z faces";
      for (int g = 0; g < 2 * (f / 2); ++g)
        if (cfg->bc[g] != MSL_BC_PERIODIC && cfg->bc[g] != MSL_BC_OUTFLOW_ZG)
          return "diffuse walls need periodic or zero-gradient lower faces";
    }
  }
  return nullptr;
}

struct Layout {
  Geo geo;
  size_t esz;
  size_t off_tab, off_planes[2], off_cls, off_newmask, off_tflag, off_blist[2], off_bcount, off_blk,
      off_red, off_flag, off_tlist, off_kn, off_pond, off_mlp, total;
  int nblk, Q[2], np[2];
  long long plane_bytes;
  int mlpF, mlpO, mlpH, mlpP, nctile, nct[3];
  size_t mlp_off[12];
};

static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }
static int roundup(int v, int m) { return (v + m - 1) / m * m; }

static void make_layout(const msl_config *cfg, Layout &L) {
  memset(&L, 0, sizeof(L));
  Geo &g = L.geo;
  g.dim = cfg->dim;
  g.nx = cfg->nx;
  g.ny = cfg->ny;
  g.nz = cfg->dim == 3 ? cfg->nz : 1;
  L.esz = store_size(cfg->store);
  const int e64 = (int)(64 / L.esz);
  g.xo = e64 > MSL_G ? e64 : MSL_G + 1;
  g.pitch = roundup(g.xo + roundup(g.nx, MSL_TX) + MSL_G + 2, e64);
  if (cfg->dim == 2) {
    g.rows = MSL_G + roundup(g.ny, 16) + MSL_G + 2;
    g.slabs = 1;
  } else {
    g.rows = MSL_G + roundup(g.ny, MSL_MTY) + MSL_G + 2;
    g.slabs = MSL_G + roundup(g.nz, 4) + MSL_G + 2;
  }
  g.plane = (long long)g.slabs * g.rows * g.pitch;
  g.ncell = (long long)g.nx * g.ny * g.nz;
  g.ntx = (g.nx + MSL_TX - 1) / MSL_TX;
  g.nty = (g.ny + MSL_MTY - 1) / MSL_MTY;
  g.ntz = g.nz;
  const int nl = cfg->n_high ? 2 : 1;
  const int ns[2] = {cfg->n_low, cfg->n_high};
  size_t off = 0;
  L.off_tab = off;
  off = align256(off + sizeof(Tab));
  for (int l = 0; l < nl; ++l) {
    L.Q[l] = cfg->dim == 2 ? ns[l] * ns[l] : ns[l] * ns[l] * ns[l];
    L.np[l] = L.Q[l] * (cfg->thermal ? 2 : 1);
    L.off_planes[l] = off;
    off = align256(off + 2 * (size_t)L.np[l] * g.plane * L.esz);
  }
  L.off_cls = off;
  off = align256(off + g.ncell);
  L.off_newmask = off;
  off = align256(off + g.ncell);
  L.off_tflag = off;
  off = align256(off + (size_t)g.ntx * g.nty * g.ntz);
  for (int l = 0; l < 2; ++l) {
    L.off_blist[l] = off;
    off = align256(off + (nl > 1 ? (size_t)g.ncell * 4 : 4));
  }
  L.off_bcount = off;
  off = align256(off + 16);
  L.nblk = (int)((g.ncell + 4095) / 4096);
  L.off_blk = off;
  off = align256(off + (size_t)3 * L.nblk * 4);
  L.off_red = off;
  off = align256(off + (size_t)1024 * 9 * 8 + 128);   // per-block partials, then results
  L.off_flag = off;
  off = align256(off + 64);
  L.off_tlist = off;   // live-tile list of the high-order set, then its count
  off = align256(off + ((size_t)g.ntx * g.nty * g.ntz + 16) * 4);
  // Knudsen-number criterion: each cell's density and mean free path
  L.off_kn = off;
  if (cfg->crit_kind == MSL_CRIT_KN && nl > 1) off = align256(off + (size_t)g.ncell * 2 * 8);
  // co-moving frames: two buffers of populations and frames, iteration counters
  L.off_pond = off;
  // (then the wall densities of the two y faces, 2 nx doubles)
  if (cfg->pond)
    off = align256(off + (size_t)g.ncell * 8 * 2 * (L.np[0] + (nl > 1 ? L.np[1] : 0) + 4) + 64 + (size_t)16 * g.nx);
  // learned closure
  if (cfg->lift_mode == MSL_LIFT_MLP && nl > 1) {
    const int q = L.Q[0], Q = L.Q[1];
    L.mlpF = 2 + cfg->dim + (q - 1 - cfg->dim);
    L.mlpO = Q - q;
    L.mlpH = cfg->mlp_hidden > 0 ? cfg->mlp_hidden : 64;
    L.mlpP = L.mlpF * L.mlpH + L.mlpH + L.mlpH * L.mlpH + L.mlpH + L.mlpH * L.mlpO + L.mlpO;
    for (int a = 0; a < 3; ++a) {
      const int n = a == 0 ? g.nx : (a == 1 ? g.ny : g.nz);
      L.nct[a] = (n + MSL_CHECK_TILE - 1) / MSL_CHECK_TILE;
    }
    L.nctile = L.nct[0] * L.nct[1] * L.nct[2];
    const size_t sizes[12] = {
        (size_t)L.mlpP * 4,                       // 0 weights
        (size_t)(2 * L.mlpF + 2 * L.mlpO) * 4,    // 1 stats
        (size_t)g.ncell * L.mlpF * 4,             // 2 features
        (size_t)g.ncell * L.mlpO * 4,             // 3 outputs
        (size_t)L.mlpP * 4,                       // 4 adam m
        (size_t)L.mlpP * 4,                       // 5 adam v
        (size_t)L.mlpP * 4,                       // 6 grad
        (size_t)MSL_MLP_LOSS_RING * 4,            // 7 loss history
        (size_t)L.nctile,                         // 8 flags
        (size_t)L.nctile * 2 * 8,                 // 9 per-tile errors
        (size_t)MSL_MLP_MAXBLK * (L.mlpP + 1) * 4,  // 10 gradient / loss partials
        (size_t)g.ncell * (L.mlpO * 4 + 16)};     // 11 check: targets, per-cell errors
    for (int k = 0; k < 12; ++k) {
      L.mlp_off[k] = off;
      off = align256(off + sizes[k]);
    }
  }
  L.total = off;
  L.plane_bytes = g.plane * (long long)L.esz;
}

// ---------------------------------------------------------------------------
// entry points
// ---------------------------------------------------------------------------
extern "C" {

int msl_workspace_bytes(const msl_config *cfg, size_t *bytes) {
  if (!bytes || check_config(cfg)) return MSL_EINVAL;
  Layout L;
  make_layout(cfg, L);
  if (L.plane_bytes >= (1ll << 31)) return MSL_EINVAL;
  *bytes = L.total;
  return MSL_OK;
}

const char *msl_last_error(const msl_ctx *c) { return c ? c->err : "null context"; }

int msl_create(const msl_config *cfg, void *ws, size_t bytes, void *stream, msl_ctx **out) {
  if (!out) return MSL_EINVAL;
  *out = nullptr;
  const char *why = check_config(cfg);
  if (why) return MSL_EINVAL;
  Layout L;
  make_layout(cfg, L);
  // planes are addressed with 32-bit byte offsets, and the stores of foreign
  // cells go to offset 2^31, which has to lie outside the plane
  if (L.plane_bytes >= (1ll << 31)) return MSL_EINVAL;
  if (!ws || bytes < L.total) return MSL_ENOMEM;
  msl_ctx *c = new (std::nothrow) msl_ctx;
  if (!c) return MSL_ENOMEM;
  memset(c, 0, sizeof(*c));
  c->cfg = *cfg;
  c->stream = (hipStream_t)stream;
  // the device of this context: its static scratch array is looked up now
  if (hipGetDevice(&c->device) != hipSuccess || msl_noalloc_setup(c->device) != MSL_OK) {
    delete c;
    return MSL_EHIP;
  }
  c->geo = L.geo;
  c->D = cfg->dim;
  c->nlat = cfg->n_high ? 2 : 1;
  c->Q[0] = L.Q[0];
  c->Q[1] = L.Q[1];
  c->ncell = L.geo.ncell;
  c->esz = L.esz;
  char *base = (char *)ws;
  // tables
  ld xs[2][MSL_MAXN], wsl[2][MSL_MAXN];
  const int ns[2] = {cfg->n_low, cfg->n_high};
  for (int l = 0; l < c->nlat; ++l)
    if (gauss_hermite(ns[l], xs[l], wsl[l])) { delete c; return MSL_EINVAL; }
  Tab &t = c->htab;
  memset(&t, 0, sizeof(t));
  // the run's frame (eq. veli); T_ref <= 0 stands for the lattice temperature 1
  const double Tref = cfg->T_ref > 0.0 ? cfg->T_ref : 1.0;
  const ld sqT = sqrtl((ld)Tref);
  double ur[3] = {0, 0, 0}, su[3] = {0, 0, 0};
  for (int a = 0; a < cfg->dim; ++a) { ur[a] = cfg->u_ref[a]; su[a] = cfg->store_u[a]; }
  // CFL = max |v_ia| dt / dx over every configured velocity set and axis (Sec. IV)
  ld vmax = 0;
  for (int l = 0; l < c->nlat; ++l)
    for (int ax = 0; ax < cfg->dim; ++ax)
      for (int a = 0; a < ns[l]; ++a) {
        const ld v = fabsl(sqT * xs[l][a] + (ld)ur[ax]);
        if (v > vmax) vmax = v;
      }
  const double dt = (double)((ld)cfg->cfl / vmax);
  const double rho0 = cfg->rho0 > 0 ? cfg->rho0 : 1.0, T0 = cfg->T0 > 0 ? cfg->T0 : 1.0;
  for (int l = 0; l < c->nlat; ++l)
    build_lat(t.lat[l], ns[l], cfg->dim, xs[l], wsl[l], dt, ur, Tref, su, rho0, T0);
  for (int l = 0; l < c->nlat; ++l)
    for (int ax = 0; ax < cfg->dim; ++ax)
      for (int a = 0; a < ns[l]; ++a)
        if (abs(t.lat[l].n0[ax][a]) + 1 > MSL_G) { delete c; return MSL_EINVAL; }
  if (c->nlat > 1) {
    const int nq = ns[0], nQ = ns[1];
    for (int a = 0; a < nQ; ++a) {
      ld coef[MSL_MAXN];
      lagrange_coeffs(nQ, xs[1], a, coef);
      for (int m = 0; m < nQ; ++m) t.Vi[a][m] = (double)coef[m];
      for (int ap = 0; ap < nq; ++ap) {
        ld sh = 0, fact = 1;
        for (int j = 0; j < nq; ++j) {
          if (j > 0) fact *= (ld)j;
          sh += hermite_he(j, xs[1][a]) * hermite_he(j, xs[0][ap]) / fact;
        }
        t.KH[a][ap] = (double)(wsl[1][a] * sh);
      }
    }
    // raw completion per axis, in the particle velocities of that axis: the
    // degree < n_q part of the high-order Lagrange basis polynomial in v,
    // evaluated at the low-order velocities
    for (int ax = 0; ax < 3; ++ax) {
      const ld u = ax < cfg->dim ? (ld)ur[ax] : 0.0L;
      ld vh[MSL_MAXN], vl[MSL_MAXN];
      for (int a = 0; a < nQ; ++a) vh[a] = sqT * xs[1][a] + u;
      for (int a = 0; a < nq; ++a) vl[a] = sqT * xs[0][a] + u;
      for (int a = 0; a < nQ; ++a) {
        ld coef[MSL_MAXN];
        lagrange_coeffs(nQ, vh, a, coef);
        for (int ap = 0; ap < nq; ++ap) {
          ld s = 0;
          for (int m = 0; m < nq; ++m) s += coef[m] * powl(vl[ap], m);
          t.K[ax][a][ap] = (double)s;
        }
      }
    }
    for (int ap = 0; ap < nq; ++ap)
      for (int a = 0; a < nQ; ++a) t.P[ap][a] = (double)lagrange_eval(nq, xs[0], ap, xs[1][a]);
  }
  t.dt = dt;
  t.cv = cfg->cv;
  t.gfac = cfg->thermal ? cfg->cv - 0.5 * cfg->dim : 0.0;
  t.tau = cfg->tau;
  t.omega = 1.0 / cfg->tau;
  t.omegaf = (float)t.omega;
  t.mu_ref = (cfg->tau - 0.5) * cfg->tau_ref_rho * cfg->tau_ref_T * dt;
  t.mu_exp = cfg->mu_exp;
  t.tau_ref_T = cfg->tau_ref_T > 0 ? cfg->tau_ref_T : 1.0;
  t.mu_T1 = t.mu_ref * pow(1.0 / t.tau_ref_T, t.mu_exp);
  t.rho0 = cfg->rho0 > 0 ? cfg->rho0 : 1.0;
  t.T0 = cfg->T0 > 0 ? cfg->T0 : 1.0;
  t.tau_mode = cfg->tau_mode;
  t.igsc = t.gfac > 0.0 ? 1.0 / (t.gfac * (cfg->T0 > 0 ? cfg->T0 : 1.0)) : 0.0;
  t.igscf = (float)t.igsc;
  t.qe = cfg->tau2 > 0.0 && cfg->tau2 != cfg->tau;
  t.qe_ratio = t.qe ? (cfg->tau2 - 0.5) / (cfg->tau - 0.5) : 1.0;
  t.thermal = cfg->thermal;
  t.dim = cfg->dim;
  t.nlat = c->nlat;
  t.lift_mode = cfg->lift_mode;
  // diffuse walls: the wall equilibrium does not change during a run, only its
  // density (set per ghost cell from the flux arriving at the wall)
  for (int f = 0; f < 2 * cfg->dim; ++f) {
    if (cfg->bc[f] != MSL_BC_DIFFUSE_WALL) continue;
    const int ax = f / 2, side = f % 2;
    const double *ws = cfg->bc_state[f];
    for (int l = 0; l < c->nlat; ++l) {
      const LatTab &Lt = t.lat[l];
      cell_feq(Lt, cfg->dim, 1.0, ws + 1, ws[4], t.wall_eq[f][l]);
      double out = 0;
      for (int i = 0; i < Lt.Q; ++i) {
        const int d = ax == 0 ? i % Lt.n : (ax == 1 ? (i / Lt.n) % Lt.n : i / (Lt.n * Lt.n));
        const double cn = Lt.v[ax][d];
        if (side ? cn < 0 : cn > 0) out += fabs(cn) * t.wall_eq[f][l][i];
      }
      t.wall_out[f][l] = out;
    }
  }
  // workspace
  c->dtab = (Tab *)(base + L.off_tab);
  for (int l = 0; l < c->nlat; ++l) {
    c->planes[l][0] = base + L.off_planes[l];
    c->planes[l][1] = base + L.off_planes[l] + (size_t)L.np[l] * L.geo.plane * L.esz;
  }
  c->cls = (uint8_t *)(base + L.off_cls);
  c->newmask = (uint8_t *)(base + L.off_newmask);
  c->tflag = (uint8_t *)(base + L.off_tflag);
  c->blist[0] = (int *)(base + L.off_blist[0]);
  c->blist[1] = (int *)(base + L.off_blist[1]);
  c->bcount = (int *)(base + L.off_bcount);
  c->blk = (int *)(base + L.off_blk);
  c->nblk = L.nblk;
  c->red = (double *)(base + L.off_red);
  c->flag = (int *)(base + L.off_flag);
  c->tlist = (int *)(base + L.off_tlist);
  c->kn_rho = (double *)(base + L.off_kn);
  c->kn_lam = c->kn_rho + L.geo.ncell;
  if (cfg->pond) {
    double *pb = (double *)(base + L.off_pond);
    for (int l = 0; l < c->nlat; ++l) {
      const size_t nf = (size_t)L.np[l] * L.geo.ncell;
      c->pond_f[l][0] = pb;
      c->pond_f[l][1] = pb + nf;
      pb += 2 * nf;
    }
    const size_t nfr = (size_t)4 * L.geo.ncell;
    c->pond_fr[0] = pb;
    c->pond_fr[1] = pb + nfr;
    c->pond_stats = (unsigned long long *)(pb + 2 * nfr);
    c->pond_wall = pb + 2 * nfr + 8;
  }
  c->tcount = c->tlist + (size_t)L.geo.ntx * L.geo.nty * L.geo.ntz;
  if (L.mlpP) {
    c->mlpF = L.mlpF; c->mlpO = L.mlpO; c->mlpH = L.mlpH; c->mlpP = L.mlpP;
    c->mlp_w = (float *)(base + L.mlp_off[0]);
    c->mlp_stats = (float *)(base + L.mlp_off[1]);
    c->mlp_feat = (float *)(base + L.mlp_off[2]);
    c->mlp_out = (float *)(base + L.mlp_off[3]);
    c->mlp_m = (float *)(base + L.mlp_off[4]);
    c->mlp_v = (float *)(base + L.mlp_off[5]);
    c->mlp_g = (float *)(base + L.mlp_off[6]);
    c->mlp_loss = (float *)(base + L.mlp_off[7]);
    c->mlp_flag = (uint8_t *)(base + L.mlp_off[8]);
    c->mlp_err = (double *)(base + L.mlp_off[9]);
    c->mlp_gpart = (float *)(base + L.mlp_off[10]);
    c->mlp_tgt = (float *)(base + L.mlp_off[11]);
    c->mlp_cerr = (double *)(base + L.mlp_off[11] + align256((size_t)L.geo.ncell * L.mlpO * 4));
    c->nctile = L.nctile;
    for (int a = 0; a < 3; ++a) c->nct[a] = L.nct[a];
  }
  // zero the whole workspace once (padding included), upload the tables,
  // start with every cell on the low-order set
  if (hipMemsetAsync(ws, 0, L.total, c->stream) != hipSuccess ||
      hipMemcpyAsync(c->dtab, &t, sizeof(Tab), hipMemcpyHostToDevice, c->stream) != hipSuccess) {
    delete c;
    return MSL_EHIP;
  }
  if (c->mlp_flag && hipMemsetAsync(c->mlp_flag, 1, c->nctile, c->stream) != hipSuccess) {
    delete c;
    return MSL_EHIP;
  }
  if (msl_launch_classify(c) != MSL_OK) { delete c; return MSL_EHIP; }
  // 2D two-set contexts without the learned closure: the stream-collide
  // launches convert the band cells (lift in the low-order launch, projection
  // in the high-order one)
  const int sc2 = cfg->lift_mode != MSL_LIFT_MLP && msl_stream_sc2_all(c);
  c->fuse = sc2 && c->nlat == 2;
  // 2D faces that are all zero-gradient or fixed: the zero-gradient ones are
  // applied inside the stream-collide launches (the fixed ghosts are
  // constant), so a step launches no ghost fill
  if (sc2) {
    int m = 0, ok = 1;
    for (int f = 0; f < 4; ++f) {
      if (cfg->bc[f] == MSL_BC_OUTFLOW_ZG) m |= 1 << f;
      else if (cfg->bc[f] != MSL_BC_FIXED_EQ) ok = 0;
    }
    c->zgm = ok ? m : 0;
  }
  // step graphs: one block per criterion period (at most 64 steps), else 16
  c->gmode = 0;
  c->gB = cfg->crit_kind && cfg->crit_every > 0 && c->nlat > 1 && cfg->crit_every <= 64 ? cfg->crit_every : 16;
  // the host copy of the tables must stay valid until the upload has run
  if (hipStreamSynchronize(c->stream) != hipSuccess) { delete c; return MSL_EHIP; }
  *out = c;
  return MSL_OK;
}

static void graph_release(msl_ctx *c);

void msl_destroy(msl_ctx *c) {
  if (c && c->prof) msl_profile(c, 0);
  if (c && c->prof_nh) hipHostFree(c->prof_nh);
  if (c) {
    graph_release(c);
    for (int k = 0; k < 2; ++k) {
      if (c->gs[k]) hipStreamDestroy(c->gs[k]);
      if (c->gev[k]) hipEventDestroy(c->gev[k]);
    }
  }
  delete c;
}

int msl_get_dt(const msl_ctx *c, double *dt) {
  if (!c || !dt) return MSL_EINVAL;
  *dt = c->htab.dt;
  return MSL_OK;
}

int msl_get_step(const msl_ctx *c, long *step) {
  if (!c || !step) return MSL_EINVAL;
  *step = c->step;
  return MSL_OK;
}

static int refresh_band(msl_ctx *c) {
  int rc = msl_launch_classify(c);
  if (rc) return rc;
  if (c->initialized && c->nlat > 1) {
    rc = msl_launch_band_convert(c, c->planes[0][c->cur], c->planes[1][c->cur]);
    if (rc) return rc;
    if (c->cfg.lift_mode == MSL_LIFT_MLP && c->mlp_on)
      rc = msl_mlp_band_lift(c, c->planes[0][c->cur], c->planes[1][c->cur]);
  }
  return rc;
}

int msl_init(msl_ctx *c, const double *rho, const double *u, const double *T) {
  if (!c || !rho || !u || (c->cfg.thermal && !T)) return MSL_EINVAL;
  if (c->cfg.pond) {
    const int rc = msl_pond_launch_init(c, rho, u, T);
    if (rc) { set_err(c, "init kernel launch failed"); return rc; }
    c->initialized = 1;
    c->step = 0;
    return MSL_OK;
  }
  int rc = msl_launch_init_eq(c, rho, u, T);
  if (!rc) rc = msl_launch_bc_fixed(c);
  if (rc) { set_err(c, "init kernel launch failed"); return rc; }
  c->initialized = 1;
  c->step = 0;
  rc = refresh_band(c);
  if (rc) set_err(c, "band conversion failed");
  return rc;
}

int msl_set_mask(msl_ctx *c, const uint8_t *mask) {
  if (!c || !mask) return MSL_EINVAL;
  if (hipMemsetAsync(c->flag, 0, sizeof(int), c->stream) != hipSuccess) return MSL_EHIP;
  int rc = msl_launch_check_mask(c, mask);
  if (rc) return rc;
  int bad = 0;
  if (hipMemcpyAsync(&bad, c->flag, sizeof(int), hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess)
    return MSL_EHIP;
  if (bad) { set_err(c, "mask values must be 0/1 (1 only with a high order)"); return MSL_EINVAL; }
  if (c->cfg.pond) return msl_pond_launch_set_mask(c, mask, c->initialized);
  rc = msl_launch_switch(c, mask);
  if (rc) return rc;
  return refresh_band(c);
}

int msl_get_mask(msl_ctx *c, uint8_t *mask) {
  if (!c || !mask) return MSL_EINVAL;
  // the order is bit 0 of the class byte
  return msl_launch_get_mask(c, mask);
}

static int mask_step(msl_ctx *c) {
  int rc = msl_launch_criterion(c);
  if (!rc) rc = msl_launch_dilate(c);
  if (rc) return rc;
  rc = msl_launch_switch(c, c->newmask);
  if (rc) return rc;
  return refresh_band(c);
}

// ---- per-kernel timing ----
// Per-class launch timing without draining the stream: records live in a ring
// of events; when the ring is three-quarters full the oldest half is read,
// whose events completed long ago.  The number of high-order cells, which sets
// the bytes of a stream-collide launch, is copied by the GPU itself into a
// pinned host ring at every mask update and read with the records.
__global__ void k_prof_snap(const int *__restrict__ src, int *__restrict__ dst) {
  if (threadIdx.x == 0) dst[0] = src[0];
}

static int prof_read(msl_ctx *c, long long upto) {
  if (upto <= c->ndone) return MSL_OK;
  MSL_HIP(hipEventSynchronize(c->ev[2 * ((upto - 1) % MSL_PROF_REC) + 1]));
  for (long long k = c->ndone; k < upto; ++k) {
    const int r = (int)(k % MSL_PROF_REC);
    float ms = 0.f;
    MSL_HIP(hipEventElapsedTime(&ms, c->ev[2 * r], c->ev[2 * r + 1]));
    double cells = c->rec_cells[r];
    if (c->rec_lat[r] >= 0) {
      const double nh = c->nlat > 1 ? (double)c->prof_nh[c->rec_slot[r]] : 0.0;
      cells = c->nlat == 1 ? (double)c->ncell : (c->rec_lat[r] == 0 ? (double)c->ncell - nh : nh);
    }
    double *st = c->pstat[c->rec_cls[r]];
    st[0] += 1.0;
    st[1] += ms;
    st[2] += cells * c->rec_bpc[r];
    st[3] += cells;
  }
  c->ndone = upto;
  return MSL_OK;
}

static void prof_snap(msl_ctx *c) {
  if (!c->prof || c->nlat < 2) return;
  const int slot = (int)(++c->nsnap % MSL_PROF_REC);
  hipLaunchKernelGGL(k_prof_snap, dim3(1), dim3(64), 0, c->stream, c->bcount + 2, c->prof_nh + slot);
}

// launches of every prof-th step are timed
static bool prof_on(const msl_ctx *c) { return c->prof && c->step % c->prof == 0; }

static void prof_begin(msl_ctx *c) {
  if (prof_on(c)) hipEventRecord(c->ev[2 * (c->nrec % MSL_PROF_REC)], c->stream);
}

// lat >= 0: a stream-collide launch of that velocity set (cells from the
// snapshot in force); otherwise `cells` as given
static int prof_end(msl_ctx *c, int cls, int lat, double bytes_per_cell, double cells) {
  if (!prof_on(c)) return MSL_OK;
  const int r = (int)(c->nrec % MSL_PROF_REC);
  hipEventRecord(c->ev[2 * r + 1], c->stream);
  c->rec_cls[r] = cls;
  c->rec_lat[r] = lat;
  c->rec_slot[r] = (int)(c->nsnap % MSL_PROF_REC);
  c->rec_bpc[r] = bytes_per_cell;
  c->rec_cells[r] = cells;
  ++c->nrec;
  if (c->nrec - c->ndone >= 3 * MSL_PROF_REC / 4) return prof_read(c, c->ndone + MSL_PROF_REC / 2);
  return MSL_OK;
}

int msl_profile(msl_ctx *c, int enable) {
  if (!c || enable < 0) return MSL_EINVAL;
  if (enable && c->prof) {
    c->prof = enable;
    return MSL_OK;
  }
  if (enable && !c->prof) {
    for (int k = 0; k < 2 * MSL_PROF_REC; ++k) MSL_HIP(hipEventCreate(&c->ev[k]));
    if (!c->prof_nh) MSL_HIP(hipHostMalloc((void **)&c->prof_nh, sizeof(int) * MSL_PROF_REC));
    memset(c->pstat, 0, sizeof(c->pstat));
    c->nrec = c->ndone = 0;
    c->nsnap = 0;
    c->prof = enable;
    if (c->nlat > 1)
      hipLaunchKernelGGL(k_prof_snap, dim3(1), dim3(64), 0, c->stream, c->bcount + 2, c->prof_nh);
    return hipGetLastError() == hipSuccess ? MSL_OK : MSL_EHIP;
  }
  if (!enable && c->prof) {
    int rc = prof_read(c, c->nrec);
    for (int k = 0; k < 2 * MSL_PROF_REC; ++k) hipEventDestroy(c->ev[k]);
    c->prof = 0;
    return rc;
  }
  return MSL_OK;
}

int msl_profile_read(msl_ctx *c, double *stats) {
  if (!c || !stats) return MSL_EINVAL;
  if (!c->prof) return MSL_ESTATE;
  int rc = prof_read(c, c->nrec);
  if (rc) return rc;
  memcpy(stats, c->pstat, sizeof(c->pstat));
  memset(c->pstat, 0, sizeof(c->pstat));
  return MSL_OK;
}

// co-moving frames: one predictor-corrector launch per step; the reach and
// positivity flags are read once at the end of the call
static int pond_step(msl_ctx *c, int nsteps) {
  if (hipMemsetAsync(c->flag, 0, sizeof(int), c->stream) != hipSuccess ||
      hipMemsetAsync(c->pond_stats, 0, 16, c->stream) != hipSuccess)
    return MSL_EHIP;
  for (int s = 0; s < nsteps; ++s) {
    const int rc = msl_pond_launch_step(c);
    if (rc) { set_err(c, "co-moving step launch failed"); return rc; }
    ++c->step;
  }
  c->pond_cells_steps = (long long)nsteps * c->ncell;
  int bad = 0;
  if (hipMemcpyAsync(&bad, c->flag, sizeof(int), hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess)
    return MSL_EHIP;
  if (bad & 1) { set_err(c, "a departure point left the two-cell reach: lower cfl"); return MSL_EUNSTABLE; }
  if (bad & 2) { set_err(c, "non-positive or non-finite density or temperature"); return MSL_EUNSTABLE; }
  return MSL_OK;
}

int msl_pond_frames(msl_ctx *c, double *out) {
  if (!c || !out || !c->cfg.pond) return MSL_EINVAL;
  if (!c->initialized) return MSL_ESTATE;
  return hipMemcpyAsync(out, c->pond_fr[c->cur], sizeof(double) * 4 * c->ncell, hipMemcpyDeviceToDevice,
                        c->stream) == hipSuccess ? MSL_OK : MSL_EHIP;
}

int msl_pond_iterations(msl_ctx *c, double *mean, int *max) {
  if (!c || !c->cfg.pond) return MSL_EINVAL;
  unsigned long long h[2] = {0, 0};
  if (hipMemcpyAsync(h, c->pond_stats, sizeof(h), hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess)
    return MSL_EHIP;
  if (mean) *mean = c->pond_cells_steps > 0 ? (double)h[0] / (double)c->pond_cells_steps : 0.0;
  if (max) *max = (int)(h[1] & 0xffffffffu);
  return MSL_OK;
}

static bool crit_step(const msl_ctx *c, long step) {
  return c->cfg.crit_kind && c->cfg.crit_every > 0 && c->nlat > 1 && step % c->cfg.crit_every == 0;
}

// the launches of one step after its criterion pass: ghost fill,
// stream-collide of each set, band conversion (and the learned lift).  fork
// (only while capturing): the high-order set's stream-collide launch goes on
// a parallel branch, forked after the ghost fill and joined before the band
// conversion
// 3D with x periodic on both faces: the x ghosts are kept current by the
// kernels that write cells (switching, stream-collide, band conversion and
// learned lift store the images of the cells x < 2 and x >= nx - 2); set
// before the step's criterion pass
static void set_xmir(msl_ctx *c) {
  c->xmir = c->D == 3 && c->cfg.bc[0] == MSL_BC_PERIODIC && c->cfg.bc[1] == MSL_BC_PERIODIC &&
            c->geo.nx >= 2 * MSL_G;
}

static int plain_step(msl_ctx *c, bool fork) {
  int rc;
  set_xmir(c);
  const int cur = c->cur, nxt = cur ^ 1;
  char *bl = c->planes[0][cur], *bh = c->nlat > 1 ? c->planes[1][cur] : nullptr;
  prof_begin(c);
  rc = msl_launch_bc(c, bl, bh);
  if (rc) { set_err(c, "ghost fill failed"); return rc; }
  if ((rc = prof_end(c, 0, -1, 0.0, 0.0))) return rc;
  fork = fork && c->nlat > 1;
  if (fork) {
    hipStream_t s0 = c->stream;
    MSL_HIP(hipEventRecord(c->gev[0], s0));
    MSL_HIP(hipStreamWaitEvent(c->gs[1], c->gev[0], 0));
    c->stream = c->gs[1];
    rc = msl_launch_stream_collide(c, 1, c->planes[1][cur], c->planes[1][nxt],
                                   c->fuse ? c->planes[0][nxt] : nullptr);
    c->stream = s0;
    MSL_HIP(hipEventRecord(c->gev[1], c->gs[1]));
    if (rc) {
      // join the branch before leaving, so that the capture can be ended
      MSL_HIP(hipStreamWaitEvent(s0, c->gev[1], 0));
      set_err(c, "stream-collide launch failed");
      return rc;
    }
  }
  for (int l = 0; l < (fork ? 1 : c->nlat); ++l) {
    // compulsory traffic: read and write every population plane of each native cell
    const double bpc = 2.0 * c->Q[l] * (c->cfg.thermal ? 2 : 1) * (double)c->esz;
    prof_begin(c);
    rc = msl_launch_stream_collide(c, l, c->planes[l][cur], c->planes[l][nxt],
                                   c->fuse ? c->planes[l ^ 1][nxt] : nullptr);
    if (rc) { set_err(c, "stream-collide launch failed"); return rc; }
    if ((rc = prof_end(c, 1 + l, l, bpc, 0.0))) return rc;
  }
  if (fork) MSL_HIP(hipStreamWaitEvent(c->stream, c->gev[1], 0));
  if (c->nlat > 1 && !c->fuse) {
    char *nl = c->planes[0][nxt], *nh = c->planes[1][nxt];
    prof_begin(c);
    rc = msl_launch_band_convert(c, nl, nh);
    if (rc) { set_err(c, "band conversion failed"); return rc; }
    if ((rc = prof_end(c, 3, -1, 0.0, 0.0))) return rc;
    if (c->cfg.lift_mode == MSL_LIFT_MLP && c->mlp_on) {
      prof_begin(c);
      rc = msl_mlp_band_lift(c, nl, nh);
      if (rc) { set_err(c, "learned lifting failed"); return rc; }
      if ((rc = prof_end(c, 5, -1, 0.0, 0.0))) return rc;
    }
  }
  c->xg_ok = c->xmir;
  c->xmir = 0;
  c->cur = nxt;
  ++c->step;
  return MSL_OK;
}

// Step graphs: contexts whose steps need no host work between launches (2D,
// no learned closure, no conservation check); timed steps (msl_profile) and
// criterion passes run outside the graphs.
static bool graph_ok(const msl_ctx *c) {
  return c->gmode > 0 && c->D == 2 && c->cfg.lift_mode != MSL_LIFT_MLP && c->cfg.check_every <= 0;
}

static void graph_release(msl_ctx *c) {
  for (int p = 0; p < 2; ++p)
    if (c->gx[p]) { hipGraphExecDestroy(c->gx[p]); c->gx[p] = nullptr; }
}

// capture gB plain steps starting from the current buffer `cur` into gx[cur];
// the context's host state (buffer parity, step counter) is left unchanged.
// A step that cannot be captured (a launch over a compact tile list, whose
// length the host reads) switches the graphs off for this context.
// the second stream and the fork / join events of the parallel branches
static int fork_streams(msl_ctx *c) {
  if (!c->gs[0]) {
    for (int k = 0; k < 2; ++k) {
      MSL_HIP(hipStreamCreateWithFlags(&c->gs[k], hipStreamNonBlocking));
      MSL_HIP(hipEventCreateWithFlags(&c->gev[k], hipEventDisableTiming));
    }
  }
  return MSL_OK;
}

static int graph_capture(msl_ctx *c) {
  if (int rc = fork_streams(c)) return rc;
  const int cur0 = c->cur;
  const long step0 = c->step;
  hipStream_t s0 = c->stream;
  c->stream = c->gs[0];
  c->capturing = 1;
  int rc = hipStreamBeginCapture(c->gs[0], hipStreamCaptureModeThreadLocal) == hipSuccess ? MSL_OK : MSL_EHIP;
  for (int k = 0; k < c->gB && rc == MSL_OK; ++k) rc = plain_step(c, c->gmode == 2);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(c->gs[0], &g);
  c->capturing = 0;
  c->stream = s0;
  c->cur = cur0;
  c->step = step0;
  c->xg_ok = 0;
  if (rc == MSL_ESTATE) {
    // not capturable: launches one by one from now on
    if (g) hipGraphDestroy(g);
    (void)hipGetLastError();
    c->gmode = 0;
    c->err[0] = 0;
    return MSL_OK;
  }
  if (rc || e != hipSuccess || !g) {
    if (g) hipGraphDestroy(g);
    set_err(c, "step graph capture failed");
    return rc ? rc : MSL_EHIP;
  }
  const hipError_t ei = hipGraphInstantiate(&c->gx[cur0], g, nullptr, nullptr, 0);
  hipGraphDestroy(g);
  if (ei != hipSuccess) {
    c->gx[cur0] = nullptr;
    set_err(c, "step graph instantiation failed");
    return MSL_EHIP;
  }
  return MSL_OK;
}

int msl_set_graph(msl_ctx *c, int mode) {
  if (!c || mode < 0 || mode > 2) return MSL_EINVAL;
  if (mode != c->gmode) graph_release(c);
  c->gmode = mode;
  return MSL_OK;
}

int msl_step(msl_ctx *c, int nsteps) {
  if (!c || nsteps < 0) return MSL_EINVAL;
  if (!c->initialized) { set_err(c, "msl_step before msl_init"); return MSL_ESTATE; }
  if (c->cfg.pond) return pond_step(c, nsteps);
  // the x ghost columns of the current buffer are taken as stale on entry
  // (the state may have been set since the last step); the live-tile list is
  // rebuilt on first use
  c->xg_ok = 0;
  c->tl_ok = 0;
  for (int s = 0; s < nsteps;) {
    int rc;
    set_xmir(c);
    if (crit_step(c, c->step)) {
      prof_begin(c);
      rc = mask_step(c);
      if (rc) { set_err(c, "criterion / switching failed"); return rc; }
      prof_snap(c);
      if ((rc = prof_end(c, 4, -1, 0.0, (double)c->ncell))) return rc;
    }
    if (c->cfg.lift_mode == MSL_LIFT_MLP && c->mlp_on && !c->mlp_manual) {
      const int every = c->cfg.mlp_check_every > 0 ? c->cfg.mlp_check_every : 20;
      if (c->step % every == 0) {
        prof_begin(c);
        if ((rc = msl_mlp_check_launch(c))) return rc;
        if ((rc = prof_end(c, 5, -1, 0.0, 0.0))) return rc;
      }
    }
    if (graph_ok(c) && nsteps - s >= c->gB) {
      // a whole block: no timed step and no criterion pass after its first step
      bool block = true;
      for (int k = 0; k < c->gB && block; ++k)
        block = !(c->prof && (c->step + k) % c->prof == 0) && (k == 0 || !crit_step(c, c->step + k));
      if (block && !c->gx[c->cur] && (rc = graph_capture(c))) return rc;
      if (block && c->gx[c->cur]) {
        MSL_HIP(hipGraphLaunch(c->gx[c->cur], c->stream));
        c->cur ^= c->gB & 1;
        c->step += c->gB;
        s += c->gB;
        continue;
      }
    }
    // mode 2 outside graphs (3D, learned closure): the two stream-collide
    // launches on parallel branches as well, except in the steps whose
    // launches are timed one by one (msl_profile)
    const bool fork = c->gmode == 2 && c->nlat > 1 && !prof_on(c);
    if (fork && (rc = fork_streams(c))) return rc;
    if ((rc = plain_step(c, fork))) return rc;
    ++s;
    if (c->cfg.check_every > 0 && c->step % c->cfg.check_every == 0) {
      double out[5];
      rc = msl_conservation(c, out);
      if (rc) return rc;
    }
  }
  return MSL_OK;
}

int msl_macros(msl_ctx *c, double *rho, double *u, double *T) {
  if (!c) return MSL_EINVAL;
  if (!c->initialized) return MSL_ESTATE;
  if (c->cfg.pond) return msl_pond_launch_macros(c, rho, u, T);
  return msl_launch_macros(c, rho, u, T);
}

int msl_get_populations(msl_ctx *c, int which, int fg, double *out) {
  if (!c || !out || which < 0 || which >= c->nlat || (fg && !c->cfg.thermal)) return MSL_EINVAL;
  if (c->cfg.pond) {
    if (!c->initialized) return MSL_ESTATE;
    const size_t n = (size_t)c->Q[which] * c->ncell;
    return hipMemcpyAsync(out, c->pond_f[which][c->cur] + (fg ? n : 0), sizeof(double) * n, hipMemcpyDeviceToDevice,
                          c->stream) == hipSuccess ? MSL_OK : MSL_EHIP;
  }
  return msl_launch_pops(c, which, fg, out, nullptr);
}

int msl_set_populations(msl_ctx *c, int which, int fg, const double *in) {
  if (!c || !in || which < 0 || which >= c->nlat || (fg && !c->cfg.thermal) || c->cfg.pond) return MSL_EINVAL;
  int rc = msl_launch_pops(c, which, fg, nullptr, in);
  if (!rc) rc = msl_launch_bc_fixed(c);
  if (rc) return rc;
  c->initialized = 1;
  return refresh_band(c);
}

int msl_conservation(msl_ctx *c, double *out) {
  if (!c || !out || c->cfg.pond) return MSL_EINVAL;
  if (!c->initialized) return MSL_ESTATE;
  double *dev = c->red + 1024 * 9;
  int rc = msl_launch_conservation(c, dev);
  if (rc) return rc;
  double h[6];
  if (hipMemcpyAsync(h, dev, sizeof(h), hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess)
    return MSL_EHIP;
  for (int m = 0; m < 5; ++m) out[m] = h[m];
  if (h[5] != 0.0) { set_err(c, "sentinel: NaN/Inf or non-positive density"); return MSL_EUNSTABLE; }
  return MSL_OK;
}

int msl_error_norms(msl_ctx *c, const double *rho_ref, const double *u_ref, const double *T_ref,
                    double *out) {
  if (!c || !out || c->cfg.pond) return MSL_EINVAL;
  if (!c->initialized) return MSL_ESTATE;
  double *dev = c->red + 1024 * 9;
  int rc = msl_launch_error_norms(c, rho_ref, u_ref, T_ref, dev);
  if (rc) return rc;
  if (hipMemcpyAsync(out, dev, 6 * sizeof(double), hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess)
    return MSL_EHIP;
  return MSL_OK;
}

// checkpoint: [header][cls][planes of each lattice (both buffers)][closure]
struct StateHeader {
  char magic[8];
  long step;
  int cur, nlat;
  long long ncell, plane_bytes[2];
  int mlpP;
};

int msl_get_state(msl_ctx *c, void *buf, size_t *bytes) {
  if (!c || !bytes || c->cfg.pond) return MSL_EINVAL;
  size_t pb[2] = {0, 0};
  for (int l = 0; l < c->nlat; ++l)
    pb[l] = (size_t)c->Q[l] * (c->cfg.thermal ? 2 : 1) * c->geo.plane * c->esz * 2;
  const size_t need = sizeof(StateHeader) + c->ncell + pb[0] + pb[1] +
                      (size_t)(c->mlpP + 2 * c->mlpF + 2 * c->mlpO) * 4 * (c->mlpP ? 1 : 0);
  if (!buf) { *bytes = need; return MSL_OK; }
  if (*bytes < need) return MSL_ENOMEM;
  StateHeader h;
  memset(&h, 0, sizeof(h));
  memcpy(h.magic, "MSLSTAT", 8);
  h.step = c->step; h.cur = c->cur; h.nlat = c->nlat; h.ncell = c->ncell;
  h.plane_bytes[0] = (long long)pb[0]; h.plane_bytes[1] = (long long)pb[1];
  h.mlpP = c->mlpP;
  char *p = (char *)buf;
  memcpy(p, &h, sizeof(h));
  p += sizeof(h);
  MSL_HIP(hipMemcpyAsync(p, c->cls, c->ncell, hipMemcpyDeviceToHost, c->stream));
  p += c->ncell;
  for (int l = 0; l < c->nlat; ++l) {
    MSL_HIP(hipMemcpyAsync(p, c->planes[l][0], pb[l], hipMemcpyDeviceToHost, c->stream));
    p += pb[l];
  }
  if (c->mlpP) {
    MSL_HIP(hipMemcpyAsync(p, c->mlp_w, (size_t)c->mlpP * 4, hipMemcpyDeviceToHost, c->stream));
    p += (size_t)c->mlpP * 4;
    MSL_HIP(hipMemcpyAsync(p, c->mlp_stats, (size_t)(2 * c->mlpF + 2 * c->mlpO) * 4,
                           hipMemcpyDeviceToHost, c->stream));
  }
  MSL_HIP(hipStreamSynchronize(c->stream));
  *bytes = need;
  return MSL_OK;
}

int msl_set_state(msl_ctx *c, const void *buf, size_t bytes) {
  if (!c || !buf || bytes < sizeof(StateHeader) || c->cfg.pond) return MSL_EINVAL;
  StateHeader h;
  memcpy(&h, buf, sizeof(h));
  size_t pb[2] = {0, 0};
  for (int l = 0; l < c->nlat; ++l)
    pb[l] = (size_t)c->Q[l] * (c->cfg.thermal ? 2 : 1) * c->geo.plane * c->esz * 2;
  if (memcmp(h.magic, "MSLSTAT", 8) || h.nlat != c->nlat || h.ncell != c->ncell ||
      h.plane_bytes[0] != (long long)pb[0] || h.plane_bytes[1] != (long long)pb[1] ||
      h.mlpP != c->mlpP) {
    set_err(c, "checkpoint does not match this configuration");
    return MSL_EINVAL;
  }
  const char *p = (const char *)buf + sizeof(h);
  MSL_HIP(hipMemcpyAsync(c->cls, p, c->ncell, hipMemcpyHostToDevice, c->stream));
  p += c->ncell;
  for (int l = 0; l < c->nlat; ++l) {
    MSL_HIP(hipMemcpyAsync(c->planes[l][0], p, pb[l], hipMemcpyHostToDevice, c->stream));
    p += pb[l];
  }
  if (c->mlpP) {
    MSL_HIP(hipMemcpyAsync(c->mlp_w, p, (size_t)c->mlpP * 4, hipMemcpyHostToDevice, c->stream));
    p += (size_t)c->mlpP * 4;
    MSL_HIP(hipMemcpyAsync(c->mlp_stats, p, (size_t)(2 * c->mlpF + 2 * c->mlpO) * 4,
                           hipMemcpyHostToDevice, c->stream));
    c->mlp_on = 1;
  }
  c->step = h.step;
  c->cur = h.cur;
  c->initialized = 1;
  // class bits, tiles and band lists follow from the restored mask
  int rc = msl_launch_classify(c);
  if (rc) return rc;
  MSL_HIP(hipStreamSynchronize(c->stream));
  return MSL_OK;
}

int msl_num_check_tiles(const msl_ctx *c, int *n) {
  if (!c || !n) return MSL_EINVAL;
  *n = c->nctile;
  return MSL_OK;
}

}  // extern "C"
