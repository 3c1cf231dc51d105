/*
 * oracle_step.c -- the multi-scale semi-Lagrangian time step, cell by cell.
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * One step, for every cell x with velocity-set order l (Sec. III.D):
 *   1. for each population i of order l, the departure point x - v_i dt and the
 *      3-point-per-axis collocation points around the nearest node, with the
 *      particle velocities v_i = sqrt(T_ref) c_i + u_ref of the run's global
 *      constant frame (eq. veli; the lattice frame is u_ref = 0, T_ref = 1);
 *   2. every collocation point of another order is converted to order l by
 *      lifting (lower order) or projection (higher order), on the fly; points
 *      outside the domain resolve through the boundary rule of their face;
 *   3. Lagrange reconstruction at the departure point (eqs. reconstructionPond,
 *      advectionPond; every point shares the one frame, so the transfer matrix
 *      is the identity);
 *   4. BGK collision towards the equilibrium in that frame (eqs. Pond_f, Pond_g
 *      with omega1 = omega2 = 1/tau; eqs. feqL, geqL with the frame as target).
 * The stored state is the post-collision population vector of each cell.
 */
#include "oracle_internal.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define REACH_MAX 3
#define SIDE_MAX (2 * REACH_MAX + 1)

struct or_ctx {
  or_config cfg;
  int D, N[3];
  int64_t ncell;
  int nlat;
  lat_t *lat[2];
  double dt;
  int reach;
  int n0[2][OR_MAXQ][3];
  double a[2][OR_MAXQ][3][3];
  double *f[2], *g[2], *fn[2], *gn[2];
  double sW[2][OR_MAXQ];   /* reduced-precision storage scale of each f population */
  uint8_t *order;
  long step;
  /* learned closure */
  int mlp_on, mlp_H, mlp_F, mlp_O, mlp_bf16;
  double *mlp_p, *xm, *xs, *tm, *ts;
  int ntile[3];
  int ntiles;
  uint8_t *flags;
  double *emlp, *egrad;
};

/* ------------------------------------------------------------------------ */

static int64_t cell_index(const or_ctx *c, const int *p) {
  return (int64_t)p[0] + (int64_t)c->N[0] * ((int64_t)p[1] + (int64_t)c->N[1] * (int64_t)p[2]);
}

static void cell_coords(const or_ctx *c, int64_t k, int *p) {
  p[0] = (int)(k % c->N[0]);
  k /= c->N[0];
  p[1] = (int)(k % c->N[1]);
  p[2] = (int)(k / c->N[1]);
}

static int tile_of(const or_ctx *c, const int *p) {
  int t0 = p[0] / OR_CHECK_TILE, t1 = p[1] / OR_CHECK_TILE, t2 = p[2] / OR_CHECK_TILE;
  return t0 + c->ntile[0] * (t1 + c->ntile[1] * t2);
}

/* storage rounding of the configured precision: FP32, or deviations
 * h = f / scale_i - 1 kept in 16 bits (scale_i = rho0 W_i unless a storage
 * reference velocity tilts it) */
static double store_round(const or_ctx *c, double v, double scale) {
  switch (c->cfg.store) {
    case 1: return (double)(float)v;
    case 2: return scale * (1.0 + or_round_fp16(v / scale - 1.0));
    case 3: return scale * (1.0 + or_round_bf16(v / scale - 1.0));
    default: return v;
  }
}

static double fscale(const or_ctx *c, int l, int i) { return c->sW[l][i]; }
static double gscale(const or_ctx *c, int l, int i) {
  return (c->cfg.cv - 0.5 * c->D) * c->cfg.T0 * c->sW[l][i];
}

/* ---- conversion of one cell's state between the two orders ---- */

static void lift_state(const or_ctx *c, const double *fq, const double *gq, int tile,
                       double *fQ, double *gQ);

static void convert(const or_ctx *c, int from, int to, const double *f, const double *g,
                    int tile, double *fo, double *go) {
  const int th = c->cfg.thermal;
  if (from == to) {
    memcpy(fo, f, sizeof(double) * c->lat[from]->Q);
    if (th) memcpy(go, g, sizeof(double) * c->lat[from]->Q);
  } else if (from < to) {
    lift_state(c, f, g, tile, fo, go);
  } else {
    lat_project(c->lat[from], c->lat[to], th, f, g, fo, go);
  }
}

/* ---- boundary resolution of a point outside the domain ---- */

typedef struct {
  int kind;            /* 0 cell, 1 equilibrium state, 2 diffuse wall */
  int64_t cell;
  double st[5];        /* rho, ux, uy, uz, T */
  double rho_w;
} src_t;

static int in_slot(const or_ctx *c, int face, const int *p) {
  const int *s = c->cfg.slot[face];
  if (s[0] >= s[1]) return 0;
  int ax = face / 2, t[2], nt = 0;
  for (int a = 0; a < c->D; a++) if (a != ax) t[nt++] = a;
  if (p[t[0]] < s[0] || p[t[0]] >= s[1]) return 0;
  if (c->D == 3 && s[2] < s[3] && (p[t[1]] < s[2] || p[t[1]] >= s[3])) return 0;
  return 1;
}

static void native_state(const or_ctx *c, int64_t k, double *f, double *g) {
  int l = c->order[k];
  for (int i = 0; i < c->lat[l]->Q; i++) {
    f[i] = c->f[l][(int64_t)i * c->ncell + k];
    if (c->cfg.thermal) g[i] = c->g[l][(int64_t)i * c->ncell + k];
  }
}

/* The highest out-of-range axis is resolved first, then the lower ones.  A
 * diffuse wall returns the wall equilibrium scaled by rho_w, chosen so that the
 * mass flux leaving the fluid cell next to the wall through the wall equals
 * the flux the wall equilibrium sends back (zero net wall-normal mass flux). */
static void resolve(const or_ctx *c, const int *pin, src_t *out) {
  int p[3] = {pin[0], pin[1], pin[2]};
  for (int ax = c->D - 1; ax >= 0; ax--) {
    if (p[ax] >= 0 && p[ax] < c->N[ax]) continue;
    int side = p[ax] < 0 ? 0 : 1;
    int face = 2 * ax + side;
    switch (c->cfg.bc[face]) {
      case 0:
        p[ax] = ((p[ax] % c->N[ax]) + c->N[ax]) % c->N[ax];
        break;
      case 2:
        p[ax] = side ? c->N[ax] - 1 : 0;
        break;
      case 1: {
        out->kind = 1;
        const double w = c->cfg.slot_edge[face];
        if (w > 0.0 && c->cfg.slot[face][0] < c->cfg.slot[face][1]) {
          /* smooth slot: weight 1/2 [tanh((t - lo + 1/2)/w) - tanh((t - hi + 1/2)/w)]
           * along each restricted tangential axis */
          int t[2], nt = 0;
          for (int a = 0; a < c->D; a++) if (a != ax) t[nt++] = a;
          const int *s = c->cfg.slot[face];
          double lam = 0.5 * (tanh((p[t[0]] - s[0] + 0.5) / w) - tanh((p[t[0]] - s[1] + 0.5) / w));
          if (c->D == 3 && s[2] < s[3])
            lam *= 0.5 * (tanh((p[t[1]] - s[2] + 0.5) / w) - tanh((p[t[1]] - s[3] + 0.5) / w));
          for (int m = 0; m < 5; m++)
            out->st[m] = c->cfg.bc_state[face][m] +
                         lam * (c->cfg.slot_state[face][m] - c->cfg.bc_state[face][m]);
          return;
        }
        const double *st = in_slot(c, face, p) ? c->cfg.slot_state[face] : c->cfg.bc_state[face];
        memcpy(out->st, st, sizeof(double) * 5);
        return;
      }
      case 3: {
        int q[3] = {p[0], p[1], p[2]};
        q[ax] = side ? c->N[ax] - 1 : 0;
        src_t adj;
        resolve(c, q, &adj);
        double f[OR_MAXQ], g[OR_MAXQ];
        int l;
        if (adj.kind == 0) {
          l = c->order[adj.cell];
          native_state(c, adj.cell, f, g);
        } else {
          l = 0;
          lat_feq(c->lat[0], adj.st[0], adj.st + 1, adj.st[4], f);
        }
        const lat_t *L = c->lat[l];
        const double *ws = c->cfg.bc_state[face];
        double weq[OR_MAXQ];
        lat_feq(L, 1.0, ws + 1, ws[4], weq);
        ld in = 0.0L, outf = 0.0L;
        for (int i = 0; i < L->Q; i++) {
          double cn = L->v[i][ax];
          int towall = side ? (cn > 0) : (cn < 0);
          int fromwall = side ? (cn < 0) : (cn > 0);
          if (towall) in += fabsl((ld)cn) * (ld)f[i];
          if (fromwall) outf += fabsl((ld)cn) * (ld)weq[i];
        }
        out->kind = 2;
        memcpy(out->st, ws, sizeof(double) * 5);
        out->st[0] = 1.0;
        out->rho_w = (double)(in / outf);
        return;
      }
      default:
        break;
    }
  }
  out->kind = 0;
  out->cell = cell_index(c, p);
}

/* state of lattice `l` at a resolved source point */
static void src_state(const or_ctx *c, const src_t *s, int l, double *f, double *g) {
  const lat_t *L = c->lat[l];
  const int th = c->cfg.thermal;
  if (s->kind == 0) {
    double fs[OR_MAXQ], gs[OR_MAXQ];
    native_state(c, s->cell, fs, gs);
    int p[3];
    cell_coords(c, s->cell, p);
    convert(c, c->order[s->cell], l, fs, gs, tile_of(c, p), f, g);
    return;
  }
  double feq[OR_MAXQ];
  lat_feq(L, 1.0, s->st + 1, s->st[4], feq);
  double rho = s->kind == 1 ? s->st[0] : s->rho_w;
  for (int i = 0; i < L->Q; i++) f[i] = rho * feq[i];
  if (th) lat_geq_from_feq(L, c->cfg.cv, s->st[4], f, g);
}

/* ---- collision ---- */

static double relax_tau(const or_ctx *c, double rho, double T) {
  if (c->cfg.tau_mode == 0) return c->cfg.tau;
  /* mu = (tau - 1/2) rho T dt (transport coefficients, R = 1), mu ~ T^s */
  double mu_ref = (c->cfg.tau - 0.5) * c->cfg.tau_ref_rho * c->cfg.tau_ref_T * c->dt;
  double mu = mu_ref * pow(T / c->cfg.tau_ref_T, c->cfg.mu_exp);
  return mu / (rho * T * c->dt) + 0.5;
}

/* Collision (eqs. Pond_f, Pond_g): relaxation towards the equilibrium at rate
 * omega1 = 1/tau, plus (omega1 - omega2)(f* - f^eq) towards the
 * quasi-equilibrium when the two rates differ.  omega2 follows tau2 at the
 * reference state; where tau varies with T the Prandtl number
 * Pr = (tau - 1/2)/(tau2 - 1/2) is kept. */
static void collide(const or_ctx *c, int l, const double *ft, const double *gt,
                    double *fo, double *go) {
  const lat_t *L = c->lat[l];
  const int th = c->cfg.thermal;
  double rho, u[3], T;
  lat_macros(L, th, c->cfg.cv, ft, gt, &rho, u, &T);
  double feq[OR_MAXQ], geq[OR_MAXQ];
  lat_feq(L, rho, u, T, feq);
  if (th) lat_geq_from_feq(L, c->cfg.cv, T, feq, geq);
  const double tl = relax_tau(c, rho, T);
  const double om = 1.0 / tl;
  const int two = c->cfg.tau2 > 0.0 && c->cfg.tau2 != c->cfg.tau;
  double fs[OR_MAXQ], gs[OR_MAXQ], om2 = om;
  if (two) {
    om2 = 1.0 / (0.5 + (tl - 0.5) * (c->cfg.tau2 - 0.5) / (c->cfg.tau - 0.5));
    lat_qeq(L, th, c->cfg.cv, rho, u, T, ft, gt, feq, geq, fs, gs);
  }
  for (int i = 0; i < L->Q; i++) {
    fo[i] = ft[i] + om * (feq[i] - ft[i]);
    if (two) fo[i] += (om - om2) * (fs[i] - feq[i]);
  }
  if (th)
    for (int i = 0; i < L->Q; i++) {
      go[i] = gt[i] + om * (geq[i] - gt[i]);
      if (two) go[i] += (om - om2) * (gs[i] - geq[i]);
    }
}

/* ---- one cell's update ---- */

typedef struct {
  double *f, *g;       /* [SIDE^D][Q] converted neighbourhood */
  uint8_t *have;
} nbhd_t;

static void nbhd_alloc(nbhd_t *nb) {
  size_t npts = SIDE_MAX * SIDE_MAX * SIDE_MAX;
  nb->f = (double *)malloc(sizeof(double) * npts * OR_MAXQ);
  nb->g = (double *)malloc(sizeof(double) * npts * OR_MAXQ);
  nb->have = (uint8_t *)malloc(npts);
}

static void nbhd_free(nbhd_t *nb) {
  free(nb->f);
  free(nb->g);
  free(nb->have);
}

static void update_cell(const or_ctx *c, int64_t k, nbhd_t *nb, double *fo, double *go) {
  const int D = c->D, R = c->reach, S = 2 * R + 1;
  const int l = c->order[k];
  const lat_t *L = c->lat[l];
  const int Q = L->Q;
  int p[3];
  cell_coords(c, k, p);
  memset(nb->have, 0, (size_t)S * S * S);
  double ft[OR_MAXQ], gt[OR_MAXQ];
  for (int i = 0; i < Q; i++) {
    ld accf = 0.0L, accg = 0.0L;
    int nsp = 1;
    for (int a = 0; a < D; a++) nsp *= 3;
    for (int s = 0; s < nsp; s++) {
      int sv[3] = {0, 0, 0}, r = s;
      double w = 1.0;
      int off[3] = {0, 0, 0};
      for (int a = 0; a < D; a++) {
        sv[a] = r % 3 - 1;
        r /= 3;
        w *= c->a[l][i][a][sv[a] + 1];
        off[a] = c->n0[l][i][a] + sv[a];
      }
      int slot = (off[0] + R) + S * ((off[1] + R) + S * (D == 3 ? off[2] + R : 0));
      double *F = nb->f + (size_t)slot * OR_MAXQ;
      double *G = nb->g + (size_t)slot * OR_MAXQ;
      if (!nb->have[slot]) {
        int q[3] = {p[0] + off[0], p[1] + off[1], D == 3 ? p[2] + off[2] : 0};
        src_t src;
        resolve(c, q, &src);
        src_state(c, &src, l, F, G);
        nb->have[slot] = 1;
      }
      accf += (ld)w * (ld)F[i];
      if (c->cfg.thermal) accg += (ld)w * (ld)G[i];
    }
    ft[i] = (double)accf;
    gt[i] = (double)accg;
  }
  collide(c, l, ft, gt, fo, go);
  for (int i = 0; i < Q; i++) {
    fo[i] = store_round(c, fo[i], fscale(c, l, i));
    if (c->cfg.thermal) go[i] = store_round(c, go[i], gscale(c, l, i));
  }
}

/* ------------------------------------------------------------------------ */

int or_create(const or_config *cfg, or_ctx **out) {
  if (!cfg || !out) return -1;
  if (cfg->dim != 2 && cfg->dim != 3) return -1;
  if (cfg->nx < 1 || cfg->ny < 1 || (cfg->dim == 3 && cfg->nz < 1)) return -1;
  if (cfg->n_low < 2 || (cfg->n_high && cfg->n_high <= cfg->n_low)) return -1;
  if (cfg->tau <= 0.5) return -1;
  if (cfg->tau2 > 0.0 && cfg->tau2 <= 0.5) return -1;
  or_ctx *c = (or_ctx *)calloc(1, sizeof(or_ctx));
  c->cfg = *cfg;
  c->D = cfg->dim;
  c->N[0] = cfg->nx;
  c->N[1] = cfg->ny;
  c->N[2] = cfg->dim == 3 ? cfg->nz : 1;
  c->ncell = (int64_t)c->N[0] * c->N[1] * c->N[2];
  c->nlat = cfg->n_high ? 2 : 1;
  c->lat[0] = lat_build(c->D, cfg->n_low);
  c->lat[1] = cfg->n_high ? lat_build(c->D, cfg->n_high) : NULL;
  if (!c->lat[0] || (cfg->n_high && !c->lat[1])) { or_destroy(c); return -2; }
  /* the run's reference frame (eq. veli); T_ref <= 0 stands for 1 */
  const double Tref = cfg->T_ref > 0.0 ? cfg->T_ref : 1.0;
  for (int l = 0; l < c->nlat; l++)
    if (lat_set_frame(c->lat[l], cfg->u_ref, Tref)) { or_destroy(c); return -2; }
  if (cfg->lift_mode == 2 && !lat_frame_trivial(c->lat[0])) { or_destroy(c); return -1; }
  /* time step from CFL = max|v_ia| dt / dx, the largest particle speed along any
   * axis over every configured velocity set */
  double vmax = 0.0;
  for (int l = 0; l < c->nlat; l++)
    for (int a = 0; a < c->D; a++)
      if (lat_vmax(c->lat[l], a) > vmax) vmax = lat_vmax(c->lat[l], a);
  c->dt = cfg->cfl / vmax;
  /* storage scale: rho0 W_i carried over to the storage reference state
   * (store_u, T0): rho0 prod_a w_a r(c_a) with r the density ratio of the
   * Gaussian N(s_a, th) to N(0, 1) at the node, s = (store_u - u_ref)/sqrt(T_ref),
   * th = T0 / T_ref; rho0 W_i when store_u = u_ref and T0 = T_ref */
  const double ths = cfg->T0 / Tref;
  for (int l = 0; l < c->nlat; l++) {
    const lat_t *L = c->lat[l];
    for (int i = 0; i < L->Q; i++) {
      double sc = cfg->rho0;
      for (int a = 0; a < c->D; a++) {
        const double sa = (cfg->store_u[a] - cfg->u_ref[a]) / sqrt(Tref);
        const double ca = L->c[i][a];
        sc *= (double)L->w[L->pw[i][a]] *
              exp(0.5 * ca * ca - 0.5 * (ca - sa) * (ca - sa) / ths) / sqrt(ths);
      }
      c->sW[l][i] = sc;
    }
  }
  c->reach = 0;
  for (int l = 0; l < c->nlat; l++) {
    const lat_t *L = c->lat[l];
    for (int i = 0; i < L->Q; i++)
      for (int a = 0; a < c->D; a++) {
        double d = -L->v[i][a] * c->dt;     /* departure point offset x - v_i dt */
        int n0 = (int)floor(d + 0.5);       /* nearest node */
        c->n0[l][i][a] = n0;
        or_lagrange3(d - n0, c->a[l][i][a]);
        int r = abs(n0) + 1;
        if (r > c->reach) c->reach = r;
      }
  }
  if (c->reach > REACH_MAX) { or_destroy(c); return -1; }
  for (int l = 0; l < c->nlat; l++) {
    size_t sz = sizeof(double) * (size_t)c->lat[l]->Q * c->ncell;
    c->f[l] = (double *)calloc(1, sz);
    c->fn[l] = (double *)calloc(1, sz);
    if (cfg->thermal) {
      c->g[l] = (double *)calloc(1, sz);
      c->gn[l] = (double *)calloc(1, sz);
    }
  }
  c->order = (uint8_t *)calloc(1, (size_t)c->ncell);
  for (int a = 0; a < 3; a++) c->ntile[a] = (c->N[a] + OR_CHECK_TILE - 1) / OR_CHECK_TILE;
  c->ntiles = c->ntile[0] * c->ntile[1] * c->ntile[2];
  c->flags = (uint8_t *)malloc((size_t)c->ntiles);
  memset(c->flags, 1, (size_t)c->ntiles);
  c->emlp = (double *)calloc((size_t)c->ntiles, sizeof(double));
  c->egrad = (double *)calloc((size_t)c->ntiles, sizeof(double));
  *out = c;
  return 0;
}

void or_destroy(or_ctx *c) {
  if (!c) return;
  for (int l = 0; l < 2; l++) {
    lat_free(c->lat[l]);
    free(c->f[l]); free(c->fn[l]); free(c->g[l]); free(c->gn[l]);
  }
  free(c->order);
  free(c->flags); free(c->emlp); free(c->egrad);
  free(c->mlp_p); free(c->xm); free(c->xs); free(c->tm); free(c->ts);
  free(c);
}

int or_qeq(const or_ctx *c, int which, const double *f, const double *g, double *fstar,
           double *gstar) {
  if (which < 0 || which >= c->nlat) return -1;
  const lat_t *L = c->lat[which];
  double rho, u[3], T, feq[OR_MAXQ], geq[OR_MAXQ];
  lat_macros(L, c->cfg.thermal, c->cfg.cv, f, g, &rho, u, &T);
  lat_feq(L, rho, u, T, feq);
  if (c->cfg.thermal) lat_geq_from_feq(L, c->cfg.cv, T, feq, geq);
  lat_qeq(L, c->cfg.thermal, c->cfg.cv, rho, u, T, f, g, feq, geq, fstar, gstar);
  return 0;
}

int or_set_threads(int n) {
#ifdef _OPENMP
  int prev = omp_get_max_threads();
  if (n >= 1) omp_set_num_threads(n);
  return prev;
#else
  (void)n;
  return 1;
#endif
}

double or_dt(const or_ctx *c) { return c->dt; }
int or_reach(const or_ctx *c) { return c->reach; }
long or_step_count(const or_ctx *c) { return c->step; }

int or_stencil(const or_ctx *c, int which, int *n0, double *a) {
  if (which < 0 || which >= c->nlat) return -1;
  const lat_t *L = c->lat[which];
  for (int i = 0; i < L->Q; i++)
    for (int ax = 0; ax < c->D; ax++) {
      n0[i * c->D + ax] = c->n0[which][i][ax];
      for (int s = 0; s < 3; s++) a[(i * c->D + ax) * 3 + s] = c->a[which][i][ax][s];
    }
  return 0;
}

int or_set_mask_raw(or_ctx *c, const uint8_t *mask) {
  for (int64_t k = 0; k < c->ncell; k++) {
    if (mask[k] > 1 || (mask[k] == 1 && c->nlat < 2)) return -1;
  }
  memcpy(c->order, mask, (size_t)c->ncell);
  return 0;
}

/* Switching (Sec. III.A): a cell whose order changes lifts or projects its own
 * state into the new velocity set. */
int or_set_mask(or_ctx *c, const uint8_t *mask) {
  for (int64_t k = 0; k < c->ncell; k++)
    if (mask[k] > 1 || (mask[k] == 1 && c->nlat < 2)) return -1;
  const int th = c->cfg.thermal;
#pragma omp parallel for schedule(dynamic, 256)
  for (int64_t k = 0; k < c->ncell; k++) {
    int from = c->order[k], to = mask[k];
    if (from == to) continue;
    double f[OR_MAXQ], g[OR_MAXQ], fo[OR_MAXQ], go[OR_MAXQ];
    native_state(c, k, f, g);
    int p[3];
    cell_coords(c, k, p);
    if (from < to && c->cfg.lift_mode == 2)
      /* a switching cell is lifted with the plain completion; the learned
       * closure only serves collocation points of the band */
      lat_lift_raw(c->lat[0], c->lat[1], th, c->cfg.cv, f, g, NULL, fo, go);
    else
      convert(c, from, to, f, g, tile_of(c, p), fo, go);
    for (int i = 0; i < c->lat[to]->Q; i++) {
      c->f[to][(int64_t)i * c->ncell + k] = store_round(c, fo[i], fscale(c, to, i));
      if (th) c->g[to][(int64_t)i * c->ncell + k] = store_round(c, go[i], gscale(c, to, i));
    }
  }
  memcpy(c->order, mask, (size_t)c->ncell);
  return 0;
}

int or_get_mask(const or_ctx *c, uint8_t *mask) {
  memcpy(mask, c->order, (size_t)c->ncell);
  return 0;
}

/* Refinement criteria of one cell: local Mach number |u|/c_s (c_s = 1
 * athermal, sqrt(gamma T) thermal), or the Frobenius norm of the
 * non-equilibrium part of the central second moment over the pressure
 * p = rho T.  (The Knudsen-number criterion needs the neighbours: below.) */
static double criterion_value(const or_ctx *c, int64_t k) {
  double f[OR_MAXQ], g[OR_MAXQ];
  native_state(c, k, f, g);
  const lat_t *L = c->lat[c->order[k]];
  double rho, u[3], T;
  lat_macros(L, c->cfg.thermal, c->cfg.cv, f, g, &rho, u, &T);
  if (c->cfg.crit_kind == 1) {
    double gam = (c->cfg.cv + 1.0) / c->cfg.cv;
    double cs = c->cfg.thermal ? sqrt(gam * T) : 1.0;
    double u2 = 0;
    for (int a = 0; a < c->D; a++) u2 += u[a] * u[a];
    return sqrt(u2) / cs;
  }
  if (c->cfg.crit_kind == 2) {
    double P[3][3] = {{0}};
    for (int i = 0; i < L->Q; i++)
      for (int a = 0; a < c->D; a++)
        for (int b = 0; b < c->D; b++)
          P[a][b] += (L->v[i][a] - u[a]) * (L->v[i][b] - u[b]) * f[i];
    double p = rho * T, s = 0;
    for (int a = 0; a < c->D; a++)
      for (int b = 0; b < c->D; b++) {
        double d = P[a][b] - (a == b ? p : 0.0);
        s += d * d;
      }
    return sqrt(s) / p;
  }
  return 0.0;
}

/* Local Knudsen number (Sec. IV.A.3): Kn = lambda / L with L = |phi / (dphi/dx)|
 * and phi the density.  The mean free path is the hard-sphere one of the
 * same section, lambda = 16/(5 sqrt(2 pi gamma)) mu a / p, evaluated with the
 * cell's own state: a = sqrt(gamma T), p = rho T and the viscosity of the
 * collision, mu = (tau - 1/2) rho T dt (transport coefficients of Sec. II.B;
 * tau the local relaxation time where it follows mu(T)).  In more than one
 * dimension L = rho / |grad rho|.  The derivative is the central difference
 * of the cell densities; across a face that is not periodic the missing
 * neighbour is the cell itself (a one-sided difference over one cell). */
static void knudsen_field(const or_ctx *c, double *kn) {
  const int64_t n = c->ncell;
  double *rho = (double *)malloc((size_t)n * sizeof(double));
  double *lam = (double *)malloc((size_t)n * sizeof(double));
  const double gam = (c->cfg.cv + 1.0) / c->cfg.cv;
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < n; k++) {
    double f[OR_MAXQ], g[OR_MAXQ], r, u[3], T;
    native_state(c, k, f, g);
    lat_macros(c->lat[c->order[k]], c->cfg.thermal, c->cfg.cv, f, g, &r, u, &T);
    const double mu = (relax_tau(c, r, T) - 0.5) * r * T * c->dt;
    const double a = sqrt(gam * T), p = r * T;
    rho[k] = r;
    lam[k] = 16.0 / (5.0 * sqrt(2.0 * acos(-1.0) * gam)) * mu * a / p;
  }
  const int ext[3] = {c->cfg.nx, c->cfg.ny, c->D == 3 ? c->cfg.nz : 1};
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < n; k++) {
    int p[3];
    cell_coords(c, k, p);
    double g2 = 0.0;
    for (int a = 0; a < c->D; a++) {
      if (ext[a] < 2) continue;
      const int periodic = c->cfg.bc[2 * a] == 0 && c->cfg.bc[2 * a + 1] == 0;
      int lo[3] = {p[0], p[1], p[2]}, hi[3] = {p[0], p[1], p[2]};
      lo[a] = p[a] - 1;
      hi[a] = p[a] + 1;
      if (periodic) {
        lo[a] = (lo[a] + ext[a]) % ext[a];
        hi[a] = hi[a] % ext[a];
      } else {
        if (lo[a] < 0) lo[a] = 0;
        if (hi[a] >= ext[a]) hi[a] = ext[a] - 1;
      }
      const double dist = periodic ? 2.0 : (double)(hi[a] - lo[a]);
      const double d = (rho[cell_index(c, hi)] - rho[cell_index(c, lo)]) / dist;
      g2 += d * d;
    }
    kn[k] = lam[k] * sqrt(g2) / rho[k];
  }
  free(rho);
  free(lam);
}

int or_eval_criterion(const or_ctx *c, uint8_t *newmask, double *value) {
  double *kn = NULL;
  if (c->cfg.crit_kind == 3) {
    kn = (double *)malloc((size_t)c->ncell * sizeof(double));
    knudsen_field(c, kn);
  }
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < c->ncell; k++) {
    double v = kn ? kn[k] : criterion_value(c, k);
    if (value) value[k] = v;
    if (newmask) newmask[k] = (c->nlat > 1 && c->cfg.crit_kind && v > c->cfg.crit_thr) ? 1 : 0;
  }
  free(kn);
  return 0;
}

int or_init(or_ctx *c, const double *rho, const double *u, const double *T) {
  const int th = c->cfg.thermal;
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < c->ncell; k++) {
    int l = c->order[k];
    const lat_t *L = c->lat[l];
    double uu[3] = {0, 0, 0};
    for (int a = 0; a < c->D; a++) uu[a] = u[(int64_t)a * c->ncell + k];
    double Tk = th ? T[k] : 1.0;
    double feq[OR_MAXQ], geq[OR_MAXQ];
    lat_feq(L, rho[k], uu, Tk, feq);
    if (th) lat_geq_from_feq(L, c->cfg.cv, Tk, feq, geq);
    for (int i = 0; i < L->Q; i++) {
      c->f[l][(int64_t)i * c->ncell + k] = store_round(c, feq[i], fscale(c, l, i));
      if (th) c->g[l][(int64_t)i * c->ncell + k] = store_round(c, geq[i], gscale(c, l, i));
    }
  }
  c->step = 0;
  return 0;
}

/* the criterion's margin: a box maximum of the selection, one axis after the
 * other (the box is separable) */
int or_dilate_mask(const or_config *cfg, const uint8_t *in, uint8_t *out) {
  const int D = cfg->dim, m = cfg->crit_margin;
  const int N[3] = {cfg->nx, cfg->ny, D == 3 ? cfg->nz : 1};
  const int64_t n = (int64_t)N[0] * N[1] * N[2];
  memcpy(out, in, (size_t)n);
  if (m <= 0) return 0;
  uint8_t *tmp = (uint8_t *)malloc((size_t)n);
  for (int a = 0; a < D; a++) {
    memcpy(tmp, out, (size_t)n);
    const int periodic = cfg->bc[2 * a] == 0 && cfg->bc[2 * a + 1] == 0;
    const int64_t stride = a == 0 ? 1 : (a == 1 ? N[0] : (int64_t)N[0] * N[1]);
    for (int64_t k = 0; k < n; k++) {
      const int p = (int)((k / stride) % N[a]);
      uint8_t v = 0;
      for (int d = -m; d <= m; d++) {
        int q = p + d;
        if (q < 0 || q >= N[a]) {
          if (!periodic) continue;
          q = ((q % N[a]) + N[a]) % N[a];
        }
        v |= tmp[k + (int64_t)(q - p) * stride];
      }
      out[k] = v;
    }
  }
  free(tmp);
  return 0;
}

int or_step(or_ctx *c, int nsteps) {
  const int th = c->cfg.thermal;
  uint8_t *nm = NULL;
  if (c->cfg.crit_kind && c->cfg.crit_every > 0 && c->nlat > 1)
    nm = (uint8_t *)malloc((size_t)c->ncell);
  for (int s = 0; s < nsteps; s++) {
    if (nm && c->step % c->cfg.crit_every == 0) {
      or_eval_criterion(c, nm, NULL);
      if (c->cfg.crit_margin > 0) {
        uint8_t *dm = (uint8_t *)malloc((size_t)c->ncell);
        or_dilate_mask(&c->cfg, nm, dm);
        memcpy(nm, dm, (size_t)c->ncell);
        free(dm);
      }
      or_set_mask(c, nm);
    }
    if (c->mlp_on && c->step % 20 == 0 && !(c->mlp_bf16 & 2)) or_mlp_check(c);
#pragma omp parallel
    {
      nbhd_t nb;
      nbhd_alloc(&nb);
      double fo[OR_MAXQ], go[OR_MAXQ];
#pragma omp for schedule(dynamic, 64)
      for (int64_t k = 0; k < c->ncell; k++) {
        int l = c->order[k];
        update_cell(c, k, &nb, fo, go);
        for (int i = 0; i < c->lat[l]->Q; i++) {
          c->fn[l][(int64_t)i * c->ncell + k] = fo[i];
          if (th) c->gn[l][(int64_t)i * c->ncell + k] = go[i];
        }
      }
      nbhd_free(&nb);
    }
    for (int l = 0; l < c->nlat; l++) {
      double *t = c->f[l]; c->f[l] = c->fn[l]; c->fn[l] = t;
      t = c->g[l]; c->g[l] = c->gn[l]; c->gn[l] = t;
    }
    c->step++;
  }
  free(nm);
  return 0;
}

int or_step_cells(const or_ctx *c, int ncells, const int64_t *cells, double *fout,
                  double *gout) {
  int Qm = c->lat[c->nlat - 1]->Q;
#pragma omp parallel
  {
    nbhd_t nb;
    nbhd_alloc(&nb);
    double fo[OR_MAXQ], go[OR_MAXQ];
#pragma omp for schedule(dynamic, 4)
    for (int n = 0; n < ncells; n++) {
      int64_t k = cells[n];
      if (k < 0 || k >= c->ncell) continue;
      update_cell(c, k, &nb, fo, go);
      int Q = c->lat[c->order[k]]->Q;
      for (int i = 0; i < Qm; i++) {
        fout[(size_t)n * Qm + i] = i < Q ? fo[i] : 0.0;
        if (gout) gout[(size_t)n * Qm + i] = (i < Q && c->cfg.thermal) ? go[i] : 0.0;
      }
    }
    nbhd_free(&nb);
  }
  return 0;
}

/* populations of lattice `which` at every cell: native values where the cell
 * uses that order, the lifted / projected native state elsewhere */
int or_get_pops(const or_ctx *c, int which, int fg, double *out) {
  if (which < 0 || which >= c->nlat || (fg && !c->cfg.thermal)) return -1;
  const int Q = c->lat[which]->Q;
#pragma omp parallel for schedule(dynamic, 256)
  for (int64_t k = 0; k < c->ncell; k++) {
    double f[OR_MAXQ], g[OR_MAXQ], fo[OR_MAXQ], go[OR_MAXQ];
    native_state(c, k, f, g);
    int p[3];
    cell_coords(c, k, p);
    convert(c, c->order[k], which, f, g, tile_of(c, p), fo, go);
    for (int i = 0; i < Q; i++) out[(int64_t)i * c->ncell + k] = fg ? go[i] : fo[i];
  }
  return 0;
}

int or_set_pops(or_ctx *c, int which, int fg, const double *in) {
  if (which < 0 || which >= c->nlat || (fg && !c->cfg.thermal)) return -1;
  const int Q = c->lat[which]->Q;
  double *dst = fg ? c->g[which] : c->f[which];
  memcpy(dst, in, sizeof(double) * (size_t)Q * c->ncell);
  return 0;
}

int or_macros(const or_ctx *c, double *rho, double *u, double *T) {
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < c->ncell; k++) {
    double f[OR_MAXQ], g[OR_MAXQ], r, uu[3], t;
    native_state(c, k, f, g);
    lat_macros(c->lat[c->order[k]], c->cfg.thermal, c->cfg.cv, f, g, &r, uu, &t);
    if (rho) rho[k] = r;
    if (u) for (int a = 0; a < c->D; a++) u[(int64_t)a * c->ncell + k] = uu[a];
    if (T) T[k] = t;
  }
  return 0;
}

/* global sums of the conserved quantities: rho, rho u (3), rho E */
int or_conservation(const or_ctx *c, double *out) {
  ld s[5] = {0, 0, 0, 0, 0};
  for (int64_t k = 0; k < c->ncell; k++) {
    const lat_t *L = c->lat[c->order[k]];
    double f[OR_MAXQ], g[OR_MAXQ];
    native_state(c, k, f, g);
    for (int i = 0; i < L->Q; i++) {
      ld fi = (ld)f[i], c2 = 0.0L;
      s[0] += fi;
      for (int a = 0; a < c->D; a++) {
        s[1 + a] += (ld)L->v[i][a] * fi;
        c2 += (ld)L->v[i][a] * (ld)L->v[i][a];
      }
      s[4] += 0.5L * c2 * fi;
      if (c->cfg.thermal) s[4] += (ld)g[i];
    }
  }
  for (int m = 0; m < 5; m++) out[m] = (double)s[m];
  return 0;
}

/* ------------------------------------------------------------------------ */
/* learned closure in the lifting step                                      */
/* ------------------------------------------------------------------------ */

int or_set_mlp(or_ctx *c, int H, const double *params, const double *xmean,
               const double *xstd, const double *tmean, const double *tstd, int bf16) {
  if (c->nlat < 2 || !lat_frame_trivial(c->lat[0])) return -1;
  int F, O;
  or_mlp_dims(c->D, c->lat[0]->n, c->lat[1]->n, &F, &O);
  int np = or_mlp_nparams(F, H, O);
  free(c->mlp_p); free(c->xm); free(c->xs); free(c->tm); free(c->ts);
  c->mlp_p = (double *)malloc(sizeof(double) * np);
  c->xm = (double *)malloc(sizeof(double) * F);
  c->xs = (double *)malloc(sizeof(double) * F);
  c->tm = (double *)malloc(sizeof(double) * O);
  c->ts = (double *)malloc(sizeof(double) * O);
  memcpy(c->mlp_p, params, sizeof(double) * np);
  memcpy(c->xm, xmean, sizeof(double) * F);
  memcpy(c->xs, xstd, sizeof(double) * F);
  memcpy(c->tm, tmean, sizeof(double) * O);
  memcpy(c->ts, tstd, sizeof(double) * O);
  c->mlp_H = H; c->mlp_F = F; c->mlp_O = O;
  /* bit 0: bf16 rounding of the network's matmul operands; bit 1: the error
   * check is not run automatically every 20 steps */
  c->mlp_bf16 = bf16;
  c->mlp_on = 1;
  memset(c->flags, 1, (size_t)c->ntiles);
  return 0;
}

int or_set_mlp_flags(or_ctx *c, const uint8_t *flags) {
  memcpy(c->flags, flags, (size_t)c->ntiles);
  return 0;
}

int or_get_mlp_flags(const or_ctx *c, uint8_t *flags, double *emlp, double *egrad) {
  if (flags) memcpy(flags, c->flags, (size_t)c->ntiles);
  if (emlp) memcpy(emlp, c->emlp, sizeof(double) * c->ntiles);
  if (egrad) memcpy(egrad, c->egrad, sizeof(double) * c->ntiles);
  return 0;
}

/* predicted non-equilibrium moments dM_{Q-q} of a low-order state */
static void mlp_predict(const or_ctx *c, const double *fq, const double *gq, double *dM,
                        double *tn) {
  const lat_t *Lq = c->lat[0], *LQ = c->lat[1];
  double feat[64], x[64], y[256];
  mlp_features_lat(Lq, c->cfg.thermal, c->cfg.cv, fq, gq, feat);
  /* standardised features, limited to +-8 standard deviations: a state far
   * outside the training data gets a bounded input instead of an arbitrary one */
  for (int k = 0; k < c->mlp_F; k++) {
    double v = (feat[k] - c->xm[k]) / c->xs[k];
    x[k] = v > 8.0 ? 8.0 : (v < -8.0 ? -8.0 : v);
  }
  mlp_forward_one(c->mlp_p, c->mlp_F, c->mlp_H, c->mlp_O, x, y, c->mlp_bf16 & 1);
  double rho, u[3], T;
  lat_macros(Lq, c->cfg.thermal, c->cfg.cv, fq, gq, &rho, u, &T);
  int k = 0;
  for (int j = 0; j < LQ->Q; j++) {
    int inq = 1, deg = 0;
    for (int a = 0; a < LQ->D; a++) {
      if (LQ->pw[j][a] >= Lq->n) inq = 0;
      deg += LQ->pw[j][a];
    }
    if (inq) continue;
    double t = y[k] * c->ts[k] + c->tm[k];   /* de-standardised normalised target */
    if (tn) tn[k] = t;
    if (dM) dM[k] = rho * pow(T, 0.5 * deg) * t;
    k++;
  }
}

/* Lifting with the learned closure: the completed moments are the equilibrium
 * moments plus the network's prediction of their non-equilibrium part, unless
 * the check tile's error test selected plain Grad lifting. */
static void lift_state(const or_ctx *c, const double *fq, const double *gq, int tile,
                       double *fQ, double *gQ) {
  const lat_t *Lq = c->lat[0], *LQ = c->lat[1];
  const int th = c->cfg.thermal;
  if (c->cfg.lift_mode == 1) {
    lat_lift_hermite(Lq, LQ, th, c->cfg.cv, fq, gq, fQ, gQ);
  } else if (c->cfg.lift_mode == 2 && c->mlp_on && c->flags[tile]) {
    double dM[OR_MAXQ];
    mlp_predict(c, fq, gq, dM, NULL);
    lat_lift_raw(Lq, LQ, th, c->cfg.cv, fq, gq, dM, fQ, gQ);
  } else {
    lat_lift_raw(Lq, LQ, th, c->cfg.cv, fq, gq, NULL, fQ, gQ);
  }
}

int or_lift_cell(const or_ctx *c, const double *fq, const double *gq, int tile,
                 double *fQ, double *gQ) {
  if (c->nlat < 2 || tile < 0 || tile >= c->ntiles) return -1;
  lift_state(c, fq, gq, tile, fQ, gQ);
  return 0;
}

/* The closure's error check against the high-order solution: on high-order
 * cells that border low-order cells, the network predicts the cells' own
 * missing moments from their projected low-order state; per check tile, the
 * network is kept only if its squared error is below that of Grad lifting
 * (which predicts no non-equilibrium part).  Tiles without such cells follow
 * the total over the domain.  Ties, including an exactly equilibrium state
 * where both errors vanish, go to Grad lifting. */
int or_mlp_check(or_ctx *c) {
  if (!c->mlp_on) return -1;
  const int D = c->D, R = c->reach, O = c->mlp_O;
  const lat_t *Lq = c->lat[0], *LQ = c->lat[1];
  memset(c->emlp, 0, sizeof(double) * c->ntiles);
  memset(c->egrad, 0, sizeof(double) * c->ntiles);
  uint8_t *has = (uint8_t *)calloc((size_t)c->ntiles, 1);
  for (int64_t k = 0; k < c->ncell; k++) {
    if (c->order[k] != 1) continue;
    int p[3];
    cell_coords(c, k, p);
    int border = 0;
    for (int dz = (D == 3 ? -R : 0); dz <= (D == 3 ? R : 0) && !border; dz++)
      for (int dy = -R; dy <= R && !border; dy++)
        for (int dx = -R; dx <= R && !border; dx++) {
          int q[3] = {p[0] + dx, p[1] + dy, p[2] + dz}, ok = 1;
          for (int a = 0; a < D; a++) {
            if (q[a] < 0 || q[a] >= c->N[a]) {
              if (c->cfg.bc[2 * a + (q[a] < 0 ? 0 : 1)] != 0) ok = 0;
              q[a] = ((q[a] % c->N[a]) + c->N[a]) % c->N[a];
            }
          }
          if (ok && c->order[cell_index(c, q)] == 0) border = 1;
        }
    if (!border) continue;
    double fQ[OR_MAXQ], gQ[OR_MAXQ], fq[OR_MAXQ], gq[OR_MAXQ], t[OR_MAXQ], tp[OR_MAXQ];
    native_state(c, k, fQ, gQ);
    lat_project(LQ, Lq, c->cfg.thermal, fQ, gQ, fq, gq);
    mlp_targets_lat(Lq, LQ, c->cfg.thermal, c->cfg.cv, fQ, gQ, t);
    mlp_predict(c, fq, gq, NULL, tp);
    int tl = tile_of(c, p);
    for (int o = 0; o < O; o++) {
      c->emlp[tl] += (tp[o] - t[o]) * (tp[o] - t[o]);
      c->egrad[tl] += t[o] * t[o];
    }
    has[tl] = 1;
  }
  double em = 0, eg = 0;
  for (int t = 0; t < c->ntiles; t++) { em += c->emlp[t]; eg += c->egrad[t]; }
  for (int t = 0; t < c->ntiles; t++)
    c->flags[t] = has[t] ? (c->emlp[t] < c->egrad[t]) : (em < eg);
  free(has);
  return 0;
}
