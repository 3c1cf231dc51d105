/*
 * oracle_pond.c -- the semi-Lagrangian step in co-moving reference frames
 * (PonD, Sec. II.C.1), one or two velocity sets, cell by cell.
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Every cell stores its post-collision populations, of its own velocity set,
 * in its own frame lambda = {u, T} (eq. reference), with particle velocities
 * v_i = sqrt(theta) c_i + u, theta = T / T_L, T_L = 1 (eq. vi).  One step at a
 * monitoring cell x of set l:
 *   predictor: lambda_0 = the cell's frame of the previous step;
 *   for n = 0, 1, ...:
 *     each population i is reconstructed at its departure point
 *     x - v_i^{lambda_n} dt by 3-point-per-axis Lagrange interpolation over the
 *     collocation points around the nearest node, every collocation point's
 *     population vector transferred from its own frame lambda_s to lambda_n
 *     first (eqs. reconstructionPond, advectionPond) with the transfer matrix
 *     G = M_{lambda_n}^{-1} M_{lambda_s} (eqs. momf, fll), M_lambda the moment
 *     matrix of eq. momf at that frame's particle velocities;
 *     corrector: rho, u, T of the reconstructed populations (eqs.
 *     correctorfields) define lambda_{n+1};
 *   until lambda stops changing (reading: the largest change of a velocity
 *   component or of T at most 1e-14, at most 60 iterations);
 *   collision in the converged frame, where the equilibria are f^eq = rho W_i
 *   and g^eq = (cv - D/2) T rho W_i (eqs. feqPond, geqPond): BGK, or the
 *   two-relaxation model with the quasi-equilibria of eqs. fqeq, gqeq.
 * With two velocity sets (Sec. III), a collocation point of the other set is
 * first lifted (Sec. III.B) or projected (Sec. III.C) into set l in its own
 * frame, with the moments taken at that frame's particle velocities, then
 * transferred like any other point.  Every `crit_every` steps the Knudsen
 * number of Sec. IV.A.3 of each cell (from its own set in its own frame)
 * selects the set, and a cell whose set changes converts its own state in its
 * own frame.
 * Collocation points outside the domain: periodic faces wrap, zero-gradient
 * faces repeat the edge cell (its populations and frame), fixed-equilibrium
 * faces give the face state's co-moving equilibrium in the face state's frame,
 * and diffuse walls give the wall state's co-moving equilibrium in the wall's
 * frame, with the density that balances the wall-normal particle flux of the
 * adjacent fluid cell.
 */
#include "oracle_internal.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define POND_MAXIT 60
#define POND_TOL 1e-14

struct or_pond {
  or_config cfg;
  int D, N[3], nlat, Q[2], NP[2];
  int64_t ncell;
  lat_t *L[2];
  double dt;
  /* per set, [NP][ncell]: f planes then g planes of the cells of that set,
   * each in its own frame (entries of the other set's cells are unused) */
  double *f[2], *fn[2];
  /* per set, during a step: the cells of the other set converted into this
   * set in their own frames */
  double *fx[2];
  double *fr, *frn;  /* [4][ncell]: u_x, u_y, u_z, T of each cell's frame */
  uint8_t *order;    /* velocity set of each cell */
  long step;
  double it_mean;
  int it_max, bad;
};

/* a frame's particle velocities and (for a target frame) the inverse of its
 * moment matrix (Q x Q, allocated for target frames only) */
typedef struct {
  ld u[3], T;
  ld v[OR_MAXQ][3];
  ld *Minv;
} pframe_t;

static ld ipowl_(ld b, int e) {
  ld r = 1.0L;
  for (int k = 0; k < e; k++) r *= b;
  return r;
}

static void frame_velocities(const lat_t *L, const ld *u, ld T, pframe_t *fr) {
  const ld st = sqrtl(T);
  for (int a = 0; a < 3; a++) fr->u[a] = a < L->D ? u[a] : 0.0L;
  fr->T = T;
  for (int i = 0; i < L->Q; i++)
    for (int a = 0; a < 3; a++) fr->v[i][a] = a < L->D ? st * L->cl[i][a] + fr->u[a] : 0.0L;
}

static int frame_target(const lat_t *L, const ld *u, ld T, pframe_t *fr) {
  frame_velocities(L, u, T, fr);
  const int Q = L->Q;
  ld *M = (ld *)malloc(sizeof(ld) * Q * Q);
  for (int j = 0; j < Q; j++)
    for (int i = 0; i < Q; i++) {
      ld v = 1.0L;
      for (int a = 0; a < L->D; a++) v *= ipowl_(fr->v[i][a], L->pw[j][a]);
      M[j * Q + i] = v;
    }
  int rc = ld_invert(Q, M, fr->Minv);
  free(M);
  return rc;
}

/* out = M_dst^{-1} M_src f: the populations f given in the frame whose
 * particle velocities are src->v, transferred to the frame dst (eq. fll) */
static void transfer(const lat_t *L, const pframe_t *src, const pframe_t *dst, const double *f,
                     ld *out) {
  const int Q = L->Q;
  ld m[OR_MAXQ];
  for (int j = 0; j < Q; j++) {
    ld s = 0.0L;
    for (int i = 0; i < Q; i++) {
      ld v = (ld)f[i];
      for (int a = 0; a < L->D; a++) v *= ipowl_(src->v[i][a], L->pw[j][a]);
      s += v;
    }
    m[j] = s;
  }
  for (int i = 0; i < Q; i++) {
    ld s = 0.0L;
    for (int j = 0; j < Q; j++) s += dst->Minv[i * Q + j] * m[j];
    out[i] = s;
  }
}

static int64_t pcell(const or_pond *c, const int *p) {
  return (int64_t)p[0] + (int64_t)c->N[0] * ((int64_t)p[1] + (int64_t)c->N[1] * p[2]);
}

/* the state of collocation point q (possibly outside the domain) in set l: its
 * f (and g) vector and its frame */
static void point_state(const or_pond *c, int l, const int *qin, double *f, double *g, ld *u, ld *T) {
  const lat_t *L = c->L[l];
  const int Q = c->Q[l];
  int q[3] = {qin[0], qin[1], qin[2]};
  for (int a = 0; a < c->D; a++) {
    if (q[a] >= 0 && q[a] < c->N[a]) continue;
    const int face = 2 * a + (q[a] < 0 ? 0 : 1);
    const int bc = c->cfg.bc[face];
    if (bc == 1) {   /* fixed equilibrium: the face state in its own frame */
      const double *st = c->cfg.bc_state[face];
      const double Tf = c->cfg.thermal ? st[4] : 1.0;
      for (int b = 0; b < 3; b++) u[b] = b < c->D ? (ld)st[1 + b] : 0.0L;
      *T = (ld)Tf;
      for (int i = 0; i < Q; i++) {
        f[i] = st[0] * L->W[i];
        if (c->cfg.thermal) g[i] = (c->cfg.cv - 0.5 * c->D) * Tf * st[0] * L->W[i];
      }
      return;
    }
  }
  /* a diffuse wall (the highest such axis): the wall state's co-moving
   * equilibrium in the wall's frame {u_w, T_w}, scaled by rho_w so that the
   * wall-normal particle flux it sends into the fluid equals the flux arriving
   * from the adjacent fluid cell, both counted in the wall's frame (the
   * adjacent cell's populations transferred there, eq. fll) */
  for (int a = c->D - 1; a >= 0; a--) {
    if (q[a] >= 0 && q[a] < c->N[a]) continue;
    const int side = q[a] < 0 ? 0 : 1, face = 2 * a + side;
    if (c->cfg.bc[face] != 3) continue;
    int qa[3] = {q[0], q[1], q[2]};
    qa[a] = side ? c->N[a] - 1 : 0;
    for (int b = 0; b < c->D; b++) {
      if (qa[b] >= 0 && qa[b] < c->N[b]) continue;
      const int fb = 2 * b + (qa[b] < 0 ? 0 : 1);
      if (c->cfg.bc[fb] == 0) qa[b] = ((qa[b] % c->N[b]) + c->N[b]) % c->N[b];
      else qa[b] = qa[b] < 0 ? 0 : c->N[b] - 1;
    }
    const int64_t ka = pcell(c, qa);
    const int o = c->order[ka];
    const lat_t *Lo = c->L[o];
    const double *ws = c->cfg.bc_state[face];
    const double Tw = c->cfg.thermal ? ws[4] : 1.0;
    const ld sTw = sqrtl((ld)Tw), uwn = (ld)ws[1 + a];
    /* the adjacent cell's populations transferred into the wall's frame */
    pframe_t *src = (pframe_t *)malloc(sizeof(pframe_t)), *dst = (pframe_t *)malloc(sizeof(pframe_t));
    dst->Minv = (ld *)malloc(sizeof(ld) * c->Q[o] * c->Q[o]);
    ld uk[3], uw[3];
    for (int b = 0; b < 3; b++) {
      uk[b] = (ld)c->fr[(int64_t)b * c->ncell + ka];
      uw[b] = b < c->D ? (ld)ws[1 + b] : 0.0L;
    }
    frame_velocities(Lo, uk, (ld)c->fr[(int64_t)3 * c->ncell + ka], src);
    frame_target(Lo, uw, (ld)Tw, dst);
    double fk[OR_MAXQ];
    ld fw[OR_MAXQ];
    for (int i = 0; i < c->Q[o]; i++) fk[i] = c->f[o][(int64_t)i * c->ncell + ka];
    transfer(Lo, src, dst, fk, fw);
    free(dst->Minv); free(src); free(dst);
    ld in = 0.0L, out = 0.0L;
    for (int i = 0; i < c->Q[o]; i++) {
      const ld vw = sTw * Lo->cl[i][a] + uwn;
      if (side ? vw > 0.0L : vw < 0.0L) in += fabsl(vw) * fw[i];
      if (side ? vw < 0.0L : vw > 0.0L) out += fabsl(vw) * Lo->Wl[i];
    }
    const double rw = (double)(in / out);
    for (int b = 0; b < 3; b++) u[b] = b < c->D ? (ld)ws[1 + b] : 0.0L;
    *T = (ld)Tw;
    for (int i = 0; i < Q; i++) {
      f[i] = rw * L->W[i];
      if (c->cfg.thermal) g[i] = (c->cfg.cv - 0.5 * c->D) * Tw * rw * L->W[i];
    }
    return;
  }
  for (int a = 0; a < c->D; a++) {
    if (q[a] >= 0 && q[a] < c->N[a]) continue;
    const int face = 2 * a + (q[a] < 0 ? 0 : 1);
    if (c->cfg.bc[face] == 0) q[a] = ((q[a] % c->N[a]) + c->N[a]) % c->N[a];
    else q[a] = q[a] < 0 ? 0 : c->N[a] - 1;   /* zero gradient */
  }
  const int64_t k = pcell(c, q);
  const double *src = c->order[k] == l ? c->f[l] : c->fx[l];
  for (int i = 0; i < Q; i++) {
    f[i] = src[(int64_t)i * c->ncell + k];
    if (c->cfg.thermal) g[i] = src[(int64_t)(Q + i) * c->ncell + k];
  }
  for (int b = 0; b < 3; b++) u[b] = (ld)c->fr[(int64_t)b * c->ncell + k];
  *T = (ld)c->fr[(int64_t)3 * c->ncell + k];
}

/* one cell's state of set `from`, given in the frame {u, T}, in set `to` in
 * the same frame: lifting (Sec. III.B; the raw completion or its Hermite
 * variant) or projection (Sec. III.C), with the moments at that frame's
 * particle velocities.  Lf: the two sets' lattices, whose frame this sets. */
static int convert_in_frame(const or_pond *c, lat_t **Lf, int from, int to, const double *f,
                            const double *g, const double *u, double T, double *fo, double *go) {
  const int th = c->cfg.thermal;
  if (from == to) {
    memcpy(fo, f, sizeof(double) * c->Q[from]);
    if (th) memcpy(go, g, sizeof(double) * c->Q[from]);
    return 0;
  }
  if (lat_set_frame(Lf[0], u, T) || lat_set_frame(Lf[1], u, T)) return -1;
  if (from < to) {
    if (c->cfg.lift_mode == 1) lat_lift_hermite(Lf[0], Lf[1], th, c->cfg.cv, f, th ? g : NULL, fo, th ? go : NULL);
    else lat_lift_raw(Lf[0], Lf[1], th, c->cfg.cv, f, th ? g : NULL, NULL, fo, th ? go : NULL);
  } else {
    lat_project(Lf[1], Lf[0], th, f, th ? g : NULL, fo, th ? go : NULL);
  }
  return 0;
}

/* cell k's own state converted into set l (its own frame) */
static int cell_in_set(const or_pond *c, lat_t **Lf, int64_t k, int l, double *fo, double *go) {
  const int o = c->order[k], Qo = c->Q[o];
  double f[OR_MAXQ], g[OR_MAXQ], u[3];
  for (int i = 0; i < Qo; i++) {
    f[i] = c->f[o][(int64_t)i * c->ncell + k];
    g[i] = c->cfg.thermal ? c->f[o][(int64_t)(Qo + i) * c->ncell + k] : 0.0;
  }
  for (int a = 0; a < 3; a++) u[a] = c->fr[(int64_t)a * c->ncell + k];
  return convert_in_frame(c, Lf, o, l, f, g, u, c->fr[(int64_t)3 * c->ncell + k], fo, go);
}

static void lats_new(const or_pond *c, lat_t **Lf) {
  Lf[0] = lat_build(c->D, c->cfg.n_low);
  Lf[1] = c->nlat > 1 ? lat_build(c->D, c->cfg.n_high) : lat_build(c->D, c->cfg.n_low);
}

static void lats_free(lat_t **Lf) {
  lat_free(Lf[0]);
  lat_free(Lf[1]);
}

/* the other set's cells in each set, in their own frames */
static int convert_all(or_pond *c) {
  if (c->nlat < 2) return 0;
  int bad = 0;
#pragma omp parallel reduction(| : bad)
  {
    lat_t *Lf[2];
    lats_new(c, Lf);
    double fo[OR_MAXQ], go[OR_MAXQ];
#pragma omp for schedule(dynamic, 64)
    for (int64_t k = 0; k < c->ncell; k++) {
      const int l = 1 - c->order[k];
      if (cell_in_set(c, Lf, k, l, fo, go)) { bad = 1; continue; }
      for (int i = 0; i < c->Q[l]; i++) {
        c->fx[l][(int64_t)i * c->ncell + k] = fo[i];
        if (c->cfg.thermal) c->fx[l][(int64_t)(c->Q[l] + i) * c->ncell + k] = go[i];
      }
    }
    lats_free(Lf);
  }
  return bad ? -4 : 0;
}

static double relax_tau_p(const or_pond *c, double rho, double T) {
  if (c->cfg.tau_mode == 0) return c->cfg.tau;
  double mu_ref = (c->cfg.tau - 0.5) * c->cfg.tau_ref_rho * c->cfg.tau_ref_T * c->dt;
  double mu = mu_ref * pow(T / c->cfg.tau_ref_T, c->cfg.mu_exp);
  return mu / (rho * T * c->dt) + 0.5;
}

#define PSIDE 5   /* collocation points lie within 2 cells: nearest node within 1 */

/* one cell's step; returns the iteration count, or -1 when a departure point
 * leaves the two-cell reach or the state is not finite */
static int pond_cell(const or_pond *c, int64_t k, double *fo, double *go, double *frame_out) {
  const int l = c->order[k];
  const lat_t *L = c->L[l];
  const int D = c->D, Q = c->Q[l], th = c->cfg.thermal;
  int p[3];
  p[0] = (int)(k % c->N[0]);
  p[1] = (int)((k / c->N[0]) % c->N[1]);
  p[2] = (int)(k / ((int64_t)c->N[0] * c->N[1]));
  const int npts = D == 3 ? PSIDE * PSIDE * PSIDE : PSIDE * PSIDE;
  /* the neighbourhood's states, read once */
  double *nf = (double *)malloc(sizeof(double) * npts * OR_MAXQ);
  double *ng = (double *)malloc(sizeof(double) * npts * OR_MAXQ);
  pframe_t *nfr = (pframe_t *)malloc(sizeof(pframe_t) * npts);
  ld *tf = (ld *)malloc(sizeof(ld) * npts * OR_MAXQ);   /* transferred to the current frame */
  ld *tg = (ld *)malloc(sizeof(ld) * npts * OR_MAXQ);
  uint8_t *have = (uint8_t *)malloc(npts);
  pframe_t *tgt = (pframe_t *)malloc(sizeof(pframe_t));
  tgt->Minv = (ld *)malloc(sizeof(ld) * Q * Q);
  for (int s = 0; s < npts; s++) {
    int q[3] = {p[0] + s % PSIDE - 2, p[1] + (s / PSIDE) % PSIDE - 2, D == 3 ? p[2] + s / (PSIDE * PSIDE) - 2 : 0};
    ld u[3], T;
    point_state(c, l, q, nf + (size_t)s * OR_MAXQ, ng + (size_t)s * OR_MAXQ, u, &T);
    frame_velocities(L, u, T, &nfr[s]);
  }
  ld u[3] = {(ld)c->fr[k], (ld)c->fr[c->ncell + k], (ld)c->fr[2 * c->ncell + k]};
  ld T = (ld)c->fr[3 * c->ncell + k];
  double ft[OR_MAXQ], gt[OR_MAXQ], rho = 0.0, Tn = 1.0;
  ld uf[3] = {u[0], u[1], u[2]}, Tfr = T;   /* the frame ft, gt are given in */
  int it, ok = 1;
  for (it = 1; it <= POND_MAXIT; it++) {
    if (frame_target(L, u, T, tgt)) { ok = 0; break; }
    for (int a = 0; a < 3; a++) uf[a] = u[a];
    Tfr = T;
    memset(have, 0, (size_t)npts);
    /* reconstruction at the departure points, in the current frame */
    for (int i = 0; i < Q; i++) {
      ld accf = 0.0L, accg = 0.0L;
      int n0[3] = {0, 0, 0};
      double wgt[3][3] = {{1, 0, 0}, {1, 0, 0}, {1, 0, 0}};
      for (int a = 0; a < D; a++) {
        const double d = -(double)tgt->v[i][a] * c->dt;
        n0[a] = (int)floor(d + 0.5);
        if (n0[a] < -1 || n0[a] > 1) ok = 0;
        or_lagrange3(d - n0[a], wgt[a]);
      }
      if (!ok) break;
      const int nsp = D == 3 ? 27 : 9;
      for (int sidx = 0; sidx < nsp; sidx++) {
        int sv[3] = {sidx % 3 - 1, (sidx / 3) % 3 - 1, D == 3 ? sidx / 9 - 1 : 0};
        ld w = 1.0L;
        int off[3] = {0, 0, 0};
        for (int a = 0; a < D; a++) {
          w *= (ld)wgt[a][sv[a] + 1];
          off[a] = n0[a] + sv[a];
        }
        const int s = (off[0] + 2) + PSIDE * ((off[1] + 2) + PSIDE * (D == 3 ? off[2] + 2 : 0));
        if (!have[s]) {
          transfer(L, &nfr[s], tgt, nf + (size_t)s * OR_MAXQ, tf + (size_t)s * OR_MAXQ);
          if (th) transfer(L, &nfr[s], tgt, ng + (size_t)s * OR_MAXQ, tg + (size_t)s * OR_MAXQ);
          have[s] = 1;
        }
        accf += w * tf[(size_t)s * OR_MAXQ + i];
        if (th) accg += w * tg[(size_t)s * OR_MAXQ + i];
      }
      ft[i] = (double)accf;
      gt[i] = th ? (double)accg : 0.0;
    }
    if (!ok) break;
    /* corrector: density, velocity and temperature in this frame's velocities */
    ld r = 0.0L, j[3] = {0, 0, 0}, e = 0.0L;
    for (int i = 0; i < Q; i++) {
      r += (ld)ft[i];
      ld v2 = 0.0L;
      for (int a = 0; a < D; a++) {
        j[a] += tgt->v[i][a] * (ld)ft[i];
        v2 += tgt->v[i][a] * tgt->v[i][a];
      }
      e += 0.5L * v2 * (ld)ft[i];
      if (th) e += (ld)gt[i];
    }
    ld nu[3] = {0, 0, 0}, nT = 1.0L, u2 = 0.0L;
    for (int a = 0; a < D; a++) {
      nu[a] = j[a] / r;
      u2 += nu[a] * nu[a];
    }
    if (th) nT = (e / r - 0.5L * u2) / (ld)c->cfg.cv;
    if (!(r > 0.0L) || !(nT > 0.0L) || !isfinite((double)r)) { ok = 0; break; }
    ld delta = fabsl(nT - T);
    for (int a = 0; a < D; a++) delta = fmaxl(delta, fabsl(nu[a] - u[a]));
    rho = (double)r;
    Tn = (double)nT;
    if (delta <= POND_TOL) break;
    for (int a = 0; a < 3; a++) u[a] = nu[a];
    T = nT;
  }
  free(nf); free(ng); free(nfr); free(tf); free(tg); free(have);
  free(tgt->Minv);
  free(tgt);
  if (!ok) return -1;
  /* collision in the converged frame (the last frame the populations were
   * reconstructed in), where f^eq = rho W_i, g^eq = (cv - D/2) T rho W_i */
  const double Tf = (double)Tfr;
  const double tl = relax_tau_p(c, rho, Tn);
  const double om = 1.0 / tl;
  const int two = c->cfg.tau2 > 0.0 && c->cfg.tau2 != c->cfg.tau;
  const double om2 = two ? 1.0 / (0.5 + (tl - 0.5) * (c->cfg.tau2 - 0.5) / (c->cfg.tau - 0.5)) : om;
  const double gq = th ? (c->cfg.cv - 0.5 * D) * Tf : 0.0;
  /* quasi-equilibria (eqs. fqeq, gqeq) in the co-moving frame: v - u = sqrt(T) c,
   * Qbar = T^{3/2} sum c c c (f - f^eq), qbar = T^{1/2} sum c (g - g^eq);
   * f* = f^eq + W T^{-3/2}/6 Qbar : (c c c - sym(c 1)), g* = g^eq + W T^{-1/2} qbar . c */
  double Qb[3][3][3] = {{{0}}}, qb[3] = {0, 0, 0};
  if (two) {
    const double s3 = pow(Tf, 1.5), s1 = sqrt(Tf);
    for (int i = 0; i < Q; i++) {
      const double nfq = ft[i] - rho * L->W[i];
      const double ngq = th ? gt[i] - gq * rho * L->W[i] : 0.0;
      for (int a = 0; a < D; a++) {
        qb[a] += s1 * L->c[i][a] * ngq;
        for (int b = 0; b < D; b++)
          for (int cc = 0; cc < D; cc++) Qb[a][b][cc] += s3 * L->c[i][a] * L->c[i][b] * L->c[i][cc] * nfq;
      }
    }
  }
  for (int i = 0; i < Q; i++) {
    const double feq = rho * L->W[i];
    fo[i] = ft[i] + om * (feq - ft[i]);
    if (two) {
      double s = 0.0;
      for (int a = 0; a < D; a++)
        for (int b = 0; b < D; b++)
          for (int cc = 0; cc < D; cc++) {
            const double ca = L->c[i][a], cb = L->c[i][b], ccc = L->c[i][cc];
            const double h3 = ca * cb * ccc - (b == cc ? ca : 0.0) - (a == cc ? cb : 0.0) - (a == b ? ccc : 0.0);
            s += Qb[a][b][cc] * h3;
          }
      fo[i] += (om - om2) * L->W[i] * s / (6.0 * pow(Tf, 1.5));
    }
    if (th) {
      const double geq = gq * rho * L->W[i];
      go[i] = gt[i] + om * (geq - gt[i]);
      if (two) {
        double s = 0.0;
        for (int a = 0; a < D; a++) s += qb[a] * L->c[i][a];
        go[i] += (om - om2) * L->W[i] * s / sqrt(Tf);
      }
    }
  }
  for (int a = 0; a < 3; a++) frame_out[a] = a < D ? (double)uf[a] : 0.0;
  frame_out[3] = Tf;
  return it > POND_MAXIT ? POND_MAXIT : it;
}

/* ------------------------------------------------------------------------ */

int or_pond_create(const or_config *cfg, or_pond **out) {
  if (!cfg || !out) return -1;
  if (cfg->dim != 2 && cfg->dim != 3) return -1;
  if (cfg->nx < 1 || cfg->ny < 1 || (cfg->dim == 3 && cfg->nz < 1)) return -1;
  if (cfg->n_low < 2 || (cfg->n_high != 0 && cfg->n_high <= cfg->n_low)) return -1;
  if (cfg->n_high != 0 && (cfg->lift_mode != 0 && cfg->lift_mode != 1)) return -1;
  if (cfg->crit_kind != 0 && cfg->crit_kind != 3) return -1;   /* fixed sets or the Knudsen number */
  if (cfg->tau <= 0.5 || (cfg->tau2 > 0.0 && cfg->tau2 <= 0.5)) return -1;
  if (cfg->store != 0) return -1;                       /* FP64 populations */
  for (int f = 0; f < 2 * cfg->dim; f++) {
    if (cfg->bc[f] < 0 || cfg->bc[f] > 3) return -1;
    if (cfg->bc[f] == 3) {   /* diffuse walls: not on x faces, lower faces periodic or zero-gradient */
      if (f < 2) return -1;
      for (int g = 0; g < 2 * (f / 2); g++)
        if (cfg->bc[g] != 0 && cfg->bc[g] != 2) return -1;
    }
  }
  or_pond *c = (or_pond *)calloc(1, sizeof(or_pond));
  c->cfg = *cfg;
  c->D = cfg->dim;
  c->N[0] = cfg->nx;
  c->N[1] = cfg->ny;
  c->N[2] = cfg->dim == 3 ? cfg->nz : 1;
  c->ncell = (int64_t)c->N[0] * c->N[1] * c->N[2];
  c->nlat = cfg->n_high ? 2 : 1;
  /* dt = CFL / the largest lattice speed of the sets (the lattice-frame rule;
   * a departure point beyond the two-cell reach in some frame is reported by
   * the step) */
  double vmax = 0.0;
  for (int l = 0; l < c->nlat; l++) {
    c->L[l] = lat_build(c->D, l ? cfg->n_high : cfg->n_low);
    if (!c->L[l]) { or_pond_destroy(c); return -2; }
    c->Q[l] = c->L[l]->Q;
    c->NP[l] = cfg->thermal ? 2 * c->Q[l] : c->Q[l];
    for (int a = 0; a < c->D; a++)
      if (lat_vmax(c->L[l], a) > vmax) vmax = lat_vmax(c->L[l], a);
    c->f[l] = (double *)calloc((size_t)c->NP[l] * c->ncell, sizeof(double));
    c->fn[l] = (double *)calloc((size_t)c->NP[l] * c->ncell, sizeof(double));
    if (c->nlat > 1) c->fx[l] = (double *)calloc((size_t)c->NP[l] * c->ncell, sizeof(double));
  }
  c->dt = cfg->cfl / vmax;
  c->fr = (double *)calloc((size_t)4 * c->ncell, sizeof(double));
  c->frn = (double *)calloc((size_t)4 * c->ncell, sizeof(double));
  c->order = (uint8_t *)calloc((size_t)c->ncell, 1);
  *out = c;
  return 0;
}

void or_pond_destroy(or_pond *c) {
  if (!c) return;
  for (int l = 0; l < 2; l++) {
    lat_free(c->L[l]);
    free(c->f[l]); free(c->fn[l]); free(c->fx[l]);
  }
  free(c->fr); free(c->frn); free(c->order);
  free(c);
}

double or_pond_dt(const or_pond *c) { return c->dt; }

/* every cell at the co-moving equilibrium of (rho, u, T) in its own frame,
 * in each set (an equilibrium is the same state in both) */
int or_pond_init(or_pond *c, const double *rho, const double *u, const double *T) {
  const int th = c->cfg.thermal;
  for (int64_t k = 0; k < c->ncell; k++) {
    const double Tk = th ? T[k] : 1.0;
    for (int l = 0; l < c->nlat; l++)
      for (int i = 0; i < c->Q[l]; i++) {
        c->f[l][(int64_t)i * c->ncell + k] = rho[k] * c->L[l]->W[i];
        if (th) c->f[l][(int64_t)(c->Q[l] + i) * c->ncell + k] = (c->cfg.cv - 0.5 * c->D) * Tk * rho[k] * c->L[l]->W[i];
      }
    for (int a = 0; a < 3; a++) c->fr[(int64_t)a * c->ncell + k] = a < c->D ? u[(int64_t)a * c->ncell + k] : 0.0;
    c->fr[(int64_t)3 * c->ncell + k] = Tk;
  }
  c->step = 0;
  return 0;
}

/* the velocity set of each cell; convert: cells whose set changes lift or
 * project their own state in their own frame */
int or_pond_set_mask(or_pond *c, const uint8_t *mask, int convert) {
  for (int64_t k = 0; k < c->ncell; k++)
    if (mask[k] > 1 || (mask[k] && c->nlat < 2)) return -1;
  int bad = 0;
  if (convert && c->nlat > 1) {
#pragma omp parallel reduction(| : bad)
    {
      lat_t *Lf[2];
      lats_new(c, Lf);
      double fo[OR_MAXQ], go[OR_MAXQ];
#pragma omp for schedule(dynamic, 64)
      for (int64_t k = 0; k < c->ncell; k++) {
        const int to = mask[k];
        if (to == c->order[k]) continue;
        if (cell_in_set(c, Lf, k, to, fo, go)) { bad = 1; continue; }
        for (int i = 0; i < c->Q[to]; i++) {
          c->f[to][(int64_t)i * c->ncell + k] = fo[i];
          if (c->cfg.thermal) c->f[to][(int64_t)(c->Q[to] + i) * c->ncell + k] = go[i];
        }
      }
      lats_free(Lf);
    }
  }
  memcpy(c->order, mask, (size_t)c->ncell);
  return bad ? -4 : 0;
}

int or_pond_get_mask(const or_pond *c, uint8_t *out) {
  memcpy(out, c->order, (size_t)c->ncell);
  return 0;
}

/* rho, u, T of cell k from its own populations in its own frame */
static void cell_macros(const or_pond *c, int64_t k, ld *rho, ld *uo, ld *To) {
  const int l = c->order[k];
  const lat_t *L = c->L[l];
  const ld Tf = (ld)c->fr[3 * c->ncell + k], st = sqrtl(Tf);
  ld r = 0, j[3] = {0, 0, 0}, e = 0;
  for (int i = 0; i < c->Q[l]; i++) {
    const ld f = (ld)c->f[l][(int64_t)i * c->ncell + k];
    ld v2 = 0;
    r += f;
    for (int a = 0; a < c->D; a++) {
      const ld v = st * L->cl[i][a] + (ld)c->fr[(int64_t)a * c->ncell + k];
      j[a] += v * f;
      v2 += v * v;
    }
    e += 0.5L * v2 * f;
    if (c->cfg.thermal) e += (ld)c->f[l][(int64_t)(c->Q[l] + i) * c->ncell + k];
  }
  ld u2 = 0;
  for (int a = 0; a < 3; a++) {
    uo[a] = a < c->D ? j[a] / r : 0.0L;
    u2 += uo[a] * uo[a];
  }
  *rho = r;
  *To = c->cfg.thermal ? (e / r - 0.5L * u2) / (ld)c->cfg.cv : 1.0L;
}

/* Knudsen-number criterion (Sec. IV.A.3): Kn = lambda |grad rho| / rho with the
 * hard-sphere mean free path lambda = 16/(5 sqrt(2 pi gamma)) mu a / p, a the
 * sound speed sqrt(gamma T), p = rho T, mu = (tau - 1/2) rho T dt at the local
 * relaxation time; central differences of the cell densities, one-sided over
 * one cell at a face that is not periodic.  Sets with Kn > crit_thr are the
 * high-order set. */
static void pond_criterion(const or_pond *c, uint8_t *newmask) {
  const int64_t n = c->ncell;
  double *rho = (double *)malloc((size_t)n * sizeof(double));
  double *lam = (double *)malloc((size_t)n * sizeof(double));
  const double gam = (c->cfg.cv + 1.0) / c->cfg.cv;
  for (int64_t k = 0; k < n; k++) {
    ld r, u[3], T;
    cell_macros(c, k, &r, u, &T);
    const double rd = (double)r, Td = (double)T;
    const double mu = (relax_tau_p(c, rd, Td) - 0.5) * rd * Td * c->dt;
    rho[k] = rd;
    lam[k] = 16.0 / (5.0 * sqrt(2.0 * acos(-1.0) * gam)) * mu * sqrt(gam * Td) / (rd * Td);
  }
  for (int64_t k = 0; k < n; k++) {
    const int p[3] = {(int)(k % c->N[0]), (int)((k / c->N[0]) % c->N[1]), (int)(k / ((int64_t)c->N[0] * c->N[1]))};
    double g2 = 0.0;
    for (int a = 0; a < c->D; a++) {
      if (c->N[a] < 2) continue;
      const int periodic = c->cfg.bc[2 * a] == 0 && c->cfg.bc[2 * a + 1] == 0;
      int lo[3] = {p[0], p[1], p[2]}, hi[3] = {p[0], p[1], p[2]};
      lo[a] = p[a] - 1;
      hi[a] = p[a] + 1;
      if (periodic) {
        lo[a] = (lo[a] + c->N[a]) % c->N[a];
        hi[a] = hi[a] % c->N[a];
      } else {
        if (lo[a] < 0) lo[a] = 0;
        if (hi[a] >= c->N[a]) hi[a] = c->N[a] - 1;
      }
      const double dist = periodic ? 2.0 : (double)(hi[a] - lo[a]);
      const double d = (rho[pcell(c, hi)] - rho[pcell(c, lo)]) / dist;
      g2 += d * d;
    }
    newmask[k] = lam[k] * sqrt(g2) / rho[k] > c->cfg.crit_thr ? 1 : 0;
  }
  free(rho);
  free(lam);
}

int or_pond_step(or_pond *c, int nsteps) {
  for (int s = 0; s < nsteps; s++) {
    if (c->nlat > 1 && c->cfg.crit_kind == 3 && c->cfg.crit_every > 0 && c->step % c->cfg.crit_every == 0) {
      uint8_t *nm = (uint8_t *)malloc((size_t)c->ncell), *dm = (uint8_t *)malloc((size_t)c->ncell);
      pond_criterion(c, nm);
      or_dilate_mask(&c->cfg, nm, dm);
      const int rc = or_pond_set_mask(c, dm, 1);
      free(nm);
      free(dm);
      if (rc) return rc;
    }
    if (convert_all(c)) return -4;
    int bad = 0, itmax = 0;
    double itsum = 0.0;
#pragma omp parallel reduction(| : bad) reduction(max : itmax) reduction(+ : itsum)
    {
      double fo[OR_MAXQ], go[OR_MAXQ], frm[4];
#pragma omp for schedule(dynamic, 16)
      for (int64_t k = 0; k < c->ncell; k++) {
        const int l = c->order[k];
        const int it = pond_cell(c, k, fo, go, frm);
        if (it < 0) { bad = 1; continue; }
        if (it > itmax) itmax = it;
        itsum += it;
        for (int i = 0; i < c->Q[l]; i++) {
          c->fn[l][(int64_t)i * c->ncell + k] = fo[i];
          if (c->cfg.thermal) c->fn[l][(int64_t)(c->Q[l] + i) * c->ncell + k] = go[i];
        }
        for (int a = 0; a < 4; a++) c->frn[(int64_t)a * c->ncell + k] = frm[a];
      }
    }
    if (bad) return -4;
    for (int l = 0; l < c->nlat; l++) {
      double *t = c->f[l]; c->f[l] = c->fn[l]; c->fn[l] = t;
    }
    double *t = c->fr; c->fr = c->frn; c->frn = t;
    c->it_mean = itsum / (double)c->ncell;
    c->it_max = itmax;
    c->step++;
  }
  return 0;
}

int or_pond_iterations(const or_pond *c, double *mean, int *max) {
  if (mean) *mean = c->it_mean;
  if (max) *max = c->it_max;
  return 0;
}

/* populations of set `which` at every cell, in each cell's own frame: native
 * where the cell uses that set, its state lifted / projected elsewhere:
 * [Q][ncell] (fg = 1: g) */
int or_pond_get_pops(const or_pond *c, int which, int fg, double *out) {
  if (which < 0 || which >= c->nlat || (fg && !c->cfg.thermal)) return -1;
  const int Q = c->Q[which];
  int bad = 0;
#pragma omp parallel reduction(| : bad)
  {
    lat_t *Lf[2];
    lats_new(c, Lf);
    double fo[OR_MAXQ], go[OR_MAXQ];
#pragma omp for schedule(dynamic, 64)
    for (int64_t k = 0; k < c->ncell; k++) {
      if (cell_in_set(c, Lf, k, which, fo, go)) { bad = 1; continue; }
      for (int i = 0; i < Q; i++) out[(int64_t)i * c->ncell + k] = fg ? go[i] : fo[i];
    }
    lats_free(Lf);
  }
  return bad ? -4 : 0;
}

int or_pond_get_frames(const or_pond *c, double *out) {
  memcpy(out, c->fr, sizeof(double) * 4 * c->ncell);
  return 0;
}

/* rho, u, T of every cell from its populations in its own frame */
int or_pond_macros(const or_pond *c, double *rho, double *u, double *T) {
  for (int64_t k = 0; k < c->ncell; k++) {
    ld r, uu[3], t;
    cell_macros(c, k, &r, uu, &t);
    if (rho) rho[k] = (double)r;
    if (u)
      for (int a = 0; a < c->D; a++) u[(int64_t)a * c->ncell + k] = (double)uu[a];
    if (T) T[k] = (double)t;
  }
  return 0;
}

/* G_{src}^{dst} f for one population vector (frames as {u_x, u_y, u_z, T}) */
int or_pond_transfer(int dim, int n, const double *src, const double *dst, const double *f,
                     double *out) {
  lat_t *L = lat_build(dim, n);
  if (!L) return -1;
  pframe_t *s = (pframe_t *)malloc(sizeof(pframe_t)), *d = (pframe_t *)malloc(sizeof(pframe_t));
  d->Minv = (ld *)malloc(sizeof(ld) * L->Q * L->Q);
  ld us[3] = {src[0], src[1], src[2]}, ud[3] = {dst[0], dst[1], dst[2]};
  frame_velocities(L, us, (ld)src[3], s);
  int rc = frame_target(L, ud, (ld)dst[3], d);
  ld o[OR_MAXQ];
  if (!rc) {
    transfer(L, s, d, f, o);
    for (int i = 0; i < L->Q; i++) out[i] = (double)o[i];
  }
  free(d->Minv);
  free(s); free(d);
  lat_free(L);
  return rc ? -2 : 0;
}
