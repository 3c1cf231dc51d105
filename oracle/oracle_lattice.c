/*
 * oracle_lattice.c -- velocity sets, moment matrices, lattice equilibrium,
 * lifting and projection, written directly from the paper's definitions.
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 */
#include "oracle_internal.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* Probabilists' Hermite polynomial He_n(x) by the three-term recurrence
 * He_{k+1} = x He_k - k He_{k-1}. */
static ld hermite(int n, ld x) {
  if (n == 0) return 1.0L;
  ld h0 = 1.0L, h1 = x;
  for (int k = 1; k < n; k++) {
    ld h2 = x * h1 - (ld)k * h0;
    h0 = h1;
    h1 = h2;
  }
  return h1;
}

/* Gauss-Hermite rule with weight exp(-c^2/2)/sqrt(2 pi) (lattice temperature 1):
 * nodes are the roots of He_n (Sec. II.A, Tab. I), located by a sign-change scan,
 * bisection and Newton polishing; weights w_k = n! / (n^2 He_{n-1}(x_k)^2). */
int gh_rule_ld(int n, ld *x, ld *w) {
  if (n < 1 || n > OR_MAXN) return -1;
  ld lim = 2.0L * sqrtl((ld)n) + 2.0L;
  int found = 0;
  const int steps = 200000;
  ld prev_x = -lim, prev_v = hermite(n, prev_x);
  for (int s = 1; s <= steps && found < n; s++) {
    ld cx = -lim + 2.0L * lim * (ld)s / (ld)steps;
    ld cv = hermite(n, cx);
    if (cv == 0.0L) {
      x[found++] = cx;
    } else if ((prev_v < 0) != (cv < 0) && prev_v != 0.0L) {
      ld lo = prev_x, hi = cx, vlo = prev_v;
      for (int it = 0; it < 200; it++) {
        ld mid = 0.5L * (lo + hi);
        ld vm = hermite(n, mid);
        if ((vm < 0) == (vlo < 0)) { lo = mid; vlo = vm; } else { hi = mid; }
      }
      ld r = 0.5L * (lo + hi);
      for (int it = 0; it < 5; it++) {  /* Newton: He_n' = n He_{n-1} */
        ld d = (ld)n * hermite(n - 1, r);
        if (d == 0.0L) break;
        r -= hermite(n, r) / d;
      }
      x[found++] = r;
    }
    prev_x = cx;
    prev_v = cv;
  }
  if (found != n) return -2;
  ld fact = 1.0L;
  for (int k = 2; k <= n; k++) fact *= (ld)k;
  for (int k = 0; k < n; k++) {
    ld h = hermite(n - 1, x[k]);
    w[k] = fact / ((ld)n * (ld)n * h * h);
  }
  /* an odd rule has an exact zero node */
  if (n % 2 == 1) x[n / 2] = 0.0L;
  return 0;
}

int or_gh_rule(int n, double *x, double *w) {
  ld xl[OR_MAXN], wl[OR_MAXN];
  int rc = gh_rule_ld(n, xl, wl);
  if (rc) return rc;
  for (int k = 0; k < n; k++) { x[k] = (double)xl[k]; w[k] = (double)wl[k]; }
  return 0;
}

/* Gauss-Jordan inverse with partial pivoting in long double. */
static int invert_ld(int n, const ld *A, ld *Ainv) {
  ld *a = (ld *)malloc(sizeof(ld) * (size_t)n * 2 * n);
  if (!a) return -2;
  for (int r = 0; r < n; r++)
    for (int c = 0; c < 2 * n; c++)
      a[r * 2 * n + c] = c < n ? A[r * n + c] : (c - n == r ? 1.0L : 0.0L);
  for (int col = 0; col < n; col++) {
    int piv = col;
    for (int r = col + 1; r < n; r++)
      if (fabsl(a[r * 2 * n + col]) > fabsl(a[piv * 2 * n + col])) piv = r;
    if (a[piv * 2 * n + col] == 0.0L) { free(a); return -3; }
    if (piv != col)
      for (int c = 0; c < 2 * n; c++) {
        ld t = a[col * 2 * n + c];
        a[col * 2 * n + c] = a[piv * 2 * n + c];
        a[piv * 2 * n + c] = t;
      }
    ld d = a[col * 2 * n + col];
    for (int c = 0; c < 2 * n; c++) a[col * 2 * n + c] /= d;
    for (int r = 0; r < n; r++) {
      if (r == col) continue;
      ld fct = a[r * 2 * n + col];
      if (fct == 0.0L) continue;
      for (int c = 0; c < 2 * n; c++) a[r * 2 * n + c] -= fct * a[col * 2 * n + c];
    }
  }
  for (int r = 0; r < n; r++)
    for (int c = 0; c < n; c++) Ainv[r * n + c] = a[r * 2 * n + n + c];
  free(a);
  return 0;
}

int ld_invert(int n, const ld *A, ld *Ainv) { return invert_ld(n, A, Ainv); }

static ld ipow_ld(ld b, int e) {
  ld r = 1.0L;
  for (int k = 0; k < e; k++) r *= b;
  return r;
}

/* Tensor-product lattice D<dim>Q<n^dim> (eqs. ci, wi), its moment matrix
 * M[j][i] = prod_a c_ia^{p_a(j)} with powers p_a(j) < n (eq. momf; the moment
 * index j uses the same base-n digits as the population index) and inverse. */
lat_t *lat_build(int dim, int n) {
  if (dim < 2 || dim > 3 || n < 2 || n > OR_MAXN) return NULL;
  int Q = 1;
  for (int a = 0; a < dim; a++) Q *= n;
  if (Q > OR_MAXQ) return NULL;
  lat_t *L = (lat_t *)calloc(1, sizeof(lat_t));
  if (!L) return NULL;
  L->D = dim; L->n = n; L->Q = Q;
  if (gh_rule_ld(n, L->x, L->w)) { free(L); return NULL; }
  for (int i = 0; i < Q; i++) {
    int r = i;
    ld W = 1.0L;
    for (int a = 0; a < dim; a++) {
      int d = r % n; r /= n;
      L->pw[i][a] = d;
      L->cl[i][a] = L->x[d];
      L->c[i][a] = (double)L->x[d];
      W *= L->w[d];
    }
    L->Wl[i] = W;
    L->W[i] = (double)W;
  }
  L->M = (ld *)malloc(sizeof(ld) * Q * Q);
  L->Minv = (ld *)malloc(sizeof(ld) * Q * Q);
  for (int j = 0; j < Q; j++)
    for (int i = 0; i < Q; i++) {
      ld v = 1.0L;
      for (int a = 0; a < dim; a++) v *= ipow_ld(L->cl[i][a], L->pw[j][a]);
      L->M[j * Q + i] = v;
    }
  if (invert_ld(Q, L->M, L->Minv)) { lat_free(L); return NULL; }
  L->Mf = (ld *)malloc(sizeof(ld) * Q * Q);
  L->Mfinv = (ld *)malloc(sizeof(ld) * Q * Q);
  const double zero[3] = {0.0, 0.0, 0.0};
  if (lat_set_frame(L, zero, 1.0)) { lat_free(L); return NULL; }
  return L;
}

void lat_free(lat_t *L) {
  if (!L) return;
  free(L->M);
  free(L->Minv);
  free(L->Mf);
  free(L->Mfinv);
  free(L);
}

/* The run's reference frame lambda_ref = {u_ref, T_ref} (eq. veli with R = 1,
 * T_L = 1): particle velocities v_i = sqrt(T_ref) c_i + u_ref, and the moment
 * matrix of eq. momf evaluated at them, M_f[j][i] = prod_a v_ia^{p_a(j)}, with
 * its inverse.  The lattice frame is u_ref = 0, T_ref = 1. */
int lat_set_frame(lat_t *L, const double *u_ref, double T_ref) {
  if (!(T_ref > 0.0)) return -1;
  const int Q = L->Q, D = L->D;
  ld st = sqrtl((ld)T_ref);
  L->Tr = (ld)T_ref;
  for (int a = 0; a < 3; a++) L->ur[a] = a < D ? (ld)u_ref[a] : 0.0L;
  for (int i = 0; i < Q; i++)
    for (int a = 0; a < 3; a++) {
      L->vl[i][a] = a < D ? st * L->cl[i][a] + L->ur[a] : 0.0L;
      L->v[i][a] = (double)L->vl[i][a];
    }
  for (int j = 0; j < Q; j++)
    for (int i = 0; i < Q; i++) {
      ld v = 1.0L;
      for (int a = 0; a < D; a++) v *= ipow_ld(L->vl[i][a], L->pw[j][a]);
      L->Mf[j * Q + i] = v;
    }
  return invert_ld(Q, L->Mf, L->Mfinv);
}

int lat_frame_trivial(const lat_t *L) {
  return L->Tr == 1.0L && L->ur[0] == 0.0L && L->ur[1] == 0.0L && L->ur[2] == 0.0L;
}

/* largest particle speed along one axis */
double lat_vmax(const lat_t *L, int axis) {
  double m = 0;
  for (int i = 0; i < L->Q; i++) if (fabs(L->v[i][axis]) > m) m = fabs(L->v[i][axis]);
  return m;
}

/* Equilibrium in the run's frame, f^ref = M_ref^{-1} M_{u,theta} (rho W)
 * (eqs. fll, feqL, feqL0 with the target frame lambda_ref): the moments of the
 * co-moving equilibrium rho W_i evaluated with the particle velocities
 * sqrt(theta) c_i + u (eqs. vi, momf), mapped to the run's frame by the inverse
 * of its moment matrix.  In the lattice frame this is f^L. */
void lat_feq(const lat_t *L, double rho, const double *u, double theta, double *out) {
  ld co[OR_MAXQ];
  for (int i = 0; i < L->Q; i++) co[i] = (ld)rho * L->Wl[i];
  lat_from_comoving(L, u, theta, co, out);
}

/* Transfer of a population vector given in the co-moving frame {u, theta}
 * (particle velocities sqrt(theta) c_i + u) to the run's frame:
 * out = M_ref^{-1} M_{u,theta} co (eqs. fll, momf). */
void lat_from_comoving(const lat_t *L, const double *u, double theta, const ld *co, double *out) {
  const int Q = L->Q, D = L->D;
  ld st = sqrtl((ld)theta);
  ld mom[OR_MAXQ];
  ld vel[OR_MAXQ][3];
  for (int i = 0; i < Q; i++)
    for (int a = 0; a < D; a++) vel[i][a] = st * L->cl[i][a] + (ld)u[a];
  for (int j = 0; j < Q; j++) {
    ld s = 0.0L;
    for (int i = 0; i < Q; i++) {
      ld v = co[i];
      for (int a = 0; a < D; a++) v *= ipow_ld(vel[i][a], L->pw[j][a]);
      s += v;
    }
    mom[j] = s;
  }
  for (int i = 0; i < Q; i++) {
    ld s = 0.0L;
    for (int j = 0; j < Q; j++) s += L->Mfinv[i * Q + j] * mom[j];
    out[i] = (double)s;
  }
}

/* Quasi-equilibria of the two-relaxation model (Sec. II.B, eqs. fqeq, gqeq),
 * in the run's frame (the quasi-equilibrium counterpart of eq. feqL).
 *   Qbar_abc = sum_i (v_i - u)_a (v_i - u)_b (v_i - u)_c (f_i - f^eq_i),
 *   qbar_a   = sum_i (v_i - u)_a (g_i - g^eq_i),
 * with the particle velocities v of the run's frame; in the co-moving frame
 * {u, T} (theta = T, R = T_L = 1, velocities sqrt(theta) c + u)
 *   f*_i = rho W_i + W_i Qbar : (theta^{3/2} c c c - T theta^{1/2} sym(c (x) 1)) / (6 T^3),
 *   g*_i = (cv - D/2) T rho W_i + W_i theta^{1/2} qbar . c / T,
 * sym(c (x) 1)_abc = c_a d_bc + c_b d_ac + c_c d_ab (the three placements, so
 * that the bracket is the third Hermite tensor and f* keeps the third central
 * moment Qbar); both are transferred to the run's frame.  g may be NULL when
 * athermal (then gstar is untouched). */
void lat_qeq(const lat_t *L, int thermal, double cv, double rho, const double *u, double T,
             const double *f, const double *g, const double *feq, const double *geq,
             double *fstar, double *gstar) {
  const int Q = L->Q, D = L->D;
  ld Qb[3][3][3] = {{{0}}}, qb[3] = {0, 0, 0};
  for (int i = 0; i < Q; i++) {
    ld d[3];
    for (int a = 0; a < D; a++) d[a] = L->vl[i][a] - (ld)u[a];
    const ld nf = (ld)f[i] - (ld)feq[i];
    for (int a = 0; a < D; a++)
      for (int b = 0; b < D; b++)
        for (int c = 0; c < D; c++) Qb[a][b][c] += d[a] * d[b] * d[c] * nf;
    if (thermal)
      for (int a = 0; a < D; a++) qb[a] += d[a] * ((ld)g[i] - (ld)geq[i]);
  }
  const ld th = (ld)T, Tl = (ld)T;
  ld cof[OR_MAXQ], cog[OR_MAXQ];
  for (int i = 0; i < Q; i++) {
    const ld *c = L->cl[i];
    ld s = 0.0L;
    for (int a = 0; a < D; a++)
      for (int b = 0; b < D; b++)
        for (int cc = 0; cc < D; cc++) {
          const ld ccc = c[a] * c[b] * c[cc];
          const ld sym = (b == cc ? c[a] : 0.0L) + (a == cc ? c[b] : 0.0L) + (a == b ? c[cc] : 0.0L);
          s += Qb[a][b][cc] * (powl(th, 1.5L) * ccc - Tl * sqrtl(th) * sym);
        }
    cof[i] = (ld)rho * L->Wl[i] + L->Wl[i] * s / (6.0L * Tl * Tl * Tl);
    if (thermal) {
      ld qc = 0.0L;
      for (int a = 0; a < D; a++) qc += qb[a] * c[a];
      cog[i] = ((ld)cv - 0.5L * D) * Tl * (ld)rho * L->Wl[i] + L->Wl[i] * sqrtl(th) * qc / Tl;
    }
  }
  lat_from_comoving(L, u, T, cof, fstar);
  if (thermal) lat_from_comoving(L, u, T, cog, gstar);
}

/* Raw lattice moments m_j = sum_i f_i prod_a c_ia^{p_a(j)} for every j of the
 * lattice's own moment set (eq. momf in the lattice frame). */
void lat_moments(const lat_t *L, const double *f, ld *m) {
  const int Q = L->Q;
  for (int j = 0; j < Q; j++) {
    ld s = 0.0L;
    for (int i = 0; i < Q; i++) s += L->M[j * Q + i] * (ld)f[i];
    m[j] = s;
  }
}

/* raw moment with powers p of populations f of lattice L, taken with the
 * particle velocities of the run's frame (eq. momf) */
static ld moment_pows(const lat_t *L, const double *f, const int *p) {
  ld s = 0.0L;
  for (int i = 0; i < L->Q; i++) {
    ld v = (ld)f[i];
    for (int a = 0; a < L->D; a++) v *= ipow_ld(L->vl[i][a], p[a]);
    s += v;
  }
  return s;
}

/* Density, velocity and temperature of one cell (conservation laws of Sec.
 * II.B): rho = sum f, rho u = sum v f, rho E = sum |v|^2/2 f + sum g with the
 * particle velocities v of the run's frame, and the ideal-gas energy
 * rho E = cv rho T + rho u^2/2 (eq. E).  Athermal: T = T_L = 1. */
void lat_macros(const lat_t *L, int thermal, double cv, const double *f, const double *g,
                double *rho, double *u, double *T) {
  ld r = 0.0L, j[3] = {0, 0, 0}, e = 0.0L;
  for (int i = 0; i < L->Q; i++) {
    ld fi = (ld)f[i];
    r += fi;
    ld c2 = 0.0L;
    for (int a = 0; a < L->D; a++) {
      j[a] += L->vl[i][a] * fi;
      c2 += L->vl[i][a] * L->vl[i][a];
    }
    e += 0.5L * c2 * fi;
    if (thermal) e += (ld)g[i];
  }
  *rho = (double)r;
  ld u2 = 0.0L;
  for (int a = 0; a < L->D; a++) {
    u[a] = (double)(j[a] / r);
    u2 += (j[a] / r) * (j[a] / r);
  }
  for (int a = L->D; a < 3; a++) u[a] = 0.0;
  if (thermal)
    *T = (double)((e - 0.5L * r * u2) / ((ld)cv * r));
  else
    *T = 1.0;
}

/* g^L = (cv - D/2) T f^L (eq. geqL, R = 1). */
void lat_geq_from_feq(const lat_t *L, double cv, double T, const double *feq, double *geq) {
  double s = (cv - 0.5 * L->D) * T;
  for (int i = 0; i < L->Q; i++) geq[i] = s * feq[i];
}

/* Lifting f_q -> f_Q (Sec. III.B, App. C): the moments of the low-order set are
 * kept, m_q; the moments the low-order set cannot hold are taken from the
 * high-order lattice equilibrium at the cell's rho, u, T, M^eq_{Q-q}; the
 * completed moment vector is inverted with M_Q^{-1}.  `dM` (may be NULL) adds a
 * correction to the completed moments M_{Q-q} (learned closure), in the order
 * of the high-order moment index.  The same map is applied to g (Sec. III.C). */
void lat_lift_raw(const lat_t *Lq, const lat_t *LQ, int thermal, double cv,
                  const double *fq, const double *gq, const double *dM,
                  double *fQ, double *gQ) {
  const int Q = LQ->Q, D = LQ->D, nq = Lq->n;
  double rho, u[3], T;
  lat_macros(Lq, thermal, cv, fq, gq, &rho, u, &T);
  double feqQ[OR_MAXQ], geqQ[OR_MAXQ];
  lat_feq(LQ, rho, u, T, feqQ);
  ld Mf[OR_MAXQ], Mg[OR_MAXQ];
  int k = 0;
  for (int j = 0; j < Q; j++) {
    int inq = 1;
    for (int a = 0; a < D; a++) if (LQ->pw[j][a] >= nq) inq = 0;
    if (inq) {
      Mf[j] = moment_pows(Lq, fq, LQ->pw[j]);
    } else {
      Mf[j] = moment_pows(LQ, feqQ, LQ->pw[j]);
      if (dM) Mf[j] += (ld)dM[k];
      k++;
    }
  }
  for (int i = 0; i < Q; i++) {
    ld s = 0.0L;
    for (int j = 0; j < Q; j++) s += LQ->Mfinv[i * Q + j] * Mf[j];
    fQ[i] = (double)s;
  }
  if (thermal && gq && gQ) {
    lat_geq_from_feq(LQ, cv, T, feqQ, geqQ);
    for (int j = 0; j < Q; j++) {
      int inq = 1;
      for (int a = 0; a < D; a++) if (LQ->pw[j][a] >= nq) inq = 0;
      Mg[j] = inq ? moment_pows(Lq, gq, LQ->pw[j]) : moment_pows(LQ, geqQ, LQ->pw[j]);
    }
    for (int i = 0; i < Q; i++) {
      ld s = 0.0L;
      for (int j = 0; j < Q; j++) s += LQ->Mfinv[i * Q + j] * Mg[j];
      gQ[i] = (double)s;
    }
  }
}

/* Hermite-coefficient variant of lifting: the Hermite coefficients
 * b_p = sum_i f_i prod_a He_{p_a}(c_ia) with every p_a < n_q are kept, the others
 * are those of the high-order equilibrium, and f_Q is rebuilt from the
 * Gauss-Hermite orthogonality f_i = W_i sum_p prod_a He_{p_a}(c_ia)/p_a! b_p. */
static void lift_hermite_one(const lat_t *Lq, const lat_t *LQ, const double *fq,
                             const double *feqQ, double *fQ) {
  const int Q = LQ->Q, D = LQ->D, nq = Lq->n;
  ld b[OR_MAXQ];
  for (int j = 0; j < Q; j++) {
    int inq = 1;
    for (int a = 0; a < D; a++) if (LQ->pw[j][a] >= nq) inq = 0;
    const lat_t *L = inq ? Lq : LQ;
    const double *f = inq ? fq : feqQ;
    ld s = 0.0L;
    for (int i = 0; i < L->Q; i++) {
      ld v = (ld)f[i];
      for (int a = 0; a < D; a++) v *= hermite(LQ->pw[j][a], L->cl[i][a]);
      s += v;
    }
    b[j] = s;
  }
  for (int i = 0; i < Q; i++) {
    ld s = 0.0L;
    for (int j = 0; j < Q; j++) {
      ld v = b[j];
      for (int a = 0; a < D; a++) {
        int p = LQ->pw[j][a];
        ld fct = 1.0L;
        for (int t = 2; t <= p; t++) fct *= (ld)t;
        v *= hermite(p, LQ->cl[i][a]) / fct;
      }
      s += v;
    }
    fQ[i] = (double)(LQ->Wl[i] * s);
  }
}

void lat_lift_hermite(const lat_t *Lq, const lat_t *LQ, int thermal, double cv,
                      const double *fq, const double *gq, double *fQ, double *gQ) {
  double rho, u[3], T;
  lat_macros(Lq, thermal, cv, fq, gq, &rho, u, &T);
  double feqQ[OR_MAXQ], geqQ[OR_MAXQ];
  lat_feq(LQ, rho, u, T, feqQ);
  lift_hermite_one(Lq, LQ, fq, feqQ, fQ);
  if (thermal && gq && gQ) {
    lat_geq_from_feq(LQ, cv, T, feqQ, geqQ);
    lift_hermite_one(Lq, LQ, gq, geqQ, gQ);
  }
}

/* Projection f_Q -> f_q (Sec. III.C, App. C): the first q moments of f_Q are
 * available exactly, m_{Q->q} = M_q, and f_q = M_q^{-1} m_{Q->q}. */
void lat_project(const lat_t *LQ, const lat_t *Lq, int thermal, const double *fQ,
                 const double *gQ, double *fq, double *gq) {
  const int q = Lq->Q;
  ld m[OR_MAXQ];
  for (int j = 0; j < q; j++) m[j] = moment_pows(LQ, fQ, Lq->pw[j]);
  for (int i = 0; i < q; i++) {
    ld s = 0.0L;
    for (int j = 0; j < q; j++) s += Lq->Mfinv[i * q + j] * m[j];
    fq[i] = (double)s;
  }
  if (thermal && gQ && gq) {
    for (int j = 0; j < q; j++) m[j] = moment_pows(LQ, gQ, Lq->pw[j]);
    for (int i = 0; i < q; i++) {
      ld s = 0.0L;
      for (int j = 0; j < q; j++) s += Lq->Mfinv[i * q + j] * m[j];
      gq[i] = (double)s;
    }
  }
}

/* ---- exported lattice-level helpers ---- */

int or_lattice_feq(int dim, int n, double rho, const double *u, double theta, double *out) {
  lat_t *L = lat_build(dim, n);
  if (!L) return -1;
  double uu[3] = {0, 0, 0};
  for (int a = 0; a < dim; a++) uu[a] = u[a];
  lat_feq(L, rho, uu, theta, out);
  lat_free(L);
  return 0;
}

int or_moment_matrix(int dim, int n, double *M, double *Minv) {
  lat_t *L = lat_build(dim, n);
  if (!L) return -1;
  for (int k = 0; k < L->Q * L->Q; k++) {
    if (M) M[k] = (double)L->M[k];
    if (Minv) Minv[k] = (double)L->Minv[k];
  }
  lat_free(L);
  return 0;
}

int or_lift(int dim, int nq, int nQ, int thermal, double cv, int mode,
            const double *fq, const double *gq, double *fQ, double *gQ) {
  if (nq >= nQ) return -1;
  lat_t *Lq = lat_build(dim, nq), *LQ = lat_build(dim, nQ);
  if (!Lq || !LQ) { lat_free(Lq); lat_free(LQ); return -1; }
  if (mode == 1)
    lat_lift_hermite(Lq, LQ, thermal, cv, fq, gq, fQ, gQ);
  else
    lat_lift_raw(Lq, LQ, thermal, cv, fq, gq, NULL, fQ, gQ);
  lat_free(Lq);
  lat_free(LQ);
  return 0;
}

int or_project(int dim, int nQ, int nq, const double *fQ, const double *gQ,
               double *fq, double *gq) {
  if (nq >= nQ) return -1;
  lat_t *Lq = lat_build(dim, nq), *LQ = lat_build(dim, nQ);
  if (!Lq || !LQ) { lat_free(Lq); lat_free(LQ); return -1; }
  lat_project(LQ, Lq, gQ != NULL && gq != NULL, fQ, gQ, fq, gq);
  lat_free(Lq);
  lat_free(LQ);
  return 0;
}

/* Lagrange basis through the nodes -1, 0, 1 evaluated at xi (the
 * reconstruction functions a_s of eq. reconstructionPond on a 3-point stencil):
 * a_s(xi) = prod_{m != s} (xi - m) / (s - m). */
int or_lagrange3(double xi, double *a) {
  for (int s = -1; s <= 1; s++) {
    ld v = 1.0L;
    for (int m = -1; m <= 1; m++)
      if (m != s) v *= ((ld)xi - (ld)m) / (ld)(s - m);
    a[s + 1] = (double)v;
  }
  return 0;
}

/* IEEE binary16 rounding to nearest, ties to even, of a double, returned as
 * the double it represents (overflow -> inf, gradual underflow kept). */
double or_round_fp16(double v) {
  if (isnan(v) || isinf(v) || v == 0.0) return v;
  double av = fabs(v);
  int e;
  frexp(av, &e);          /* av = m * 2^e, m in [0.5, 1) */
  int ex = e - 1;          /* av in [2^ex, 2^(ex+1)) */
  if (ex < -14) ex = -14;  /* subnormal spacing 2^-24 */
  double ulp = ldexp(1.0, ex - 10);
  double q = av / ulp;     /* exact: scaling by a power of two */
  double fl = floor(q);
  double rem = q - fl;
  double r;
  if (rem > 0.5) r = fl + 1;
  else if (rem < 0.5) r = fl;
  else r = fmod(fl, 2.0) == 0.0 ? fl : fl + 1;
  double out = r * ulp;
  if (out > 65504.0) out = INFINITY;
  return v < 0 ? -out : out;
}

/* bfloat16 (8 significant bits, float32 exponent range) rounding to nearest,
 * ties to even. */
double or_round_bf16(double v) {
  if (isnan(v) || isinf(v) || v == 0.0) return v;
  double av = fabs(v);
  int e;
  frexp(av, &e);
  int ex = e - 1;
  if (ex < -126) ex = -126;
  double ulp = ldexp(1.0, ex - 7);
  double q = av / ulp;
  double fl = floor(q);
  double rem = q - fl;
  double r;
  if (rem > 0.5) r = fl + 1;
  else if (rem < 0.5) r = fl;
  else r = fmod(fl, 2.0) == 0.0 ? fl : fl + 1;
  double out = r * ulp;
  if (out >= ldexp(1.0, 128)) out = INFINITY;
  return v < 0 ? -out : out;
}
