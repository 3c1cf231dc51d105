/*
 * oracle_mlp.c -- FP64 reference of the learned lifting closure: features,
 * targets, a two-hidden-layer perceptron with SiLU activations, its mean-square
 * loss gradient by back-propagation, and Adam.  TEST INFRASTRUCTURE ONLY.
 *
 * The closure replaces the equilibrium completion M_{Q-q} = M^eq_{Q-q} of the
 * lifting step (Sec. III.B) by M^eq_{Q-q} + rho T^{|p|/2} t(p), where t is the
 * network's estimate of the normalised non-equilibrium part of each missing raw
 * moment, computed from the normalised low-order moments of the cell.
 */
#include "oracle_internal.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

int or_mlp_nparams(int F, int H, int O) { return F * H + H + H * H + H + H * O + O; }

int or_mlp_dims(int dim, int nq, int nQ, int *F, int *O) {
  int q = 1, Q = 1;
  for (int a = 0; a < dim; a++) { q *= nq; Q *= nQ; }
  *F = 2 + dim + (q - 1 - dim);
  *O = Q - q;
  return 0;
}

static ld ipw(ld b, int e) {
  ld r = 1.0L;
  for (int k = 0; k < e; k++) r *= b;
  return r;
}

/* features: rho, u/sqrt(T), T, then the central moments
 * sum_i f_i prod_a (c_ia - u_a)^{p_a} / (rho T^{|p|/2}) of every low-order
 * moment index p with |p| >= 2, in ascending moment index */
int mlp_features_lat(const lat_t *Lq, int thermal, double cv, const double *fq,
                     const double *gq, double *feat) {
  double rho, u[3], T;
  lat_macros(Lq, thermal, cv, fq, gq, &rho, u, &T);
  const int D = Lq->D;
  int k = 0;
  feat[k++] = rho;
  for (int a = 0; a < D; a++) feat[k++] = u[a] / sqrt(T);
  feat[k++] = T;
  for (int j = 0; j < Lq->Q; j++) {
    int deg = 0;
    for (int a = 0; a < D; a++) deg += Lq->pw[j][a];
    if (deg < 2) continue;
    ld s = 0.0L;
    for (int i = 0; i < Lq->Q; i++) {
      ld v = (ld)fq[i];
      for (int a = 0; a < D; a++) v *= ipw(Lq->cl[i][a] - (ld)u[a], Lq->pw[j][a]);
      s += v;
    }
    feat[k++] = (double)(s / ((ld)rho * powl((ld)T, 0.5L * deg)));
  }
  return k;
}

/* targets: normalised non-equilibrium part of each raw moment the low-order
 * set cannot hold, (M_p - M^eq_p) / (rho T^{|p|/2}), in ascending moment index
 * of the high-order set */
int mlp_targets_lat(const lat_t *Lq, const lat_t *LQ, int thermal, double cv,
                    const double *fQ, const double *gQ, double *targ) {
  double rho, u[3], T;
  lat_macros(LQ, thermal, cv, fQ, gQ, &rho, u, &T);
  double feq[OR_MAXQ];
  lat_feq(LQ, rho, u, T, feq);
  ld m[OR_MAXQ], meq[OR_MAXQ];
  lat_moments(LQ, fQ, m);
  lat_moments(LQ, feq, meq);
  int k = 0;
  for (int j = 0; j < LQ->Q; j++) {
    int inq = 1, deg = 0;
    for (int a = 0; a < LQ->D; a++) {
      if (LQ->pw[j][a] >= Lq->n) inq = 0;
      deg += LQ->pw[j][a];
    }
    if (inq) continue;
    targ[k++] = (double)((m[j] - meq[j]) / ((ld)rho * powl((ld)T, 0.5L * deg)));
  }
  return k;
}

int or_mlp_features(int dim, int nq, int thermal, double cv, const double *fq,
                    const double *gq, double *feat) {
  lat_t *L = lat_build(dim, nq);
  if (!L) return -1;
  mlp_features_lat(L, thermal, cv, fq, gq, feat);
  lat_free(L);
  return 0;
}

int or_mlp_targets(int dim, int nq, int nQ, int thermal, double cv, const double *fQ,
                   const double *gQ, double *targ) {
  lat_t *Lq = lat_build(dim, nq), *LQ = lat_build(dim, nQ);
  if (!Lq || !LQ) { lat_free(Lq); lat_free(LQ); return -1; }
  mlp_targets_lat(Lq, LQ, thermal, cv, fQ, gQ, targ);
  lat_free(Lq);
  lat_free(LQ);
  return 0;
}

static double sigm(double z) { return 1.0 / (1.0 + exp(-z)); }
static double silu(double z) { return z * sigm(z); }
static double silu_d(double z) {
  double s = sigm(z);
  return s * (1.0 + z * (1.0 - s));
}
static double rb(double v, int bf16) { return bf16 ? or_round_bf16(v) : v; }

/* y = W3^T s(W2^T s(W1^T x + b1) + b2) + b3 with s = SiLU.  With `bf16` set,
 * the operands of each product (input, weights, hidden activations) are
 * rounded to bfloat16 first, as a reduced-precision matrix unit consumes them;
 * sums and biases stay in double. */
void mlp_forward_one(const double *p, int F, int H, int O, const double *x, double *y,
                     int bf16) {
  const double *W1 = p, *b1 = W1 + F * H, *W2 = b1 + H, *b2 = W2 + H * H, *W3 = b2 + H,
               *b3 = W3 + H * O;
  double h1[256], h2[256];
  for (int j = 0; j < H; j++) {
    double s = b1[j];
    for (int k = 0; k < F; k++) s += rb(x[k], bf16) * rb(W1[k * H + j], bf16);
    h1[j] = silu(s);
  }
  for (int j = 0; j < H; j++) {
    double s = b2[j];
    for (int k = 0; k < H; k++) s += rb(h1[k], bf16) * rb(W2[k * H + j], bf16);
    h2[j] = silu(s);
  }
  for (int j = 0; j < O; j++) {
    double s = b3[j];
    for (int k = 0; k < H; k++) s += rb(h2[k], bf16) * rb(W3[k * O + j], bf16);
    y[j] = s;
  }
}

int or_mlp_forward(const double *p, int F, int H, int O, int n, const double *X,
                   double *Y, int bf16) {
  if (H > 256) return -1;
  for (int r = 0; r < n; r++) mlp_forward_one(p, F, H, O, X + (size_t)r * F, Y + (size_t)r * O, bf16);
  return 0;
}

/* loss = mean over samples and outputs of (y - t)^2; gradient by the chain
 * rule through the three affine maps and the two SiLU activations */
int or_mlp_loss_grad(const double *p, int F, int H, int O, int n, const double *X,
                     const double *T, double *loss, double *grad) {
  if (H > 256 || O > 256) return -1;
  const double *W1 = p, *b1 = W1 + F * H, *W2 = b1 + H, *b2 = W2 + H * H, *W3 = b2 + H,
               *b3 = W3 + H * O;
  const int np = or_mlp_nparams(F, H, O);
  memset(grad, 0, sizeof(double) * np);
  double *gW1 = grad, *gb1 = gW1 + F * H, *gW2 = gb1 + H, *gb2 = gW2 + H * H, *gW3 = gb2 + H,
         *gb3 = gW3 + H * O;
  (void)b3;
  double L = 0.0;
  const double scale = 2.0 / ((double)n * O);
  for (int r = 0; r < n; r++) {
    const double *x = X + (size_t)r * F, *t = T + (size_t)r * O;
    double z1[256], h1[256], z2[256], h2[256];
    for (int j = 0; j < H; j++) {
      double s = b1[j];
      for (int k = 0; k < F; k++) s += x[k] * W1[k * H + j];
      z1[j] = s;
      h1[j] = silu(s);
    }
    for (int j = 0; j < H; j++) {
      double s = b2[j];
      for (int k = 0; k < H; k++) s += h1[k] * W2[k * H + j];
      z2[j] = s;
      h2[j] = silu(s);
    }
    double dy[256], dh2[256], dz2[256], dh1[256], dz1[256];
    for (int j = 0; j < O; j++) {
      double s = b3[j];
      for (int k = 0; k < H; k++) s += h2[k] * W3[k * O + j];
      double e = s - t[j];
      L += e * e;
      dy[j] = scale * e;
    }
    for (int k = 0; k < H; k++) {
      double s = 0.0;
      for (int j = 0; j < O; j++) {
        gW3[k * O + j] += h2[k] * dy[j];
        s += W3[k * O + j] * dy[j];
      }
      dh2[k] = s;
      dz2[k] = s * silu_d(z2[k]);
    }
    for (int j = 0; j < O; j++) gb3[j] += dy[j];
    for (int k = 0; k < H; k++) {
      double s = 0.0;
      for (int j = 0; j < H; j++) {
        gW2[k * H + j] += h1[k] * dz2[j];
        s += W2[k * H + j] * dz2[j];
      }
      dh1[k] = s;
      dz1[k] = s * silu_d(z1[k]);
    }
    for (int j = 0; j < H; j++) gb2[j] += dz2[j];
    for (int k = 0; k < F; k++)
      for (int j = 0; j < H; j++) gW1[k * H + j] += x[k] * dz1[j];
    for (int j = 0; j < H; j++) gb1[j] += dz1[j];
    (void)dh1;
    (void)dh2;
  }
  *loss = L / ((double)n * O);
  return 0;
}

/* Adam (Kingma & Ba 2015) with bias-corrected first and second moments */
int or_adam(double *p, double *m, double *v, const double *g, int np, int t, double lr,
            double b1, double b2, double eps) {
  double c1 = 1.0 - pow(b1, t), c2 = 1.0 - pow(b2, t);
  for (int k = 0; k < np; k++) {
    m[k] = b1 * m[k] + (1.0 - b1) * g[k];
    v[k] = b2 * v[k] + (1.0 - b2) * g[k] * g[k];
    double mh = m[k] / c1, vh = v[k] / c2;
    p[k] -= lr * mh / (sqrt(vh) + eps);
  }
  return 0;
}
