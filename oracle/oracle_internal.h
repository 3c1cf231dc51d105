/* oracle_internal.h -- shared declarations of the oracle's own translation
 * units.  TEST INFRASTRUCTURE ONLY. */
#ifndef MSL_ORACLE_INTERNAL_H
#define MSL_ORACLE_INTERNAL_H
#include "oracle.h"

#define OR_MAXN 8
#define OR_MAXQ 216
#define OR_CHECK_TILE 64

typedef long double ld;

typedef struct lat_t {
  int D, n, Q;
  ld x[OR_MAXN], w[OR_MAXN];   /* 1D nodes and weights */
  ld cl[OR_MAXQ][3];           /* velocities (long double) */
  double c[OR_MAXQ][3];        /* velocities (double) */
  ld Wl[OR_MAXQ];
  double W[OR_MAXQ];
  int pw[OR_MAXQ][3];          /* base-n digits of the population / moment index */
  ld *M, *Minv;                /* Q x Q moment matrix and its inverse */
  /* reference frame of the run (eq. veli): v_ia = sqrt(T_ref) c_ia + u_ref,a */
  ld ur[3], Tr;
  ld vl[OR_MAXQ][3];
  double v[OR_MAXQ][3];
  ld *Mf, *Mfinv;              /* moment matrix at the particle velocities v and its inverse */
} lat_t;

int gh_rule_ld(int n, ld *x, ld *w);
int ld_invert(int n, const ld *A, ld *Ainv);   /* Gauss-Jordan, partial pivoting */
lat_t *lat_build(int dim, int n);
void lat_free(lat_t *L);
int lat_set_frame(lat_t *L, const double *u_ref, double T_ref);
int lat_frame_trivial(const lat_t *L);
double lat_vmax(const lat_t *L, int axis);
void lat_feq(const lat_t *L, double rho, const double *u, double theta, double *out);
void lat_from_comoving(const lat_t *L, const double *u, double theta, const ld *co, double *out);
void lat_qeq(const lat_t *L, int thermal, double cv, double rho, const double *u, double T,
             const double *f, const double *g, const double *feq, const double *geq,
             double *fstar, double *gstar);
void lat_moments(const lat_t *L, const double *f, ld *m);
void lat_macros(const lat_t *L, int thermal, double cv, const double *f, const double *g,
                double *rho, double *u, double *T);
void lat_geq_from_feq(const lat_t *L, double cv, double T, const double *feq, double *geq);
void lat_lift_raw(const lat_t *Lq, const lat_t *LQ, int thermal, double cv,
                  const double *fq, const double *gq, const double *dM,
                  double *fQ, double *gQ);
void lat_lift_hermite(const lat_t *Lq, const lat_t *LQ, int thermal, double cv,
                      const double *fq, const double *gq, double *fQ, double *gQ);
void lat_project(const lat_t *LQ, const lat_t *Lq, int thermal, const double *fQ,
                 const double *gQ, double *fq, double *gq);

/* closure helpers (oracle_mlp.c) */
int mlp_features_lat(const lat_t *Lq, int thermal, double cv, const double *fq,
                     const double *gq, double *feat);
int mlp_targets_lat(const lat_t *Lq, const lat_t *LQ, int thermal, double cv,
                    const double *fQ, const double *gQ, double *targ);
void mlp_forward_one(const double *p, int F, int H, int O, const double *x, double *y,
                     int bf16);
#endif
