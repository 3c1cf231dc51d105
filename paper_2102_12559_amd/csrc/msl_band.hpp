// msl_band.hpp -- lifting and projection of one cell with compile-time
// velocity-set sizes (FP64, register resident), used by the band conversion
// and the switching kernels.
#pragma once
#include "msl_device.hpp"

template <int D, int N> struct Pow { static constexpr int v = D == 2 ? N * N : N * N * N; };

// (Ax x Ay (x Az)) applied to a tensor-product array: out[NO^D] = A_a[NO][NI]
// along each axis a of in[NI^D]
template <int D, int NO, int NI>
__device__ __forceinline__ void tensor_apply_t(const double (*Ax)[MSL_MAXN], const double (*Ay)[MSL_MAXN],
                                               const double (*Az)[MSL_MAXN], const double *in,
                                               double *out) {
  if constexpr (D == 2) {
    double t[NI * NO];
#pragma unroll
    for (int b = 0; b < NO; ++b)
#pragma unroll
      for (int ap = 0; ap < NI; ++ap) {
        double s = 0;
#pragma unroll
        for (int bp = 0; bp < NI; ++bp) s += Ay[b][bp] * in[ap + NI * bp];
        t[ap + NI * b] = s;
      }
#pragma unroll
    for (int b = 0; b < NO; ++b)
#pragma unroll
      for (int a = 0; a < NO; ++a) {
        double s = 0;
#pragma unroll
        for (int ap = 0; ap < NI; ++ap) s += Ax[a][ap] * t[ap + NI * b];
        out[a + NO * b] = s;
      }
  } else {
    double t1[NI * NI * NO], t2[NI * NO * NO];
#pragma unroll
    for (int c = 0; c < NO; ++c)
#pragma unroll
      for (int bp = 0; bp < NI; ++bp)
#pragma unroll
        for (int ap = 0; ap < NI; ++ap) {
          double s = 0;
#pragma unroll
          for (int cp = 0; cp < NI; ++cp) s += Az[c][cp] * in[ap + NI * (bp + NI * cp)];
          t1[ap + NI * (bp + NI * c)] = s;
        }
#pragma unroll
    for (int c = 0; c < NO; ++c)
#pragma unroll
      for (int b = 0; b < NO; ++b)
#pragma unroll
        for (int ap = 0; ap < NI; ++ap) {
          double s = 0;
#pragma unroll
          for (int bp = 0; bp < NI; ++bp) s += Ay[b][bp] * t1[ap + NI * (bp + NI * c)];
          t2[ap + NI * (b + NO * c)] = s;
        }
#pragma unroll
    for (int c = 0; c < NO; ++c)
#pragma unroll
      for (int b = 0; b < NO; ++b)
#pragma unroll
        for (int a = 0; a < NO; ++a) {
          double s = 0;
#pragma unroll
          for (int ap = 0; ap < NI; ++ap) s += Ax[a][ap] * t2[ap + NI * (b + NO * c)];
          out[a + NO * (b + NO * c)] = s;
        }
  }
}

template <int D, int N>
__device__ __forceinline__ void macros_t(const LatTab &L, bool thermal, double cv, const double *f,
                                         const double *g, double &rho, double *u, double &T) {
  double r = 0, j[3] = {0, 0, 0}, e = 0;
#pragma unroll
  for (int i = 0; i < Pow<D, N>::v; ++i) {
    const int a = i % N, b = (i / N) % N, c = D == 3 ? i / (N * N) : 0;
    const double cx = L.v[0][a], cy = L.v[1][b], cz = D == 3 ? L.v[2][c] : 0.0;
    r += f[i];
    j[0] += cx * f[i];
    j[1] += cy * f[i];
    if (D == 3) j[2] += cz * f[i];
    e += 0.5 * (cx * cx + cy * cy + cz * cz) * f[i];
    if (thermal) e += g[i];
  }
  rho = r;
  u[0] = j[0] / r;
  u[1] = j[1] / r;
  u[2] = D == 3 ? j[2] / r : 0.0;
  T = thermal ? (e - 0.5 * r * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2])) / (cv * r) : 1.0;
}

template <int D, int N>
__device__ __forceinline__ void feq_t(const LatTab &L, double rho, const double *u, double T,
                                      double *feq) {
  double P[3][N];
#pragma unroll
  for (int a = 0; a < D; ++a) eq_axis<double, N>(L, (u[a] - L.ur[a]) * L.isq, T * L.iTr, P[a]);
#pragma unroll
  for (int i = 0; i < Pow<D, N>::v; ++i) {
    double v = rho * P[0][i % N] * P[1][(i / N) % N];
    if (D == 3) v *= P[2][i / (N * N)];
    feq[i] = v;
  }
}

// Lifting (Sec. III.B, App. C): f_Q = f^L_Q + (Kx x Ky (x Kz)) (f_q - f^L_q),
// K_a the degree < n_q part of the high-order Lagrange basis in the particle
// velocities along axis a, evaluated at the low nodes (or the Hermite
// completion matrix); the learned closure adds (Vi x Vi) dM.  With TH false
// the energy populations are known to be absent at compile time.
template <int D, int NL, int NH, bool TH = true>
__device__ __forceinline__ void lift_t(const Tab *tab, const double *fq, const double *gq,
                                       const double *dM, double *fQ, double *gQ) {
  const LatTab &Lq = tab->lat[0], &LQ = tab->lat[1];
  constexpr int q = Pow<D, NL>::v, Q = Pow<D, NH>::v;
  double rho, u[3], T;
  const bool th = TH && tab->thermal;
  macros_t<D, NL>(Lq, th, tab->cv, fq, gq, rho, u, T);
  double eq_q[q], eq_Q[Q], neq[q], corr[Q];
  feq_t<D, NL>(Lq, rho, u, T, eq_q);
  feq_t<D, NH>(LQ, rho, u, T, eq_Q);
  const bool herm = tab->lift_mode == MSL_LIFT_GRAD_HERMITE;
  const double (*Kx)[MSL_MAXN] = herm ? tab->KH : tab->K[0];
  const double (*Ky)[MSL_MAXN] = herm ? tab->KH : tab->K[1];
  const double (*Kz)[MSL_MAXN] = herm ? tab->KH : tab->K[2];
#pragma unroll
  for (int i = 0; i < q; ++i) neq[i] = fq[i] - eq_q[i];
  tensor_apply_t<D, NH, NL>(Kx, Ky, Kz, neq, corr);
#pragma unroll
  for (int i = 0; i < Q; ++i) fQ[i] = eq_Q[i] + corr[i];
  if (dM) {
    tensor_apply_t<D, NH, NH>(tab->Vi, tab->Vi, tab->Vi, dM, corr);
#pragma unroll
    for (int i = 0; i < Q; ++i) fQ[i] += corr[i];
  }
  if (th) {
    const double s = tab->gfac * T;
#pragma unroll
    for (int i = 0; i < q; ++i) neq[i] = gq[i] - s * eq_q[i];
    tensor_apply_t<D, NH, NL>(Kx, Ky, Kz, neq, corr);
#pragma unroll
    for (int i = 0; i < Q; ++i) gQ[i] = s * eq_Q[i] + corr[i];
  }
}

// Projection (Sec. III.C, App. C): f_q = (P x P) f_Q, P the low-order
// Lagrange basis evaluated at the high-order nodes.
template <int D, int NL, int NH, bool TH = true>
__device__ __forceinline__ void project_t(const Tab *tab, const double *fQ, const double *gQ,
                                          double *fq, double *gq) {
  tensor_apply_t<D, NL, NH>(tab->P, tab->P, tab->P, fQ, fq);
  if (TH && tab->thermal) tensor_apply_t<D, NL, NH>(tab->P, tab->P, tab->P, gQ, gq);
}

template <typename S, int D, int N, bool TH = true>
__device__ __forceinline__ void read_cell_t(const Tab *tab, const Geo &g, const char *base, int l,
                                            int off, double *f, double *gg) {
  const LatTab &L = tab->lat[l];
  constexpr int Q = Pow<D, N>::v;
  const S *p = (const S *)base;
  const double gs = tab->gfac * tab->T0;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    f[i] = load_pop<S>(p + (long long)i * g.plane, off, L.sc[i]);
    if (TH && tab->thermal) gg[i] = load_pop<S>(p + (long long)(Q + i) * g.plane, off, gs * L.sc[i]);
  }
}

template <typename S, int D, int N, bool TH = true>
__device__ __forceinline__ void write_cell_t(const Tab *tab, const Geo &g, char *base, int l,
                                             int off, const double *f, const double *gg) {
  const LatTab &L = tab->lat[l];
  constexpr int Q = Pow<D, N>::v;
  S *p = (S *)base;
  const double gs = tab->gfac * tab->T0;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    store_pop<S>(p + (long long)i * g.plane, off, f[i], L.sc[i]);
    if (TH && tab->thermal) store_pop<S>(p + (long long)(Q + i) * g.plane, off, gg[i], gs * L.sc[i]);
  }
}

// Dispatch a functor templated on (D, NL, NH) over the supported pairs.
template <typename F>
__host__ inline int msl_pair_dispatch(int D, int nl, int nh, F &&f) {
  if (D == 2) {
    if (nl == 3 && nh == 4) return f.template operator()<2, 3, 4>();
    if (nl == 3 && nh == 5) return f.template operator()<2, 3, 5>();
    if (nl == 3 && nh == 6) return f.template operator()<2, 3, 6>();
    if (nl == 4 && nh == 5) return f.template operator()<2, 4, 5>();
    if (nl == 4 && nh == 6) return f.template operator()<2, 4, 6>();
    if (nl == 5 && nh == 6) return f.template operator()<2, 5, 6>();
  } else {
    if (nl == 3 && nh == 4) return f.template operator()<3, 3, 4>();
  }
  return MSL_EINVAL;
}
