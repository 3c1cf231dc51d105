// msl_device.hpp -- device helpers shared by the kernels: precision selection,
// the lattice equilibrium in Hermite product form, per-population deviation
// scales, and the macroscopic moments of one cell.
#pragma once
#include "msl_internal.hpp"

template <typename C> __device__ __forceinline__ C tsel(double d, float f);
template <> __device__ __forceinline__ double tsel<double>(double d, float) { return d; }
template <> __device__ __forceinline__ float tsel<float>(double, float f) { return f; }

// Register budget heuristic: cells per thread along the marching axis so that
// the interpolated populations of all planes fit in about `budget` VGPRs.
__host__ __device__ constexpr int msl_rows_for(int nplanes, int words, int budget) {
  return budget / (nplanes * words) >= 4 ? 4 : (budget / (nplanes * words) >= 2 ? 2 : 1);
}

// 1D factor of the lattice equilibrium: the populations w_a P(c_a) whose first
// n moments are those of a Gaussian with mean u and variance theta.  With
// Gauss-Hermite orthogonality P(c) = sum_{j<n} He_j(c) b_j / j!, where
// b_j = E[He_j(X)], X ~ N(u, theta), follows from the generating function
// exp(u t + (theta - 1) t^2 / 2):  b_0 = 1, b_1 = u,
// b_{j+1} = u b_j + j (theta - 1) b_{j-1}.  The tensor product of the 1D factors
// (times rho) is the lattice-frame equilibrium f^L of eqs. feqL / feqL0.
// (LT: the lattice table, possibly in the constant address space)
template <typename C, int N, typename LT = LatTab>
__device__ __forceinline__ void eq_axis(const LT &L, C u, C theta, C *P) {
  C b[N];
  b[0] = C(1);
  if (N > 1) b[1] = u;
  const C tm1 = theta - C(1);
#pragma unroll
  for (int j = 1; j + 1 < N; ++j) b[j + 1] = u * b[j] + C(j) * tm1 * b[j - 1];
#pragma unroll
  for (int a = 0; a < N; ++a) {
    C s = C(0);
#pragma unroll
    for (int j = 0; j < N; ++j) s += tsel<C>(L.hw[a][j], L.hwf[a][j]) * b[j];
    P[a] = s;
  }
}

// Per-axis factors of the quasi-equilibria (eqs. fqeq, gqeq) in the run's
// frame.  A co-moving population w_a He_k(c_a) (Hermite order k along one axis)
// maps to the run's frame as theta'^{k/2} A[k][a] with
//   A[k][a] = sum_{k <= j < N} w_a He_j(c_a)/j! * j!/(j-k)! * b_{j-k},
// b_j the Hermite coefficients of the equilibrium factor (eq_axis), from the
// generating function E[He_k(Z) exp(t (sqrt(theta') Z + u') - t^2/2)] =
// theta'^{k/2} t^k exp(u' t + (theta' - 1) t^2/2).  A[0] is the equilibrium
// factor itself.
template <typename C, int N>
__device__ __forceinline__ void qe_axis(const LatTab &L, double u, double theta, C (*A)[N]) {
  double b[N];
  b[0] = 1.0;
  if (N > 1) b[1] = u;
#pragma unroll
  for (int j = 1; j + 1 < N; ++j) b[j + 1] = u * b[j] + (double)j * (theta - 1.0) * b[j - 1];
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int a = 0; a < N; ++a) {
      double s = 0.0;
#pragma unroll
      for (int j = k; j < N; ++j) {
        double fall = 1.0;
        for (int m = 0; m < k; ++m) fall *= (double)(j - m);
        s += L.hw[a][j] * fall * b[j - k];
      }
      A[k][a] = (C)s;
    }
}

// runtime-N variant (FP64), used by the auxiliary kernels and the host tables
__host__ __device__ __forceinline__ void eq_axis_rt(const LatTab &L, double u, double theta, double *P) {
  double b[MSL_MAXN];
  const int N = L.n;
  b[0] = 1.0;
  b[1] = u;
  for (int j = 1; j + 1 < N; ++j) b[j + 1] = u * b[j] + (double)j * (theta - 1.0) * b[j - 1];
  for (int a = 0; a < N; ++a) {
    double s = 0.0;
    for (int j = 0; j < N; ++j) s += L.hw[a][j] * b[j];
    P[a] = s;
  }
}

// XCD-aware tile order.  Workgroups are handed to the 8 XCDs in turn (linear
// workgroup id modulo 8), and each XCD has its own L2.  Mapping the workgroups
// an XCD receives onto one contiguous range of tiles (row-major) keeps the
// halo rows and columns that neighbouring tiles share inside one L2.
#define MSL_NXCD 8
__device__ __forceinline__ int msl_xcd_tile(int b, int nb) {
  const int per = nb / MSL_NXCD, rem = nb % MSL_NXCD;
  const int xcd = b % MSL_NXCD, slot = b / MSL_NXCD;
  return xcd < rem ? xcd * (per + 1) + slot : rem * (per + 1) + (xcd - rem) * per + slot;
}

// interior coordinates of cell k (x fastest)
__device__ __forceinline__ void cell_coords(const Geo &g, long long k, int &x, int &y, int &z) {
  x = (int)(k % g.nx);
  k /= g.nx;
  y = (int)(k % g.ny);
  z = (int)(k / g.ny);
}

template <typename S>
__device__ __forceinline__ double load_pop(const S *p, long long k, double scale) {
  using T = StoreTraits<S>;
  double v = (double)T::load(p[k]);
  return T::dev ? scale * (1.0 + v) : v;
}

template <typename S>
__device__ __forceinline__ void store_pop(S *p, long long k, double v, double scale) {
  using T = StoreTraits<S>;
  using C = typename T::C;
  p[k] = T::store(T::dev ? (C)(v / scale - 1.0) : (C)v);
}

// Moments of one cell's populations of set L in FP64: rho, u, T (conservation
// laws of Sec. II.B with the particle velocities v of the run's frame; T from
// rho E = cv rho T + rho u^2/2, eq. E; athermal T = 1).
__device__ __forceinline__ void cell_macros(const LatTab &L, int dim, int thermal, double cv,
                                            const double *f, const double *g, double &rho,
                                            double *u, double &T) {
  const int n = L.n, Q = L.Q;
  double r = 0, j[3] = {0, 0, 0}, e = 0;
  for (int i = 0; i < Q; ++i) {
    const double cx = L.v[0][i % n], cy = L.v[1][(i / n) % n], cz = dim == 3 ? L.v[2][i / (n * n)] : 0.0;
    r += f[i];
    j[0] += cx * f[i];
    j[1] += cy * f[i];
    j[2] += cz * f[i];
    e += 0.5 * (cx * cx + cy * cy + cz * cz) * f[i];
    if (thermal) e += g[i];
  }
  rho = r;
  u[0] = j[0] / r;
  u[1] = j[1] / r;
  u[2] = j[2] / r;
  const double u2 = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  T = thermal ? (e - 0.5 * r * u2) / (cv * r) : 1.0;
}

// Equilibrium of set L at (rho, u, T) in the run's frame, FP64, all Q
// populations: per axis the 1D factor at the frame-relative velocity
// (u - u_ref) / sqrt(T_ref) and reduced temperature T / T_ref.
__host__ __device__ __forceinline__ void cell_feq(const LatTab &L, int dim, double rho, const double *u,
                                         double T, double *feq) {
  double P[3][MSL_MAXN];
  for (int a = 0; a < dim; ++a) eq_axis_rt(L, (u[a] - L.ur[a]) * L.isq, T * L.iTr, P[a]);
  const int n = L.n;
  for (int i = 0; i < L.Q; ++i) {
    double v = rho * P[0][i % n] * P[1][(i / n) % n];
    if (dim == 3) v *= P[2][i / (n * n)];
    feq[i] = v;
  }
}
