// msl_stream.hpp -- the fused stream-and-collide kernel, one instantiation per
// (dimension, velocity-set order, storage precision, thermal model).
//
// This file holds the register-staged 2D kernel used where the LDS-resident
// one (msl_stream2.hpp) does not fit, and the launcher; 3D runs use the
// chunked kernel of msl_stream3.hpp.
//
// One workgroup owns a tile of 64 x TY cells.
// For each population plane (f_0..f_{Q-1}, then g_0..g_{Q-1}) the workgroup
// stages the plane's (64+2) x (TY+2) neighbourhood of the departure points into
// LDS -- the departure offset x - c_i dt is the same for every cell of a plane,
// so the staged window is the tile shifted by the population's base offset --
// while the next plane's global loads are in flight (double-buffered LDS, one
// barrier per plane).  Each thread interpolates its cells separably (rows,
// then columns; eq. reconstructionPond with 3-point Lagrange functions) into
// registers.  After the last plane every cell holds all its streamed
// populations and is collided in registers: moments, Hermite product-form
// equilibrium, BGK (eqs. Pond_f/g, omega1 = omega2), and stored coalesced.
// Cells of the other velocity set are skipped; tiles without a cell of this
// set exit before loading anything.
#pragma once
#include <utility>

#include "msl_device.hpp"
#include "msl_stream2.hpp"
#include "msl_stream3.hpp"
#include "msl_stream3z.hpp"

template <typename S, bool TH, int N, int D>
struct SCTraits {
  using T = StoreTraits<S>;
  using C = typename T::C;
  static constexpr int Q = D == 2 ? N * N : N * N * N;
  static constexpr int NP = TH ? 2 * Q : Q;
#ifndef MSL_ROWS_OVERRIDE
  static constexpr int R = msl_rows_for(NP, (int)(sizeof(C) / 4), D == 2 ? 96 : 128);
#else
  static constexpr int R = MSL_ROWS_OVERRIDE;
#endif
  // occupancy target: registers for the streamed values of all planes plus
  // the collision of one cell
  static constexpr int VREG = NP * R * (int)(sizeof(C) / 4) + 2 * Q * (int)(sizeof(C) / 4) + 48;
#ifndef MSL_WAVES_OVERRIDE
  static constexpr int WAVES = 512 / VREG >= 8 ? 8 : (512 / VREG < 1 ? 1 : 512 / VREG);
#else
  static constexpr int WAVES = MSL_WAVES_OVERRIDE;
#endif
};

// Collision of the R cells of one thread; ft[k][r] holds the streamed value of
// plane k (raw storage domain) at cell r.
template <typename S, bool TH, int N, int D, int R, int NP, bool QE = false>
__device__ __forceinline__ void collide_store(const Tab *__restrict__ tab, int lat, const Geo &g,
                                              typename StoreTraits<S>::C (&ft)[NP][R],
                                              S *__restrict__ out, const uint8_t *__restrict__ cls,
                                              int x, int y0, int z0, int ystep, int zstep) {
  using T = StoreTraits<S>;
  using C = typename T::C;
  constexpr int Q = D == 2 ? N * N : N * N * N;
  const LatTab &L = tab->lat[lat];
  const C gsc0 = (C)(tab->gfac * tab->T0);   // g scale over the f scale
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int y = y0 + r * ystep, z = z0 + r * zstep;
    // every lane collides (values of foreign or outside cells are discarded at
    // the store): a branch here would let the compiler sink the interpolation
    // into it and keep the staged window values alive across the collision
    const bool inside = x < g.nx && y < g.ny && (D == 2 || z < g.nz);
    const long long cell = inside ? ((long long)z * g.ny + y) * g.nx + x : 0;
    const bool mine = inside && (cls[cell] & 1) == lat;
    C f[Q];
    C gg[TH ? Q : 1];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const C W = tsel<C>(L.sc[i], L.scf[i]);   // storage scale of f_i
      f[i] = T::dev ? W * (C(1) + ft[i][r]) : ft[i][r];
      if (TH) gg[TH ? i : 0] = T::dev ? gsc0 * W * (C(1) + ft[TH ? Q + i : 0][r]) : ft[TH ? Q + i : 0][r];
    }
    // moments (Sec. II.B)
    C rho = C(0), jx = C(0), jy = C(0), jz = C(0), e = C(0);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const int a = i % N, b = (i / N) % N, cc = D == 3 ? i / (N * N) : 0;
      const C cx = tsel<C>(L.v[0][a], L.vf[0][a]), cy = tsel<C>(L.v[1][b], L.vf[1][b]);
      const C cz = D == 3 ? tsel<C>(L.v[2][cc], L.vf[2][cc]) : C(0);
      rho += f[i];
      jx += cx * f[i];
      jy += cy * f[i];
      if (D == 3) jz += cz * f[i];
      if (TH) e += C(0.5) * (cx * cx + cy * cy + cz * cz) * f[i] + gg[TH ? i : 0];
    }
    // the equilibrium factors are evaluated in FP64 for every storage type:
    // single-precision Hermite tables would bias the equilibrium's mass and
    // momentum by their rounding, the same way every step
    const double rd = (double)rho, ird = 1.0 / rd;
    const double ux = (double)jx * ird, uy = (double)jy * ird, uz = (double)jz * ird;
    double Tm = 1.0;
    if (TH) Tm = ((double)e - 0.5 * rd * (ux * ux + uy * uy + uz * uz)) / (tab->cv * rd);
    C om = tsel<C>(tab->omega, tab->omegaf);
    double tl = tab->tau;
    if (tab->tau_mode == 1) {
      const double mu = TH ? tab->mu_ref * pow(Tm / tab->tau_ref_T, tab->mu_exp) : tab->mu_T1;
      tl = mu / (rd * Tm * tab->dt) + 0.5;
      om = (C)(1.0 / tl);
    }
    double Px[N], Py[N], Pz[N];
    eq_axis<double, N>(L, (ux - L.ur[0]) * L.isq, Tm * L.iTr, Px);
    eq_axis<double, N>(L, (uy - L.ur[1]) * L.isq, Tm * L.iTr, Py);
    if (D == 3) eq_axis<double, N>(L, (uz - L.ur[2]) * L.isq, Tm * L.iTr, Pz);
#pragma unroll
    for (int a = 0; a < N; ++a) Px[a] *= rd;
    const C gf = (C)(tab->gfac * Tm);
    // two-relaxation model (2D; eqs. Pond_f/g with the quasi-equilibria of
    // eqs. fqeq, gqeq in the run's frame): Qbar, qbar of the cell folded with
    // (omega1 - omega2) and the constants of f* - f^eq and g* - g^eq
    C Ax[QE ? 4 : 1][N], Ay[QE ? 4 : 1][N], Qb[4] = {C(0), C(0), C(0), C(0)}, qb[2] = {C(0), C(0)};
    if constexpr (QE) {
      static_assert(D == 2, "the two-relaxation model is built for 2D");
      qe_axis<C, N>(L, (ux - L.ur[0]) * L.isq, Tm * L.iTr, Ax);
      qe_axis<C, N>(L, (uy - L.ur[1]) * L.isq, Tm * L.iTr, Ay);
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        const int a = i % N, b = (i / N) % N;
        const C dx = tsel<C>(L.v[0][a], L.vf[0][a]) - (C)ux, dy = tsel<C>(L.v[1][b], L.vf[1][b]) - (C)uy;
        const C feq = (C)(Px[a] * Py[b]);
        const C nf = f[i] - feq;
        Qb[0] += dx * dx * dx * nf;
        Qb[1] += dx * dx * dy * nf;
        Qb[2] += dx * dy * dy * nf;
        Qb[3] += dy * dy * dy * nf;
        if (TH) {
          const C ng = gg[TH ? i : 0] - gf * feq;
          qb[0] += dx * ng;
          qb[1] += dy * ng;
        }
      }
      const C dom = (C)(1.0 / tl - 1.0 / (0.5 + (tl - 0.5) * tab->qe_ratio));
      const C cf = (C)(L.isq * L.isq * L.isq / 6.0) * dom, cg = (C)L.isq * dom;
      Qb[0] *= cf;
      Qb[1] *= C(3) * cf;
      Qb[2] *= C(3) * cf;
      Qb[3] *= cf;
      qb[0] *= cg;
      qb[1] *= cg;
    }
    const unsigned boff = (unsigned)g.idx(x, y, z) * (unsigned)sizeof(S);
    S so[Q];
    S sg[TH ? Q : 1];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const int a = i % N, b = (i / N) % N, cc = D == 3 ? i / (N * N) : 0;
      double feqd = Px[a] * Py[b];
      if (D == 3) feqd *= Pz[cc];
      const C feq = (C)feqd;
      C fo = f[i] + om * (feq - f[i]);
      if constexpr (QE)
        fo += Qb[0] * Ax[3][a] * Ay[0][b] + Qb[1] * Ax[2][a] * Ay[1][b] + Qb[2] * Ax[1][a] * Ay[2][b] +
              Qb[3] * Ax[0][a] * Ay[3][b];
      const C W = tsel<C>(L.sc[i], L.scf[i]);
      so[i] = T::store(T::dev ? fo / W - C(1) : fo);
      if (TH) {
        C go = gg[TH ? i : 0] + om * (gf * feq - gg[TH ? i : 0]);
        if constexpr (QE) go += qb[0] * Ax[1][a] * Ay[0][b] + qb[1] * Ax[0][a] * Ay[1][b];
        sg[TH ? i : 0] = T::store(T::dev ? go / (gsc0 * W) - C(1) : go);
      }
    }
    if (mine) {
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        *(S *)((char *)(out + (long long)i * g.plane) + boff) = so[i];
        if (TH) *(S *)((char *)(out + (long long)(Q + i) * g.plane) + boff) = sg[TH ? i : 0];
      }
    }
  }
}

template <int NP, typename F>
__device__ __forceinline__ void for_planes(F &&f) {
  [&]<int... Ks>(std::integer_sequence<int, Ks...>) {
    (f.template operator()<Ks>(), ...);
  }(std::make_integer_sequence<int, NP>{});
}

template <typename S, bool TH, int N, bool QE = false>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(SCTraits<S, TH, N, 2>::WAVES)))
k_sc2d(const Tab *__restrict__ tab, int lat, Geo g, const S *__restrict__ in, S *__restrict__ out,
       const uint8_t *__restrict__ cls, const uint8_t *__restrict__ tflag) {
  using Tr = SCTraits<S, TH, N, 2>;
  using T = typename Tr::T;
  using C = typename Tr::C;
  constexpr int Q = Tr::Q, NP = Tr::NP, R = Tr::R;
  constexpr int TY = MSL_MTY * R;
  constexpr int LW = MSL_TX + 2, LR = TY + 2, NE = LW * LR, NLD = (NE + 255) / 256;
  __shared__ C sm[2][NE];
  const LatTab &L = tab->lat[lat];
  const int bx = blockIdx.x, by = blockIdx.y;
  const int x0 = bx * MSL_TX, y0 = by * TY;
  {
    uint8_t any = 0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int my = by * R + r;
      if (my < g.nty) any |= tflag[my * g.ntx + bx];
    }
    if (!(any & (1 << lat))) return;
  }
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  // per-thread offsets of the staged window elements (plane independent)
  int eoff[NLD];
#pragma unroll
  for (int m = 0; m < NLD; ++m) {
    int e = threadIdx.x + 256 * m;
    e = e < NE ? e : NE - 1;
    const int rr = e / LW, cc = e - rr * LW;
    eoff[m] = (rr * g.pitch + cc) * (int)sizeof(S);   // byte offset from the window origin
  }
  C ft[NP][R];
  C reg[NLD];
  auto gload = [&]<int K>() {
    constexpr int i = K % Q, a = i % N, b = i / N;
    const int ox = L.n0[0][a] - 1, oy = L.n0[1][b] - 1;
    const S *base = in + (long long)K * g.plane + g.idx(x0 + ox, y0 + oy, 0);
#pragma unroll
    for (int m = 0; m < NLD; ++m)
      reg[m] = (C)T::load(*(const S *)((const char *)base + (unsigned)eoff[m]));
  };
  auto lstore = [&](int buf) {
#pragma unroll
    for (int m = 0; m < NLD; ++m) {
      const int e = threadIdx.x + 256 * m;
      if (NE % 256 == 0 || m + 1 < NLD || e < NE) sm[buf][e] = reg[m];
    }
  };
  auto step = [&]<int K>() {
    if constexpr (K + 1 < NP) gload.template operator()<K + 1>();
    constexpr int i = K % Q, a = i % N, b = i / N;
    constexpr int buf = K & 1;
    const C wx0 = tsel<C>(L.a[0][a][0], L.af[0][a][0]), wx1 = tsel<C>(L.a[0][a][1], L.af[0][a][1]),
            wx2 = tsel<C>(L.a[0][a][2], L.af[0][a][2]);
    const C wy0 = tsel<C>(L.a[1][b][0], L.af[1][b][0]), wy1 = tsel<C>(L.a[1][b][1], L.af[1][b][1]),
            wy2 = tsel<C>(L.a[1][b][2], L.af[1][b][2]);
    // differenced form: the centre weight is 1 - w0 - w2 exactly, so a
    // uniform field is reproduced without a rounding bias in the weights
    (void)wx1;
    (void)wy1;
    C h[R + 2];
#pragma unroll
    for (int r = 0; r < R + 2; ++r) {
      const C *row = &sm[buf][(ty * R + r) * LW + tx];
      h[r] = row[1] + wx0 * (row[0] - row[1]) + wx2 * (row[2] - row[1]);
    }
#pragma unroll
    for (int r = 0; r < R; ++r) ft[K][r] = h[r + 1] + wy0 * (h[r] - h[r + 1]) + wy2 * (h[r + 2] - h[r + 1]);
    if constexpr (K + 1 < NP) lstore((K + 1) & 1);
    __syncthreads();
  };
  gload.template operator()<0>();
  lstore(0);
  __syncthreads();
  for_planes<NP>(step);
  collide_store<S, TH, N, 2, R, NP, QE>(tab, lat, g, ft, out, cls, x0 + tx, y0 + ty * R, 0, 1, 0);
}

// 2D, every plane resident in LDS (k_sc2d_res); NO > 0: the launch also
// converts its band cells into the other set's planes `oth` (NO nodes per axis)
template <typename S, bool TH, int N, bool QE, int NO>
static int launch_sc2(msl_ctx *c, int lat, const char *in, char *out, char *oth) {
  const Geo &g = c->geo;
  dim3 block(256);
  S *os = (S *)oth;
  // non-temporal stores for FP32 / FP64 D2Q9 planes when the set's buffer
  // exceeds the 256 MB last-level cache
  const int nt = N == 3 && sizeof(S) >= 4 &&
                 (double)g.plane * sizeof(S) * c->Q[lat] * (c->cfg.thermal ? 2 : 1) > 256.0 * (1 << 20);
  const long long tiles8 = (long long)((g.nx + MSL_TX - 1) / MSL_TX) * ((g.ny + 7) / 8);
  bool small = false;
  if constexpr (N == 3) {
    // D2Q9 on a grid of fewer than 8 tiles of 8 rows per CU: 4-row tiles,
    // twice as many workgroups
    using T2 = SC2Traits<S, TH, N, true>;
    static_assert(T2::fits && T2::TY == 4, "4-row D2Q9 tile");
    small = tiles8 < 2048;
    if (small) {
      dim3 grid((g.nx + MSL_TX - 1) / MSL_TX, (g.ny + T2::TY - 1) / T2::TY);
      hipLaunchKernelGGL((k_sc2d_res<S, TH, N, true, false, QE, NO>), grid, block, 0, c->stream, c->dtab, lat, g,
                         (const S *)in, (S *)out, c->cls, c->tflag, lat == 0, nt, nullptr, nullptr, os, c->zgm);
    }
  }
  if constexpr (N > 3 && NO < N) {
    using T2 = SC2Traits<S, TH, N>;
    const long long tiles = (long long)g.ntx * ((g.ny + T2::TY - 1) / T2::TY);
    const long long fit = 256LL * (T2::WGS < 1 ? 1 : T2::WGS);
    if (!small && lat != 0 && tiles > 4 * fit) {
      // the high-order set on a large grid: one workgroup per live tile of
      // the compact list, whose length is read back (one stream
      // synchronisation each time the tile flags change, i.e. once per
      // criterion pass); smaller grids launch the whole tile grid, where
      // tiles without cells of the set exit at once
      if (c->capturing) return MSL_ESTATE;   // the list length is read by the host
      if (!c->tl_ok) {
        if (msl_launch_tile_list(c, lat, T2::R, 1)) return MSL_EHIP;
        int n = 0;
        if (hipMemcpyAsync(&n, c->tcount, sizeof(int), hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
            hipStreamSynchronize(c->stream) != hipSuccess)
          return MSL_EHIP;
        c->tl_n = n;
        c->tl_ok = 1;
      }
      if (c->tl_n == 0) return MSL_OK;
      dim3 grid((unsigned)c->tl_n);
      hipLaunchKernelGGL((k_sc2d_res<S, TH, N, false, true, QE, NO>), grid, block, 0, c->stream, c->dtab, lat,
                         g, (const S *)in, (S *)out, c->cls, c->tflag, 0, nt, c->tlist, c->tcount, os, c->zgm);
      return hipGetLastError() == hipSuccess ? MSL_OK : MSL_EHIP;
    }
  }
  if (!small) {
    using T2 = SC2Traits<S, TH, N>;
    dim3 grid((g.nx + MSL_TX - 1) / MSL_TX, (g.ny + T2::TY - 1) / T2::TY);
    hipLaunchKernelGGL((k_sc2d_res<S, TH, N, false, false, QE, NO>), grid, block, 0, c->stream, c->dtab, lat, g,
                       (const S *)in, (S *)out, c->cls, c->tflag, lat == 0, nt, nullptr, nullptr, os, c->zgm);
  }
  return hipGetLastError() == hipSuccess ? MSL_OK : MSL_EHIP;
}

// whether the launches of set `lat` can convert its band cells themselves
// (2D kernels with every plane resident in LDS)
template <typename S, bool TH, int N>
static bool fusable_n(int D) {
  return D == 2 && SC2Traits<S, TH, N>::fits;
}

template <typename S, bool TH, int N, int D, bool QE = false>
static int launch_one(msl_ctx *c, int lat, const char *in, char *out, char *oth) {
  using Tr = SCTraits<S, TH, N, D>;
  const Geo &g = c->geo;
  dim3 block(256);
  if constexpr (D == 2 && SC2Traits<S, TH, N>::fits) {
    switch (oth ? c->htab.lat[lat ^ 1].n : 0) {
      case 0: return launch_sc2<S, TH, N, QE, 0>(c, lat, in, out, nullptr);
      case 3: if constexpr (N != 3) return launch_sc2<S, TH, N, QE, 3>(c, lat, in, out, oth); break;
      case 4: if constexpr (N != 4) return launch_sc2<S, TH, N, QE, 4>(c, lat, in, out, oth); break;
      case 5: if constexpr (N != 5) return launch_sc2<S, TH, N, QE, 5>(c, lat, in, out, oth); break;
      case 6: if constexpr (N != 6) return launch_sc2<S, TH, N, QE, 6>(c, lat, in, out, oth); break;
    }
    return MSL_EINVAL;
  } else if constexpr (D == 2) {
    if (oth) return MSL_EINVAL;
    dim3 grid((g.nx + MSL_TX - 1) / MSL_TX, (g.ny + MSL_MTY * Tr::R - 1) / (MSL_MTY * Tr::R));
    hipLaunchKernelGGL((k_sc2d<S, TH, N, QE>), grid, block, 0, c->stream, c->dtab, lat, g,
                       (const S *)in, (S *)out, c->cls, c->tflag);
  } else {
    if (oth) return MSL_EINVAL;
    if constexpr (SC3ZTraits<S, TH, N>::fits) {
      // 3D: columns of 64 x 4 x ZC cells walked along z; the high-order set
      // of a large grid runs over the compact list of its live columns
      using T3 = SC3ZTraits<S, TH, N>;
      {
        const int ncz = (g.nz + T3::ZC - 1) / T3::ZC;
        const long long tiles = (long long)g.ntx * g.nty * ncz;
        const long long fit = 256LL * ((160 * 1024) / T3::LDS_BYTES);
        if (lat != 0 && tiles > 4 * fit) {
          if (c->capturing) return MSL_ESTATE;   // the list length is read by the host
        if (!c->tl_ok) {
            if (msl_launch_tile_list(c, lat, 1, T3::ZC)) return MSL_EHIP;
            int n = 0;
            if (hipMemcpyAsync(&n, c->tcount, sizeof(int), hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
                hipStreamSynchronize(c->stream) != hipSuccess)
              return MSL_EHIP;
            c->tl_n = n;
            c->tl_ok = 1;
          }
          if (c->tl_n == 0) return MSL_OK;
          hipLaunchKernelGGL((k_sc3d_zm<S, TH, N, true>), dim3((unsigned)c->tl_n), dim3(T3::NT), 0, c->stream,
                             c->dtab, lat, g, (const S *)in, (S *)out, c->cls, c->tflag, 0, c->xmir,
                             c->tlist, c->tcount);
          return hipGetLastError() == hipSuccess ? MSL_OK : MSL_EHIP;
        }
        dim3 grid((g.nx + MSL_TX - 1) / MSL_TX, (g.ny + MSL_MTY - 1) / MSL_MTY, ncz);
        hipLaunchKernelGGL((k_sc3d_zm<S, TH, N>), grid, dim3(T3::NT), 0, c->stream, c->dtab, lat, g,
                           (const S *)in, (S *)out, c->cls, c->tflag, lat == 0, c->xmir, nullptr, nullptr);
        return hipGetLastError() == hipSuccess ? MSL_OK : MSL_EHIP;
      }
    }
    // 3D sets whose planes do not fit the walk's register budget: planes
    // streamed through LDS in chunks; the high-order set of a large grid runs
    // over the compact list of its live tiles (as in 2D)
    using T3 = SC3Traits<S, TH, N>;
    const long long tiles = (long long)g.ntx * g.nty * ((g.ntz + T3::RZ - 1) / T3::RZ);
    const long long fit = 256LL * ((160 * 1024) / T3::LDS_BYTES);
    {
      if (lat != 0 && tiles > 4 * fit) {
        if (c->capturing) return MSL_ESTATE;   // the list length is read by the host
        if (!c->tl_ok) {
          if (msl_launch_tile_list(c, lat, 1, T3::RZ)) return MSL_EHIP;
          int n = 0;
          if (hipMemcpyAsync(&n, c->tcount, sizeof(int), hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
              hipStreamSynchronize(c->stream) != hipSuccess)
            return MSL_EHIP;
          c->tl_n = n;
          c->tl_ok = 1;
        }
        if (c->tl_n == 0) return MSL_OK;
        hipLaunchKernelGGL((k_sc3d_res<S, TH, N, true>), dim3((unsigned)c->tl_n), block, 0, c->stream,
                           c->dtab, lat, g, (const S *)in, (S *)out, c->cls, c->tflag, 0, c->xmir,
                           c->tlist, c->tcount);
        return hipGetLastError() == hipSuccess ? MSL_OK : MSL_EHIP;
      }
    }
    dim3 grid((g.nx + MSL_TX - 1) / MSL_TX, (g.ny + MSL_MTY - 1) / MSL_MTY, (g.nz + T3::RZ - 1) / T3::RZ);
    hipLaunchKernelGGL((k_sc3d_res<S, TH, N>), grid, block, 0, c->stream, c->dtab, lat, g,
                       (const S *)in, (S *)out, c->cls, c->tflag, lat == 0, c->xmir, nullptr, nullptr);
  }
  return hipGetLastError() == hipSuccess ? MSL_OK : MSL_EHIP;
}

template <typename S, bool TH>
static int launch_n(msl_ctx *c, int lat, const char *in, char *out, char *oth) {
  const int n = c->htab.lat[lat].n;
  if (c->D == 2) {
    if (c->htab.qe) {
      switch (n) {
        case 3: return launch_one<S, TH, 3, 2, true>(c, lat, in, out, oth);
        case 4: return launch_one<S, TH, 4, 2, true>(c, lat, in, out, oth);
        case 5: return launch_one<S, TH, 5, 2, true>(c, lat, in, out, oth);
        case 6: return launch_one<S, TH, 6, 2, true>(c, lat, in, out, oth);
      }
      return MSL_EINVAL;
    }
    switch (n) {
      case 3: return launch_one<S, TH, 3, 2>(c, lat, in, out, oth);
      case 4: return launch_one<S, TH, 4, 2>(c, lat, in, out, oth);
      case 5: return launch_one<S, TH, 5, 2>(c, lat, in, out, oth);
      case 6: return launch_one<S, TH, 6, 2>(c, lat, in, out, oth);
    }
  } else {
    switch (n) {
      case 3: return launch_one<S, TH, 3, 3>(c, lat, in, out, oth);
      case 4: return launch_one<S, TH, 4, 3>(c, lat, in, out, oth);
    }
  }
  return MSL_EINVAL;
}

// stream-and-collide of set `lat` for one storage type and energy variant;
// oth: the other set's new planes when the launch converts its band cells
template <typename S, bool TH>
int msl_launch_store_th(msl_ctx *c, int lat, const char *in, char *out, char *oth) {
  return launch_n<S, TH>(c, lat, in, out, oth);
}

// every set of a 2D context runs the kernel with all planes resident in LDS
// (which can convert band cells and apply zero-gradient faces itself)
template <typename S, bool TH>
int msl_sc2_all_th(const msl_ctx *c) {
  if (c->D != 2) return 0;
  for (int l = 0; l < c->nlat; ++l) {
    bool ok = false;
    switch (c->htab.lat[l].n) {
      case 3: ok = fusable_n<S, TH, 3>(2); break;
      case 4: ok = fusable_n<S, TH, 4>(2); break;
      case 5: ok = fusable_n<S, TH, 5>(2); break;
      case 6: ok = fusable_n<S, TH, 6>(2); break;
    }
    if (!ok) return 0;
  }
  return 1;
}
