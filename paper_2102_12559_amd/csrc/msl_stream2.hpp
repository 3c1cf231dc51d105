// msl_stream2.hpp -- the 2D stream-and-collide kernel with every population
// plane resident in LDS.
//
// A workgroup owns a tile of 64 x TY cells.  It first issues, for every plane
// (f_0..f_{Q-1}, then g_0..g_{Q-1}), direct-to-LDS buffer loads of the plane's
// (66 x (TY+2)) window around the departure points of the tile (the departure
// offset x - c_i dt is the same for all cells of a plane, so the window is
// the tile shifted by the plane's base offset).  All windows are in flight at
// once -- tens of KB per workgroup -- and no VGPR stages them.  After one wait
// and one barrier follow:
//   1. separable 3-point Lagrange reconstruction of every population
//      (eq. reconstructionPond) into registers, accumulating rho, rho u
//      (, rho E);
//   2. the per-axis equilibrium factors of each cell (FP64);
//   3. BGK relaxation of the reconstructed values towards the Hermite
//      product-form lattice equilibrium (eqs. Pond_f/g, feqL, geqL) and the
//      store, with buffer stores whose out-of-range offset drops the writes of
//      foreign or outside cells.
// A wave owns R rows of 64 cells, so the reconstructed values take NP * R
// registers per lane; every window element is read from LDS (R + 2) / R
// times per population instead of 3.
#pragma once
#include <utility>

#include "msl_device.hpp"

typedef __attribute__((address_space(3))) void msl_lds_t;
#define MSL_RSRC_WORD3 0x00020000   // raw buffer, gfx9-family descriptor word 3

template <typename S, bool TH, int N, bool SMALL = false>
struct SC2Traits {
  using T = StoreTraits<S>;
  using C = typename T::C;
  static constexpr int Q = N * N;
  static constexpr int NP = TH ? 2 * Q : Q;
  static constexpr int SZ = (int)sizeof(S);
  // a window row is loaded in 16-byte chunks (one per lane and DMA
  // instruction): 66 elements plus the misalignment of the row start (its
  // address is only 4-byte aligned), rounded up to whole chunks
  static constexpr int CPR = (66 * SZ + 3 + 15) / 16;   // chunks per row
  static constexpr int LWD = 4 * CPR;                    // dwords per row
  static constexpr int chunks_per_plane(int ty) { return (ty + 2) * CPR; }
  static constexpr int dwords_per_plane(int ty) { return 4 * chunks_per_plane(ty); }
  static constexpr int LDS_BUDGET = 72 * 1024;
  // tile height: the tallest of 16 / 8 / 4 rows whose windows fit the LDS
  // budget and whose reconstructed values (NP x TY/4 per lane) fit a register
  // budget of 48; D2Q9 takes at most 8 rows (smaller workgroups, more of them
  // resident per CU: measured faster at every storage type), and 4 on grids
  // too small to give every CU several tiles of 8 rows (SMALL)
  static constexpr int REGW = SZ == 8 ? 2 : 1;
  static constexpr bool tile_ok(int ty) {
    return NP * dwords_per_plane(ty) * 4 <= LDS_BUDGET && NP * (ty / 4) * REGW <= 48;
  }
  static constexpr int TY = SMALL ? 4 : (N == 3 && tile_ok(8)) ? 8 : (tile_ok(16) ? 16 : (tile_ok(8) ? 8 : 4));
  static constexpr int R = TY / 4;
  static constexpr int PD = dwords_per_plane(TY);     // LDS dwords per plane window
  static constexpr int CP = chunks_per_plane(TY);      // 16-byte chunks per plane window
  static constexpr int M = (CP + 255) / 256;           // DMA instructions per wave per plane
  static constexpr int LDS_BYTES = NP * PD * 4;
  static constexpr bool fits = LDS_BYTES <= 150 * 1024;
  // workgroups per CU allowed by LDS (160 KB); with 4 waves per workgroup that
  // is also the waves per SIMD the register budget has to allow (capped where
  // a tighter register budget would spill: 3 in general, 4 for athermal
  // D2Q9, 8 for the 4-row D2Q9 tile)
  static constexpr int WGS = (160 * 1024) / LDS_BYTES;
  static constexpr int WCAP = SMALL ? 8 : (N == 3 && !TH ? 4 : 3);
  static constexpr int WAVES = WGS >= WCAP ? WCAP : (WGS < 1 ? 1 : WGS);
};

template <int NP, typename F>
__device__ __forceinline__ void msl_for_planes(F &&f) {
  [&]<int... Ks>(std::integer_sequence<int, Ks...>) {
    (f.template operator()<Ks>(), ...);
  }(std::make_integer_sequence<int, NP>{});
}

template <typename S>
__device__ __forceinline__ float lds_elem(const char *p);
template <>
__device__ __forceinline__ float lds_elem<float>(const char *p) { return *(const float *)p; }
template <>
__device__ __forceinline__ float lds_elem<_Float16>(const char *p) { return (float)*(const _Float16 *)p; }
template <>
__device__ __forceinline__ float lds_elem<bf16_t>(const char *p) {
  return __uint_as_float(((uint32_t)*(const uint16_t *)p) << 16);
}
template <typename S>
__device__ __forceinline__ double lds_elem_d(const char *p) { return *(const double *)p; }

// The value a lane of the wave holds (a wave-uniform copy, v_readlane).
template <typename V>
__device__ __forceinline__ V msl_lane_get(V v, int lane) {
  if constexpr (sizeof(V) == 8) {
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, lane);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), lane);
    return __builtin_bit_cast(V, ((unsigned long long)hi << 32) | lo);
  } else {
    return __builtin_bit_cast(V, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), lane));
  }
}

// A wave whose band cells number at most this many lifts them one cell at a
// time across its lanes (one output node per lane); more, and every lane
// lifts its own cell.
#define MSL_LIFT_COOP 4

// NO > 0: the other velocity set of a two-set run has NO nodes per axis, and
// the kernel also converts its band cells (bit 1 of the class byte) into that
// set, in the new buffer `oth` of the other set's planes: the low-order
// launch lifts (NO > N), the high-order launch projects (NO < N), each from
// the post-collision populations it holds in registers.
template <typename S, bool TH, int N, bool SMALL, bool LIST = false, bool QE = false, int NO = 0>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(SC2Traits<S, TH, N, SMALL>::WAVES)))
k_sc2d_res(const Tab *__restrict__ tab, int lat, Geo g, const S *__restrict__ in,
           S *__restrict__ out, const uint8_t *__restrict__ cls,
           const uint8_t *__restrict__ tflag, int remap, int nt, const int *__restrict__ tlist,
           const int *__restrict__ tcount, S *__restrict__ oth, int zgm) {
  using Tr = SC2Traits<S, TH, N, SMALL>;
  using T = typename Tr::T;
  using C = typename Tr::C;
  constexpr int Q = Tr::Q, NP = Tr::NP, R = Tr::R, TY = Tr::TY, PD = Tr::PD, M = Tr::M;
  constexpr int LWD = Tr::LWD, SZ = Tr::SZ;
  constexpr int LR = TY + 2;
  __shared__ uint32_t sm[NP * PD];
  constexpr bool LIFT = NO > N, PROJ = NO > 0 && NO < N;
  constexpr int QO = NO * NO;
  constexpr int NTAB = LIFT ? NO * NO + 2 * NO * N + QO : (PROJ ? NO * N + QO : 1);
  __shared__ double stab[NTAB];
  const LatTab &L = tab->lat[lat];
  auto tile_body = [&](const int bx, const int by) {
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
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int tx = lane, ty = w;
  const unsigned pitch_b = (unsigned)g.pitch * SZ;
  const unsigned plane_b = (unsigned)g.plane * SZ;
  // plane-independent byte offsets of this lane's window chunks (16 bytes)
  constexpr int CPR = Tr::CPR, CP = Tr::CP;
  unsigned voff[M];
#pragma unroll
  for (int m = 0; m < M; ++m) {
    int d = lane + 64 * (w + 4 * m);
    d = d < CP ? d : CP - 1;
    const int row = d / CPR, col = d - row * CPR;
    voff[m] = (unsigned)row * pitch_b + (unsigned)col * 16u;
  }
  // 1. every plane's window in flight at once (direct-to-LDS loads)
  auto issue = [&]<int K>() {
    constexpr int i = K % Q, a = i % N, b = i / N;
    const int ox = L.n0[0][a] - 1, oy = L.n0[1][b] - 1;
    const unsigned org = (unsigned)g.idx(x0 + ox, y0 + oy, 0) * SZ;   // window origin (bytes)
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        (void *)(in + (long long)K * g.plane), (short)0, (int)plane_b, MSL_RSRC_WORD3);
    const int soff = (int)(org & ~3u);
#pragma unroll
    for (int m = 0; m < M; ++m)
      if ((m + 1) * 256 <= CP || lane + 64 * (w + 4 * m) < CP)   // chunk of the window
        __builtin_amdgcn_raw_ptr_buffer_load_lds(
            rs, (msl_lds_t *)(sm + K * PD + 256 * (w + 4 * m)), 16, (int)voff[m], soff, 0, 0);
  };
  msl_for_planes<NP>(issue);
  // band conversion tables of the other set, staged in LDS while the windows
  // load (uniform reads later, no scalar-load round trips in the epilogue):
  // lifting: the Hermite basis of the high-order nodes (NO x NO), the per-axis
  // completion matrices (NO x N, x then y), the reciprocal storage scales
  // (NO^2); projection: the low-order basis at the high-order nodes (NO x N),
  // the reciprocal scales
  if constexpr (NO > 0) {
    const LatTab &LO = tab->lat[LIFT ? 1 : 0];
    const int t = threadIdx.x;
    if constexpr (LIFT) {
      const bool herm = tab->lift_mode == MSL_LIFT_GRAD_HERMITE;
      if (t < NO * NO) {
        stab[t] = LO.hw[t / NO][t % NO];
      } else if (t < NO * NO + 2 * NO * N) {
        const int k = t - NO * NO, ax = k / (NO * N), e = k % (NO * N);
        stab[t] = herm ? tab->KH[e / N][e % N] : tab->K[ax][e / N][e % N];
      } else if (t < NTAB) {
        stab[t] = LO.isc[t - NO * NO - 2 * NO * N];
      }
    } else {
      if (t < NO * N) stab[t] = tab->P[t / N][t % N];
      else if (t < NTAB) stab[t] = LO.isc[t - NO * N];
    }
  }
  // my cells: inside the domain and of this velocity set; band: also
  // converted into the other set
  bool mine[R], band[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int x = x0 + tx, y = y0 + ty * R + r;
    const bool inside = x < g.nx && y < g.ny;
    const uint8_t cb = cls[inside ? (long long)y * g.nx + x : 0];
    mine[r] = inside && (cb & 1) == lat;
    band[r] = NO > 0 && mine[r] && (cb & 2);
  }
  __syncthreads();   // the compiler waits for the loads before the barrier
  // zero-gradient faces (bits of zgm: x low, x high, y low, y high) applied to
  // the staged windows instead of a ghost fill: a ghost takes the value of
  // the edge cell of its row (x faces), then ghost rows copy the edge row,
  // x ghosts included (y faces), the order of the separable ghost passes.
  // Fixed faces keep their stored ghosts.  Only tiles whose windows reach a
  // ghost layer of such a face take part (a uniform condition).
  if (zgm && (((zgm & 1) && x0 < MSL_G) || ((zgm & 2) && x0 + MSL_TX + MSL_G > g.nx) ||
              ((zgm & 4) && y0 < MSL_G) || ((zgm & 8) && y0 + TY + MSL_G > g.ny))) {
    auto origin = [&](int K, int &wx, int &wy, int &boff) {
      const int i = K % Q, a = i % N, b = i / N;
      wx = x0 + L.n0[0][a] - 1;
      wy = y0 + L.n0[1][b] - 1;
      boff = (int)(((unsigned)g.idx(wx, wy, 0) * SZ) & 3u);
    };
    // x ghosts of the rows inside the domain: (plane, window row, ghost column)
    if (zgm & 3) {
      for (int it = threadIdx.x; it < NP * LR * 2 * MSL_G; it += 256) {
        const int K = it / (LR * 2 * MSL_G), rem = it % (LR * 2 * MSL_G);
        const int r = rem / (2 * MSL_G), gc = rem % (2 * MSL_G);
        const int side = gc / MSL_G;
        if (!(zgm & (1 << side))) continue;
        int wx, wy, boff;
        origin(K, wx, wy, boff);
        const int Y = wy + r;
        const int X = side ? g.nx + (gc - MSL_G) : gc - MSL_G;
        const int j = X - wx, js = (side ? g.nx - 1 : 0) - wx;
        if (Y < 0 || Y >= g.ny || j < 0 || j >= MSL_TX + 2) continue;
        char *row = (char *)(sm + K * PD + r * LWD) + boff;
        *(S *)(row + j * SZ) = *(const S *)(row + js * SZ);
      }
      __syncthreads();
    }
    // ghost rows: whole padded rows in 16-byte chunks (a plane's rows share
    // one alignment)
    if (zgm & 12) {
      for (int it = threadIdx.x; it < NP * 2 * MSL_G * CPR; it += 256) {
        const int K = it / (2 * MSL_G * CPR), rem = it % (2 * MSL_G * CPR);
        const int gr = rem / CPR, ch = rem % CPR;
        const int side = gr / MSL_G;
        if (!(zgm & (4 << side))) continue;
        int wx, wy, boff;
        origin(K, wx, wy, boff);
        const int Y = side ? g.ny + (gr - MSL_G) : gr - MSL_G;
        const int r = Y - wy, rs = (side ? g.ny - 1 : 0) - wy;
        if (r < 0 || r >= LR) continue;
        uint4 *dst = (uint4 *)(sm + K * PD + r * LWD) + ch;
        *dst = *((const uint4 *)(sm + K * PD + rs * LWD) + ch);
      }
      __syncthreads();
    }
  }

  // reconstruction of plane K at this thread's R cells (raw storage domain)
  auto recon = [&]<int K>(C (&ft)[R]) {
    constexpr int i = K % Q, a = i % N, b = i / N;
    const int ox = L.n0[0][a] - 1, oy = L.n0[1][b] - 1;
    const unsigned org = (unsigned)g.idx(x0 + ox, y0 + oy, 0) * SZ;
    const char *base = (const char *)(sm + K * PD) + (org & 3u);
    const C wx0 = tsel<C>(L.a[0][a][0], L.af[0][a][0]), wx2 = tsel<C>(L.a[0][a][2], L.af[0][a][2]);
    const C wy0 = tsel<C>(L.a[1][b][0], L.af[1][b][0]), wy2 = tsel<C>(L.a[1][b][2], L.af[1][b][2]);
    const C wx1 = tsel<C>(L.a[0][a][1], L.af[0][a][1]), wy1 = tsel<C>(L.a[1][b][1], L.af[1][b][1]);
    C h[R + 2];
#pragma unroll
    for (int r = 0; r < R + 2; ++r) {
      const char *row = base + (ty * R + r) * LWD * 4 + tx * SZ;
      C v0, v1, v2;
      if constexpr (SZ == 8) {
        v0 = (C)lds_elem_d<S>(row); v1 = (C)lds_elem_d<S>(row + 8); v2 = (C)lds_elem_d<S>(row + 16);
      } else {
        v0 = (C)lds_elem<S>(row); v1 = (C)lds_elem<S>(row + SZ); v2 = (C)lds_elem<S>(row + 2 * SZ);
      }
      // FP32 / FP64: the differenced form, centre weight 1 - w0 - w2 exactly;
      // 16-bit deviations: the three weights (one operation fewer per row on
      // the arithmetic-bound 16-bit path; the difference is below the storage
      // rounding)
      if constexpr (SZ == 2) h[r] = wx0 * v0 + wx1 * v1 + wx2 * v2;
      else h[r] = v1 + wx0 * (v0 - v1) + wx2 * (v2 - v1);
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if constexpr (SZ == 2) ft[r] = wy0 * h[r] + wy1 * h[r + 1] + wy2 * h[r + 2];
      else ft[r] = h[r + 1] + wy0 * (h[r] - h[r + 1]) + wy2 * (h[r + 2] - h[r + 1]);
    }
  };

  const C gsc0 = (C)(tab->gfac * tab->T0);   // g scale over the f scale
  // 2. reconstruction and moments
  C rho[R], jx[R], jy[R], en[R];
#pragma unroll
  for (int r = 0; r < R; ++r) { rho[r] = C(0); jx[r] = C(0); jy[r] = C(0); en[r] = C(0); }
  C ftk[NP][R];   // reconstructed populations (storage domain)
  auto pass1 = [&]<int K>() {
    constexpr int i = K % Q, a = i % N, b = i / N;
    recon.template operator()<K>(ftk[K]);
    const C W = tsel<C>(L.sc[i], L.scf[i]);   // storage scale of f_i
    const C cx = tsel<C>(L.v[0][a], L.vf[0][a]), cy = tsel<C>(L.v[1][b], L.vf[1][b]);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if constexpr (K < Q) {
        const C f = T::dev ? W * (C(1) + ftk[K][r]) : ftk[K][r];
        rho[r] += f;
        jx[r] += cx * f;
        jy[r] += cy * f;
        if (TH) en[r] += C(0.5) * (cx * cx + cy * cy) * f;
      } else {
        en[r] += T::dev ? gsc0 * W * (C(1) + ftk[K][r]) : ftk[K][r];
      }
    }
  };
  msl_for_planes<NP>(pass1);

  // 3. equilibrium factors per cell, in FP64 (no rounding bias in the
  //    equilibrium's mass and momentum), kept in the compute precision
  C Px[R][N], Py[R][N], om[R], gf[R];
  // two-relaxation model: velocity, omega1 - omega2 and the per-axis factors
  // of the quasi-equilibria (without rho) of each cell
  C uxr[QE ? R : 1], uyr[QE ? R : 1], dom[QE ? R : 1];
  C Ax[QE ? R : 1][4][N], Ay[QE ? R : 1][4][N];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const double rd = (double)rho[r], ird = 1.0 / rd;
    const double ux = (double)jx[r] * ird, uy = (double)jy[r] * ird;
    double Tm = 1.0;
    if (TH) Tm = ((double)en[r] - 0.5 * rd * (ux * ux + uy * uy)) / (tab->cv * rd);
    double px[N], py[N];
    eq_axis<double, N>(L, (ux - L.ur[0]) * L.isq, Tm * L.iTr, px);
    eq_axis<double, N>(L, (uy - L.ur[1]) * L.isq, Tm * L.iTr, py);
#pragma unroll
    for (int q = 0; q < N; ++q) {
      Px[r][q] = (C)(px[q] * rd);
      Py[r][q] = (C)py[q];
    }
    om[r] = tsel<C>(tab->omega, tab->omegaf);
    double tl = tab->tau;
    // temperature-dependent viscosity mu = mu_ref (T / T_ref)^s, tau = mu / (rho T dt)
    // + 1/2 (athermal: T = 1, the power is a table constant)
    if (tab->tau_mode == 1) {
      const double mu = TH ? tab->mu_ref * pow(Tm / tab->tau_ref_T, tab->mu_exp) : tab->mu_T1;
      tl = mu / (rd * Tm * tab->dt) + 0.5;
      om[r] = (C)(1.0 / tl);
    }
    gf[r] = (C)(tab->gfac * Tm);
    if constexpr (QE) {
      uxr[r] = (C)ux;
      uyr[r] = (C)uy;
      dom[r] = (C)(1.0 / tl - 1.0 / (0.5 + (tl - 0.5) * tab->qe_ratio));
      qe_axis<C, N>(L, (ux - L.ur[0]) * L.isq, Tm * L.iTr, Ax[r]);
      qe_axis<C, N>(L, (uy - L.ur[1]) * L.isq, Tm * L.iTr, Ay[r]);
    }
  }
  // two-relaxation model (eqs. Pond_f/g with the quasi-equilibria of eqs. fqeq,
  // gqeq in the run's frame): the non-equilibrium third central moment Qbar and
  // heat flux qbar of each cell, folded with (omega1 - omega2) and the
  // constants of f* - f^eq = T_ref^{-3/2}/6 sum_{|k|=3} mult(k) Qbar_k prod A^(k),
  // g* - g^eq = T_ref^{-1/2} sum_a qbar_a A^(1)_a prod A^(0)
  C Qb[QE ? R : 1][4], qb[QE ? R : 1][2];
  if constexpr (QE) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      Qb[r][0] = Qb[r][1] = Qb[r][2] = Qb[r][3] = C(0);
      qb[r][0] = qb[r][1] = C(0);
    }
    auto qacc = [&]<int K>() {
      constexpr int i = K % Q, a = i % N, b = i / N;
      const C W = tsel<C>(L.sc[i], L.scf[i]);
      const C sc = K < Q ? W : gsc0 * W;
      const C cx = tsel<C>(L.v[0][a], L.vf[0][a]), cy = tsel<C>(L.v[1][b], L.vf[1][b]);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const C feq = Px[r][a] * Py[r][b];
        const C v = T::dev ? sc * (C(1) + ftk[K][r]) : ftk[K][r];
        const C dx = cx - uxr[r], dy = cy - uyr[r];
        if constexpr (K < Q) {
          const C nf = v - feq;
          Qb[r][0] += dx * dx * dx * nf;
          Qb[r][1] += dx * dx * dy * nf;
          Qb[r][2] += dx * dy * dy * nf;
          Qb[r][3] += dy * dy * dy * nf;
        } else {
          const C ng = v - gf[r] * feq;
          qb[r][0] += dx * ng;
          qb[r][1] += dy * ng;
        }
      }
    };
    msl_for_planes<NP>(qacc);
    const C cf = (C)(L.isq * L.isq * L.isq / 6.0), cg = (C)L.isq;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      Qb[r][0] *= dom[r] * cf;
      Qb[r][1] *= dom[r] * C(3) * cf;
      Qb[r][2] *= dom[r] * C(3) * cf;
      Qb[r][3] *= dom[r] * cf;
      qb[r][0] *= dom[r] * cg;
      qb[r][1] *= dom[r] * cg;
    }
  }
  // band conversion state: lifting keeps the non-equilibrium part of every
  // post-collision population (f - f^eq, g - gfac T f^eq); projection
  // accumulates (P x P) f of each output node while the populations are
  // stored (only in waves that hold a band cell).  The conversions compute in
  // FP64 whatever the storage precision.
  C nq[LIFT ? NP : 1][R];
  double acc[PROJ ? (TH ? 2 : 1) * QO : 1][R];   // (P x P) f per output node
  double tp[PROJ ? NO : 1][R];                   // P along x of the current row
  double Pp[PROJ ? NO : 1][PROJ ? N : 1];        // P[a'][a], from LDS
  bool wband = false;
  if constexpr (NO > 0) {
    bool b = false;
#pragma unroll
    for (int r = 0; r < R; ++r) b |= band[r];
    wband = __any(b);
  }
  if constexpr (PROJ) {
#pragma unroll
    for (int k = 0; k < (TH ? 2 : 1) * QO; ++k)
#pragma unroll
      for (int r = 0; r < R; ++r) acc[k][r] = 0.0;
#pragma unroll
    for (int k = 0; k < NO; ++k)
#pragma unroll
      for (int r = 0; r < R; ++r) tp[k][r] = 0.0;
    if (wband) {
#pragma unroll
      for (int ap = 0; ap < NO; ++ap)
#pragma unroll
        for (int a = 0; a < N; ++a) Pp[ap][a] = stab[ap * N + a];
    }
  }
  // 4. collide and store
  unsigned soff_cell[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int x = x0 + tx, y = y0 + ty * R + r;
    soff_cell[r] = mine[r] ? (unsigned)g.idx(x, y, 0) * SZ : 0x80000000u;
  }
  auto pass2 = [&]<int K>() {
    constexpr int i = K % Q, a = i % N, b = i / N;
    const C W = tsel<C>(L.sc[i], L.scf[i]);
    // decoded scale of a 16-bit deviation and its reciprocal (one per plane)
    const C sc = K < Q ? W : gsc0 * W;
    const C isc = T::dev ? tsel<C>(L.isc[i], L.iscf[i]) * (K < Q ? C(1) : tsel<C>(tab->igsc, tab->igscf)) : C(1);
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        (void *)(out + (long long)K * g.plane), (short)0, (int)plane_b, MSL_RSRC_WORD3);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const C feq = Px[r][a] * Py[r][b];
      const C v = T::dev ? sc * (C(1) + ftk[K][r]) : ftk[K][r];
      C vo;
      if constexpr (K < Q) vo = v + om[r] * (feq - v);
      else vo = v + om[r] * (gf[r] * feq - v);
      if constexpr (QE) {
        if constexpr (K < Q)
          vo += Qb[r][0] * Ax[r][3][a] * Ay[r][0][b] + Qb[r][1] * Ax[r][2][a] * Ay[r][1][b] +
                Qb[r][2] * Ax[r][1][a] * Ay[r][2][b] + Qb[r][3] * Ax[r][0][a] * Ay[r][3][b];
        else
          vo += qb[r][0] * Ax[r][1][a] * Ay[r][0][b] + qb[r][1] * Ax[r][0][a] * Ay[r][1][b];
      }
      if constexpr (LIFT) nq[K][r] = vo - (K < Q ? feq : gf[r] * feq);
      if constexpr (PROJ) {
        // separable: along x within the row b, then along y at its end
        if (wband) {
          const double vd = (double)vo;
#pragma unroll
          for (int ap = 0; ap < NO; ++ap) tp[ap][r] += Pp[ap][a] * vd;
          if constexpr (a == N - 1) {
#pragma unroll
            for (int bp = 0; bp < NO; ++bp)
#pragma unroll
              for (int ap = 0; ap < NO; ++ap)
                acc[(K < Q ? 0 : QO) + ap + NO * bp][r] += Pp[bp][b] * tp[ap][r];
#pragma unroll
            for (int ap = 0; ap < NO; ++ap) tp[ap][r] = 0.0;
          }
        }
      }
      const C o = T::dev ? vo * isc - C(1) : vo;
      const S sv = T::store(o);
      // nt: non-temporal stores (cache policy bit 1) when the output buffer is
      // far larger than the caches and is read back only in the next step
      // (D2Q9 in FP32 / FP64 on large grids; the test is compiled out elsewhere)
      constexpr bool NTOK = N == 3 && !SMALL && SZ >= 4;
      if constexpr (SZ == 8) {
        typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
        if (NTOK && nt) __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, sv), rs, (int)soff_cell[r], 0, 2);
        else __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, sv), rs, (int)soff_cell[r], 0, 0);
      } else if constexpr (SZ == 4) {
        if (NTOK && nt) __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, sv), rs, (int)soff_cell[r], 0, 2);
        else __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, sv), rs, (int)soff_cell[r], 0, 0);
      } else {
        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(uint16_t, sv), rs, (int)soff_cell[r], 0, 0);
      }
    }
  };
  msl_for_planes<NP>(pass2);
  // 5. band cells into the other set (Sec. III.B-C, App. C): lifting
  //    f_Q = f^eq_Q + (Kx x Ky)(f_q - f^eq_q) at the cell's rho, u, T (the
  //    collision conserves them), projection f_q = (P x P) f_Q
  if constexpr (NO > 0) {
    if (wband) {
      const LatTab &LO = tab->lat[LIFT ? 1 : 0];
      const double igs = tab->igsc;
      const double *isct = stab + (LIFT ? NO * NO + 2 * NO * N : NO * N);   // 1 / storage scales
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if constexpr (LIFT) {
          if (!__ballot(band[r])) continue;
        } else {
          if (!band[r]) continue;
        }
        // buffer stores: the plane's base in scalar registers, one 32-bit
        // byte offset per lane (a 64-bit address per store would not fit in
        // the registers of an eight-wave launch)
        const int cidx = (int)g.idx(x0 + tx, y0 + ty * R + r, 0);
        const int boff = (int)((unsigned)cidx * SZ);
        auto put = [&](const int k, const double v, const double is) {
          const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
              (void *)(oth + (long long)k * g.plane), (short)0, (int)plane_b, MSL_RSRC_WORD3);
          const S sv = T::store(T::dev ? (C)(v * is - 1.0) : (C)v);
          if constexpr (SZ == 8) {
            typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
            __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, sv), rs, boff, 0, 0);
          } else if constexpr (SZ == 4) {
            __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, sv), rs, boff, 0, 0);
          } else {
            __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(uint16_t, sv), rs, boff, 0, 0);
          }
        };
        if constexpr (LIFT) {
          // every lane widens its cell's moments (only band lanes' are used)
          const double rd = (double)rho[r], ux = (double)jx[r] / rd, uy = (double)jy[r] / rd;
          double Tm = 1.0;
          if (TH) Tm = ((double)en[r] - 0.5 * rd * (ux * ux + uy * uy)) / (tab->cv * rd);
          const double tm1 = Tm * LO.iTr - 1.0;
          const double uxs = (ux - LO.ur[0]) * LO.isq, uys = (uy - LO.ur[1]) * LO.isq;
          unsigned long long bmask = __ballot(band[r]);
          if (__popcll(bmask) <= MSL_LIFT_COOP) {
            // few band cells in the wave: the wave lifts them one at a time,
            // lane i computing output node i (its Hermite factors and the
            // separable completion at that node), with the cell's moments
            // and non-equilibrium populations read from its lane
            while (bmask) {
              const int src = __builtin_ctzll(bmask);
              bmask &= bmask - 1;
              const double crd = msl_lane_get(rd, src), cux = msl_lane_get(uxs, src);
              const double cuy = msl_lane_get(uys, src), ctm = msl_lane_get(tm1, src);
              const double cT = TH ? msl_lane_get(Tm, src) : 1.0;
              const long long cid = (long long)__builtin_amdgcn_readlane(cidx, src);
              C cq[TH ? 2 * Q : Q];
#pragma unroll
              for (int k = 0; k < (TH ? 2 * Q : Q); ++k) cq[k] = msl_lane_get(nq[k][r], src);
              if (lane < QO) {
                const int a = lane % NO, b = lane / NO;
                double px = stab[a * NO], py = stab[b * NO];
                double xm = 1.0, xj = cux, ym = 1.0, yj = cuy;
#pragma unroll
                for (int j = 1; j < NO; ++j) {
                  px += stab[a * NO + j] * xj;
                  py += stab[b * NO + j] * yj;
                  const double xn = cux * xj + (double)j * ctm * xm;
                  const double yn = cuy * yj + (double)j * ctm * ym;
                  xm = xj;
                  xj = xn;
                  ym = yj;
                  yj = yn;
                }
                const double feq = crd * px * py;
#pragma unroll
                for (int h = 0; h < (TH ? 2 : 1); ++h) {
                  double cr = 0.0;
#pragma unroll
                  for (int bp = 0; bp < N; ++bp) {
                    double t = 0.0;
#pragma unroll
                    for (int ap = 0; ap < N; ++ap) t += stab[NO * NO + a * N + ap] * (double)cq[h * Q + ap + N * bp];
                    cr += stab[NO * NO + NO * N + b * N + bp] * t;
                  }
                  const double v = (h ? tab->gfac * cT : 1.0) * feq + cr;
                  const double is = h ? igs * isct[lane] : isct[lane];
                  oth[(long long)(h * QO + lane) * g.plane + cid] = T::store(T::dev ? (C)(v * is - 1.0) : (C)v);
                }
              }
            }
            continue;
          }
          if (!band[r]) continue;
          // many band cells: each lane lifts its own.  Equilibrium factors
          // of the high-order nodes (eq_axis with the basis from LDS): all of
          // y here, x per output column below (its Hermite coefficients
          // recomputed there: fewer values live)
          double PY[NO];
          {
            double by[NO];
            by[0] = 1.0;
            by[1] = uys;
#pragma unroll
            for (int j = 1; j + 1 < NO; ++j) by[j + 1] = uys * by[j] + (double)j * tm1 * by[j - 1];
#pragma unroll
            for (int b = 0; b < NO; ++b) {
              double sy = 0.0;
#pragma unroll
              for (int j = 0; j < NO; ++j) sy += stab[b * NO + j] * by[j];
              PY[b] = sy;
            }
          }
          // one output column a at a time (not unrolled: a few values live).
          // The tables come from the uniform table memory (scalar loads into
          // scalar registers, the same for every lane: no LDS round trips in
          // the loop), the populations are widened inside the loop (an empty
          // statement tied to the column index keeps the conversion there:
          // hoisted, the FP64 copies would exceed the registers of an
          // eight-wave launch and spill)
          const bool herm = tab->lift_mode == MSL_LIFT_GRAD_HERMITE;
          const double *KxT = herm ? &tab->KH[0][0] : &tab->K[0][0][0];
          const double *KyT = herm ? &tab->KH[0][0] : &tab->K[1][0][0];
#pragma unroll 1
          for (int a = 0; a < NO; ++a) {
            double px = LO.hw[a][0], bm = 1.0, bj = uxs;
#pragma unroll
            for (int j = 1; j < NO; ++j) {
              px += LO.hw[a][j] * bj;
              const double bn = uxs * bj + (double)j * tm1 * bm;
              bm = bj;
              bj = bn;
            }
            px *= rd;
#pragma unroll
            for (int h = 0; h < (TH ? 2 : 1); ++h) {
              const double sg = h ? tab->gfac * Tm : 1.0;
              double t[N];
#pragma unroll
              for (int bp = 0; bp < N; ++bp) {
                double sum = 0.0;
#pragma unroll
                for (int ap = 0; ap < N; ++ap) {
                  C q = nq[h * Q + ap + N * bp][r];
                  asm("" : "+v"(q) : "s"(a));
                  sum += KxT[a * MSL_MAXN + ap] * (double)q;
                }
                t[bp] = sum;
              }
#pragma unroll
              for (int b = 0; b < NO; ++b) {
                double cr = 0.0;
#pragma unroll
                for (int bp = 0; bp < N; ++bp) cr += KyT[b * MSL_MAXN + bp] * t[bp];
                const int i = a + NO * b;
                put(h * QO + i, sg * px * PY[b] + cr, h ? igs * isct[i] : isct[i]);
              }
            }
          }
        } else {
#pragma unroll
          for (int h = 0; h < (TH ? 2 : 1); ++h)
#pragma unroll
            for (int i = 0; i < QO; ++i)
              put(h * QO + i, acc[h * QO + i][r], h ? igs * isct[i] : isct[i]);
        }
      }
    }
  }
  };
  if constexpr (LIST) {
    // sparse launch: one workgroup per entry of the compact list of live
    // tiles (ascending tile order), so no workgroup is spent on a tile
    // without cells of this set; the XCD-aware order over the list gives
    // each XCD a contiguous run of it (vertically adjacent tiles, whose
    // windows overlap, share that XCD's L2)
    const int n = *tcount;
    if ((int)blockIdx.x < n) {
      const int tile = tlist[msl_xcd_tile((int)blockIdx.x, n)];
      tile_body(tile % g.ntx, tile / g.ntx);
    }
  } else {
    // dense launches take the XCD-aware tile order; the others the linear
    // order, which spreads their active tiles over all XCDs
    const int lin = (int)(blockIdx.y * gridDim.x + blockIdx.x);
    const int tile = remap ? msl_xcd_tile(lin, (int)(gridDim.x * gridDim.y)) : lin;
    tile_body(tile % (int)gridDim.x, tile / (int)gridDim.x);
  }
}
