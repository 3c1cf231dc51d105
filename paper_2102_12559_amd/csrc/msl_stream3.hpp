// msl_stream3.hpp -- the 3D stream-and-collide kernel: population planes
// streamed through LDS in chunks, the reconstructed values held in registers.
//
// A workgroup owns 64 x 4 x RZ cells, RZ cells per lane along z (2 for D3Q27,
// 1 for D3Q64).  The planes
// (f_0..f_{Q-1}, then g_0..g_{Q-1}) are taken CH at a time: direct-to-LDS
// buffer loads of every plane's 66 x 6 x (RZ + 2) window around the departure points
// of the tile (the departure offset x - c_i dt is the same for every cell of a
// plane), one wait and barrier, the separable 3-point Lagrange reconstruction
// (eq. reconstructionPond: along x on nine rows, then y, then z) of each
// lane's cell into registers, and a barrier before the chunk's LDS is reused.
// After the last chunk every lane holds all its reconstructed populations:
// moments, FP64 equilibrium factors, BGK relaxation (eqs. Pond_f/g, feqL,
// geqL) and buffer stores whose out-of-range offset drops the writes of
// foreign or outside cells.  Several workgroups per CU overlap one another's
// loads and arithmetic.
#pragma once
#include <utility>

#include "msl_device.hpp"
#include "msl_stream2.hpp"

template <typename S, bool TH, int N>
struct SC3Traits {
  using T = StoreTraits<S>;
  using C = typename T::C;
  static constexpr int Q = N * N * N;
  static constexpr int NP = TH ? 2 * Q : Q;
  static constexpr int SZ = (int)sizeof(S);
  static constexpr int LWD = (66 * SZ + 3) / 4 + (SZ < 4 ? 1 : 0);   // dwords per window row
  // z cells per lane: a D3Q27 tile is 64 x 4 x RZ cells, whose window's
  // RZ + 2 z slabs serve RZ cells (a 64 x 4 x 1 tile reads three slabs for
  // one cell); RZ = 3 for 16-bit storage, 4 for FP32, 2 for FP64 (measured
  // on the 256^3 run; the register budget bounds it), and 2 (1 in FP64) with
  // the g populations.  D3Q64: two cells per lane in FP32, one otherwise
  // (measured; with 16-bit storage the extra registers cost more than the
  // saved reads).
  static constexpr int RZ = N != 3 ? (!TH && SZ == 4 ? 2 : 1) : TH ? (SZ == 8 ? 1 : 2) : (SZ == 2 ? 3 : (SZ == 4 ? 4 : 2));
  static constexpr int ROWS = 6 * (RZ + 2);                           // (4 + 2) y rows x (RZ + 2) z slabs
  static constexpr int PD = (ROWS * LWD + 255) / 256 * 256;           // dwords per plane window
  static constexpr int M = PD / 256;                                  // DMA instructions per wave
  // LDS budget of a chunk: 24 KB for D3Q27, 40 KB for D3Q64 (measured on the
  // 256^3 run; D3Q27 with two cells per lane is insensitive to 24-48 KB)
  static constexpr int BUDGET = (N == 3 ? 24 : 40) * 1024;
  static constexpr int CHMAX = BUDGET / (PD * 4) < 1 ? 1 : BUDGET / (PD * 4);
  static constexpr int NCH = (NP + CHMAX - 1) / CHMAX;                // chunks
  static constexpr int CH = (NP + NCH - 1) / NCH;                     // planes per chunk
  static constexpr int LDS_BYTES = CH * PD * 4;
  static constexpr int REGW = SZ == 8 ? 2 : 1;
  static constexpr int VREG = NP * REGW * RZ + 80;
  static constexpr int WG_LDS = (160 * 1024) / LDS_BYTES;
  static constexpr int W_REG = 512 / VREG;
  static constexpr int WAVES0 = WG_LDS < W_REG ? WG_LDS : W_REG;
  static constexpr int WAVES = WAVES0 > 8 ? 8 : (WAVES0 < 1 ? 1 : WAVES0);
};

template <int K0, int K1, typename F>
__device__ __forceinline__ void msl_for_range(F &&f) {
  [&]<int... Ks>(std::integer_sequence<int, Ks...>) {
    (f.template operator()<K0 + Ks>(), ...);
  }(std::make_integer_sequence<int, K1 - K0>{});
}

template <typename S, bool TH, int N, bool LIST = false>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(SC3Traits<S, TH, N>::WAVES)))
k_sc3d_res(const Tab *__restrict__ tab, int lat, Geo g, const S *__restrict__ in,
           S *__restrict__ out, const uint8_t *__restrict__ cls,
           const uint8_t *__restrict__ tflag, int remap, int xmir, const int *__restrict__ tlist,
           const int *__restrict__ tcount) {
  using Tr = SC3Traits<S, TH, N>;
  using T = typename Tr::T;
  using C = typename Tr::C;
  constexpr int Q = Tr::Q, NP = Tr::NP, PD = Tr::PD, M = Tr::M, CH = Tr::CH, NCH = Tr::NCH;
  constexpr int LWD = Tr::LWD, SZ = Tr::SZ, ROWS = Tr::ROWS, RZ = Tr::RZ;
  __shared__ uint32_t sm[CH * PD];
  const LatTab &L = tab->lat[lat];
  // the tile: from the grid (XCD-aware order for dense launches), or (LIST:
  // sparse launches on large grids) one workgroup per entry of the compact
  // list of live tiles, in XCD-aware order over the list
  int tile;
  if constexpr (LIST) {
    const int n = *tcount;
    if ((int)blockIdx.x >= n) return;
    tile = tlist[msl_xcd_tile((int)blockIdx.x, n)];
  } else {
    const int lin = (int)((blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x);
    tile = remap ? msl_xcd_tile(lin, (int)(gridDim.x * gridDim.y * gridDim.z)) : lin;
  }
  const int bx = tile % g.ntx, by = (tile / g.ntx) % g.nty;
  const int z0 = tile / (g.ntx * g.nty) * RZ;
  const int x0 = bx * MSL_TX, y0 = by * MSL_MTY;
  {
    uint8_t any = 0;
#pragma unroll
    for (int rz = 0; rz < RZ; ++rz)
      if (z0 + rz < g.nz) any |= tflag[((long long)(z0 + rz) * g.nty + by) * g.ntx + bx];
    if (!(any & (1 << lat))) return;
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const unsigned pitch_b = (unsigned)g.pitch * SZ;
  const unsigned plane_b = (unsigned)g.plane * SZ;
  // plane-independent byte offsets of this lane's window dwords
  unsigned voff[M];
#pragma unroll
  for (int m = 0; m < M; ++m) {
    int d = lane + 64 * (w + 4 * m);
    d = d < ROWS * LWD ? d : ROWS * LWD - 1;
    const int row = d / LWD, col = d - row * LWD;
    const int rz = row / 6, ry = row - 6 * rz;
    voff[m] = ((unsigned)rz * (unsigned)g.rows + (unsigned)ry) * pitch_b + (unsigned)col * 4u;
  }
  const int x = x0 + lane, y = y0 + w;
  bool mine[RZ];
#pragma unroll
  for (int rz = 0; rz < RZ; ++rz) {
    const int z = z0 + rz;
    const bool inside = x < g.nx && y < g.ny && z < g.nz;
    mine[rz] = inside && (cls[inside ? ((long long)z * g.ny + y) * g.nx + x : 0] & 1) == lat;
  }

  // per-node tables of each axis: interpolation weights and the window offset
  // of the departure stencil
  C wlo[3][N], wmid[3][N], whi[3][N];
  int offx[N], offy[N], offz[N];
#pragma unroll
  for (int a = 0; a < N; ++a) {
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      wlo[ax][a] = tsel<C>(L.a[ax][a][0], L.af[ax][a][0]);
      wmid[ax][a] = tsel<C>(L.a[ax][a][1], L.af[ax][a][1]);
      whi[ax][a] = tsel<C>(L.a[ax][a][2], L.af[ax][a][2]);
    }
    offx[a] = L.n0[0][a] - 1;
    offy[a] = (L.n0[1][a] - 1) * g.pitch;
    offz[a] = (L.n0[2][a] - 1) * g.rows * g.pitch;
  }
  const int org0 = g.idx(x0, y0, z0);
  // DMA of planes [k0, k1) into the chunk's LDS (a scalar loop: plane k's
  // window origin and buffer descriptor are computed when it is issued)
  auto issue = [&](int k0, int k1) {
#pragma unroll 1
    for (int k = k0; k < k1; ++k) {
      const int i = k % Q, a = i % N, b = (i / N) % N, cc = i / (N * N);
      const unsigned org =
          (unsigned)(org0 + (L.n0[0][a] - 1) + (L.n0[1][b] - 1) * g.pitch + (L.n0[2][cc] - 1) * g.rows * g.pitch) *
          SZ;
      const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
          (void *)(in + (long long)k * g.plane), (short)0, (int)plane_b, MSL_RSRC_WORD3);
#pragma unroll
      for (int m = 0; m < M; ++m)
        __builtin_amdgcn_raw_ptr_buffer_load_lds(
            rs, (msl_lds_t *)(sm + (k - k0) * PD + 64 * (w + 4 * m)), 4, (int)voff[m],
            (int)(org & ~3u), 0, 0);
    }
  };
  C ftk[NP][RZ];   // reconstructed populations (storage domain)
  auto recon = [&]<int K>() {
    constexpr int i = K % Q, a = i % N, b = (i / N) % N, cc = i / (N * N);
    const unsigned org = (unsigned)(org0 + offx[a] + offy[b] + offz[cc]) * SZ;
    // an opaque window address per plane: the loads of different planes are
    // neither merged nor hoisted together, so one plane's values are live at a time
    unsigned lofs = (unsigned)((K % CH) * PD * 4) + (org & 3u) + (unsigned)(lane * SZ);
    asm volatile("" : "+v"(lofs));
    const char *base = (const char *)sm + lofs;
    const C wx0 = wlo[0][a], wx2 = whi[0][a], wy0 = wlo[1][b], wy2 = whi[1][b], wz0 = wlo[2][cc],
            wz2 = whi[2][cc];
    C hz[RZ + 2];   // x- then y-interpolated values of the window's z slabs
#pragma unroll
    for (int dz = 0; dz < RZ + 2; ++dz) {
      C hy[3];
#pragma unroll
      for (int dy = 0; dy < 3; ++dy) {
        const char *row = base + (6 * dz + w + dy) * LWD * 4;
        C v0, v1, v2;
        if constexpr (SZ == 8) {
          v0 = (C)lds_elem_d<S>(row); v1 = (C)lds_elem_d<S>(row + 8); v2 = (C)lds_elem_d<S>(row + 16);
        } else {
          v0 = (C)lds_elem<S>(row); v1 = (C)lds_elem<S>(row + SZ); v2 = (C)lds_elem<S>(row + 2 * SZ);
        }
        // FP32 / FP64: differenced form, centre weight 1 - w0 - w2 exactly;
        // 16-bit deviations: the three weights (one operation fewer)
        if constexpr (SZ == 2) hy[dy] = wx0 * v0 + wmid[0][a] * v1 + wx2 * v2;
        else hy[dy] = v1 + wx0 * (v0 - v1) + wx2 * (v2 - v1);
      }
      if constexpr (SZ == 2) hz[dz] = wy0 * hy[0] + wmid[1][b] * hy[1] + wy2 * hy[2];
      else hz[dz] = hy[1] + wy0 * (hy[0] - hy[1]) + wy2 * (hy[2] - hy[1]);
    }
#pragma unroll
    for (int rz = 0; rz < RZ; ++rz) {
      if constexpr (SZ == 2) ftk[K][rz] = wz0 * hz[rz] + wmid[2][cc] * hz[rz + 1] + wz2 * hz[rz + 2];
      else ftk[K][rz] = hz[rz + 1] + wz0 * (hz[rz] - hz[rz + 1]) + wz2 * (hz[rz + 2] - hz[rz + 1]);
      // the value is final here: without this the interpolation would be sunk
      // to its first use after the last chunk, keeping every window value of
      // every plane alive until then
      asm volatile("" : "+v"(ftk[K][rz]));
    }
  };
  auto chunk = [&]<int CI>() {
    constexpr int k0 = CI * CH, k1 = k0 + CH < NP ? k0 + CH : NP;
    issue(k0, k1);
    __syncthreads();   // the compiler waits for the loads before the barrier
    msl_for_range<k0, k1>(recon);
    __syncthreads();   // the chunk's LDS is reused by the next chunk
  };
  msl_for_planes<NCH>(chunk);

  const C gsc0 = (C)(tab->gfac * tab->T0);   // g scale over the f scale
  // periodic x (xmir, nx >= 4): the cells x < 2 and x >= nx - 2 are also
  // stored into the ghost columns of the other side, which the next step's
  // windows read; only the tiles at the two x ends take the second store
  const bool xedge = xmir && (x0 < MSL_G || x0 + MSL_TX > g.nx - MSL_G);
  // moments, equilibrium, collision and stores of the lane's cell z0 + rz
  auto finish = [&]<int rz>() {
  const int z = z0 + rz;
  // moments (Sec. II.B)
  C rho = C(0), jx = C(0), jy = C(0), jz = C(0), en = C(0);
  auto moments = [&]<int K>() {
    constexpr int i = K % Q, a = i % N, b = (i / N) % N, cc = i / (N * N);
    const C W = tsel<C>(L.sc[i], L.scf[i]);   // storage scale of f_i
    if constexpr (K < Q) {
      const C cx = tsel<C>(L.v[0][a], L.vf[0][a]), cy = tsel<C>(L.v[1][b], L.vf[1][b]),
              cz = tsel<C>(L.v[2][cc], L.vf[2][cc]);
      const C f = T::dev ? W * (C(1) + ftk[K][rz]) : ftk[K][rz];
      rho += f;
      jx += cx * f;
      jy += cy * f;
      jz += cz * f;
      if (TH) en += C(0.5) * (cx * cx + cy * cy + cz * cz) * f;
    } else {
      en += T::dev ? gsc0 * W * (C(1) + ftk[K][rz]) : ftk[K][rz];
    }
  };
  msl_for_planes<NP>(moments);
  // equilibrium factors in FP64 (no rounding bias in the equilibrium's mass
  // and momentum), kept in the compute precision
  const double rd = (double)rho, ird = 1.0 / rd;
  const double ux = (double)jx * ird, uy = (double)jy * ird, uz = (double)jz * ird;
  double Tm = 1.0;
  if (TH) Tm = ((double)en - 0.5 * rd * (ux * ux + uy * uy + uz * uz)) / (tab->cv * rd);
  C om = tsel<C>(tab->omega, tab->omegaf);
  if (tab->tau_mode == 1) {
    const double mu = TH ? tab->mu_ref * pow(Tm / tab->tau_ref_T, tab->mu_exp) : tab->mu_T1;
    om = (C)(1.0 / (mu / (rd * Tm * tab->dt) + 0.5));
  }
  C Px[N], Py[N], Pz[N];
  {
    double px[N], py[N], pz[N];
    eq_axis<double, N>(L, (ux - L.ur[0]) * L.isq, Tm * L.iTr, px);
    eq_axis<double, N>(L, (uy - L.ur[1]) * L.isq, Tm * L.iTr, py);
    eq_axis<double, N>(L, (uz - L.ur[2]) * L.isq, Tm * L.iTr, pz);
#pragma unroll
    for (int q = 0; q < N; ++q) {
      Px[q] = (C)(px[q] * rd);
      Py[q] = (C)py[q];
      Pz[q] = (C)pz[q];
    }
  }
  const C gf = (C)(tab->gfac * Tm);
  const unsigned soff = mine[rz] ? (unsigned)g.idx(x, y, z) * SZ : 0x80000000u;
  const unsigned ioff = (mine[rz] && x < MSL_G) ? soff + (unsigned)g.nx * SZ
                        : (mine[rz] && x >= g.nx - MSL_G) ? soff - (unsigned)g.nx * SZ : 0x80000000u;
  // collide and store
  auto store = [&]<int K>() {
    constexpr int i = K % Q, a = i % N, b = (i / N) % N, cc = i / (N * N);
    const C W = tsel<C>(L.sc[i], L.scf[i]);
    const C sc = K < Q ? W : gsc0 * W;
    const C isc = T::dev ? tsel<C>(L.isc[i], L.iscf[i]) * (K < Q ? C(1) : tsel<C>(tab->igsc, tab->igscf)) : C(1);
    const C feq = Px[a] * Py[b] * Pz[cc];
    const C v = T::dev ? sc * (C(1) + ftk[K][rz]) : ftk[K][rz];
    C vo;
    if constexpr (K < Q) vo = v + om * (feq - v);
    else vo = v + om * (gf * feq - v);
    const S sv = T::store(T::dev ? vo * isc - C(1) : vo);
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        (void *)(out + (long long)K * g.plane), (short)0, (int)plane_b, MSL_RSRC_WORD3);
    auto put = [&](unsigned o) {
      if constexpr (SZ == 8) {
        typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, sv), rs, (int)o, 0, 0);
      } else if constexpr (SZ == 4) {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, sv), rs, (int)o, 0, 0);
      } else {
        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(uint16_t, sv), rs, (int)o, 0, 0);
      }
    };
    put(soff);
    if (xedge) put(ioff);
  };
  msl_for_planes<NP>(store);
  };
  msl_for_planes<RZ>(finish);
}
