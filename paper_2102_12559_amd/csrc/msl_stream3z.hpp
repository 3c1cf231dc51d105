// msl_stream3z.hpp -- the 3D stream-and-collide kernel that marches along z.
//
// A workgroup owns a column of 64 x 4 x ZC cells (one y row per wave, one x
// cell per lane; 16-bit D3Q64: four waves per row, each with the planes of
// one z node) and walks it from its lowest z cell upwards.  At each step
// of the walk it brings one z slab of every plane's departure window into
// LDS (direct-to-LDS buffer loads of 6 rows x 66 cells: the departure offset
// x - v_i dt is the same for every cell of a plane, so the slab is the
// column's cross-section shifted by the plane's base offset), interpolates
// the slab along x and y (eq. reconstructionPond, 3-point Lagrange weights),
// and combines it with the two slabs before it, which each lane keeps in
// registers, into the population streamed to its cell (the z interpolation).
// Every slab of a column's window is read once per column instead of once
// per group of z cells, and each lane reconstructs one new slab per
// population and step instead of all three.  The cell then collides in
// registers: moments, FP64 equilibrium factors in the run's frame, BGK
// relaxation (eqs. Pond_f/g, feqL, geqL) and buffer stores whose
// out-of-range offset drops the writes of foreign or outside cells.  The
// loads of the next slab are issued before the collision, so they are in
// flight while it runs.
//
// Each lane holds three values per population (two partial sums or slabs and
// the streamed value), so the kernel serves the velocity sets whose planes fit
// the register file: athermal D3Q27 in 16-bit and FP32 storage (three waves
// per SIMD) and athermal D3Q64 in 16-bit storage (one wave per SIMD).  The
// others use the chunked kernel of msl_stream3.hpp.
#pragma once
#include <utility>

#include "msl_stream3.hpp"

// s_waitcnt for the vector memory counter only (gfx9 encoding: vmcnt in bits
// 3:0 and 15:14, expcnt 6:4 and lgkmcnt 11:8 left at their maxima): wait until
// at most NV vector memory operations of this wave are outstanding
template <int NV>
__device__ __forceinline__ void msl_wait_vm() {
  static_assert(NV >= 0 && NV <= 63, "vmcnt is a 6-bit field");
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_waitcnt((NV & 15) | (7 << 4) | (15 << 8) | ((NV >> 4) << 14));
  asm volatile("" ::: "memory");
}

// workgroup barrier for LDS traffic only: this wave's LDS reads have returned
// (lgkmcnt 0) and no memory operation moves across it; unlike
// __syncthreads() it does not wait for outstanding global stores
__device__ __forceinline__ void msl_lds_barrier() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_waitcnt(15 | (7 << 4) | (0 << 8) | (3 << 14));
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

// a 16-bit stored element (the low 16 bits of u) as float
template <typename S>
__device__ __forceinline__ float half_elem(uint32_t u);
template <>
__device__ __forceinline__ float half_elem<_Float16>(uint32_t u) {
  return (float)__builtin_bit_cast(_Float16, (uint16_t)u);
}
template <>
__device__ __forceinline__ float half_elem<bf16_t>(uint32_t u) { return __uint_as_float(u << 16); }
template <typename S>
__device__ __forceinline__ float half_elem(uint32_t) { return 0.0f; }

template <typename S, bool TH, int N>
struct SC3ZTraits {
  using T = StoreTraits<S>;
  using C = typename T::C;
  static constexpr int Q = N * N * N;
  static constexpr int NP = TH ? 2 * Q : Q;
  static constexpr int SZ = (int)sizeof(S);
  static constexpr int LWD = (66 * SZ + 3) / 4 + (SZ < 4 ? 1 : 0);   // dwords per window row
  static constexpr int SD = 6 * LWD;                                  // dwords of a plane's slab
  static constexpr int M = (SD + 255) / 256;                          // DMA instructions per wave
  // LDS dwords per plane: 16-bit slabs (204 dwords) are padded to the 256
  // that one DMA instruction of the four waves writes, so that every lane
  // loads (no exec-mask branch per plane and step); FP32 slabs (396 dwords)
  // keep their size, the padding would cost a wave per SIMD of LDS occupancy
  static constexpr bool PAD = SZ == 2;
  static constexpr int SDP = PAD ? M * 256 : SD;
  static constexpr int ZC = 32;                                       // cells per column along z
  static_assert(ZC <= 32, "the lane's cells of a column are kept as bits of a 32-bit word");
  // planes per LDS chunk: every plane of a step in one chunk where 64 KB hold them
  static constexpr int BUDGET = 64 * 1024;
  static constexpr int CHMAX = BUDGET / (SDP * 4) < 1 ? 1 : BUDGET / (SDP * 4);
  static constexpr int NCH = (NP + CHMAX - 1) / CHMAX;
  static constexpr int CH = (NP + NCH - 1) / NCH;
  static constexpr int LDS_BYTES = CH * SDP * 4;
  static constexpr int REGW = SZ == 8 ? 2 : 1;
  // 16-bit D3Q64: four waves per row of cells, each holding the 16 planes of
  // one z node (the parts differ by a plane offset and a z-node offset;
  // partial moments summed through LDS), so that four waves per SIMD fit the
  // register file instead of one
  static constexpr bool SPLIT = !TH && N == 4 && SZ == 2;
  static constexpr int NHW = SPLIT ? 4 : 1;   // waves per row of cells
  static constexpr int NT = 256 * NHW;        // threads per workgroup
  static constexpr int NPW = NP / NHW;        // planes per wave
  // registers per lane: three per plane and about 50 besides (D3Q27: 167
  // VGPRs, three waves per SIMD); D3Q64 with all planes in one wave needs
  // about 300, VGPRs and AGPRs together
  static constexpr int VREG = 3 * NPW * REGW + (N == 3 ? 48 : 110);
  // athermal D3Q27 in 16-bit and FP32 storage, athermal D3Q64 in 16-bit
  // storage (at one wave per SIMD: 3355 against 3541 us for the chunked
  // kernel on a 256^3 grid, while FP32 D3Q64 ran slower, 4941 against 4245
  // us); FP64 values and the g planes of the thermal model would spill
  static constexpr bool fits = !TH && (N == 3 ? SZ <= 4 : (N == 4 && SZ == 2));
  static constexpr int WG_LDS = (160 * 1024) / LDS_BYTES;
  static constexpr int W_REG = 512 / VREG;
  // waves per SIMD: NHW per resident workgroup
  static constexpr int WAVES0 = WG_LDS * NHW < W_REG ? WG_LDS * NHW : W_REG;
  static constexpr int WAVES1 = WAVES0 / NHW * NHW < NHW ? NHW : WAVES0 / NHW * NHW;
  static constexpr int WAVES = WAVES1 > 8 ? 8 : WAVES1;
};

template <typename S, bool TH, int N, bool LIST = false>
__global__ void __launch_bounds__((SC3ZTraits<S, TH, N>::NT))
    __attribute__((amdgpu_waves_per_eu(SC3ZTraits<S, TH, N>::WAVES)))
k_sc3d_zm(const Tab *__restrict__ tab, int lat, Geo g, const S *__restrict__ in,
          S *__restrict__ out, const uint8_t *__restrict__ cls,
          const uint8_t *__restrict__ tflag, int remap, int xmir, const int *__restrict__ tlist,
          const int *__restrict__ tcount) {
  using Tr = SC3ZTraits<S, TH, N>;
  using T = typename Tr::T;
  using C = typename Tr::C;
  constexpr int Q = Tr::Q, NP = Tr::NP, SD = Tr::SD, SDP = Tr::SDP, M = Tr::M, CH = Tr::CH, NCH = Tr::NCH;
  constexpr int LWD = Tr::LWD, SZ = Tr::SZ, ZC = Tr::ZC;
  constexpr bool SPL = Tr::SPLIT;
  constexpr int NPW = Tr::NPW;
  static_assert(!SPL || (NCH == 1 && NP == Q), "the split walk: one chunk, f planes only");
  __shared__ uint32_t sm[CH * SDP];
  __shared__ float smom[SPL ? Tr::NHW : 1][SPL ? 4 : 1][SPL ? 256 : 1];   // partial moments per part
  const LatTab &L = tab->lat[lat];
  // the column: from the grid (XCD-aware order for dense launches), or one
  // workgroup per entry of the compact list of live columns (sparse launches)
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
  const int z0 = tile / (g.ntx * g.nty) * ZC;
  const int x0 = bx * MSL_TX, y0 = by * MSL_MTY;
  const int zn = g.nz - z0 < ZC ? g.nz - z0 : ZC;   // cells of the column (>= 1)
  {
    uint8_t any = 0;
    for (int k = 0; k < zn; ++k) any |= tflag[((long long)(z0 + k) * g.nty + by) * g.ntx + bx];
    if (!(any & (1 << lat))) return;
  }
  // (the wave index as a scalar: the LDS destinations of the DMA are formed
  // in scalar registers)
  // w: the wave's row of cells; hf: its half of the planes (split walk), which
  // starts at plane kb and z node ccb
  const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int w = wv & 3, hf = SPL ? wv >> 2 : 0;
  const int kb = hf * NPW, ccb = kb / (N * N);
  const unsigned pitch_b = (unsigned)g.pitch * SZ;
  const unsigned plane_b = (unsigned)g.plane * SZ;
  const unsigned slab_b = (unsigned)g.rows * pitch_b;
  // plane-independent byte offsets of this lane's slab dwords; lanes past the
  // slab's SD dwords issue no load
  unsigned voff[M];
  bool vld[M];
#pragma unroll
  for (int m = 0; m < M; ++m) {
    const int d = lane + 64 * (w + 4 * m);
    vld[m] = Tr::PAD || d < SD;   // padded: lanes past the slab load a valid dword into the pad
    const int dd = d < SD ? d : SD - 1;
    const int row = dd / LWD, col = dd - row * LWD;
    voff[m] = (unsigned)row * pitch_b + (unsigned)col * 4u;
  }
  // per-node tables of each axis: interpolation weights and the window offset
  // of the departure stencil (the z offset selects the first slab)
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
  // z tables from the wave's first z node on (split walk; ccb = 0 otherwise)
  if constexpr (SPL) {
#pragma unroll
    for (int a = 0; a < N; ++a) {
      const int az = a + ccb < N ? a + ccb : N - 1;
      wlo[2][a] = tsel<C>(L.a[2][az][0], L.af[2][az][0]);
      wmid[2][a] = tsel<C>(L.a[2][az][1], L.af[2][az][1]);
      whi[2][a] = tsel<C>(L.a[2][az][2], L.af[2][az][2]);
      offz[a] = (L.n0[2][az] - 1) * g.rows * g.pitch;
    }
  }
  // byte offset of the column's first slab window (before the plane's shift)
  const unsigned org0b = (unsigned)g.idx(x0, y0, z0) * SZ;
  // DMA of step t's slab of planes [K0, K1) into LDS: slab z0 + n0_z - 1 + t.
  // Each plane has its own buffer descriptor (the range of one plane); the
  // base offsets pass through an empty asm at every call, so the per-plane
  // descriptors and offsets are formed here rather than hoisted out of the
  // walk (4 + 1 scalar registers per plane)
  const long long plane_b64 = g.plane * SZ;
  auto issue = [&]<int K0, int K1>(const int t) {
    unsigned ob = org0b + (unsigned)t * slab_b;
    const char *pp = (const char *)in + (kb + K0) * plane_b64;
    asm volatile("" : "+s"(ob), "+s"(pp));
    msl_for_range<K0, K1>([&]<int K>() {
      constexpr int i = K % Q, a = i % N, b = (i / N) % N, cc = i / (N * N);
      const unsigned so = (ob + (unsigned)(offx[a] + offy[b] + offz[cc]) * SZ) & ~3u;
      const __amdgpu_buffer_rsrc_t rs =
          __builtin_amdgcn_make_buffer_rsrc((void *)pp, (short)0, (int)plane_b, MSL_RSRC_WORD3);
#pragma unroll
      for (int m = 0; m < M; ++m)
        if (vld[m])
          __builtin_amdgcn_raw_ptr_buffer_load_lds(
              rs, (msl_lds_t *)(sm + (SPL ? kb + K : K - K0) * SDP + 64 * (w + 4 * m)), 4, (int)voff[m], (int)so, 0, 0);
      pp += plane_b64;
    });
  };
  // LDS byte offset of the lane's first element in its wave's first window
  // row.  Rows start 64-byte aligned in HBM (the pitch is a multiple of 64
  // bytes and the column's x0 a multiple of 64 cells), so a plane's window
  // starts at byte (offx SZ) mod 4 of its first dword: 0 or 2 for 16-bit
  // storage, 0 otherwise.  The 16-bit elements are read one by one with
  // 16-bit LDS reads (volatile, so that the compiler does not merge two of
  // them into a 4-byte read at a 2-byte boundary, which stalls the LDS pipeline)
  unsigned rb[N];
#pragma unroll
  for (int a = 0; a < N; ++a)
    rb[a] = (unsigned)(w * LWD * 4 + lane * SZ) + (SZ == 2 ? (unsigned)(offx[a] & 1) * 2u : 0u);
  // per plane: the two slabs before the new one (FP32 / FP64: x, y
  // interpolated values ha = slab t - 2, hb = slab t - 1), or (16-bit storage)
  // the z interpolation's partial sums of the next two cells
  // (ha = w0 h_{t-2} + w1 h_{t-1}, hb = w0 h_{t-1}), which need no register moves
  // as the walk advances; ftk: the streamed value
  C ha[NPW], hb[NPW], ftk[NPW];   // (the wave's planes: all, or its half)
#pragma unroll
  for (int k = 0; k < NPW; ++k) ha[k] = hb[k] = C(0);
  // the new slab of plane K: x then y interpolation, then the z interpolation
  // of the three slabs into the streamed value of cell z0 + t - 2
  auto recon = [&]<int K>() {
    constexpr int i = K % Q, a = i % N, b = (i / N) % N, cc = i / (N * N);
    const char *base = (const char *)sm + ((SPL ? kb : 0) + K % CH) * SDP * 4 + rb[a];
    const C wx0 = wlo[0][a], wx2 = whi[0][a], wy0 = wlo[1][b], wy2 = whi[1][b], wz0 = wlo[2][cc],
            wz2 = whi[2][cc];
    C hy[3];
#pragma unroll
    for (int dy = 0; dy < 3; ++dy) {
      const char *row = base + dy * LWD * 4;
      C v0, v1, v2;
      if constexpr (SZ == 8) {
        v0 = (C)lds_elem_d<S>(row); v1 = (C)lds_elem_d<S>(row + 8); v2 = (C)lds_elem_d<S>(row + 16);
      } else if constexpr (SZ == 4) {
        v0 = (C)lds_elem<S>(row); v1 = (C)lds_elem<S>(row + SZ); v2 = (C)lds_elem<S>(row + 2 * SZ);
      } else {
        typedef volatile const __attribute__((address_space(3))) uint16_t lds_u16;
        v0 = (C)half_elem<S>(*(lds_u16 *)row);
        v1 = (C)half_elem<S>(*(lds_u16 *)(row + 2));
        v2 = (C)half_elem<S>(*(lds_u16 *)(row + 4));
      }
      // FP32 / FP64: differenced form, centre weight 1 - w0 - w2 exactly;
      // 16-bit deviations: the three weights (one operation fewer)
      // (the innermost product is an FMA with 0, so that FP16 values enter
      // all three as mixed-precision FMAs without a conversion)
      if constexpr (SZ == 2) hy[dy] = __builtin_fmaf(wx0, v0, __builtin_fmaf(wmid[0][a], v1, __builtin_fmaf(wx2, v2, 0.0f)));
      else hy[dy] = v1 + wx0 * (v0 - v1) + wx2 * (v2 - v1);
    }
    C hn;
    if constexpr (SZ == 2) {
      hn = wy0 * hy[0] + wmid[1][b] * hy[1] + wy2 * hy[2];
      // three-address FMAs: with the two-address form the compiler keeps
      // the partial sums in fixed registers through two moves per plane
      const C wzm = wmid[2][cc];
      asm("v_fma_f32 %0, %1, %2, %3" : "=v"(ftk[K]) : "s"(wz2), "v"(hn), "v"(ha[K]));
      asm("v_fma_f32 %0, %1, %2, %3" : "=v"(ha[K]) : "s"(wzm), "v"(hn), "v"(hb[K]));
      hb[K] = wz0 * hn;
      asm("" : "+v"(hb[K]));
    } else {
      hn = hy[1] + wy0 * (hy[0] - hy[1]) + wy2 * (hy[2] - hy[1]);
      ftk[K] = hb[K] + wz0 * (ha[K] - hb[K]) + wz2 * (hn - hb[K]);
      ha[K] = hb[K];
      hb[K] = hn;
      asm("" : "+v"(ftk[K]), "+v"(hb[K]));
    }
    // (the empty asm statements fix the final values: without them the
    // interpolation would be sunk into the collision, keeping the LDS values
    // of every plane alive until then; they are not volatile, so the LDS reads
    // of the next planes may be issued before them.)  The plane's arithmetic
    // stays before this point; only LDS reads and scalar instructions of later
    // planes may move above it
    __builtin_amdgcn_sched_barrier(0x0104);
  };

  const C gsc0 = (C)(tab->gfac * tab->T0);   // g scale over the f scale
  const int x = x0 + lane, y = y0 + w;
  // the lane's cells of this velocity set along the column (bit k: z0 + k),
  // read before the walk so that no load waits behind the slab loads in it
  uint32_t mine_bits = 0;
  if (x < g.nx && y < g.ny)
    for (int k = 0; k < zn; ++k)
      mine_bits |= (uint32_t)((cls[((long long)(z0 + k) * g.ny + y) * g.nx + x] & 1) == lat) << k;
  // periodic x (xmir, nx >= 4): the cells x < 2 and x >= nx - 2 are also
  // stored into the ghost columns of the other side, which the next step's
  // windows read; only the columns at the two x ends take the second store
  const bool xedge = xmir && (x0 < MSL_G || x0 + MSL_TX > g.nx - MSL_G);
  // byte offset of the lane's cell at z0 and the stride of one z step
  const unsigned cell0 = (unsigned)g.idx(x < g.nx ? x : 0, y < g.ny ? y : 0, z0) * SZ;
  const unsigned zstride = slab_b;
  // moments, equilibrium, collision and stores of the lane's cell at z
  auto finish = [&]<bool XE>(const int z) {
    const bool mine = (mine_bits >> (z - z0)) & 1u;
    // the per-plane scales and velocities are loaded here at every cell
    // (scalar loads) rather than hoisted out of the walk into 2 NP + 3 N
    // scalar registers
    // (through the constant address space: the table is read-only for the
    // kernel's lifetime, which the empty asm would otherwise hide, turning
    // the scalar loads into vector loads)
    typedef const __attribute__((address_space(4))) LatTab cLatTab;
    typedef const __attribute__((address_space(4))) Tab cTab;
    cLatTab *Lp = (cLatTab *)&L;
    cTab *tp = (cTab *)tab;
    // plane K's base, advanced plane by plane (from the wave's first plane)
    const char *op = (const char *)out + (long long)kb * plane_b64;
    asm volatile("" : "+s"(Lp), "+s"(tp), "+s"(op));
    auto &L = *Lp;
    C rho = C(0), jx = C(0), jy = C(0), jz = C(0), en = C(0);
    auto moments = [&]<int K>() {
      constexpr int i = K % Q, a = i % N, b = (i / N) % N, cc = i / (N * N);
      // (split walk: population kb + i, z node ccb + cc)
      const C W = tsel<C>(L.sc[kb + i], L.scf[kb + i]);   // storage scale of f_i
      if constexpr (K < Q) {
        const C cx = tsel<C>(L.v[0][a], L.vf[0][a]), cy = tsel<C>(L.v[1][b], L.vf[1][b]),
                cz = tsel<C>(L.v[2][ccb + cc], L.vf[2][ccb + cc]);
        const C f = T::dev ? W * (C(1) + ftk[K]) : ftk[K];
        ftk[K] = f;   // the population itself from here on
        rho += f;
        jx += cx * f;
        jy += cy * f;
        jz += cz * f;
        if (TH) en += C(0.5) * (cx * cx + cy * cy + cz * cz) * f;
      } else {
        ftk[K] = T::dev ? gsc0 * W * (C(1) + ftk[K]) : ftk[K];
        en += ftk[K];
      }
    };
    msl_for_planes<NPW>(moments);
    if constexpr (SPL) {
      // the other half's partial sums (a + b == b + a: both waves of a row
      // hold the same sums)
      const int ci = w * 64 + lane;
      smom[hf][0][ci] = rho;
      smom[hf][1][ci] = jx;
      smom[hf][2][ci] = jy;
      smom[hf][3][ci] = jz;
      msl_lds_barrier();
      rho = smom[0][0][ci];
      jx = smom[0][1][ci];
      jy = smom[0][2][ci];
      jz = smom[0][3][ci];
#pragma unroll
      for (int h = 1; h < Tr::NHW; ++h) {
        rho += smom[h][0][ci];
        jx += smom[h][1][ci];
        jy += smom[h][2][ci];
        jz += smom[h][3][ci];
      }
    }
    // equilibrium factors in FP64 (no rounding bias in the equilibrium's mass
    // and momentum), kept in the compute precision
    const double rd = (double)rho, ird = 1.0 / rd;
    const double ux = (double)jx * ird, uy = (double)jy * ird, uz = (double)jz * ird;
    double Tm = 1.0;
    if (TH) Tm = ((double)en - 0.5 * rd * (ux * ux + uy * uy + uz * uz)) / (tp->cv * rd);
    C om = tsel<C>(tp->omega, tp->omegaf);
    if (tp->tau_mode == 1) {
      const double mu = TH ? tp->mu_ref * pow(Tm / tp->tau_ref_T, tp->mu_exp) : tp->mu_T1;
      om = (C)(1.0 / (mu / (rd * Tm * tp->dt) + 0.5));
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
      if constexpr (SPL) {   // z factors from the wave's first z node on
#pragma unroll
        for (int q = 0; q < N; ++q) {
          C v = Pz[q];
#pragma unroll
          for (int r = q + 1; r < N; ++r)
            if (r == q + ccb) v = (C)pz[r];
          Pz[q] = v;
        }
      }
    }
    const C gf = (C)(tp->gfac * Tm);
    const unsigned soff = mine ? cell0 + (unsigned)(z - z0) * zstride : 0x80000000u;
    const unsigned ioff = (mine && x < MSL_G) ? soff + (unsigned)g.nx * SZ
                          : (mine && x >= g.nx - MSL_G) ? soff - (unsigned)g.nx * SZ : 0x80000000u;
    auto store = [&]<int K>() {
      constexpr int i = K % Q, a = i % N, b = (i / N) % N, cc = i / (N * N);
      const C isc = T::dev ? tsel<C>(L.isc[kb + i], L.iscf[kb + i]) * (K < Q ? C(1) : tsel<C>(tp->igsc, tp->igscf)) : C(1);
      const C feq = Px[a] * Py[b] * Pz[cc];
      const C v = ftk[K];
      C vo;
      if constexpr (K < Q) vo = v + om * (feq - v);
      else vo = v + om * (gf * feq - v);
      const S sv = T::store(T::dev ? vo * isc - C(1) : vo);
      const __amdgpu_buffer_rsrc_t rsout =
          __builtin_amdgcn_make_buffer_rsrc((void *)op, (short)0, (int)plane_b, MSL_RSRC_WORD3);
      op += plane_b64;
      auto put = [&](unsigned o) {
        if constexpr (SZ == 8) {
          typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
          __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, sv), rsout, (int)o, 0, 0);
        } else if constexpr (SZ == 4) {
          __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, sv), rsout, (int)o, 0, 0);
        } else {
          __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(uint16_t, sv), rsout, (int)o, 0, 0);
        }
      };
      put(soff);
      if constexpr (XE) put(ioff);
    };
    msl_for_planes<NPW>(store);
  };

  // the walk: slabs t = 0 .. zn + 1; from t = 2 on, cell z0 + t - 2 is complete.
  // The first chunk of the next slab is loaded while the current cell
  // collides.  The barriers are plain s_barrier with the waits spelt out: a
  // __syncthreads() would also wait for the cell's stores (its release fence),
  // exposing their latency at every step, while the slab's loads only need
  // the loads issued before them (vector memory operations complete in issue
  // order, so waiting until the stores of one cell are all that is
  // outstanding waits for exactly the slab).
  // (vmcnt holds at most 63: with more stores per cell the wait also takes
  // the oldest of them)
  constexpr int VW1 = NPW < 63 ? NPW : 63, VW2 = 2 * NPW < 63 ? 2 * NPW : 63;
  constexpr int CH0 = CH < NPW ? CH : NPW;   // (split walk: the wave's half)
  issue.template operator()<0, CH0>(0);
  msl_wait_vm<0>();
  for (int t = 0; t < zn + 2; ++t) {
    // the row offsets pass through an empty asm at every step, so that the
    // per-plane LDS addresses are formed in the walk, not hoisted out of it
    // into NP registers
#pragma unroll
    for (int a = 0; a < N; ++a) asm volatile("" : "+v"(rb[a]));
    auto chunk = [&]<int CI>() {
      constexpr int k0 = CI * CH, k1 = k0 + CH < NP ? k0 + CH : NP;
      if constexpr (CI > 0) {
        issue.template operator()<k0, k1>(t);
        msl_wait_vm<0>();
      }
      msl_lds_barrier();   // every wave's share of the slab is in LDS
      msl_for_range<k0, (k1 < NPW ? k1 : NPW)>(recon);
      msl_lds_barrier();   // the chunk's LDS values are read; the next load may overwrite them
    };
    msl_for_planes<NCH>(chunk);
    if (t + 1 < zn + 2) issue.template operator()<0, CH0>(t + 1);
    if (t >= 2) {
      if (xedge) {
        finish.template operator()<true>(z0 + t - 2);
        msl_wait_vm<VW2>();
      } else {
        finish.template operator()<false>(z0 + t - 2);
        msl_wait_vm<VW1>();
      }
    } else {
      msl_wait_vm<0>();
    }
  }
}
