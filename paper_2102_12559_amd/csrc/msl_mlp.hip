// msl_mlp.hip -- the learned lifting closure: features and targets of band
// cells, a F -> H -> H -> O perceptron (SiLU) on the BF16 matrix cores with
// FP32 accumulation (forward, backward, Adam), snapshot collection, the
// learned lift of the low-order band cells and the per-tile error check that
// falls back to Grad lifting.
//
// Matrix-core fragments (v_mfma_f32_16x16x16_bf16, wave64): lane l holds
//   A[m = l%16][k = 4(l/16)+i], B[k = 4(l/16)+i][n = l%16], D[m = 4(l/16)+i][n = l%16]
// for i = 0..3.  One wavefront carries a tile of 16 samples through all three
// layers; weights live in LDS as BF16, activations pass through LDS to turn
// the D layout of one layer into the A layout of the next.
#include <stdio.h>
#include <string.h>

#include <mutex>

#include "msl_band.hpp"
#include "msl_device.hpp"

typedef short s4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ short f2bf(float v) {
  uint32_t b = __float_as_uint(v);
  if ((b & 0x7fffffffu) > 0x7f800000u) return (short)((b >> 16) | 0x40u);
  b += 0x7fffu + ((b >> 16) & 1u);
  return (short)(b >> 16);
}
// LDS written by other lanes of the same wavefront becomes visible
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
__device__ __forceinline__ float silu(float z) { return z / (1.0f + __expf(-z)); }
__device__ __forceinline__ float silu_d(float z) {
  const float s = 1.0f / (1.0f + __expf(-z));
  return s * (1.0f + z * (1.0f - s));
}

// ---------------------------------------------------------------------------
// features and targets (FP64)
// ---------------------------------------------------------------------------

// standardised feature, limited to +-8 standard deviations: a state far
// outside the training data gets a bounded input instead of an arbitrary one
#define MSL_MLP_XCLIP 8.0
__device__ __forceinline__ double std_feature(double v, float mean, float sd) {
  const double z = (v - mean) / sd;
  return z > MSL_MLP_XCLIP ? MSL_MLP_XCLIP : (z < -MSL_MLP_XCLIP ? -MSL_MLP_XCLIP : z);
}

// number of features (rho, u, T and the low-order moments of degree >= 2) and
// of outputs (the raw moments the low-order set cannot hold)
template <int D, int NL>
constexpr int nfeat() {
  int n = 2 + D;
  for (int j = 0; j < Pow<D, NL>::v; ++j)
    if (j % NL + (j / NL) % NL + (D == 3 ? j / (NL * NL) : 0) >= 2) ++n;
  return n;
}
template <int D, int NL, int NH>
constexpr int nout() { return Pow<D, NH>::v - Pow<D, NL>::v; }
// position of high-order moment index j (3D) among the network's outputs: the
// indices outside the low-order block, in ascending order
template <int NL, int NH>
__host__ __device__ constexpr int out_index(int j) {
  int o = 0;
  for (int k = 0; k < j; ++k)
    if (!(k % NH < NL && (k / NH) % NH < NL && k / (NH * NH) < NL)) ++o;
  return o;
}

// M[p] = sum_i f_i prod_a (c_{i_a} - s_a)^{p_a} for every moment index p < N per
// axis, by one contraction per axis of the tensor-product population array
template <int D, int N>
__device__ __forceinline__ void moments_sep(const double *c, const double *sft, const double *f,
                                            double *M) {
  double pw[D][N][N];   // pw[a][p][node]
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int k = 0; k < N; ++k) {
      const double d = c[k] - sft[a];
      double v = 1.0;
#pragma unroll
      for (int p = 0; p < N; ++p) {
        pw[a][p][k] = v;
        v *= d;
      }
    }
  if constexpr (D == 2) {
    double t[N][N];   // t[p0][b]
#pragma unroll
    for (int p0 = 0; p0 < N; ++p0)
#pragma unroll
      for (int b = 0; b < N; ++b) {
        double s = 0;
#pragma unroll
        for (int k = 0; k < N; ++k) s += pw[0][p0][k] * f[k + N * b];
        t[p0][b] = s;
      }
#pragma unroll
    for (int p1 = 0; p1 < N; ++p1)
#pragma unroll
      for (int p0 = 0; p0 < N; ++p0) {
        double s = 0;
#pragma unroll
        for (int b = 0; b < N; ++b) s += pw[1][p1][b] * t[p0][b];
        M[p0 + N * p1] = s;
      }
  } else {
    double t1[N * N * N], t2[N * N * N];
#pragma unroll
    for (int p0 = 0; p0 < N; ++p0)
#pragma unroll
      for (int bc = 0; bc < N * N; ++bc) {
        double s = 0;
#pragma unroll
        for (int k = 0; k < N; ++k) s += pw[0][p0][k] * f[k + N * bc];
        t1[p0 + N * bc] = s;   // [p0][b][c]
      }
#pragma unroll
    for (int p1 = 0; p1 < N; ++p1)
#pragma unroll
      for (int p0 = 0; p0 < N; ++p0)
#pragma unroll
        for (int cc = 0; cc < N; ++cc) {
          double s = 0;
#pragma unroll
          for (int k = 0; k < N; ++k) s += pw[1][p1][k] * t1[p0 + N * (k + N * cc)];
          t2[p0 + N * (p1 + N * cc)] = s;
        }
#pragma unroll
    for (int p2 = 0; p2 < N; ++p2)
#pragma unroll
      for (int p01 = 0; p01 < N * N; ++p01) {
        double s = 0;
#pragma unroll
        for (int k = 0; k < N; ++k) s += pw[2][p2][k] * t2[p01 + N * N * k];
        M[p01 + N * N * p2] = s;
      }
  }
}

// rho, u/sqrt(T), T, then the normalised central moments
// sum_i f_i prod_a (c_ia - u_a)^{p_a} / (rho T^{|p|/2}) of every low-order moment
// index p with |p| >= 2, in ascending moment index
template <int D, int NL, bool TH = true>
__device__ void features_t(const Tab *tab, const double *fq, const double *gq, double *feat) {
  const LatTab &L = tab->lat[0];
  double rho, u[3], T;
  macros_t<D, NL>(L, TH && tab->thermal, tab->cv, fq, gq, rho, u, T);
  int k = 0;
  feat[k++] = rho;
  const double sT = sqrt(T);
  for (int a = 0; a < D; ++a) feat[k++] = u[a] / sT;
  feat[k++] = T;
  constexpr int q = Pow<D, NL>::v;
  double M[q], den[D * (NL - 1) + 1];
  moments_sep<D, NL>(L.cr, u, fq, M);
  den[0] = rho;
#pragma unroll
  for (int d = 1; d <= D * (NL - 1); ++d) den[d] = den[d - 1] * sT;
#pragma unroll
  for (int j = 0; j < q; ++j) {
    const int p0 = j % NL, p1 = (j / NL) % NL, p2 = D == 3 ? j / (NL * NL) : 0;
    const int deg = p0 + p1 + p2;
    if (deg < 2) continue;
    feat[k++] = M[j] / den[deg];
  }
}

// normalised non-equilibrium parts (M_p - M^eq_p) / (rho T^{|p|/2}) of the raw
// moments the low-order set cannot hold, in ascending high-order moment index
template <int D, int NL, int NH, bool TH = true>
__device__ void targets_t(const Tab *tab, const double *fQ, const double *gQ, double *t) {
  const LatTab &LQ = tab->lat[1];
  constexpr int Q = Pow<D, NH>::v;
  double rho, u[3], T, dv[Q], M[Q];
  macros_t<D, NH>(LQ, TH && tab->thermal, tab->cv, fQ, gQ, rho, u, T);
  feq_t<D, NH>(LQ, rho, u, T, dv);
#pragma unroll
  for (int i = 0; i < Q; ++i) dv[i] = fQ[i] - dv[i];
  const double zero[3] = {0.0, 0.0, 0.0};
  moments_sep<D, NH>(LQ.cr, zero, dv, M);
  const double sT = sqrt(T);
  double den[D * (NH - 1) + 1];
  den[0] = rho;
#pragma unroll
  for (int d = 1; d <= D * (NH - 1); ++d) den[d] = den[d - 1] * sT;
  int k = 0;
#pragma unroll
  for (int j = 0; j < Q; ++j) {
    const int p0 = j % NH, p1 = (j / NH) % NH, p2 = D == 3 ? j / (NH * NH) : 0;
    if (p0 < NL && p1 < NL && p2 < NL) continue;
    t[k++] = M[j] / den[p0 + p1 + p2];
  }
}

// ---------------------------------------------------------------------------
// the perceptron on the matrix cores
// ---------------------------------------------------------------------------
template <int FP, int H, int OP>
struct MlpLds {
  short w1[FP * H], w2[H * H], w3[H * OP];
  float b1[H], b2[H], b3[OP];
  short act1[4][16 * H], act2[4][16 * H], dz2[4][16 * H], dy[4][16 * OP];
  float red[4];
};

// mode 0: forward (Y[n][O] out); mode 1: forward + backward of the mean-square
// loss over `inv_count` (gradient and loss partials of this workgroup)
template <int FP, int H, int OP, int MODE>
__global__ void __launch_bounds__(256)
k_mlp(const float *__restrict__ prm, int F, int O, const float *__restrict__ X,
      const float *__restrict__ Y, int n_host, const int *__restrict__ n_dev,
      float *__restrict__ out, float *__restrict__ gpart, long long lbase, float inv_count) {
  __shared__ MlpLds<FP, H, OP> s;
  __shared__ float sg[MODE == 1 ? (FP * H + H + H * H + H + H * OP + OP) : 1];
  const int P = F * H + H + H * H + H + H * O + O;
  const float *W1 = prm, *B1 = W1 + F * H, *W2 = B1 + H, *B2 = W2 + H * H, *W3 = B2 + H,
              *B3 = W3 + H * O;
  for (int k = threadIdx.x; k < FP * H; k += 256) {
    const int f = k / H, h = k % H;
    s.w1[k] = f2bf(f < F ? W1[f * H + h] : 0.f);
  }
  for (int k = threadIdx.x; k < H * H; k += 256) s.w2[k] = f2bf(W2[k]);
  for (int k = threadIdx.x; k < H * OP; k += 256) {
    const int h = k / OP, o = k % OP;
    s.w3[k] = f2bf(o < O ? W3[h * O + o] : 0.f);
  }
  for (int k = threadIdx.x; k < H; k += 256) { s.b1[k] = B1[k]; s.b2[k] = B2[k]; }
  for (int k = threadIdx.x; k < OP; k += 256) s.b3[k] = k < O ? B3[k] : 0.f;
  if (MODE == 1)
    for (int k = threadIdx.x; k < FP * H + H + H * H + H + H * OP + OP; k += 256) sg[k] = 0.f;
  __syncthreads();

  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int lr = lane & 15, lg = lane >> 4;
  const int n = n_dev ? *n_dev : n_host;
  const int ntiles = (n + 15) / 16;
  short *a1 = s.act1[w], *a2 = s.act2[w], *dz = s.dz2[w], *dyb = s.dy[w];

  // gradient accumulators (mode 1)
  f4 gw1[FP / 16][H / 16], gw2[H / 16][H / 16], gw3[H / 16][OP / 16];
  float gb1[H / 16], gb2[H / 16], gb3[OP / 16];
  float lossacc = 0.f;
  if (MODE == 1) {
#pragma unroll
    for (int a = 0; a < H / 16; ++a) {
      gb1[a] = gb2[a] = 0.f;
#pragma unroll
      for (int b = 0; b < FP / 16; ++b) gw1[b][a] = f4{0, 0, 0, 0};
#pragma unroll
      for (int b = 0; b < H / 16; ++b) gw2[a][b] = f4{0, 0, 0, 0};
#pragma unroll
      for (int b = 0; b < OP / 16; ++b) gw3[a][b] = f4{0, 0, 0, 0};
    }
#pragma unroll
    for (int b = 0; b < OP / 16; ++b) gb3[b] = 0.f;
  }

  // forward only: the weight fragments stay in registers for every tile
  s4 bw1[MODE == 0 ? FP / 16 : 1][MODE == 0 ? H / 16 : 1];
  s4 bw2[MODE == 0 ? H / 16 : 1][MODE == 0 ? H / 16 : 1];
  s4 bw3[MODE == 0 ? H / 16 : 1][MODE == 0 ? OP / 16 : 1];
  if constexpr (MODE == 0) {
#pragma unroll
    for (int nt = 0; nt < H / 16; ++nt)
#pragma unroll
      for (int kc = 0; kc < FP / 16; ++kc)
#pragma unroll
        for (int i = 0; i < 4; ++i) bw1[kc][nt][i] = s.w1[(kc * 16 + 4 * lg + i) * H + nt * 16 + lr];
#pragma unroll
    for (int nt = 0; nt < H / 16; ++nt)
#pragma unroll
      for (int kc = 0; kc < H / 16; ++kc)
#pragma unroll
        for (int i = 0; i < 4; ++i) bw2[kc][nt][i] = s.w2[(kc * 16 + 4 * lg + i) * H + nt * 16 + lr];
#pragma unroll
    for (int nt = 0; nt < OP / 16; ++nt)
#pragma unroll
      for (int kc = 0; kc < H / 16; ++kc)
#pragma unroll
        for (int i = 0; i < 4; ++i) bw3[kc][nt][i] = s.w3[(kc * 16 + 4 * lg + i) * OP + nt * 16 + lr];
  }

  const int tstride = MODE == 1 ? 1 << 30 : gridDim.x * 4;
  for (int tile = blockIdx.x * 4 + w; tile < ntiles; tile += tstride) {
    const int r0 = tile * 16;
    // ---- layer 1: z1 = x W1 + b1 ----
    f4 z1[H / 16], z2[H / 16];
#pragma unroll
    for (int nt = 0; nt < H / 16; ++nt) {
      f4 acc;
      const float bb = s.b1[nt * 16 + lr];
      acc = f4{bb, bb, bb, bb};
#pragma unroll
      for (int kc = 0; kc < FP / 16; ++kc) {
        s4 av, bv;
        const int row = r0 + lr;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int col = kc * 16 + 4 * lg + i;
          av[i] = f2bf(row < n && col < F ? X[(long long)row * F + col] : 0.f);
          if constexpr (MODE == 0) bv[i] = bw1[kc][nt][i];
          else bv[i] = s.w1[(kc * 16 + 4 * lg + i) * H + nt * 16 + lr];
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc, 0, 0, 0);
      }
      z1[nt] = acc;
#pragma unroll
      for (int i = 0; i < 4; ++i) a1[(4 * lg + i) * H + nt * 16 + lr] = f2bf(silu(acc[i]));
    }
    wave_sync();
    // ---- layer 2: z2 = h1 W2 + b2 ----
#pragma unroll
    for (int nt = 0; nt < H / 16; ++nt) {
      const float bb = s.b2[nt * 16 + lr];
      f4 acc = f4{bb, bb, bb, bb};
#pragma unroll
      for (int kc = 0; kc < H / 16; ++kc) {
        const s4 av = *(const s4 *)&a1[lr * H + kc * 16 + 4 * lg];
        s4 bv;
        if constexpr (MODE == 0) bv = bw2[kc][nt];
        else
#pragma unroll
          for (int i = 0; i < 4; ++i) bv[i] = s.w2[(kc * 16 + 4 * lg + i) * H + nt * 16 + lr];
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc, 0, 0, 0);
      }
      z2[nt] = acc;
#pragma unroll
      for (int i = 0; i < 4; ++i) a2[(4 * lg + i) * H + nt * 16 + lr] = f2bf(silu(acc[i]));
    }
    wave_sync();
    // ---- layer 3: y = h2 W3 + b3 ----
    f4 yv[OP / 16];
#pragma unroll
    for (int nt = 0; nt < OP / 16; ++nt) {
      const float bb = s.b3[nt * 16 + lr];
      f4 acc = f4{bb, bb, bb, bb};
#pragma unroll
      for (int kc = 0; kc < H / 16; ++kc) {
        const s4 av = *(const s4 *)&a2[lr * H + kc * 16 + 4 * lg];
        s4 bv;
        if constexpr (MODE == 0) bv = bw3[kc][nt];
        else
#pragma unroll
          for (int i = 0; i < 4; ++i) bv[i] = s.w3[(kc * 16 + 4 * lg + i) * OP + nt * 16 + lr];
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc, 0, 0, 0);
      }
      yv[nt] = acc;
    }
    if (MODE == 0) {
#pragma unroll
      for (int nt = 0; nt < OP / 16; ++nt)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int row = r0 + 4 * lg + i, col = nt * 16 + lr;
          if (row < n && col < O) out[(long long)row * O + col] = yv[nt][i];
        }
      continue;
    }
    // ---- backward ----
    // dY = 2 (y - t) / count
#pragma unroll
    for (int nt = 0; nt < OP / 16; ++nt) {
      float cs = 0.f;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = r0 + 4 * lg + i, col = nt * 16 + lr;
        float d = 0.f;
        if (row < n && col < O) {
          const float e = yv[nt][i] - Y[(long long)row * O + col];
          lossacc += e * e;
          d = 2.f * e * inv_count;
        }
        dyb[(4 * lg + i) * OP + col] = f2bf(d);
        cs += d;
      }
      gb3[nt] += cs;
    }
    wave_sync();
    // dW3 += h2^T dY   (M = H features, K = 16 samples, N = OP)
#pragma unroll
    for (int mt = 0; mt < H / 16; ++mt) {
      s4 av;
#pragma unroll
      for (int i = 0; i < 4; ++i) av[i] = a2[(4 * lg + i) * H + mt * 16 + lr];
#pragma unroll
      for (int nt = 0; nt < OP / 16; ++nt) {
        s4 bv;
#pragma unroll
        for (int i = 0; i < 4; ++i) bv[i] = dyb[(4 * lg + i) * OP + nt * 16 + lr];
        gw3[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, gw3[mt][nt], 0, 0, 0);
      }
    }
    // dH2 = dY W3^T, dZ2 = dH2 * silu'(z2)
#pragma unroll
    for (int nt = 0; nt < H / 16; ++nt) {
      f4 acc = f4{0, 0, 0, 0};
#pragma unroll
      for (int kc = 0; kc < OP / 16; ++kc) {
        const s4 av = *(const s4 *)&dyb[lr * OP + kc * 16 + 4 * lg];
        const s4 bv = *(const s4 *)&s.w3[(nt * 16 + lr) * OP + kc * 16 + 4 * lg];
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc, 0, 0, 0);
      }
      float cs = 0.f;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float d = acc[i] * silu_d(z2[nt][i]);
        dz[(4 * lg + i) * H + nt * 16 + lr] = f2bf(d);
        cs += d;
      }
      gb2[nt] += cs;
    }
    wave_sync();
    // dW2 += h1^T dZ2
#pragma unroll
    for (int mt = 0; mt < H / 16; ++mt) {
      s4 av;
#pragma unroll
      for (int i = 0; i < 4; ++i) av[i] = a1[(4 * lg + i) * H + mt * 16 + lr];
#pragma unroll
      for (int nt = 0; nt < H / 16; ++nt) {
        s4 bv;
#pragma unroll
        for (int i = 0; i < 4; ++i) bv[i] = dz[(4 * lg + i) * H + nt * 16 + lr];
        gw2[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, gw2[mt][nt], 0, 0, 0);
      }
    }
    // dH1 = dZ2 W2^T, dZ1 = dH1 * silu'(z1)   (kept in act2, no longer needed)
#pragma unroll
    for (int nt = 0; nt < H / 16; ++nt) {
      f4 acc = f4{0, 0, 0, 0};
#pragma unroll
      for (int kc = 0; kc < H / 16; ++kc) {
        const s4 av = *(const s4 *)&dz[lr * H + kc * 16 + 4 * lg];
        const s4 bv = *(const s4 *)&s.w2[(nt * 16 + lr) * H + kc * 16 + 4 * lg];
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc, 0, 0, 0);
      }
      float cs = 0.f;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float d = acc[i] * silu_d(z1[nt][i]);
        a2[(4 * lg + i) * H + nt * 16 + lr] = f2bf(d);
        cs += d;
      }
      gb1[nt] += cs;
    }
    wave_sync();
    // dW1 += x^T dZ1
#pragma unroll
    for (int mt = 0; mt < FP / 16; ++mt) {
      s4 av;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = r0 + 4 * lg + i, col = mt * 16 + lr;
        av[i] = f2bf(row < n && col < F ? X[(long long)row * F + col] : 0.f);
      }
#pragma unroll
      for (int nt = 0; nt < H / 16; ++nt) {
        s4 bv;
#pragma unroll
        for (int i = 0; i < 4; ++i) bv[i] = a2[(4 * lg + i) * H + nt * 16 + lr];
        gw1[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, gw1[mt][nt], 0, 0, 0);
      }
    }
  }
  if (MODE != 1) return;
  // ---- deterministic workgroup reduction: waves add in order ----
  // bias sums: combine the four lane groups of each column
#pragma unroll
  for (int a = 0; a < H / 16; ++a) {
    gb1[a] += __shfl_xor(gb1[a], 16);
    gb1[a] += __shfl_xor(gb1[a], 32);
    gb2[a] += __shfl_xor(gb2[a], 16);
    gb2[a] += __shfl_xor(gb2[a], 32);
  }
#pragma unroll
  for (int a = 0; a < OP / 16; ++a) {
    gb3[a] += __shfl_xor(gb3[a], 16);
    gb3[a] += __shfl_xor(gb3[a], 32);
  }
  for (int m = 1; m < 64; m <<= 1) lossacc += __shfl_xor(lossacc, m);
  const int oW1 = 0, oB1 = FP * H, oW2 = oB1 + H, oB2 = oW2 + H * H, oW3 = oB2 + H,
            oB3 = oW3 + H * OP;
  for (int wv = 0; wv < 4; ++wv) {
    if (w == wv) {
#pragma unroll
      for (int mt = 0; mt < FP / 16; ++mt)
#pragma unroll
        for (int nt = 0; nt < H / 16; ++nt)
#pragma unroll
          for (int i = 0; i < 4; ++i)
            sg[oW1 + (mt * 16 + 4 * lg + i) * H + nt * 16 + lr] += gw1[mt][nt][i];
#pragma unroll
      for (int mt = 0; mt < H / 16; ++mt)
#pragma unroll
        for (int nt = 0; nt < H / 16; ++nt)
#pragma unroll
          for (int i = 0; i < 4; ++i)
            sg[oW2 + (mt * 16 + 4 * lg + i) * H + nt * 16 + lr] += gw2[mt][nt][i];
#pragma unroll
      for (int mt = 0; mt < H / 16; ++mt)
#pragma unroll
        for (int nt = 0; nt < OP / 16; ++nt)
#pragma unroll
          for (int i = 0; i < 4; ++i)
            sg[oW3 + (mt * 16 + 4 * lg + i) * OP + nt * 16 + lr] += gw3[mt][nt][i];
      if (lg == 0) {
#pragma unroll
        for (int a = 0; a < H / 16; ++a) {
          sg[oB1 + a * 16 + lr] += gb1[a];
          sg[oB2 + a * 16 + lr] += gb2[a];
        }
#pragma unroll
        for (int a = 0; a < OP / 16; ++a) sg[oB3 + a * 16 + lr] += gb3[a];
      }
      if (lane == 0) s.red[wv] = lossacc;
    }
    __syncthreads();
  }
  // unpadded layout of this workgroup's partial
  float *gp = gpart + (long long)blockIdx.x * P;
  for (int k = threadIdx.x; k < P; k += 256) {
    float v;
    if (k < F * H) v = sg[oW1 + (k / H) * H + k % H];
    else if (k < F * H + H) v = sg[oB1 + (k - F * H)];
    else if (k < F * H + H + H * H) v = sg[oW2 + (k - F * H - H)];
    else if (k < F * H + 2 * H + H * H) v = sg[oB2 + (k - F * H - H - H * H)];
    else if (k < F * H + 2 * H + H * H + H * O) {
      const int r = k - (F * H + 2 * H + H * H);
      v = sg[oW3 + (r / O) * OP + r % O];
    } else {
      v = sg[oB3 + (k - (F * H + 2 * H + H * H + H * O))];
    }
    gp[k] = v;
  }
  if (threadIdx.x == 0) gpart[lbase + blockIdx.x] = s.red[0] + s.red[1] + s.red[2] + s.red[3];
}

// sum of the workgroup partials in a fixed order; optionally Adam
__global__ void k_mlp_reduce_adam(float *__restrict__ prm, float *__restrict__ m,
                                  float *__restrict__ v, float *__restrict__ gout,
                                  const float *__restrict__ gpart, long long lbase, int P, int nblk,
                                  int apply, int t, float lr, float b1, float b2, float eps,
                                  float *__restrict__ loss_out, float loss_scale) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k == 0 && loss_out) {
    float L = 0.f;
    for (int b = 0; b < nblk; ++b) L += gpart[lbase + b];
    *loss_out = L * loss_scale;
  }
  if (k >= P) return;
  float g = 0.f;
  for (int b = 0; b < nblk; ++b) g += gpart[(long long)b * P + k];
  if (gout) gout[k] = g;
  if (!apply) return;
  const float mk = b1 * m[k] + (1.f - b1) * g;
  const float vk = b2 * v[k] + (1.f - b2) * g * g;
  m[k] = mk;
  v[k] = vk;
  const float mh = mk / (1.f - powf(b1, (float)t)), vh = vk / (1.f - powf(b2, (float)t));
  prm[k] -= lr * mh / (sqrtf(vh) + eps);
}

// ---------------------------------------------------------------------------
// band cells: features -> network -> learned lift; error check
// ---------------------------------------------------------------------------
__device__ __forceinline__ int check_tile(const Geo &g, int x, int y, int z, const int *nct) {
  return x / MSL_CHECK_TILE + nct[0] * (y / MSL_CHECK_TILE + nct[1] * (z / MSL_CHECK_TILE));
}

// standardised features of the low-order band cells (from the state in bl)
template <typename S, int D, int NL, bool TH>
__global__ void __launch_bounds__(64)
k_band_features(const Tab *__restrict__ tab, Geo g, const char *bl, const int *__restrict__ list,
                const int *__restrict__ count, const float *__restrict__ stats,
                float *__restrict__ feat) {
  constexpr int q = Pow<D, NL>::v, F = nfeat<D, NL>();
  const int n = *count;
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < n;
       t += (long long)gridDim.x * blockDim.x) {
    int x, y, z;
    cell_coords(g, list[t], x, y, z);
    double f[q], gg[TH ? q : 1], ft[F];
    read_cell_t<S, D, NL, TH>(tab, g, bl, 0, g.idx(x, y, z), f, gg);
    features_t<D, NL, TH>(tab, f, gg, ft);
#pragma unroll
    for (int a = 0; a < F; ++a) feat[t * F + a] = (float)std_feature(ft[a], stats[a], stats[F + a]);
  }
}

// the learned lift of the low-order band cells: completed moments
// M^eq_{Q-q} + rho T^{|p|/2} t_p, t_p the de-standardised network output;
// cells of check tiles that failed the error check get t = 0 (Grad lifting)
template <typename S, int D, int NL, int NH, bool TH>
__global__ void __launch_bounds__(64)
k_band_lift_mlp(const Tab *__restrict__ tab, Geo g, const char *bl, char *bh,
                const int *__restrict__ list, const int *__restrict__ count,
                const float *__restrict__ stats, const float *__restrict__ yout,
                const uint8_t *__restrict__ flags, int nct0, int nct1, int xmir) {
  constexpr int q = Pow<D, NL>::v, Q = Pow<D, NH>::v, F = nfeat<D, NL>(), O = nout<D, NL, NH>();
  const int n = *count;
  const int nct[3] = {nct0, nct1, 1};
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < n;
       t += (long long)gridDim.x * blockDim.x) {
    int x, y, z;
    cell_coords(g, list[t], x, y, z);
    const int off = g.idx(x, y, z);
    double f[q], gg[TH ? q : 1], fo[Q], go[TH ? Q : 1], dM[Q];
    read_cell_t<S, D, NL, TH>(tab, g, bl, 0, off, f, gg);
    const bool use = flags[check_tile(g, x, y, z, nct)] != 0;
    double rho, u[3], T;
    macros_t<D, NL>(tab->lat[0], TH && tab->thermal, tab->cv, f, gg, rho, u, T);
    // rho T^{|p|/2} for every degree
    const double sT = sqrt(T);
    double sc[D * (NH - 1) + 1];
    sc[0] = use ? rho : 0.0;
#pragma unroll
    for (int d = 1; d <= D * (NH - 1); ++d) sc[d] = sc[d - 1] * sT;
    const float *yo = yout + t * O;
    int o = 0;
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      const int p0 = j % NH, p1 = (j / NH) % NH, p2 = D == 3 ? j / (NH * NH) : 0;
      if (p0 < NL && p1 < NL && p2 < NL) { dM[j] = 0.0; continue; }
      const double tn = (double)yo[o] * stats[2 * F + O + o] + stats[2 * F + o];
      dM[j] = sc[p0 + p1 + p2] * tn;
      ++o;
    }
    lift_t<D, NL, NH, TH>(tab, f, gg, dM, fo, go);
    write_cell_t<S, D, NH, TH>(tab, g, bh, 1, off, fo, go);
    // 3D, x periodic: the image in the ghost column on the other side
    if constexpr (D == 3)
      if (xmir && (x < MSL_G || x >= g.nx - MSL_G))
        write_cell_t<S, D, NH, TH>(tab, g, bh, 1, x < MSL_G ? off + g.nx : off - g.nx, fo, go);
  }
}

// The learned lift of 3D athermal band cells, 64 cells per workgroup: wave 0
// reads the cells' populations, forms rho, u and the non-equilibrium parts
// f - f^eq (LDS), waves 1-3 stage the network outputs (LDS); then wave w
// computes the output layer c = w (the NH^2 high-order populations with
// z node c) of every cell, one cell per lane: the z, y, x passes of the
// separable completion and of the inverse-Vandermonde map of the learned
// moments, restricted to that layer (the same operations as the whole-cell
// form), so the stores of a wave are 64 consecutive cells of one plane.
// One wave per cell and set would hold every population and both transforms
// in registers (one wave per SIMD, with spills).
template <typename S, int NL, int NH>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
k_band_lift_mlp3(const Tab *__restrict__ tab, Geo g, const char *bl, char *bh,
                 const int *__restrict__ list, const int *__restrict__ count,
                 const float *__restrict__ stats, const float *__restrict__ yout,
                 const uint8_t *__restrict__ flags, int nct0, int nct1, int xmir) {
  constexpr int q = NL * NL * NL, Q = NH * NH * NH, F = nfeat<3, NL>(), O = nout<3, NL, NH>();
  static_assert(NH == 4, "one output layer per wave of four");
  __shared__ double s_neq[q][64];
  __shared__ float s_y[O][64];
  __shared__ double s_m[4][64];   // rho, u of each cell
  __shared__ int s_off[64], s_ioff[64];
  __shared__ uint8_t s_use[64], s_img[64];
  const LatTab &Lq = tab->lat[0], &LQ = tab->lat[1];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int n = *count;
  const int nct[3] = {nct0, nct1, 1};
  // the completion matrices, the inverse Vandermonde matrix and the output
  // statistics in LDS (read as broadcasts where they are used; as scalar
  // loads they were hoisted out of the walk over the cells into more scalar
  // registers than there are)
  __shared__ double s_K[3][NH][NL], s_V[NH][NH];
  __shared__ float s_mu[O], s_sd[O];
  // and the Hermite bases (for eq_axis) and storage scales of both sets
  struct EqTab {
    double hw[MSL_MAXN][MSL_MAXN];
    float hwf[MSL_MAXN][MSL_MAXN];
  };
  __shared__ EqTab s_eq[2];
  __shared__ double s_sc[2][Q];
  {
    for (int e = threadIdx.x; e < 2 * MSL_MAXN * MSL_MAXN; e += blockDim.x) {
      const int l = e / (MSL_MAXN * MSL_MAXN), r = (e / MSL_MAXN) % MSL_MAXN, cc = e % MSL_MAXN;
      s_eq[l].hw[r][cc] = tab->lat[l].hw[r][cc];
      s_eq[l].hwf[r][cc] = tab->lat[l].hwf[r][cc];
    }
    for (int e = threadIdx.x; e < 2 * Q; e += blockDim.x) s_sc[e / Q][e % Q] = tab->lat[e / Q].sc[e % Q];
    const bool herm = tab->lift_mode == MSL_LIFT_GRAD_HERMITE;
    for (int e = threadIdx.x; e < 3 * NH * NL; e += blockDim.x) {
      const int ax = e / (NH * NL), r = (e / NL) % NH, cc = e % NL;
      s_K[ax][r][cc] = herm ? tab->KH[r][cc] : tab->K[ax][r][cc];
    }
    for (int e = threadIdx.x; e < NH * NH; e += blockDim.x) s_V[e / NH][e % NH] = tab->Vi[e / NH][e % NH];
    for (int e = threadIdx.x; e < O; e += blockDim.x) {
      s_mu[e] = stats[2 * F + e];
      s_sd[e] = stats[2 * F + O + e];
    }
  }
  __syncthreads();
  for (long long t0 = (long long)blockIdx.x * 64; t0 < n; t0 += (long long)gridDim.x * 64) {
    const double (*Kx)[NL] = s_K[0];
    const double (*Ky)[NL] = s_K[1];
    const double (*Kz)[NL] = s_K[2];
    const double (*Vi)[NH] = s_V;
    const float *mu = s_mu, *sd = s_sd;
    const double *scq = s_sc[0], *scQ = s_sc[1];
    const EqTab *eqt = s_eq;
    const long long t = t0 + lane;
    const bool live = t < n;
    if (w == 0) {
      double f[q];
      double rho = 1.0, u[3] = {0.0, 0.0, 0.0};
      int off = 0, x = 0, y = 0, z = 0;
      if (live) {
        cell_coords(g, list[t], x, y, z);
        off = g.idx(x, y, z);
        const S *pl = (const S *)bl;
#pragma unroll
        for (int i = 0; i < q; ++i) f[i] = load_pop<S>(pl + (long long)i * g.plane, off, scq[i]);
        double T;
        macros_t<3, NL>(Lq, false, tab->cv, f, nullptr, rho, u, T);
      } else {
#pragma unroll
        for (int i = 0; i < q; ++i) f[i] = 0.0;
      }
      double Pq[3][NL];
#pragma unroll
      for (int a = 0; a < 3; ++a) eq_axis<double, NL>(eqt[0], (u[a] - Lq.ur[a]) * Lq.isq, Lq.iTr, Pq[a]);
#pragma unroll
      for (int i = 0; i < q; ++i) {
        const double e = rho * Pq[0][i % NL] * Pq[1][(i / NL) % NL] * Pq[2][i / (NL * NL)];
        s_neq[i][lane] = live ? f[i] - e : 0.0;
      }
      s_m[0][lane] = rho;
      s_m[1][lane] = u[0];
      s_m[2][lane] = u[1];
      s_m[3][lane] = u[2];
      s_off[lane] = off;
      s_ioff[lane] = x < MSL_G ? off + g.nx : off - g.nx;   // x image (periodic x)
      s_use[lane] = live && flags[check_tile(g, x, y, z, nct)] != 0;
      s_img[lane] = live && xmir && (x < MSL_G || x >= g.nx - MSL_G);
    } else {
      for (int o = w - 1; o < O; o += 3) s_y[o][lane] = live ? yout[t * O + o] : 0.f;
    }
    __syncthreads();
    const int c = __builtin_amdgcn_readfirstlane(w);   // this wave's output layer along z
    const double rho = s_m[0][lane];
    const double u[3] = {s_m[1][lane], s_m[2][lane], s_m[3][lane]};
    // equilibrium factors of the high-order set (T = 1)
    double PQ[3][NH];
#pragma unroll
    for (int a = 0; a < 3; ++a) eq_axis<double, NH>(eqt[1], (u[a] - LQ.ur[a]) * LQ.isq, LQ.iTr, PQ[a]);
    double pz = PQ[2][0];   // the layer's z factor
#pragma unroll
    for (int k = 1; k < NH; ++k)
      if (c == k) pz = PQ[2][k];
    // completion of the non-equilibrium part: z (to layer c), then y, then x
    double t1[NL * NL], t2[NL * NH];
#pragma unroll
    for (int k = 0; k < NL * NL; ++k) {
      double acc = 0;
#pragma unroll
      for (int cp = 0; cp < NL; ++cp) acc += Kz[c][cp] * s_neq[k + NL * NL * cp][lane];
      t1[k] = acc;
    }
#pragma unroll
    for (int b = 0; b < NH; ++b)
#pragma unroll
      for (int ap = 0; ap < NL; ++ap) {
        double acc = 0;
#pragma unroll
        for (int bp = 0; bp < NL; ++bp) acc += Ky[b][bp] * t1[ap + NL * bp];
        t2[ap + NL * b] = acc;
      }
    // the learned moments dM_p = rho T^{|p|/2} t_p (T = 1: rho) of the
    // indices p outside the low-order block, mapped by (Vi x Vi x Vi)
    const double sc0 = s_use[lane] ? rho : 0.0;
    double v1[NH * NH], v2[NH * NH];
#pragma unroll
    for (int k = 0; k < NH * NH; ++k) {
      double acc = 0;
#pragma unroll
      for (int cp = 0; cp < NH; ++cp) {
        const int j = k + NH * NH * cp, p0 = j % NH, p1 = (j / NH) % NH;
        if (p0 < NL && p1 < NL && cp < NL) continue;   // dM = 0 in the low-order block
        const int o = out_index<NL, NH>(j);
        const double tn = (double)s_y[o][lane] * sd[o] + mu[o];
        acc += Vi[c][cp] * (sc0 * tn);
      }
      v1[k] = acc;
    }
#pragma unroll
    for (int b = 0; b < NH; ++b)
#pragma unroll
      for (int ap = 0; ap < NH; ++ap) {
        double acc = 0;
#pragma unroll
        for (int bp = 0; bp < NH; ++bp) acc += Vi[b][bp] * v1[ap + NH * bp];
        v2[ap + NH * b] = acc;
      }
    const bool live2 = t0 + lane < n;
    const int off = s_off[lane];
    const bool img = s_img[lane];
    const int ioff = s_ioff[lane];
    S *p = (S *)bh;
#pragma unroll
    for (int b = 0; b < NH; ++b)
#pragma unroll
      for (int a = 0; a < NH; ++a) {
        double ck = 0, cv = 0;   // the x passes of the two maps
#pragma unroll
        for (int ap = 0; ap < NL; ++ap) ck += Kx[a][ap] * t2[ap + NL * b];
#pragma unroll
        for (int ap = 0; ap < NH; ++ap) cv += Vi[a][ap] * v2[ap + NH * b];
        const int i = a + NH * (b + NH * c);
        double fo = rho * PQ[0][a] * PQ[1][b] * pz + ck;
        fo += cv;
        if (live2) {
          store_pop<S>(p + (long long)i * g.plane, off, fo, scQ[i]);
          if (img) store_pop<S>(p + (long long)i * g.plane, ioff, fo, scQ[i]);
        }
      }
    __syncthreads();   // the next group overwrites the staged values
  }
}

// error check, stage 1: for the high-order band cells, the standardised
// features of their projected state and their true normalised targets
template <typename S, int D, int NL, int NH, bool TH>
__global__ void __launch_bounds__(64)
k_check_prepare(const Tab *__restrict__ tab, Geo g, const char *bh, const int *__restrict__ list,
                const int *__restrict__ count, const float *__restrict__ stats,
                float *__restrict__ feat, float *__restrict__ tgt) {
  constexpr int q = Pow<D, NL>::v, Q = Pow<D, NH>::v, F = nfeat<D, NL>(), O = nout<D, NL, NH>();
  const int n = *count;
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < n;
       t += (long long)gridDim.x * blockDim.x) {
    int x, y, z;
    cell_coords(g, list[t], x, y, z);
    double fQ[Q], gQ[TH ? Q : 1], fq[q], gq[TH ? q : 1], ft[F], tt[O];
    read_cell_t<S, D, NH, TH>(tab, g, bh, 1, g.idx(x, y, z), fQ, gQ);
    project_t<D, NL, NH, TH>(tab, fQ, gQ, fq, gq);
    features_t<D, NL, TH>(tab, fq, gq, ft);
    targets_t<D, NL, NH, TH>(tab, fQ, gQ, tt);
#pragma unroll
    for (int a = 0; a < F; ++a) feat[t * F + a] = (float)std_feature(ft[a], stats[a], stats[F + a]);
#pragma unroll
    for (int a = 0; a < O; ++a) tgt[t * O + a] = (float)tt[a];
  }
}

// stage 2: per-cell squared errors of the network and of Grad (zero) lifting
__global__ void __launch_bounds__(256)
k_check_cells(const int *__restrict__ count, const float *__restrict__ stats, int F,
                              int O, const float *__restrict__ yout, const float *__restrict__ tgt,
                              double *__restrict__ cerr) {
  const int n = *count;
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < n;
       t += (long long)gridDim.x * blockDim.x) {
    double em = 0, eg = 0;
    for (int o = 0; o < O; ++o) {
      const double tn = (double)yout[t * O + o] * stats[2 * F + O + o] + stats[2 * F + o];
      const double tr = tgt[t * O + o];
      em += (tn - tr) * (tn - tr);
      eg += tr * tr;
    }
    cerr[2 * t] = em;
    cerr[2 * t + 1] = eg;
  }
}

// stage 3: per check tile sums.  One block per tile.  The list is ascending in
// cell index, so the cells of a tile lie in the slab of list entries whose
// outermost coordinate falls in the tile's range; the block finds that slab by
// bisection and sums the entries of its own tile in a fixed order (strided per
// thread, then a fixed tree), so the sums do not depend on scheduling.
__global__ void __launch_bounds__(256)
k_check_tiles(Geo g, const int *__restrict__ list, const int *__restrict__ count,
              const double *__restrict__ cerr, int nct0, int nct1, double *__restrict__ terr) {
  __shared__ double rem[256], reg[256];
  __shared__ int rhas[256];
  __shared__ int range[2];
  const int tl = blockIdx.x;
  const int nct[3] = {nct0, nct1, 1};
  if (threadIdx.x < 2) {
    const int n = *count;
    const int outer = g.dim == 3 ? tl / (nct0 * nct1) : tl / nct0;
    const long long S = g.dim == 3 ? (long long)g.nx * g.ny : (long long)g.nx;
    const int NO = g.dim == 3 ? g.nz : g.ny;
    const int e = min((outer + threadIdx.x) * MSL_CHECK_TILE, NO);
    const long long key = (long long)e * S;
    int lo = 0, hi = n;           // first entry with list[t] >= key
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if ((long long)list[mid] < key) lo = mid + 1;
      else hi = mid;
    }
    range[threadIdx.x] = lo;
  }
  __syncthreads();
  double em = 0, eg = 0;
  int has = 0;
  for (int t = range[0] + threadIdx.x; t < range[1]; t += blockDim.x) {
    int x, y, z;
    cell_coords(g, list[t], x, y, z);
    if (check_tile(g, x, y, z, nct) != tl) continue;
    em += cerr[2 * t];
    eg += cerr[2 * t + 1];
    has = 1;
  }
  rem[threadIdx.x] = em;
  reg[threadIdx.x] = eg;
  rhas[threadIdx.x] = has;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      rem[threadIdx.x] += rem[threadIdx.x + w];
      reg[threadIdx.x] += reg[threadIdx.x + w];
      rhas[threadIdx.x] |= rhas[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    terr[2 * tl] = rem[0];
    terr[2 * tl + 1] = rhas[0] ? reg[0] : -1.0;
  }
}

// stage 4: the flags.  A tile uses the network where its summed error is below
// the Grad completion's; tiles without high-order band cells follow the totals
// over the domain; ties (an equilibrium state, where both vanish) go to Grad.
// One block, fixed-order sums.
__global__ void __launch_bounds__(256)
k_check_flags(int ntile, const double *__restrict__ terr, uint8_t *__restrict__ flags) {
  __shared__ double rem[256], reg[256];
  double em = 0, eg = 0;
  for (int tl = threadIdx.x; tl < ntile; tl += blockDim.x)
    if (terr[2 * tl + 1] >= 0) {
      em += terr[2 * tl];
      eg += terr[2 * tl + 1];
    }
  rem[threadIdx.x] = em;
  reg[threadIdx.x] = eg;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      rem[threadIdx.x] += rem[threadIdx.x + w];
      reg[threadIdx.x] += reg[threadIdx.x + w];
    }
    __syncthreads();
  }
  const double tm = rem[0], tg = reg[0];
  for (int tl = threadIdx.x; tl < ntile; tl += blockDim.x) {
    const bool has = terr[2 * tl + 1] >= 0;
    flags[tl] = has ? (terr[2 * tl] < terr[2 * tl + 1]) : (tm < tg);
  }
}

// snapshots from a run on the high-order set: every cell's projected features
// and true targets (rows in cell order)
template <typename S, int D, int NL, int NH, bool TH>
__global__ void __launch_bounds__(64)
k_snapshots(const Tab *__restrict__ tab, Geo g, const char *bh, long long nmax,
            float *__restrict__ feat, float *__restrict__ tgt) {
  constexpr int q = Pow<D, NL>::v, Q = Pow<D, NH>::v, F = nfeat<D, NL>(), O = nout<D, NL, NH>();
  const long long n = g.ncell < nmax ? g.ncell : nmax;
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < n;
       k += (long long)gridDim.x * blockDim.x) {
    int x, y, z;
    cell_coords(g, k, x, y, z);
    double fQ[Q], gQ[TH ? Q : 1], fq[q], gq[TH ? q : 1], ft[F], tt[O];
    read_cell_t<S, D, NH, TH>(tab, g, bh, 1, g.idx(x, y, z), fQ, gQ);
    project_t<D, NL, NH, TH>(tab, fQ, gQ, fq, gq);
    features_t<D, NL, TH>(tab, fq, gq, ft);
    targets_t<D, NL, NH, TH>(tab, fQ, gQ, tt);
#pragma unroll
    for (int a = 0; a < F; ++a) feat[k * F + a] = (float)ft[a];
#pragma unroll
    for (int a = 0; a < O; ++a) tgt[k * O + a] = (float)tt[a];
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static inline int lerr() { return hipGetLastError() == hipSuccess ? MSL_OK : MSL_EHIP; }

// gpart: gradient partials [nblk][P] followed, at lbase, by the loss partials
// (nullptr: the workspace's, laid out for MSL_MLP_MAXBLK workgroups)
template <int MODE>
static int mlp_launch(msl_ctx *c, const float *X, const float *Y, int n, const int *n_dev,
                      float *out, float inv_count, int nblk, float *gpart = nullptr,
                      long long lbase = -1) {
  const int F = c->mlpF, O = c->mlpO, H = c->mlpH;
  const int FPd = (F + 15) / 16 * 16, OPd = (O + 15) / 16 * 16;
  const dim3 grid(nblk), block(256);
  if (!gpart) {
    gpart = c->mlp_gpart;
    lbase = (long long)MSL_MLP_MAXBLK * c->mlpP;
  }
#define MLP_CASE(FPv, Hv, OPv)                                                                    \
  if (FPd == FPv && H == Hv && OPd == OPv) {                                                      \
    hipLaunchKernelGGL((k_mlp<FPv, Hv, OPv, MODE>), grid, block, 0, c->stream, c->mlp_w, F, O, X, \
                       Y, n, n_dev, out, gpart, lbase, inv_count);                                \
    return lerr();                                                                                \
  }
  MLP_CASE(16, 64, 16)
  MLP_CASE(16, 64, 32)
  MLP_CASE(16, 64, 48)
  MLP_CASE(32, 64, 48)
  MLP_CASE(32, 64, 32)
  MLP_CASE(16, 32, 16)
  MLP_CASE(16, 32, 32)
  MLP_CASE(32, 32, 48)
#undef MLP_CASE
  return MSL_EINVAL;
}

template <typename F>
static int store_dispatch(int store, F &&f) {
  switch (store) {
    case MSL_FP64: return f.template operator()<double>();
    case MSL_FP32: return f.template operator()<float>();
    case MSL_FP16_DEV: return f.template operator()<_Float16>();
    case MSL_BF16_DEV: return f.template operator()<bf16_t>();
  }
  return MSL_EINVAL;
}

template <typename F>
static int thermal_dispatch(int thermal, F &&f) {
  return thermal ? f.template operator()<true>() : f.template operator()<false>();
}

int msl_mlp_band_lift(msl_ctx *c, char *bl, char *bh) {
  if (!c->mlp_on) return MSL_OK;
  int rc = store_dispatch(c->cfg.store, [&]<typename S>() {
    return msl_pair_dispatch(c->D, c->htab.lat[0].n, c->htab.lat[1].n, [&]<int D, int NL, int NH>() {
      if (nfeat<D, NL>() != c->mlpF || nout<D, NL, NH>() != c->mlpO) return (int)MSL_EINVAL;
      return thermal_dispatch(c->cfg.thermal, [&]<bool TH>() {
        hipLaunchKernelGGL((k_band_features<S, D, NL, TH>), dim3(2048), dim3(64), 0, c->stream,
                           c->dtab, c->geo, bl, c->blist[0], c->bcount, c->mlp_stats, c->mlp_feat);
        return lerr();
      });
    });
  });
  if (rc) return rc;
  // 768 workgroups: three per CU, as many as its LDS (50 KB each) and
  // registers hold (measured 6 % faster than two per CU on the 3D band)
  rc = mlp_launch<0>(c, c->mlp_feat, nullptr, 0, c->bcount, c->mlp_out, 0.f, 768);
  if (rc) return rc;
  return store_dispatch(c->cfg.store, [&]<typename S>() {
    return msl_pair_dispatch(c->D, c->htab.lat[0].n, c->htab.lat[1].n, [&]<int D, int NL, int NH>() {
      return thermal_dispatch(c->cfg.thermal, [&]<bool TH>() {
        if constexpr (D == 3 && !TH) {
          hipLaunchKernelGGL((k_band_lift_mlp3<S, NL, NH>), dim3(512), dim3(256), 0, c->stream,
                             c->dtab, c->geo, bl, bh, c->blist[0], c->bcount, c->mlp_stats,
                             c->mlp_out, c->mlp_flag, c->nct[0], c->nct[1], c->xmir);
        } else {
          hipLaunchKernelGGL((k_band_lift_mlp<S, D, NL, NH, TH>), dim3(2048), dim3(64), 0, c->stream,
                             c->dtab, c->geo, bl, bh, c->blist[0], c->bcount, c->mlp_stats,
                             c->mlp_out, c->mlp_flag, c->nct[0], c->nct[1], c->xmir);
        }
        return lerr();
      });
    });
  });
}

int msl_mlp_check_launch(msl_ctx *c) {
  if (!c->mlp_on) return MSL_OK;
  char *bh = c->planes[1][c->cur];
  int rc = store_dispatch(c->cfg.store, [&]<typename S>() {
    return msl_pair_dispatch(c->D, c->htab.lat[0].n, c->htab.lat[1].n, [&]<int D, int NL, int NH>() {
      if (nfeat<D, NL>() != c->mlpF || nout<D, NL, NH>() != c->mlpO) return (int)MSL_EINVAL;
      return thermal_dispatch(c->cfg.thermal, [&]<bool TH>() {
        hipLaunchKernelGGL((k_check_prepare<S, D, NL, NH, TH>), dim3(2048), dim3(64), 0, c->stream,
                           c->dtab, c->geo, bh, c->blist[1], c->bcount + 1, c->mlp_stats,
                           c->mlp_feat, c->mlp_tgt);
        return lerr();
      });
    });
  });
  if (rc) return rc;
  rc = mlp_launch<0>(c, c->mlp_feat, nullptr, 0, c->bcount + 1, c->mlp_out, 0.f, 768);
  if (rc) return rc;
  hipLaunchKernelGGL(k_check_cells, dim3(512), dim3(256), 0, c->stream, c->bcount + 1,
                     c->mlp_stats, c->mlpF, c->mlpO, c->mlp_out, c->mlp_tgt, c->mlp_cerr);
  hipLaunchKernelGGL(k_check_tiles, dim3(c->nctile), dim3(256), 0, c->stream, c->geo, c->blist[1],
                     c->bcount + 1, c->mlp_cerr, c->nct[0], c->nct[1], c->mlp_err);
  hipLaunchKernelGGL(k_check_flags, dim3(1), dim3(256), 0, c->stream, c->nctile, c->mlp_err,
                     c->mlp_flag);
  return lerr();
}

// ---- gradient without workspace scratch ----
// The gradient and loss partials of msl_mlp_grad_noalloc live in this
// file-scope device array (one copy per GPU, held until the process ends)
// instead of the context's workspace.  Host code never passes the array's
// name to a kernel or a copy: it uses the device address that
// hipGetSymbolAddress returns, looked up once per device when the first
// context is created on that device.
#define MSL_NOALLOC_FLOATS (1 << 20)   // 4 MiB
static __device__ __align__(256) float scratch[MSL_NOALLOC_FLOATS];
#define MSL_NOALLOC_MAXDEV 64
static float *g_scratch_ptr[MSL_NOALLOC_MAXDEV];
static std::mutex g_scratch_mu;

// called by msl_create with `device` current
int msl_noalloc_setup(int device) {
  if (device < 0 || device >= MSL_NOALLOC_MAXDEV) return MSL_EINVAL;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return MSL_OK;
  void *ptr = nullptr;
  if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return MSL_EHIP;
  g_scratch_ptr[device] = (float *)ptr;
  return MSL_OK;
}

extern "C" {

int msl_mlp_dims(const msl_ctx *c, int *F, int *O, int *H, int *P) {
  if (!c) return MSL_EINVAL;
  if (F) *F = c->mlpF;
  if (O) *O = c->mlpO;
  if (H) *H = c->mlpH;
  if (P) *P = c->mlpP;
  return MSL_OK;
}

int msl_collect_snapshots(msl_ctx *c, float *feats, float *targets, int max, int *n) {
  if (!c || !feats || !targets || !n || max < 0 || !c->mlpP) return MSL_EINVAL;
  if (!c->initialized) return MSL_ESTATE;
  int nh = 0;
  MSL_HIP(hipMemcpyAsync(&nh, c->bcount + 2, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  MSL_HIP(hipStreamSynchronize(c->stream));
  if (nh != c->ncell) return MSL_ESTATE;   // snapshots come from a run on the high-order set
  char *bh = c->planes[1][c->cur];
  int rc = store_dispatch(c->cfg.store, [&]<typename S>() {
    return msl_pair_dispatch(c->D, c->htab.lat[0].n, c->htab.lat[1].n, [&]<int D, int NL, int NH>() {
      if (nfeat<D, NL>() != c->mlpF || nout<D, NL, NH>() != c->mlpO) return (int)MSL_EINVAL;
      return thermal_dispatch(c->cfg.thermal, [&]<bool TH>() {
        hipLaunchKernelGGL((k_snapshots<S, D, NL, NH, TH>), dim3(4096), dim3(64), 0, c->stream,
                           c->dtab, c->geo, bh, (long long)max, feats, targets);
        return lerr();
      });
    });
  });
  if (rc) return rc;
  MSL_HIP(hipStreamSynchronize(c->stream));
  *n = (int)(c->ncell < max ? c->ncell : max);
  return MSL_OK;
}

int msl_mlp_set_weights(msl_ctx *c, const float *params, const float *xmean, const float *xstd,
                        const float *tmean, const float *tstd) {
  if (!c || !params || !xmean || !xstd || !tmean || !tstd || !c->mlpP) return MSL_EINVAL;
  const int F = c->mlpF, O = c->mlpO;
  float *st = (float *)malloc(sizeof(float) * (2 * F + 2 * O));
  memcpy(st, xmean, sizeof(float) * F);
  memcpy(st + F, xstd, sizeof(float) * F);
  memcpy(st + 2 * F, tmean, sizeof(float) * O);
  memcpy(st + 2 * F + O, tstd, sizeof(float) * O);
  for (int a = 0; a < F; ++a)
    if (!(st[F + a] > 0.f)) st[F + a] = 1.f;
  for (int a = 0; a < O; ++a)
    if (!(st[2 * F + O + a] > 0.f)) st[2 * F + O + a] = 1.f;
  hipError_t e1 = hipMemcpyAsync(c->mlp_w, params, sizeof(float) * c->mlpP, hipMemcpyHostToDevice, c->stream);
  hipError_t e2 = hipMemcpyAsync(c->mlp_stats, st, sizeof(float) * (2 * F + 2 * O), hipMemcpyHostToDevice, c->stream);
  hipError_t e3 = hipMemsetAsync(c->mlp_m, 0, sizeof(float) * c->mlpP, c->stream);
  hipError_t e4 = hipMemsetAsync(c->mlp_v, 0, sizeof(float) * c->mlpP, c->stream);
  hipError_t e5 = hipStreamSynchronize(c->stream);
  free(st);
  if (e1 || e2 || e3 || e4 || e5) return MSL_EHIP;
  c->mlp_steps = 0;
  c->mlp_on = 1;
  return MSL_OK;
}

int msl_mlp_get_weights(msl_ctx *c, float *params) {
  if (!c || !params || !c->mlpP) return MSL_EINVAL;
  MSL_HIP(hipMemcpyAsync(params, c->mlp_w, sizeof(float) * c->mlpP, hipMemcpyDeviceToHost, c->stream));
  MSL_HIP(hipStreamSynchronize(c->stream));
  return MSL_OK;
}

int msl_mlp_forward(msl_ctx *c, const float *X, int n, float *Yout) {
  if (!c || !X || !Yout || n < 0 || !c->mlpP) return MSL_EINVAL;
  int rc = mlp_launch<0>(c, X, nullptr, n, nullptr, Yout, 0.f, 256);
  if (rc) return rc;
  MSL_HIP(hipStreamSynchronize(c->stream));
  return MSL_OK;
}

static int grad_step(msl_ctx *c, const float *X, const float *Y, int n, int apply, float lr,
                     float *gout, float *loss_dev, float *gpart = nullptr, long long lbase = -1) {
  if (n <= 0 || n > MSL_MLP_MAXBLK * 64) return MSL_EINVAL;
  const int nblk = (n + 63) / 64;
  if (!gpart) {
    gpart = c->mlp_gpart;
    lbase = (long long)MSL_MLP_MAXBLK * c->mlpP;
  }
  const float invc = 1.f / ((float)n * (float)c->mlpO);
  int rc = mlp_launch<1>(c, X, Y, n, nullptr, nullptr, invc, nblk, gpart, lbase);
  if (rc) return rc;
  const int t = apply ? (int)(++c->mlp_steps) : 1;
  hipLaunchKernelGGL(k_mlp_reduce_adam, dim3((c->mlpP + 255) / 256), dim3(256), 0, c->stream,
                     c->mlp_w, c->mlp_m, c->mlp_v, gout, gpart, lbase, c->mlpP, nblk, apply, t,
                     lr, 0.9f, 0.999f, 1e-8f, loss_dev, invc);
  return lerr();
}

int msl_mlp_grad(msl_ctx *c, const float *X, const float *Y, int n, float *loss, float *grad) {
  if (!c || !X || !Y || !grad || !c->mlpP) return MSL_EINVAL;
  int rc = grad_step(c, X, Y, n, 0, 0.f, grad, c->mlp_loss);
  if (rc) return rc;
  float l = 0.f;
  MSL_HIP(hipMemcpyAsync(&l, c->mlp_loss, sizeof(float), hipMemcpyDeviceToHost, c->stream));
  MSL_HIP(hipStreamSynchronize(c->stream));
  if (loss) *loss = l;
  return MSL_OK;
}

int msl_mlp_grad_noalloc(msl_ctx *c, const float *X, const float *Y, int n, float *loss,
                         float *grad) {
  if (!c || !X || !Y || !grad || !c->mlpP || n <= 0 || n > MSL_MLP_MAXBLK * 64) return MSL_EINVAL;
  const int nblk = (n + 63) / 64;
  // gradient partials [nblk][P], loss partials [nblk], the loss
  const long long need = (long long)nblk * c->mlpP + nblk + 1;
  if (need > MSL_NOALLOC_FLOATS) {
    snprintf(c->err, sizeof(c->err),
             "msl_mlp_grad_noalloc: %d rows need %lld floats of scratch, the static array holds %d",
             n, need, MSL_NOALLOC_FLOATS);
    return MSL_EINVAL;
  }
  float *sp = c->device >= 0 && c->device < MSL_NOALLOC_MAXDEV ? g_scratch_ptr[c->device] : nullptr;
  if (!sp) return MSL_ESTATE;
  const long long lbase = (long long)nblk * c->mlpP;
  float *loss_dev = sp + lbase + nblk;
  int rc = grad_step(c, X, Y, n, 0, 0.f, grad, loss_dev, sp, lbase);
  if (rc) return rc;
  float l = 0.f;
  MSL_HIP(hipMemcpyAsync(&l, loss_dev, sizeof(float), hipMemcpyDeviceToHost, c->stream));
  MSL_HIP(hipStreamSynchronize(c->stream));
  if (loss) *loss = l;
  return MSL_OK;
}

int msl_mlp_train(msl_ctx *c, const float *X, const float *Y, int n, int batch, int epochs,
                  float lr, float *loss_log) {
  if (!c || !X || !Y || n <= 0 || batch <= 0 || batch > MSL_MLP_MAXBLK * 64 || epochs < 0 ||
      !c->mlpP)
    return MSL_EINVAL;
  if (!c->mlp_on) return MSL_ESTATE;   // weights must be installed first
  const int steps_per_epoch = (n + batch - 1) / batch;
  long s = 0;
  for (int e = 0; e < epochs; ++e)
    for (int b = 0; b < steps_per_epoch; ++b, ++s) {
      const int r0 = b * batch, rows = n - r0 < batch ? n - r0 : batch;
      int rc = grad_step(c, X + (long long)r0 * c->mlpF, Y + (long long)r0 * c->mlpO, rows, 1, lr,
                         nullptr, c->mlp_loss + (s % MSL_MLP_LOSS_RING));
      if (rc) return rc;
    }
  MSL_HIP(hipStreamSynchronize(c->stream));
  if (loss_log) {
    const long keep = s < MSL_MLP_LOSS_RING ? s : MSL_MLP_LOSS_RING;
    MSL_HIP(hipMemcpy(loss_log, c->mlp_loss, sizeof(float) * keep, hipMemcpyDeviceToHost));
  }
  return MSL_OK;
}

int msl_mlp_get_flags(msl_ctx *c, uint8_t *flags) {
  if (!c || !flags || !c->mlpP) return MSL_EINVAL;
  MSL_HIP(hipMemcpyAsync(flags, c->mlp_flag, c->nctile, hipMemcpyDeviceToDevice, c->stream));
  return MSL_OK;
}

int msl_mlp_set_flags(msl_ctx *c, const uint8_t *flags) {
  if (!c || !flags || !c->mlpP) return MSL_EINVAL;
  MSL_HIP(hipMemcpyAsync(c->mlp_flag, flags, c->nctile, hipMemcpyDeviceToDevice, c->stream));
  c->mlp_manual = 1;
  return MSL_OK;
}

}  // extern "C"
