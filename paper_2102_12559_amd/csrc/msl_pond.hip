// msl_pond.hip -- the step in co-moving reference frames (PonD, Sec. II.C.1),
// one or two velocity sets, 2D, FP64.
//
// Every cell keeps its post-collision populations in its own frame
// lambda = {u, T} (eq. reference; particle velocities sqrt(T) c_i + u, eq. vi,
// with T_L = 1).  A group of GS lanes (GS = the power of two >= Q) owns one
// cell, one lane per population; a workgroup's cells are one x segment of a
// row, and the 5-row neighbourhood of the segment (populations and frames,
// boundary rules applied) is staged in LDS once.  Per iteration of the
// predictor-corrector:
// each lane finds its population's departure point x - v_i dt in the current
// frame, and for each of the 3 x 3 collocation points around the nearest node
// transfers that point's population vector from its own frame to the current
// one and keeps its own component (eqs. reconstructionPond, fll).  The
// transfer G = M_target^{-1} M_source of the moment matrices of eq. momf
// factorises per axis, and its one-axis factor is the Lagrange basis of the
// lattice nodes evaluated at the source nodes mapped into the target frame:
//   G_x[a][a'] = l_a((sqrt(T_s) c_a' + u_s,x - u_x) / sqrt(T)),
// because the inverse of a Vandermonde matrix holds the Lagrange basis
// polynomials of its nodes.  The group then sums rho, j, E of the
// reconstructed populations (shuffles within the group), which define the
// next frame (eqs. correctorfields), until neither a velocity component nor T
// changes by more than 1e-14 (at most 60 passes).  The collision runs in the
// converged frame, where f^eq = rho W_i and g^eq = (cv - 1) T rho W_i (eqs.
// feqPond, geqPond), BGK or two-relaxation (eqs. fqeq, gqeq in the co-moving
// frame).
// With two velocity sets (Sec. III) the step launches once per set, over the
// cells of that set; afterwards every band cell (within two cells of the other
// set) converts its new state into the other set in its own new frame
// (lifting or projection, Sec. III.B-C), so a collocation point of the other
// set holds this set's populations in its own frame when the next step reads
// it.  The Knudsen-number criterion re-selects the sets every crit_every
// steps from each cell's own state; a cell whose set changes converts its
// state in its own frame.
#include <hip/hip_runtime.h>

#include "msl_band.hpp"

#define POND_MAXIT 60
#define POND_TOL 1e-14

struct PondArgs {
  int nx, ny;
  long long ncell;
  int bc[4];
  double st[4][5];   // fixed-equilibrium face states rho, ux, uy, uz, T
};

template <int GS>
__device__ __forceinline__ double group_sum(double v) {
#pragma unroll
  for (int o = GS / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, GS);
  return v;
}

template <int N, bool TH>
struct PondTraits {
  static constexpr int Q = N * N;
  static constexpr int NP = TH ? 2 * Q : Q;
  static constexpr int GS = Q <= 16 ? 16 : (Q <= 32 ? 32 : 64);
  static constexpr int TW = 256 / GS;         // cells of a workgroup: one x segment of a row
  static constexpr int SW = TW + 4;           // staged columns (two on each side)
  static constexpr int SP = SW * 5;           // staged collocation points (five rows)
  static constexpr int STRIDE = NP + 4;       // doubles per staged point: populations, frame
};

// the collocation point (x, y) (possibly outside the domain): the cell index
// whose state it takes, -1 - face for a fixed-equilibrium face state, or
// -5 - (side nx + x) for the diffuse wall point of column x on the low (side
// 0) or high y face
__device__ __forceinline__ long long pond_resolve(const PondArgs &pa, int x, int y) {
  if (x < 0 && pa.bc[0] == MSL_BC_FIXED_EQ) return -1;
  if (x >= pa.nx && pa.bc[1] == MSL_BC_FIXED_EQ) return -2;
  if (y < 0 && pa.bc[2] == MSL_BC_FIXED_EQ) return -3;
  if (y >= pa.ny && pa.bc[3] == MSL_BC_FIXED_EQ) return -4;
  if (x < 0 || x >= pa.nx) x = pa.bc[0] == MSL_BC_PERIODIC ? (x + pa.nx) % pa.nx : (x < 0 ? 0 : pa.nx - 1);
  if (y < 0 && pa.bc[2] == MSL_BC_DIFFUSE_WALL) return -5 - (long long)x;
  if (y >= pa.ny && pa.bc[3] == MSL_BC_DIFFUSE_WALL) return -5 - ((long long)pa.nx + x);
  if (y < 0 || y >= pa.ny) y = pa.bc[2] == MSL_BC_PERIODIC ? (y + pa.ny) % pa.ny : (y < 0 ? 0 : pa.ny - 1);
  return (long long)y * pa.nx + x;
}

template <int N, bool TH, bool QE>
__global__ void __launch_bounds__(256)
k_pond_step(const Tab *__restrict__ tab, int lat, const uint8_t *__restrict__ cls, PondArgs pa,
            const double *__restrict__ fin, const double *__restrict__ frin, double *__restrict__ fout,
            double *__restrict__ frout, int *__restrict__ flag, unsigned long long *__restrict__ itsum,
            int *__restrict__ itmax, const double *__restrict__ wrho) {
  using Tr = PondTraits<N, TH>;
  constexpr int Q = Tr::Q, NP = Tr::NP, GS = Tr::GS, TW = Tr::TW, SW = Tr::SW, SP = Tr::SP,
                STRIDE = Tr::STRIDE;
  // the workgroup's cells: x in [x0, x0 + TW) of row y; their collocation
  // points lie within two cells, so the SW x 5 points around the segment
  // (populations and frames, boundary rules applied) are staged in LDS once
  __shared__ double stg[SP * STRIDE];
  const LatTab &L = tab->lat[lat];
  const int x0 = blockIdx.x * TW, y = blockIdx.y;
  const double dt = tab->dt, cv = tab->cv;
  for (int e = threadIdx.x; e < SP * STRIDE; e += 256) {
    const int sp = e / STRIDE, m = e - sp * STRIDE;
    const int sx = x0 - 2 + sp % SW, sy = y - 2 + sp / SW;
    const long long q = pond_resolve(pa, sx, sy);
    double v;
    if (q >= 0) {
      v = m < NP ? fin[(long long)m * pa.ncell + q] : frin[(long long)(m - NP) * pa.ncell + q];
    } else {
      // a fixed-equilibrium face state, or a diffuse wall point at the wall
      // state with the column's wall density: rho W_i (and (cv - 1) T rho W_i)
      // in its own frame
      const bool wall = q <= -5;
      const long long wi = wall ? -5 - q : 0;
      const double *st = wall ? pa.st[wi < pa.nx ? 2 : 3] : pa.st[-1 - q];
      const double rs = wall ? wrho[wi] : st[0];
      const double Ts = TH ? st[4] : 1.0;
      const int j = m % Q;
      const double fj = rs * L.w[j % N] * L.w[j / N];
      if (m < Q) v = fj;
      else if (m < NP) v = (cv - 1.0) * Ts * fj;
      else v = m - NP == 0 ? st[1] : (m - NP == 1 ? st[2] : (m - NP == 2 ? 0.0 : Ts));
    }
    stg[e] = v;
  }
  __syncthreads();
  const int c = threadIdx.x / GS, li = threadIdx.x % GS;
  const int px = x0 + c, py = y;
  const long long k = (long long)py * pa.nx + (px < pa.nx ? px : 0);
  // cells of this launch's velocity set (with two sets)
  const bool cell_ok = px < pa.nx && (cls[k] & 1) == lat;
  const bool act = cell_ok && li < Q;
  const int i = act ? li : 0, a = i % N, b = i / N;
  // lattice nodes and the Lagrange denominators 1 / prod_{c != a} (x_a - x_c)
  double xn[N], den[N];
#pragma unroll
  for (int m = 0; m < N; ++m) xn[m] = L.cr[m];
#pragma unroll
  for (int m = 0; m < N; ++m) {
    double p = 1.0;
#pragma unroll
    for (int cc = 0; cc < N; ++cc)
      if (cc != m) p *= xn[m] - xn[cc];
    den[m] = 1.0 / p;
  }
  const double *own = stg + ((2) * SW + (c + 2)) * STRIDE + NP;
  double ux = own[0], uy = own[1], T = own[3];
  double ft = 0.0, gt = 0.0, rho = 0.0, Tn = 1.0;
  bool done = !cell_ok;
  int it = 0;
  for (int pass = 1; pass <= POND_MAXIT; ++pass) {
    double r = 0.0, jx = 0.0, jy = 0.0, e = 0.0;
    if (!done) {
      it = pass;
      const double sT = sqrt(T), isT = 1.0 / sT;
      const double vx = sT * xn[a] + ux, vy = sT * xn[b] + uy;
      const double dx = -vx * dt, dy = -vy * dt;
      const int nx0 = (int)floor(dx + 0.5), ny0 = (int)floor(dy + 0.5);
      const bool out = nx0 < -1 || nx0 > 1 || ny0 < -1 || ny0 > 1;
      if (act && out) atomicOr(flag, 1);
      // (a lane whose stencil left the reach reads the nearest staged points
      // instead; its cell is reported and its result is not used)
      const int ox = out ? 0 : nx0, oy = out ? 0 : ny0;
      const double xi = dx - nx0, yi = dy - ny0;
      // 3-point Lagrange weights through -1, 0, 1
      const double wx[3] = {0.5 * xi * (xi - 1.0), 1.0 - xi * xi, 0.5 * xi * (xi + 1.0)};
      const double wy[3] = {0.5 * yi * (yi - 1.0), 1.0 - yi * yi, 0.5 * yi * (yi + 1.0)};
      double accf = 0.0, accg = 0.0;
      for (int sy = -1; sy <= 1; ++sy)
        for (int sx = -1; sx <= 1; ++sx) {
          const double *pt = stg + ((oy + sy + 2) * SW + (c + 2 + ox + sx)) * STRIDE;
          const double usx = pt[NP], usy = pt[NP + 1], Ts = pt[NP + 3];
          // the transfer's rows of this lane's nodes a (x) and b (y)
          const double sTs = sqrt(Ts);
          double gx[N], gy[N];
#pragma unroll
          for (int m = 0; m < N; ++m) {
            const double zx = (sTs * xn[m] + usx - ux) * isT, zy = (sTs * xn[m] + usy - uy) * isT;
            double px_ = den[a], py_ = den[b];
#pragma unroll
            for (int cc = 0; cc < N; ++cc) {
              if (cc != a) px_ *= zx - xn[cc];
              if (cc != b) py_ *= zy - xn[cc];
            }
            gx[m] = px_;
            gy[m] = py_;
          }
          double vf = 0.0, vg = 0.0;
#pragma unroll
          for (int mb = 0; mb < N; ++mb) {
            double sf = 0.0, sg = 0.0;
#pragma unroll
            for (int ma = 0; ma < N; ++ma) {
              const int j = ma + N * mb;
              sf += gx[ma] * pt[j];
              if (TH) sg += gx[ma] * pt[Q + j];
            }
            vf += gy[mb] * sf;
            if (TH) vg += gy[mb] * sg;
          }
          const double w = wx[sx + 1] * wy[sy + 1];
          accf += w * vf;
          if (TH) accg += w * vg;
        }
      ft = accf;
      gt = TH ? accg : 0.0;
      if (act) {
        r = ft;
        jx = vx * ft;
        jy = vy * ft;
        e = 0.5 * (vx * vx + vy * vy) * ft + gt;
      }
    }
    // corrector: the group's sums (every lane of the wave takes part)
    r = group_sum<GS>(r);
    jx = group_sum<GS>(jx);
    jy = group_sum<GS>(jy);
    e = group_sum<GS>(e);
    if (!done) {
      const double nux = jx / r, nuy = jy / r;
      const double nT = TH ? (e / r - 0.5 * (nux * nux + nuy * nuy)) / cv : 1.0;
      if (!(r > 0.0) || !(nT > 0.0) || !isfinite(r)) {
        if (li == 0) atomicOr(flag, 2);
        done = true;
      } else {
        const double delta = fmax(fabs(nT - T), fmax(fabs(nux - ux), fabs(nuy - uy)));
        rho = r;
        Tn = nT;
        if (delta <= POND_TOL || pass == POND_MAXIT) {
          done = true;
        } else {
          ux = nux;
          uy = nuy;
          T = nT;
        }
      }
    }
    if (__all(done)) break;
  }
  // collision in the converged frame {ux, uy, T}
  double tl = tab->tau;
  if (tab->tau_mode == 1) tl = tab->mu_ref * pow(Tn / tab->tau_ref_T, tab->mu_exp) / (rho * Tn * dt) + 0.5;
  const double om = 1.0 / tl;
  const double W = L.w[a] * L.w[b];
  const double feq = rho * W, gq = (cv - 1.0) * T, geq = gq * rho * W;
  double fo = ft + om * (feq - ft), go = gt + om * (geq - gt);
  if constexpr (QE) {
    // quasi-equilibria in the co-moving frame (v - u = sqrt(T) c):
    // Qbar = T^{3/2} sum c c c (f - f^eq), qbar = T^{1/2} sum c (g - g^eq)
    const double om2 = 1.0 / (0.5 + (tl - 0.5) * tab->qe_ratio);
    const double cx = xn[a], cy = xn[b];
    const double nf = act ? ft - feq : 0.0, ng = act && TH ? gt - geq : 0.0;
    const double Qxxx = group_sum<GS>(cx * cx * cx * nf), Qxxy = group_sum<GS>(cx * cx * cy * nf);
    const double Qxyy = group_sum<GS>(cx * cy * cy * nf), Qyyy = group_sum<GS>(cy * cy * cy * nf);
    const double qx = group_sum<GS>(cx * ng), qy = group_sum<GS>(cy * ng);
    // f* - f^eq = W T^{-3/2}/6 Qbar : He3(c), Qbar = T^{3/2} (sums above)
    const double h = Qxxx * (cx * cx * cx - 3.0 * cx) + 3.0 * Qxxy * (cx * cx * cy - cy) +
                     3.0 * Qxyy * (cx * cy * cy - cx) + Qyyy * (cy * cy * cy - 3.0 * cy);
    fo += (om - om2) * W * h / 6.0;
    if (TH) go += (om - om2) * W * (qx * cx + qy * cy);
  }
  if (act) {
    fout[(long long)i * pa.ncell + k] = fo;
    if (TH) fout[(long long)(Q + i) * pa.ncell + k] = go;
    if (li == 0) {
      frout[k] = ux;
      frout[pa.ncell + k] = uy;
      frout[2 * pa.ncell + k] = 0.0;
      frout[3 * pa.ncell + k] = T;
      atomicAdd(itsum, (unsigned long long)it);
      atomicMax(itmax, it);
    }
  }
}

// every cell at the co-moving equilibrium of (rho, u, T) in its own frame, in
// each set (an equilibrium is the same state in both)
__global__ void k_pond_init(const Tab *__restrict__ tab, long long ncell, int thermal, int nlat,
                            const double *rho, const double *u, const double *T, double *f0, double *f1,
                            double *fr) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= ncell) return;
  const double Tk = thermal ? T[k] : 1.0;
  for (int l = 0; l < nlat; ++l) {
    const LatTab &L = tab->lat[l];
    double *f = l ? f1 : f0;
    for (int i = 0; i < L.Q; ++i) {
      const double W = L.w[i % L.n] * L.w[i / L.n];
      f[(long long)i * ncell + k] = rho[k] * W;
      if (thermal) f[(long long)(L.Q + i) * ncell + k] = (tab->cv - 1.0) * Tk * rho[k] * W;
    }
  }
  fr[k] = u[k];
  fr[ncell + k] = u[ncell + k];
  fr[2 * ncell + k] = 0.0;
  fr[3 * ncell + k] = Tk;
}

// rho, u, T of cell k from its populations (set l) in its own frame
__device__ __forceinline__ void pond_cell_macros(const Tab *tab, int l, long long ncell, int thermal,
                                                 const double *f, const double *fr, long long k, double &r,
                                                 double &ux, double &uy, double &T) {
  const LatTab &L = tab->lat[l];
  const double sT = sqrt(fr[3 * ncell + k]), fx = fr[k], fy = fr[ncell + k];
  double jx = 0, jy = 0, e = 0;
  r = 0;
  for (int i = 0; i < L.Q; ++i) {
    const double fi = f[(long long)i * ncell + k];
    const double vx = sT * L.cr[i % L.n] + fx, vy = sT * L.cr[i / L.n] + fy;
    r += fi;
    jx += vx * fi;
    jy += vy * fi;
    e += 0.5 * (vx * vx + vy * vy) * fi;
    if (thermal) e += f[(long long)(L.Q + i) * ncell + k];
  }
  ux = jx / r;
  uy = jy / r;
  T = thermal ? (e / r - 0.5 * (ux * ux + uy * uy)) / tab->cv : 1.0;
}

// rho, u, T of every cell from its own set's populations in its own frame
__global__ void k_pond_macros(const Tab *__restrict__ tab, long long ncell, int thermal, const double *f0,
                              const double *f1, const uint8_t *__restrict__ cls, const double *fr, double *rho,
                              double *u, double *T) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= ncell) return;
  const int l = cls[k] & 1;
  double r, ux, uy, t;
  pond_cell_macros(tab, l, ncell, thermal, l ? f1 : f0, fr, k, r, ux, uy, t);
  if (rho) rho[k] = r;
  if (u) {
    u[k] = ux;
    u[ncell + k] = uy;
  }
  if (T) T[k] = t;
}

// Knudsen-number criterion (Sec. IV.A.3), pass 1 on the co-moving state: each
// cell's density and hard-sphere mean free path
// lambda = 16/(5 sqrt(2 pi gamma)) mu a / p from its own set in its own frame
__global__ void k_pond_kn_fields(const Tab *__restrict__ tab, long long ncell, int thermal, const double *f0,
                                 const double *f1, const uint8_t *__restrict__ cls, const double *fr,
                                 double *__restrict__ rho, double *__restrict__ lam) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= ncell) return;
  const int l = cls[k] & 1;
  double r, ux, uy, T;
  pond_cell_macros(tab, l, ncell, thermal, l ? f1 : f0, fr, k, r, ux, uy, T);
  const double mu = tab->tau_mode == 1 ? tab->mu_ref * pow(T / tab->tau_ref_T, tab->mu_exp)
                                       : (tab->tau - 0.5) * r * T * tab->dt;
  const double gam = (tab->cv + 1.0) / tab->cv;
  rho[k] = r;
  lam[k] = 16.0 / (5.0 * sqrt(2.0 * M_PI * gam)) * mu * sqrt(gam * T) / (r * T);
}

// Raw completion along one axis in the frame v = s c + u: the degree < NL
// part of each high-order Lagrange basis polynomial written in the particle
// velocity v, evaluated at the low-order velocities.  The basis in c has the
// monomial coefficients Vi (the inverse Vandermonde matrix of the high-order
// nodes); ((v - u)/s)^k = s^-k sum_p C(k, p) v^p (-u)^(k-p) re-expands it in v.
template <int NL, int NH>
__device__ __forceinline__ void frame_completion(const Tab *tab, double s, double u, double (*K)[NL]) {
  const LatTab &Lq = tab->lat[0];
  double C[NH][NH], mu[NH];
#pragma unroll
  for (int k = 0; k < NH; ++k)
#pragma unroll
    for (int p = 0; p < NH; ++p) C[k][p] = (p == 0 || p == k) ? 1.0 : (p > k ? 0.0 : C[k - 1][p - 1] + C[k - 1][p]);
  mu[0] = 1.0;
#pragma unroll
  for (int k = 1; k < NH; ++k) mu[k] = mu[k - 1] * (-u);
  const double is = 1.0 / s;
#pragma unroll
  for (int A = 0; A < NH; ++A) {
    double beta[NL];
#pragma unroll
    for (int p = 0; p < NL; ++p) beta[p] = 0.0;
    double isk = 1.0;
#pragma unroll
    for (int k = 0; k < NH; ++k) {
      const double ck = tab->Vi[A][k] * isk;
#pragma unroll
      for (int p = 0; p < NL; ++p)
        if (p <= k) beta[p] += ck * C[k][p] * mu[k - p];
      isk *= is;
    }
#pragma unroll
    for (int a = 0; a < NL; ++a) {
      const double v = s * Lq.cr[a] + u;
      double acc = 0.0, vp = 1.0;
#pragma unroll
      for (int p = 0; p < NL; ++p) {
        acc += beta[p] * vp;
        vp *= v;
      }
      K[A][a] = acc;
    }
  }
}

// One cell's state of one set, given in its own frame {ufx, ufy, Tf}, in the
// other set in the same frame (Sec. III.B-C, App. C).  Lifting keeps the
// moments of the low-order set taken at the frame's particle velocities and
// completes the others from the high-order equilibrium: the low-order
// non-equilibrium part through the frame's completion matrices on top of the
// high-order equilibrium, both equilibria at the cell's rho, u, T taken in the
// frame (equilibrium factors at the reduced velocity (u - u_f)/sqrt(T_f) and
// temperature T/T_f); the Hermite variant keeps Hermite coefficients in the
// reduced velocities, whose matrix serves every frame.  Projection applies
// the low-order Lagrange basis at the high-order nodes (the moments it keeps
// span the same polynomials in every frame).
template <int NL, int NH, bool TH>
__device__ void pond_lift(const Tab *tab, const double *f, const double *g, double ufx, double ufy, double Tf,
                          double *fo, double *go) {
  constexpr int q = NL * NL;
  const LatTab &Lq = tab->lat[0], &LQ = tab->lat[1];
  const double sT = sqrt(Tf);
  double r = 0, jx = 0, jy = 0, e = 0;
#pragma unroll
  for (int i = 0; i < q; ++i) {
    const double vx = sT * Lq.cr[i % NL] + ufx, vy = sT * Lq.cr[i / NL] + ufy;
    r += f[i];
    jx += vx * f[i];
    jy += vy * f[i];
    e += 0.5 * (vx * vx + vy * vy) * f[i];
    if (TH) e += g[i];
  }
  const double ux = jx / r, uy = jy / r;
  const double T = TH ? (e / r - 0.5 * (ux * ux + uy * uy)) / tab->cv : 1.0;
  const double uxr = (ux - ufx) / sT, uyr = (uy - ufy) / sT, th = T / Tf;
  double pxl[NL], pyl[NL], pxh[NH], pyh[NH];
  eq_axis<double, NL>(Lq, uxr, th, pxl);
  eq_axis<double, NL>(Lq, uyr, th, pyl);
  eq_axis<double, NH>(LQ, uxr, th, pxh);
  eq_axis<double, NH>(LQ, uyr, th, pyh);
  double Kx[NH][NL], Ky[NH][NL];
  if (tab->lift_mode == MSL_LIFT_GRAD_HERMITE) {
#pragma unroll
    for (int A = 0; A < NH; ++A)
#pragma unroll
      for (int a = 0; a < NL; ++a) Kx[A][a] = Ky[A][a] = tab->KH[A][a];
  } else {
    frame_completion<NL, NH>(tab, sT, ufx, Kx);
    frame_completion<NL, NH>(tab, sT, ufy, Ky);
  }
#pragma unroll
  for (int h = 0; h < (TH ? 2 : 1); ++h) {
    const double s = h ? tab->gfac * T : 1.0;
    const double *in = h ? g : f;
    double *out = h ? go : fo;
    double neq[q];
#pragma unroll
    for (int i = 0; i < q; ++i) neq[i] = in[i] - s * r * pxl[i % NL] * pyl[i / NL];
#pragma unroll
    for (int A = 0; A < NH; ++A) {
      double t[NL];
#pragma unroll
      for (int b = 0; b < NL; ++b) {
        double sum = 0.0;
#pragma unroll
        for (int a = 0; a < NL; ++a) sum += Kx[A][a] * neq[a + NL * b];
        t[b] = sum;
      }
#pragma unroll
      for (int B = 0; B < NH; ++B) {
        double cr = 0.0;
#pragma unroll
        for (int b = 0; b < NL; ++b) cr += Ky[B][b] * t[b];
        out[A + NH * B] = s * r * pxh[A] * pyh[B] + cr;
      }
    }
  }
}

template <int NL, int NH, bool TH>
__device__ void pond_project(const Tab *tab, const double *f, const double *g, double *fo, double *go) {
#pragma unroll
  for (int h = 0; h < (TH ? 2 : 1); ++h) {
    const double *in = h ? g : f;
    double *out = h ? go : fo;
#pragma unroll
    for (int bp = 0; bp < NL; ++bp) {
      double t[NH];   // along y first: t[A] = sum_B P[bp][B] f[A + NH B]
#pragma unroll
      for (int A = 0; A < NH; ++A) {
        double sum = 0.0;
#pragma unroll
        for (int B = 0; B < NH; ++B) sum += tab->P[bp][B] * in[A + NH * B];
        t[A] = sum;
      }
#pragma unroll
      for (int ap = 0; ap < NL; ++ap) {
        double sum = 0.0;
#pragma unroll
        for (int A = 0; A < NH; ++A) sum += tab->P[ap][A] * t[A];
        out[ap + NL * bp] = sum;
      }
    }
  }
}

// mode 0: every band cell of buffer (f0, f1, fr) converts its own set's state
// into the other set; mode 1: every cell whose set differs from mask[] converts
// its state into the new set (conv = 0: only its set changes) and takes it
template <int NL, int NH, bool TH>
__global__ void __launch_bounds__(256)
k_pond_convert(const Tab *__restrict__ tab, long long ncell, int mode, int conv, double *f0, double *f1,
               const double *__restrict__ fr, uint8_t *__restrict__ cls, const uint8_t *__restrict__ mask) {
  constexpr int q = NL * NL, Q = NH * NH;
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= ncell) return;
  const uint8_t cb = cls[k];
  const int o = cb & 1;
  int to;
  if (mode == 0) {
    if (!(cb & 2)) return;
    to = o ^ 1;
  } else {
    to = mask[k] & 1;
    if (to == o) return;
    cls[k] = (uint8_t)to;
    if (!conv) return;
  }
  const double ufx = fr[k], ufy = fr[ncell + k], Tf = fr[3 * ncell + k];
  if (o == 0) {
    double f[q], g[TH ? q : 1], fo[Q], go[TH ? Q : 1];
#pragma unroll
    for (int i = 0; i < q; ++i) {
      f[i] = f0[(long long)i * ncell + k];
      if (TH) g[i] = f0[(long long)(q + i) * ncell + k];
    }
    pond_lift<NL, NH, TH>(tab, f, g, ufx, ufy, Tf, fo, go);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      f1[(long long)i * ncell + k] = fo[i];
      if (TH) f1[(long long)(Q + i) * ncell + k] = go[i];
    }
  } else {
    double f[Q], g[TH ? Q : 1], fo[q], go[TH ? q : 1];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      f[i] = f1[(long long)i * ncell + k];
      if (TH) g[i] = f1[(long long)(Q + i) * ncell + k];
    }
    pond_project<NL, NH, TH>(tab, f, g, fo, go);
#pragma unroll
    for (int i = 0; i < q; ++i) {
      f0[(long long)i * ncell + k] = fo[i];
      if (TH) f0[(long long)(q + i) * ncell + k] = go[i];
    }
  }
}

// Diffuse y walls: per column, the density rho_w of the wall state's co-moving
// equilibrium {u_w, T_w} that balances the wall-normal particle flux of the
// adjacent fluid cell, both fluxes counted in the wall's frame: the cell's
// populations (its own set, its own frame) are transferred to the wall's frame
// with the per-axis Lagrange rows of the step kernel.
template <int N>
__device__ double pond_wall_density(const Tab *tab, int l, const double *f, long long ncell, long long k,
                                    const double *fr, const double *ws, int side, int thermal) {
  constexpr int Q = N * N;
  const LatTab &L = tab->lat[l];
  double xn[N], den[N];
#pragma unroll
  for (int m = 0; m < N; ++m) xn[m] = L.cr[m];
#pragma unroll
  for (int m = 0; m < N; ++m) {
    double p = 1.0;
#pragma unroll
    for (int cc = 0; cc < N; ++cc)
      if (cc != m) p *= xn[m] - xn[cc];
    den[m] = 1.0 / p;
  }
  const double Tw = thermal ? ws[4] : 1.0, sTw = sqrt(Tw), isTw = 1.0 / sTw;
  const double sTk = sqrt(fr[3 * ncell + k]), ukx = fr[k], uky = fr[ncell + k];
  // G[a][a'] = l_a((sqrt(T_k) c_a' + u_k - u_w) / sqrt(T_w)) along x and y
  double Gx[N][N], Gy[N][N];
#pragma unroll
  for (int m = 0; m < N; ++m) {
    const double zx = (sTk * xn[m] + ukx - ws[1]) * isTw, zy = (sTk * xn[m] + uky - ws[2]) * isTw;
#pragma unroll
    for (int a = 0; a < N; ++a) {
      double px = den[a], py = den[a];
#pragma unroll
      for (int cc = 0; cc < N; ++cc)
        if (cc != a) {
          px *= zx - xn[cc];
          py *= zy - xn[cc];
        }
      Gx[a][m] = px;
      Gy[a][m] = py;
    }
  }
  double in = 0.0, out = 0.0;
#pragma unroll
  for (int b = 0; b < N; ++b) {
    // the wall-normal (y) velocity of the wall frame's node b
    const double vw = sTw * xn[b] + ws[2];
    const bool towall = side ? vw > 0.0 : vw < 0.0, fromwall = side ? vw < 0.0 : vw > 0.0;
    if (!towall && !fromwall) continue;
#pragma unroll
    for (int a = 0; a < N; ++a) {
      if (towall) {
        double s = 0.0;
#pragma unroll
        for (int bp = 0; bp < N; ++bp) {
          double t = 0.0;
#pragma unroll
          for (int ap = 0; ap < N; ++ap) t += Gx[a][ap] * f[(long long)(ap + N * bp) * ncell + k];
          s += Gy[b][bp] * t;
        }
        in += fabs(vw) * s;
      } else {
        out += fabs(vw) * L.w[a] * L.w[b];
      }
    }
  }
  (void)Q;
  return in / out;
}

__global__ void k_pond_wall(const Tab *__restrict__ tab, PondArgs pa, int thermal, int faces, const double *f0,
                            const double *f1, const uint8_t *__restrict__ cls, const double *__restrict__ fr,
                            double *__restrict__ wrho) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int nx = pa.nx, ny = pa.ny;
  const long long ncell = pa.ncell;
  if (t >= 2 * nx) return;
  const int side = t / nx, x = t % nx;
  if (!(faces & (1 << side))) return;
  const long long k = (long long)(side ? ny - 1 : 0) * nx + x;
  const int l = cls[k] & 1;
  const double *f = l ? f1 : f0;
  const double *ws = pa.st[2 + side];
  double r = 0.0;
  switch (tab->lat[l].n) {
    case 3: r = pond_wall_density<3>(tab, l, f, ncell, k, fr, ws, side, thermal); break;
    case 4: r = pond_wall_density<4>(tab, l, f, ncell, k, fr, ws, side, thermal); break;
    case 5: r = pond_wall_density<5>(tab, l, f, ncell, k, fr, ws, side, thermal); break;
    case 6: r = pond_wall_density<6>(tab, l, f, ncell, k, fr, ws, side, thermal); break;
  }
  wrho[t] = r;
}

static PondArgs pond_args(const msl_ctx *c) {
  PondArgs pa;
  pa.nx = c->geo.nx;
  pa.ny = c->geo.ny;
  pa.ncell = c->ncell;
  for (int f = 0; f < 4; ++f) {
    pa.bc[f] = c->cfg.bc[f];
    for (int m = 0; m < 5; ++m) pa.st[f][m] = c->cfg.bc_state[f][m];
  }
  return pa;
}

static unsigned pond_blocks(const msl_ctx *c) { return (unsigned)((c->ncell + 255) / 256); }

int msl_pond_launch_init(msl_ctx *c, const double *rho, const double *u, const double *T) {
  hipLaunchKernelGGL(k_pond_init, dim3(pond_blocks(c)), dim3(256), 0, c->stream, c->dtab, c->ncell,
                     c->cfg.thermal, c->nlat, rho, u, T, c->pond_f[0][c->cur],
                     c->nlat > 1 ? c->pond_f[1][c->cur] : nullptr, c->pond_fr[c->cur]);
  return hipGetLastError() == hipSuccess ? MSL_OK : MSL_EHIP;
}

int msl_pond_launch_macros(msl_ctx *c, double *rho, double *u, double *T) {
  hipLaunchKernelGGL(k_pond_macros, dim3(pond_blocks(c)), dim3(256), 0, c->stream, c->dtab, c->ncell,
                     c->cfg.thermal, c->pond_f[0][c->cur], c->nlat > 1 ? c->pond_f[1][c->cur] : nullptr,
                     c->cls, c->pond_fr[c->cur], rho, u, T);
  return hipGetLastError() == hipSuccess ? MSL_OK : MSL_EHIP;
}

// conversion launch over buffer `buf` (mode and mask as in k_pond_convert)
static int pond_convert(msl_ctx *c, int buf, int mode, int conv, const uint8_t *mask) {
  return msl_pair_dispatch(2, c->htab.lat[0].n, c->htab.lat[1].n, [&]<int D, int NL, int NH>() {
    if (c->cfg.thermal)
      hipLaunchKernelGGL((k_pond_convert<NL, NH, true>), dim3(pond_blocks(c)), dim3(256), 0, c->stream, c->dtab,
                         c->ncell, mode, conv, c->pond_f[0][buf], c->pond_f[1][buf], c->pond_fr[buf], c->cls, mask);
    else
      hipLaunchKernelGGL((k_pond_convert<NL, NH, false>), dim3(pond_blocks(c)), dim3(256), 0, c->stream, c->dtab,
                         c->ncell, mode, conv, c->pond_f[0][buf], c->pond_f[1][buf], c->pond_fr[buf], c->cls, mask);
    return hipGetLastError() == hipSuccess ? MSL_OK : MSL_EHIP;
  });
}

// new sets from `mask` (converting the cells that change when conv), then the
// band of the current buffer
int msl_pond_launch_set_mask(msl_ctx *c, const uint8_t *mask, int conv) {
  if (c->nlat < 2) return MSL_OK;   // the mask check admits only zeros
  int rc = pond_convert(c, c->cur, 1, conv, mask);
  if (!rc) rc = msl_launch_classify(c);
  if (!rc && conv) rc = pond_convert(c, c->cur, 0, 1, nullptr);
  return rc;
}

template <int N, bool TH, bool QE>
static int pond_step_n(msl_ctx *c, int lat) {
  constexpr int TW = PondTraits<N, TH>::TW;
  const PondArgs pa = pond_args(c);
  const dim3 grid((unsigned)((pa.nx + TW - 1) / TW), (unsigned)pa.ny);
  hipLaunchKernelGGL((k_pond_step<N, TH, QE>), grid, dim3(256), 0, c->stream, c->dtab, lat, c->cls, pa,
                     c->pond_f[lat][c->cur], c->pond_fr[c->cur], c->pond_f[lat][c->cur ^ 1],
                     c->pond_fr[c->cur ^ 1], c->flag, c->pond_stats, (int *)(c->pond_stats + 1), c->pond_wall);
  return hipGetLastError() == hipSuccess ? MSL_OK : MSL_EHIP;
}

template <bool TH, bool QE>
static int pond_step_th(msl_ctx *c, int lat) {
  switch (c->htab.lat[lat].n) {
    case 3: return pond_step_n<3, TH, QE>(c, lat);
    case 4: return pond_step_n<4, TH, QE>(c, lat);
    case 5: return pond_step_n<5, TH, QE>(c, lat);
    case 6: return pond_step_n<6, TH, QE>(c, lat);
  }
  return MSL_EINVAL;
}

// one step: [the Knudsen-number criterion pass], one launch per set, the band
// of the new buffer; the new buffers become current
int msl_pond_launch_step(msl_ctx *c) {
  int rc;
  if (c->nlat > 1 && c->cfg.crit_kind == MSL_CRIT_KN && c->cfg.crit_every > 0 &&
      c->step % c->cfg.crit_every == 0) {
    hipLaunchKernelGGL(k_pond_kn_fields, dim3(pond_blocks(c)), dim3(256), 0, c->stream, c->dtab, c->ncell,
                       c->cfg.thermal, c->pond_f[0][c->cur], c->pond_f[1][c->cur], c->cls, c->pond_fr[c->cur],
                       c->kn_rho, c->kn_lam);
    if (hipGetLastError() != hipSuccess) return MSL_EHIP;
    if ((rc = msl_launch_kn_mask(c))) return rc;
    if ((rc = msl_launch_dilate(c))) return rc;
    if ((rc = msl_pond_launch_set_mask(c, c->newmask, 1))) return rc;
  }
  const int faces = (c->cfg.bc[2] == MSL_BC_DIFFUSE_WALL ? 1 : 0) | (c->cfg.bc[3] == MSL_BC_DIFFUSE_WALL ? 2 : 0);
  if (faces) {
    // the wall densities from the current state (the wall states travel in
    // the kernel arguments)
    const PondArgs pa = pond_args(c);
    hipLaunchKernelGGL(k_pond_wall, dim3((unsigned)((2 * pa.nx + 255) / 256)), dim3(256), 0, c->stream, c->dtab,
                       pa, c->cfg.thermal, faces, c->pond_f[0][c->cur],
                       c->nlat > 1 ? c->pond_f[1][c->cur] : nullptr, c->cls, c->pond_fr[c->cur], c->pond_wall);
    if (hipGetLastError() != hipSuccess) return MSL_EHIP;
  }
  for (int l = 0; l < c->nlat; ++l) {
    if (c->cfg.thermal) rc = c->htab.qe ? pond_step_th<true, true>(c, l) : pond_step_th<true, false>(c, l);
    else rc = c->htab.qe ? pond_step_th<false, true>(c, l) : pond_step_th<false, false>(c, l);
    if (rc) return rc;
  }
  if (c->nlat > 1 && (rc = pond_convert(c, c->cur ^ 1, 0, 1, nullptr))) return rc;
  c->cur ^= 1;
  return MSL_OK;
}
