// msl_aux.hip -- the kernels around the fused stream-and-collide: equilibrium
// initialisation, ghost-layer fill (boundary rules), band conversion by lifting
// and projection, refinement criterion and switching, class / band / tile
// bookkeeping with an ordered compaction of the band cells, macroscopic
// fields, population import/export and the deterministic FP64 reductions.
#include "msl_band.hpp"
#include "msl_device.hpp"

#define AUX_BLOCK 256

// ---------------------------------------------------------------------------
// per-cell state access (FP64 view of the stored planes)
// ---------------------------------------------------------------------------
template <typename S>
__device__ __forceinline__ void read_cell(const Tab *tab, const Geo &g, const char *base, int l,
                                          int off, double *f, double *gg) {
  const LatTab &L = tab->lat[l];
  const S *p = (const S *)base;
  const double gs = tab->gfac * tab->T0;
  for (int i = 0; i < L.Q; ++i) {
    f[i] = load_pop<S>(p + (long long)i * g.plane, off, L.sc[i]);
    if (tab->thermal) gg[i] = load_pop<S>(p + (long long)(L.Q + i) * g.plane, off, gs * L.sc[i]);
  }
}

template <typename S>
__device__ __forceinline__ void write_cell(const Tab *tab, const Geo &g, char *base, int l, int off,
                                           const double *f, const double *gg) {
  const LatTab &L = tab->lat[l];
  S *p = (S *)base;
  const double gs = tab->gfac * tab->T0;
  for (int i = 0; i < L.Q; ++i) {
    store_pop<S>(p + (long long)i * g.plane, off, f[i], L.sc[i]);
    if (tab->thermal) store_pop<S>(p + (long long)(L.Q + i) * g.plane, off, gg[i], gs * L.sc[i]);
  }
}

// ---------------------------------------------------------------------------
// initialisation: lattice equilibrium of each cell's own velocity set
// ---------------------------------------------------------------------------
template <typename S>
__global__ void k_init_eq(const Tab *__restrict__ tab, Geo g, char *b0, char *b1,
                          const uint8_t *__restrict__ cls, const double *__restrict__ rho,
                          const double *__restrict__ u, const double *__restrict__ T) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= g.ncell) return;
  int x, y, z;
  cell_coords(g, k, x, y, z);
  const int l = cls[k] & 1;
  double uu[3] = {0, 0, 0};
  for (int a = 0; a < g.dim; ++a) uu[a] = u[a * g.ncell + k];
  const double Tk = (tab->thermal && T) ? T[k] : 1.0;
  double f[MSL_MAXQ], gg[MSL_MAXQ];
  cell_feq(tab->lat[l], g.dim, rho[k], uu, Tk, f);
  for (int i = 0; i < tab->lat[l].Q; ++i) gg[i] = tab->gfac * Tk * f[i];
  write_cell<S>(tab, g, l ? b1 : b0, l, g.idx(x, y, z), f, gg);
}

// ---------------------------------------------------------------------------
// ghost layers, one pass per axis (x, then y over the x ghosts, then z over
// the x and y ghosts), matching the resolution order highest axis first
// ---------------------------------------------------------------------------
struct BCArgs {
  int bc[6];
  double st[6][5];
  double slot_st[6][5];
  int slot[6][4];
  double slot_edge[6];
};

__device__ __forceinline__ int in_slot(const BCArgs &b, int face, int dim, const int *p) {
  const int *s = b.slot[face];
  if (s[0] >= s[1]) return 0;
  const int ax = face / 2;
  int t[2], nt = 0;
  for (int a = 0; a < dim; ++a)
    if (a != ax) t[nt++] = a;
  if (p[t[0]] < s[0] || p[t[0]] >= s[1]) return 0;
  if (dim == 3 && s[2] < s[3] && (p[t[1]] < s[2] || p[t[1]] >= s[3])) return 0;
  return 1;
}

// ghost cells of one axis pass: lower axes with ghosts, the axis itself in its
// 2G ghost layers, higher axes interior
__device__ __forceinline__ long long pass_cells(const Geo &g, int ax, int *ext, int *lo) {
  const int N[3] = {g.nx, g.ny, g.nz};
  long long tot = 1;
  for (int a = 0; a < 3; ++a) {
    if (a >= g.dim) { ext[a] = 1; lo[a] = 0; }
    else if (a < ax) { ext[a] = N[a] + 2 * MSL_G; lo[a] = -MSL_G; }
    else if (a == ax) { ext[a] = 2 * MSL_G; lo[a] = 0; }
    else { ext[a] = N[a]; lo[a] = 0; }
    tot *= ext[a];
  }
  return tot;
}

// 2D: periodic and zero-gradient ghosts of every axis in one launch (the
// step of a small 2D grid is latency-bound: one launch instead of two); one
// thread per (ghost cell, plane).  A ghost cell belongs to the pass of its highest
// out-of-range axis (that axis' ghost layers, lower axes with their ghosts,
// higher axes interior), so the passes partition the ghost cells.  A cell
// whose owning face is a copy rule takes the value at the point where every
// out-of-range coordinate is mapped by its own face's rule (wrap, clamp),
// except fixed and diffuse faces of lower axes, whose ghost coordinate is
// kept (constant ghosts, or diffuse ghosts filled earlier in the step): the
// same values as filling the axes one after the other.
template <typename S>
__global__ void __launch_bounds__(AUX_BLOCK)
k_bc_copy(const Tab *__restrict__ tab, Geo g, BCArgs b, char *bl, char *bh, int np0) {
  // blockIdx.y: plane; x: ghost cell, passes in axis order (32-bit indexing:
  // the ghost layers of any admissible grid hold fewer than 2^31 cells)
  const int N[3] = {g.nx, g.ny, g.nz};
  int ext[3][3], lo[3][3], cnt[3] = {0, 0, 0};
  for (int a = 0; a < g.dim; ++a) {
    cnt[a] = 1;
    for (int e = 0; e < 3; ++e) {
      if (e >= g.dim) { ext[a][e] = 1; lo[a][e] = 0; }
      else if (e < a) { ext[a][e] = N[e] + 2 * MSL_G; lo[a][e] = -MSL_G; }
      else if (e == a) { ext[a][e] = 2 * MSL_G; lo[a][e] = 0; }
      else { ext[a][e] = N[e]; lo[a][e] = 0; }
      cnt[a] *= ext[a][e];
    }
  }
  int cellid = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (cellid >= cnt[0] + cnt[1] + cnt[2]) return;
  const int plane = (int)blockIdx.y;
  int ax = 0;
  while (cellid >= cnt[ax]) cellid -= cnt[ax++];
  int p[3];
  int r = cellid;
  for (int e = 0; e < 3; ++e) {
    p[e] = lo[ax][e] + r % ext[ax][e];
    r /= ext[ax][e];
  }
  const int gi = p[ax];
  const int side = gi < MSL_G ? 0 : 1;
  p[ax] = side ? N[ax] + (gi - MSL_G) : gi - MSL_G;
  const int rule = b.bc[2 * ax + side];
  if (rule != MSL_BC_PERIODIC && rule != MSL_BC_OUTFLOW_ZG) return;
  int q[3] = {p[0], p[1], p[2]};
  for (int a = 0; a <= ax; ++a) {
    if (q[a] >= 0 && q[a] < N[a]) continue;
    const int ra = b.bc[2 * a + (q[a] < 0 ? 0 : 1)];
    if (ra == MSL_BC_PERIODIC) q[a] = q[a] < 0 ? q[a] + N[a] : q[a] - N[a];
    else if (ra == MSL_BC_OUTFLOW_ZG) q[a] = q[a] < 0 ? 0 : N[a] - 1;
  }
  S *pl = plane < np0 ? (S *)bl + (long long)plane * g.plane : (S *)bh + (long long)(plane - np0) * g.plane;
  pl[g.idx(p[0], p[1], p[2])] = pl[g.idx(q[0], q[1], q[2])];
}

// 3D: periodic and zero-gradient ghosts, one axis after the other: x, then y,
// then z.  A ghost takes the value at the point where its out-of-range
// coordinate is mapped by its face's rule (wrap, clamp).  The x pass covers
// the interior rows; the y pass then copies whole rows (x ghosts included)
// and the z pass whole slabs (y ghost rows included), so edges and corners
// get every axis' rule in turn.  Fixed and diffuse faces keep their own
// ghosts, which later passes copy like any other value.

// x faces: one thread per (ghost cell of an interior row, plane)
template <typename S>
__global__ void __launch_bounds__(AUX_BLOCK)
k_bc_xcopy(Geo g, BCArgs b, char *bl, char *bh, int np0) {
  const int nz = g.dim == 3 ? g.nz : 1;
  const int t = (int)(blockIdx.x * blockDim.x + threadIdx.x);   // < 4 ny nz < 2^31
  if (t >= 2 * MSL_G * g.ny * nz) return;
  const int gi = t % (2 * MSL_G), r = t / (2 * MSL_G);
  const int y = r % g.ny, z = r / g.ny;
  const int side = gi < MSL_G ? 0 : 1;
  const int rule = b.bc[side];
  if (rule != MSL_BC_PERIODIC && rule != MSL_BC_OUTFLOW_ZG) return;
  const int x = side ? g.nx + (gi - MSL_G) : gi - MSL_G;
  const int xs = rule == MSL_BC_PERIODIC ? (side ? x - g.nx : x + g.nx) : (side ? g.nx - 1 : 0);
  const int plane = (int)blockIdx.y;
  S *pl = plane < np0 ? (S *)bl + (long long)plane * g.plane : (S *)bh + (long long)(plane - np0) * g.plane;
  pl[g.idx(x, y, z)] = pl[g.idx(xs, y, z)];
}

// y faces (A = 1: whole rows of interior slabs) and z faces (A = 2: whole
// slabs): 16-byte chunks, one per thread.  Rows and slabs span the full pitch
// and row count, so the padding beyond the ghost layers is copied too (it
// holds no value any cell reads).
template <int A>
__global__ void __launch_bounds__(AUX_BLOCK)
k_bc_blocks(Geo g, BCArgs b, char *bl, char *bh, int np0, int esz) {
  const long long blk16 = A == 1 ? (long long)g.pitch * esz / 16 : (long long)g.rows * g.pitch * esz / 16;
  const int nblk = A == 1 ? 2 * MSL_G * (g.dim == 3 ? g.nz : 1) : 2 * MSL_G;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= blk16 * nblk) return;
  const int blk = (int)(t / blk16);
  const long long ch = t - (long long)blk * blk16;
  const int gi = blk % (2 * MSL_G), zz = blk / (2 * MSL_G);
  const int n = A == 1 ? g.ny : g.nz;
  const int side = gi < MSL_G ? 0 : 1;
  const int rule = b.bc[2 * A + side];
  if (rule != MSL_BC_PERIODIC && rule != MSL_BC_OUTFLOW_ZG) return;
  const int c = side ? n + (gi - MSL_G) : gi - MSL_G;
  const int cs = rule == MSL_BC_PERIODIC ? (side ? c - n : c + n) : (side ? n - 1 : 0);
  // element offsets of the ghost block and of its source
  long long dst, src;
  if (A == 1) {
    const long long zoff = g.dim == 3 ? (long long)(zz + MSL_G) * g.rows : 0;
    dst = (zoff + c + MSL_G) * g.pitch;
    src = (zoff + cs + MSL_G) * g.pitch;
  } else {
    dst = (long long)(c + MSL_G) * g.rows * g.pitch;
    src = (long long)(cs + MSL_G) * g.rows * g.pitch;
  }
  const int plane = (int)blockIdx.y;
  char *pl = plane < np0 ? bl + (long long)plane * g.plane * esz : bh + (long long)(plane - np0) * g.plane * esz;
  uint4 *d = (uint4 *)(pl + dst * esz) + ch;
  const uint4 *s = (const uint4 *)(pl + src * esz) + ch;
  *d = *s;
}

// fixed-equilibrium ghosts: constant, written once per buffer when a state is
// loaded
template <typename S>
__global__ void __launch_bounds__(AUX_BLOCK)
k_bc_fixed(const Tab *__restrict__ tab, Geo g, int ax, BCArgs b, char *bl, char *bh) {
  const int N[3] = {g.nx, g.ny, g.nz};
  int ext[3], lo[3];
  const long long tot = pass_cells(g, ax, ext, lo);
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= tot) return;
  int p[3];
  long long r = t;
  for (int a = 0; a < 3; ++a) {
    p[a] = lo[a] + (int)(r % ext[a]);
    r /= ext[a];
  }
  const int gi = p[ax];
  const int side = gi < MSL_G ? 0 : 1;
  p[ax] = side ? N[ax] + (gi - MSL_G) : gi - MSL_G;
  const int face = 2 * ax + side;
  if (b.bc[face] != MSL_BC_FIXED_EQ) return;
  char *bases[2] = {bl, bh};
  const int dst = g.idx(p[0], p[1], p[2]);
  double stb[5];
  const double *st = in_slot(b, face, g.dim, p) ? b.slot_st[face] : b.st[face];
  const int *s = b.slot[face];
  const double w = b.slot_edge[face];
  if (w > 0.0 && s[0] < s[1]) {
    // smooth slot profile: tanh edges of width w
    int t[2], nt = 0;
    for (int a = 0; a < g.dim; ++a)
      if (a != ax) t[nt++] = a;
    double lam = 0.5 * (tanh((p[t[0]] - s[0] + 0.5) / w) - tanh((p[t[0]] - s[1] + 0.5) / w));
    if (g.dim == 3 && s[2] < s[3])
      lam *= 0.5 * (tanh((p[t[1]] - s[2] + 0.5) / w) - tanh((p[t[1]] - s[3] + 0.5) / w));
    for (int m = 0; m < 5; ++m) stb[m] = b.st[face][m] + lam * (b.slot_st[face][m] - b.st[face][m]);
    st = stb;
  }
  for (int l = 0; l < tab->nlat; ++l) {
    double f[MSL_MAXQ], gg[MSL_MAXQ];
    cell_feq(tab->lat[l], g.dim, st[0], st + 1, st[4], f);
    for (int i = 0; i < tab->lat[l].Q; ++i) gg[i] = tab->gfac * st[4] * f[i];
    write_cell<S>(tab, g, bases[l], l, dst, f, gg);
  }
}

// diffuse walls (every step): the ghost holds the wall equilibrium scaled so
// that as many particles leave the wall as arrive at it from the adjacent
// fluid cell (zero net wall-normal mass flux).  The unit-density equilibrium
// and its outgoing flux come from the tables; a thread reads only the arriving
// populations of its adjacent cell and writes every plane of its ghost cell.
template <typename S>
__global__ void __launch_bounds__(AUX_BLOCK)
k_bc_diffuse(const Tab *__restrict__ tab, Geo g, int ax, BCArgs b, char *bl, char *bh,
             const uint8_t *__restrict__ cls) {
  const int N[3] = {g.nx, g.ny, g.nz};
  int ext[3], lo[3];
  const long long tot = pass_cells(g, ax, ext, lo);
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= tot) return;
  int p[3];
  long long r = t;
  for (int a = 0; a < 3; ++a) {
    p[a] = lo[a] + (int)(r % ext[a]);
    r /= ext[a];
  }
  const int gi = p[ax];
  const int side = gi < MSL_G ? 0 : 1;
  p[ax] = side ? N[ax] + (gi - MSL_G) : gi - MSL_G;
  const int face = 2 * ax + side;
  if (b.bc[face] != MSL_BC_DIFFUSE_WALL) return;
  // adjacent fluid point; lower-axis ghosts map through their own rule
  int q[3] = {p[0], p[1], p[2]};
  q[ax] = side ? N[ax] - 1 : 0;
  int use_low = 0;
  for (int a = 0; a < ax; ++a) {
    if (q[a] >= 0 && q[a] < N[a]) continue;
    const int fr = b.bc[2 * a + (q[a] < 0 ? 0 : 1)];
    if (fr == MSL_BC_PERIODIC) q[a] = (q[a] % N[a] + N[a]) % N[a];
    else if (fr == MSL_BC_OUTFLOW_ZG) q[a] = q[a] < 0 ? 0 : N[a] - 1;
    else use_low = 1;
  }
  const int m = use_low ? 0 : (cls[((long long)q[2] * g.ny + q[1]) * g.nx + q[0]] & 1);
  const LatTab &Lm = tab->lat[m];
  const S *pm = (const S *)(m ? bh : bl);
  const int src = g.idx(q[0], q[1], q[2]);
  const int n = Lm.n;
  const int stride = ax == 0 ? 1 : (ax == 1 ? n : n * n);
  // populations arriving at the wall: v_ax < 0 at the lower face, > 0 at the upper
  double in = 0;
  for (int i = 0; i < Lm.Q; ++i) {
    const double cn = Lm.v[ax][(i / stride) % n];
    if (side ? cn > 0 : cn < 0)
      in += fabs(cn) * load_pop<S>(pm + (long long)i * g.plane, src, Lm.sc[i]);
  }
  const double rw = in / tab->wall_out[face][m];
  const double Tw = b.st[face][4];
  const int dst = g.idx(p[0], p[1], p[2]);
  for (int l = 0; l < tab->nlat; ++l) {
    const LatTab &L = tab->lat[l];
    S *pl = (S *)(l ? bh : bl);
    for (int i = 0; i < L.Q; ++i) {
      const double f = rw * tab->wall_eq[face][l][i];
      store_pop<S>(pl + (long long)i * g.plane, dst, f, L.sc[i]);
      if (tab->thermal)
        store_pop<S>(pl + (long long)(L.Q + i) * g.plane, dst, tab->gfac * Tw * f,
                     tab->gfac * tab->T0 * L.sc[i]);
    }
  }
}

// ---------------------------------------------------------------------------
// refinement criterion, switching, classes, tiles, band compaction
// ---------------------------------------------------------------------------
// criterion value of one cell of order N: local Mach number |u| / c_s, or the
// Frobenius norm of the non-equilibrium central second moment over p = rho T
template <typename S, int D, int N, bool TH>
__device__ __forceinline__ double crit_value(const Tab *tab, const Geo &g, const char *base, int l,
                                             int off, int kind) {
  constexpr int Q = Pow<D, N>::v;
  const LatTab &L = tab->lat[l];
  double f[Q], gg[TH ? Q : 1], rho, u[3], T;
  read_cell_t<S, D, N, TH>(tab, g, base, l, off, f, gg);
  macros_t<D, N>(L, TH && tab->thermal, tab->cv, f, gg, rho, u, T);
  if (kind == MSL_CRIT_MA) {
    const double gam = (tab->cv + 1.0) / tab->cv;
    const double cs = TH && tab->thermal ? sqrt(gam * T) : 1.0;
    return sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]) / cs;
  }
  double P[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const double c[3] = {L.v[0][i % N], L.v[1][(i / N) % N], D == 3 ? L.v[2][i / (N * N)] : 0.0};
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
      for (int bb = 0; bb < D; ++bb) P[a][bb] += (c[a] - u[a]) * (c[bb] - u[bb]) * f[i];
  }
  const double p = rho * T;
  double s = 0;
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int bb = 0; bb < D; ++bb) {
      const double d = P[a][bb] - (a == bb ? p : 0.0);
      s += d * d;
    }
  return sqrt(s) / p;
}

// refinement criterion of every cell (Sec. III.A), from its own populations
template <typename S, int D, int NL, int NH, bool TH>
__global__ void __launch_bounds__(AUX_BLOCK)
k_criterion_t(const Tab *__restrict__ tab, Geo g, const char *bl, const char *bh,
              const uint8_t *__restrict__ cls, uint8_t *__restrict__ newmask, int kind, double thr) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= g.ncell) return;
  int x, y, z;
  cell_coords(g, k, x, y, z);
  const int off = g.idx(x, y, z);
  const double v = (cls[k] & 1) ? crit_value<S, D, NH, TH>(tab, g, bh, 1, off, kind)
                                : crit_value<S, D, NL, TH>(tab, g, bl, 0, off, kind);
  newmask[k] = v > thr ? 1 : 0;
}


// Knudsen-number criterion (Sec. IV.A.3), pass 1: the density and the
// hard-sphere mean free path lambda = 16/(5 sqrt(2 pi gamma)) mu a / p of every
// cell from its own populations (a = sqrt(gamma T), p = rho T, and the
// viscosity of the collision: mu = (tau - 1/2) rho T dt, or mu_ref (T/T_ref)^s
// where tau follows mu(T))
template <typename S, int D, int N, bool TH>
__device__ __forceinline__ void kn_cell(const Tab *tab, const Geo &g, const char *base, int l, int off,
                                        double &rho, double &lam) {
  constexpr int Q = Pow<D, N>::v;
  const LatTab &L = tab->lat[l];
  double f[Q], gg[TH ? Q : 1], u[3], T;
  read_cell_t<S, D, N, TH>(tab, g, base, l, off, f, gg);
  macros_t<D, N>(L, TH && tab->thermal, tab->cv, f, gg, rho, u, T);
  const double mu = tab->tau_mode == 1 ? tab->mu_ref * pow(T / tab->tau_ref_T, tab->mu_exp)
                                       : (tab->tau - 0.5) * rho * T * tab->dt;
  const double gam = (tab->cv + 1.0) / tab->cv;
  lam = 16.0 / (5.0 * sqrt(2.0 * M_PI * gam)) * mu * sqrt(gam * T) / (rho * T);
}

template <typename S, int D, int NL, int NH, bool TH>
__global__ void __launch_bounds__(AUX_BLOCK)
k_kn_fields(const Tab *__restrict__ tab, Geo g, const char *bl, const char *bh,
            const uint8_t *__restrict__ cls, double *__restrict__ rho, double *__restrict__ lam) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= g.ncell) return;
  int x, y, z;
  cell_coords(g, k, x, y, z);
  const int off = g.idx(x, y, z);
  double r, l;
  if (cls[k] & 1) kn_cell<S, D, NH, TH>(tab, g, bh, 1, off, r, l);
  else kn_cell<S, D, NL, TH>(tab, g, bl, 0, off, r, l);
  rho[k] = r;
  lam[k] = l;
}

// pass 2: Kn = lambda |grad rho| / rho with central differences of the cell
// densities; across a face that is not periodic (bit a of per clear) the
// missing neighbour is the cell itself, a one-sided difference over one cell
__global__ void __launch_bounds__(AUX_BLOCK)
k_kn_mask(Geo g, const double *__restrict__ rho, const double *__restrict__ lam, int per, double thr,
          uint8_t *__restrict__ newmask) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= g.ncell) return;
  int p[3];
  cell_coords(g, k, p[0], p[1], p[2]);
  const int ext[3] = {g.nx, g.ny, g.nz};
  const long long stride[3] = {1, g.nx, (long long)g.nx * g.ny};
  double g2 = 0.0;
  for (int a = 0; a < g.dim; ++a) {
    if (ext[a] < 2) continue;
    int lo = p[a] - 1, hi = p[a] + 1;
    double dist = 2.0;
    if ((per >> a) & 1) {
      lo = lo < 0 ? lo + ext[a] : lo;
      hi = hi >= ext[a] ? hi - ext[a] : hi;
    } else {
      lo = lo < 0 ? 0 : lo;
      hi = hi >= ext[a] ? ext[a] - 1 : hi;
      dist = (double)(hi - lo);
    }
    const double d = (rho[k + (hi - p[a]) * stride[a]] - rho[k + (lo - p[a]) * stride[a]]) / dist;
    g2 += d * d;
  }
  newmask[k] = lam[k] * sqrt(g2) / rho[k] > thr ? 1 : 0;
}

__global__ void k_mask_out(const uint8_t *__restrict__ cls, long long n, uint8_t *__restrict__ m) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) m[k] = cls[k] & 1;
}

__global__ void k_check_mask(const uint8_t *__restrict__ m, long long n, int allow_high,
                             int *__restrict__ flag) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  if (m[k] > 1 || (m[k] == 1 && !allow_high)) atomicOr(flag, 1);
}

// one velocity set: the class bytes take the new mask (every value is 0)
__global__ void k_switch_one(uint8_t *__restrict__ cls, const uint8_t *__restrict__ newmask, long long n) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) cls[k] = (uint8_t)(newmask[k] & 1);
}

// class bytes of a run with one velocity set: no band cells
__global__ void k_classify(Geo g, int bc_periodic_mask, uint8_t *__restrict__ cls) {
  (void)bc_periodic_mask;
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < g.ncell) cls[k] = (uint8_t)(cls[k] & 1);
}

// Band classification by separable box extrema: a cell is a band cell when a
// cell of the other order lies within Chebyshev distance MSL_G (the stencil
// reach), i.e. when the maximum and the minimum of the order bit over the box
// of +-MSL_G cells differ.  One pass per axis (periodic faces wrap, the others
// clamp to the boundary cell); a pass writes code = max << 1 | min, the last
// one sets bit 1 of the class byte.
__global__ void k_order_extrema(Geo g, int ax, int bc_periodic_mask, const uint8_t *__restrict__ in,
                                int from_cls, uint8_t *__restrict__ out, int last) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= g.ncell) return;
  int p[3];
  cell_coords(g, k, p[0], p[1], p[2]);
  const int N[3] = {g.nx, g.ny, g.nz};
  const long long stride = ax == 0 ? 1 : (ax == 1 ? (long long)g.nx : (long long)g.nx * g.ny);
  int mx = 0, mn = 1;
  for (int d = -MSL_G; d <= MSL_G; ++d) {
    int q = p[ax] + d;
    if (q < 0 || q >= N[ax]) {
      const int side = q < 0 ? 0 : 1;
      if (bc_periodic_mask & (1 << (2 * ax + side))) q = (q % N[ax] + N[ax]) % N[ax];
      else q = side ? N[ax] - 1 : 0;
    }
    const uint8_t v = in[k + (long long)(q - p[ax]) * stride];
    mx |= from_cls ? (v & 1) : ((v >> 1) & 1);
    mn &= v & 1;
  }
  if (last) out[k] = (uint8_t)((out[k] & 1) | ((mx != mn) << 1));
  else out[k] = (uint8_t)((mx << 1) | mn);
}

// The live tiles of velocity set `lat` in ascending order: a launch tile is
// 64 x 4R cells (2D) or 64 x 4 x RZ cells (3D, R = 1) and live when one of
// its micro-tiles holds a cell of the set.  One workgroup compacts the tile
// grid in chunks of 1024 x TL_TPT tiles: each thread takes TL_TPT consecutive
// tiles (their flag loads in flight together), an exclusive scan of the
// per-thread counts (wave shuffles, then the wave totals in LDS) gives each
// thread its place; the list holds (bz * rows + by) * ntx + bx.
#define TL_TPT 16
__global__ void __launch_bounds__(1024)
k_tile_list(Geo g, const uint8_t *__restrict__ tflag, int lat, int R, int RZ, int *__restrict__ list,
            int *__restrict__ count) {
  __shared__ int wsum[16];
  __shared__ int base;
  const int rows = (g.nty + R - 1) / R;
  const int ntiles = g.ntx * rows * ((g.ntz + RZ - 1) / RZ);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (threadIdx.x == 0) base = 0;
  __syncthreads();
  for (int c0 = 0; c0 < ntiles; c0 += 1024 * TL_TPT) {
    const int t0 = c0 + (int)threadIdx.x * TL_TPT;
    unsigned live = 0;   // bit j: tile t0 + j is live
    // coordinates of tile t0, then stepped along x (no division per tile)
    int bx = t0 % g.ntx, by = (t0 / g.ntx) % rows, bz = t0 / g.ntx / rows;
#pragma unroll
    for (int j = 0; j < TL_TPT; ++j) {
      const int t = t0 + j;
      if (t < ntiles) {
        uint8_t any = 0;
        for (int rz = 0; rz < RZ; ++rz) {
          const int mz = bz * RZ + rz;
          if (mz < g.ntz)
            for (int r = 0; r < R; ++r) {
              const int my = by * R + r;
              if (my < g.nty) any |= tflag[((long long)mz * g.nty + my) * g.ntx + bx];
            }
        }
        live |= (unsigned)((any >> lat) & 1) << j;
      }
      if (++bx == g.ntx) {
        bx = 0;
        if (++by == rows) { by = 0; ++bz; }
      }
    }
    const int n = __popc(live);
    int incl = n;   // inclusive scan of the counts over the wave
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int v = __shfl_up(incl, d);
      if (lane >= d) incl += v;
    }
    if (lane == 63) wsum[wv] = incl;
    __syncthreads();
    int off = base + incl - n;
    for (int k = 0; k < wv; ++k) off += wsum[k];
    for (int j = 0; j < TL_TPT; ++j)
      if ((live >> j) & 1u) list[off++] = t0 + j;
    __syncthreads();
    if (threadIdx.x == 0) {
      int tot = 0;
      for (int k = 0; k < 16; ++k) tot += wsum[k];
      base += tot;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) *count = base;
}

int msl_launch_tile_list(msl_ctx *c, int lat, int rows_per_tile, int planes_per_tile) {
  hipLaunchKernelGGL(k_tile_list, dim3(1), dim3(1024), 0, c->stream, c->geo, c->tflag, lat, rows_per_tile,
                     planes_per_tile, c->tlist, c->tcount);
  return hipGetLastError() == hipSuccess ? MSL_OK : MSL_EHIP;
}

// per micro-tile (64 x 4 (x 1)) presence of each order
__global__ void k_tileflags(Geo g, const uint8_t *__restrict__ cls, uint8_t *__restrict__ tflag) {
  const long long t = blockIdx.x;   // one 64-thread block per micro-tile
  const int mx = (int)(t % g.ntx);
  const int my = (int)((t / g.ntx) % g.nty);
  const int mz = (int)(t / ((long long)g.ntx * g.nty));
  const int x = mx * MSL_TX + threadIdx.x;
  uint32_t bits = 0;
  if (x < g.nx)
    for (int r = 0; r < MSL_MTY; ++r) {
      const int y = my * MSL_MTY + r;
      if (y < g.ny) bits |= 1u << (cls[((long long)mz * g.ny + y) * g.nx + x] & 1);
    }
  __shared__ uint32_t s[64];
  s[threadIdx.x] = bits;
  __syncthreads();
  for (int w = 32; w > 0; w >>= 1) {
    if (threadIdx.x < w) s[threadIdx.x] |= s[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) tflag[t] = (uint8_t)s[0];
}

// ordered compaction of the band cells of each order: counts per block of
// 4096 cells, one scan over the blocks, then an ordered scatter
#define CMP_CELLS 4096
__global__ void k_band_count(Geo g, const uint8_t *__restrict__ cls, int *__restrict__ blk, int nblk) {
  // lists: 0 low-order band cells, 1 high-order band cells, 2 all high-order cells
  const long long base = (long long)blockIdx.x * CMP_CELLS;
  int c0 = 0, c1 = 0, c2 = 0;
  for (int j = threadIdx.x; j < CMP_CELLS; j += blockDim.x) {
    const long long k = base + j;
    if (k < g.ncell) {
      const uint8_t v = cls[k];
      if (v & 2) { if (v & 1) ++c1; else ++c0; }
      c2 += v & 1;
    }
  }
  __shared__ int s0[AUX_BLOCK], s1[AUX_BLOCK], s2[AUX_BLOCK];
  s0[threadIdx.x] = c0;
  s1[threadIdx.x] = c1;
  s2[threadIdx.x] = c2;
  __syncthreads();
  for (int w = AUX_BLOCK / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      s0[threadIdx.x] += s0[threadIdx.x + w];
      s1[threadIdx.x] += s1[threadIdx.x + w];
      s2[threadIdx.x] += s2[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    blk[blockIdx.x] = s0[0];
    blk[nblk + blockIdx.x] = s1[0];
    blk[2 * nblk + blockIdx.x] = s2[0];
  }
}

__global__ void __launch_bounds__(1024) k_band_scan(int *__restrict__ blk, int nblk, int *__restrict__ counts) {
  // one workgroup per list (blockIdx.x): exclusive prefix sum of the
  // per-block counts in chunks of 1024 (shuffle scan within each wave, the
  // wave totals in LDS, a running carry between chunks); the list length
  // goes to counts[list]
  __shared__ int wsum[16];
  __shared__ int carry;
  int *b = blk + (long long)blockIdx.x * nblk;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int c0 = 0; c0 < nblk; c0 += 1024) {
    const int i = c0 + (int)threadIdx.x;
    const int v = i < nblk ? b[i] : 0;
    int x = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int y = __shfl_up(x, d);
      if (lane >= d) x += y;
    }
    if (lane == 63) wsum[wv] = x;
    __syncthreads();
    int before = carry;
    for (int k = 0; k < wv; ++k) before += wsum[k];
    if (i < nblk) b[i] = before + x - v;
    __syncthreads();
    if (threadIdx.x == 0) {
      int t = 0;
      for (int k = 0; k < 16; ++k) t += wsum[k];
      carry += t;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) counts[blockIdx.x] = carry;
}

__global__ void __launch_bounds__(256) k_band_scatter(Geo g, const uint8_t *__restrict__ cls,
                                                      const int *__restrict__ blk, int nblk,
                                                      int *__restrict__ lo, int *__restrict__ hi) {
  // four waves per block, each owning a quarter of its 4096 cells: count the
  // quarter's band cells, offset each wave by the counts of the waves before
  // it, then walk the quarter again in 64-cell chunks, in order
  constexpr int QC = CMP_CELLS / 4;
  __shared__ int wc[2][4];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const long long base = (long long)blockIdx.x * CMP_CELLS + (long long)wv * QC;
  const unsigned long long below = lane ? (~0ull >> (64 - lane)) : 0ull;
  int n0 = 0, n1 = 0;
  for (int j = 0; j < QC; j += 64) {
    const long long k = base + j + lane;
    const uint8_t v = k < g.ncell ? cls[k] : 0;
    n0 += __popcll(__ballot((v & 2) && !(v & 1)));
    n1 += __popcll(__ballot((v & 2) && (v & 1)));
  }
  if (lane == 0) {
    wc[0][wv] = n0;
    wc[1][wv] = n1;
  }
  __syncthreads();
  int off0 = blk[blockIdx.x], off1 = blk[nblk + blockIdx.x];
  for (int k = 0; k < wv; ++k) {
    off0 += wc[0][k];
    off1 += wc[1][k];
  }
  for (int j = 0; j < QC; j += 64) {
    const long long k = base + j + lane;
    const uint8_t v = k < g.ncell ? cls[k] : 0;
    const bool p0 = (v & 2) && !(v & 1), p1 = (v & 2) && (v & 1);
    const unsigned long long m0 = __ballot(p0), m1 = __ballot(p1);
    if (p0) lo[off0 + __popcll(m0 & below)] = (int)k;
    if (p1) hi[off1 + __popcll(m1 & below)] = (int)k;
    off0 += __popcll(m0);
    off1 += __popcll(m1);
  }
}

// ---------------------------------------------------------------------------
// macroscopic fields, population import / export
// ---------------------------------------------------------------------------
template <typename S>
__global__ void k_macros(const Tab *__restrict__ tab, Geo g, const char *bl, const char *bh,
                         const uint8_t *__restrict__ cls, double *rho, double *u, double *T) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= g.ncell) return;
  int x, y, z;
  cell_coords(g, k, x, y, z);
  const int l = cls[k] & 1;
  double f[MSL_MAXQ], gg[MSL_MAXQ], r, uu[3], t;
  read_cell<S>(tab, g, l ? bh : bl, l, g.idx(x, y, z), f, gg);
  cell_macros(tab->lat[l], g.dim, tab->thermal, tab->cv, f, gg, r, uu, t);
  if (rho) rho[k] = r;
  if (u)
    for (int a = 0; a < g.dim; ++a) u[a * g.ncell + k] = uu[a];
  if (T) T[k] = t;
}

template <typename S>
__global__ void k_pops(const Tab *__restrict__ tab, Geo g, char *base, int l, int fg,
                       const uint8_t *__restrict__ cls, double *out, const double *in) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= g.ncell) return;
  int x, y, z;
  cell_coords(g, k, x, y, z);
  const int off = g.idx(x, y, z);
  const LatTab &L = tab->lat[l];
  S *p = (S *)base;
  for (int i = 0; i < L.Q; ++i) {
    const double sc = fg ? tab->gfac * tab->T0 * L.sc[i] : L.sc[i];
    S *pl = p + (long long)(fg * L.Q + i) * g.plane;
    if (out) out[(long long)i * g.ncell + k] = load_pop<S>(pl, off, sc);
    else if ((cls[k] & 1) == l) store_pop<S>(pl, off, in[(long long)i * g.ncell + k], sc);
  }
}

// ---------------------------------------------------------------------------
// deterministic FP64 sums of rho, rho u, rho E over each cell's own state, with
// a sentinel for NaN / Inf / rho <= 0
// ---------------------------------------------------------------------------
#define RED_BLOCKS 1024
// Block reduction of NV FP64 values (bit m of maxmask: a NaN-propagating
// maximum, otherwise a sum): a butterfly over the 64 lanes of each wave
// (shuffles, fixed order), then the waves' results in wave order through LDS.
// Deterministic for a given launch shape; the result is in thread 0.
__device__ __forceinline__ double red_max(double a, double b) {
  return a != a ? a : ((b != b || b > a) ? b : a);
}

template <int NV>
__device__ __forceinline__ void block_reduce(double (&a)[NV], unsigned maxmask) {
  constexpr int NW = AUX_BLOCK / 64;
  __shared__ double s[NV][NW];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1)
#pragma unroll
    for (int m = 0; m < NV; ++m) {
      const double o = __shfl_xor(a[m], off, 64);
      a[m] = ((maxmask >> m) & 1u) ? red_max(a[m], o) : a[m] + o;
    }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int m = 0; m < NV; ++m) s[m][w] = a[m];
  __syncthreads();
  if (threadIdx.x == 0)
#pragma unroll
    for (int m = 0; m < NV; ++m) {
      double v = s[m][0];
      for (int k = 1; k < NW; ++k) v = ((maxmask >> m) & 1u) ? red_max(v, s[m][k]) : v + s[m][k];
      a[m] = v;
    }
}

// second pass: one block reduces the per-block partials part[b * NV + m]
template <int NV>
__device__ __forceinline__ void reduce_partials(const double *part, int nb, unsigned maxmask, double (&a)[NV]) {
#pragma unroll
  for (int m = 0; m < NV; ++m) a[m] = 0.0;
  for (int b = threadIdx.x; b < nb; b += blockDim.x)
#pragma unroll
    for (int m = 0; m < NV; ++m) {
      const double v = part[b * NV + m];
      a[m] = ((maxmask >> m) & 1u) ? red_max(a[m], v) : a[m] + v;
    }
  block_reduce<NV>(a, maxmask);
}

template <typename S>
__global__ void __launch_bounds__(AUX_BLOCK)
k_conserve_partial(const Tab *__restrict__ tab, Geo g, const char *bl, const char *bh,
                   const uint8_t *__restrict__ cls, double *__restrict__ part) {
  double acc[6] = {0, 0, 0, 0, 0, 0};
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < g.ncell;
       k += (long long)gridDim.x * blockDim.x) {
    int x, y, z;
    cell_coords(g, k, x, y, z);
    const int l = cls[k] & 1;
    const LatTab &L = tab->lat[l];
    double f[MSL_MAXQ], gg[MSL_MAXQ];
    read_cell<S>(tab, g, l ? bh : bl, l, g.idx(x, y, z), f, gg);
    const int n = L.n;
    double r = 0;
    for (int i = 0; i < L.Q; ++i) {
      const double c[3] = {L.v[0][i % n], L.v[1][(i / n) % n], g.dim == 3 ? L.v[2][i / (n * n)] : 0.0};
      r += f[i];
      acc[1] += c[0] * f[i];
      acc[2] += c[1] * f[i];
      acc[3] += c[2] * f[i];
      acc[4] += 0.5 * (c[0] * c[0] + c[1] * c[1] + c[2] * c[2]) * f[i];
      if (tab->thermal) acc[4] += gg[i];
    }
    acc[0] += r;
    if (!(r > 0.0) || isinf(r)) acc[5] = 1.0;
  }
  block_reduce<6>(acc, 1u << 5);
  if (threadIdx.x == 0)
    for (int m = 0; m < 6; ++m) part[blockIdx.x * 6 + m] = acc[m];
}

__global__ void __launch_bounds__(AUX_BLOCK)
k_conserve_final(const double *__restrict__ part, int nb, double *__restrict__ out) {
  double a[6];
  reduce_partials<6>(part, nb, 1u << 5, a);
  if (threadIdx.x == 0) {
    for (int m = 0; m < 5; ++m) out[m] = a[m];
    // a NaN anywhere propagates into the sums
    const bool bad = a[5] > 0.0 || isnan(a[0]) || isnan(a[4]) || isinf(a[0]) || isinf(a[4]);
    out[5] = bad ? 1.0 : 0.0;
  }
}

// Error norms of the macroscopic fields (each cell from its own populations)
// against caller reference fields: per block the sums of |x - x_ref|^2 and
// |x_ref|^2 and the maximum of |x - x_ref| for rho, u (Euclidean norm over
// the components) and T
template <typename S>
__global__ void __launch_bounds__(AUX_BLOCK)
k_errnorm_partial(const Tab *__restrict__ tab, Geo g, const char *bl, const char *bh,
                  const uint8_t *__restrict__ cls, const double *__restrict__ rref,
                  const double *__restrict__ uref, const double *__restrict__ Tref, double *__restrict__ part) {
  double acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < g.ncell;
       k += (long long)gridDim.x * blockDim.x) {
    int x, y, z;
    cell_coords(g, k, x, y, z);
    const int l = cls[k] & 1;
    double f[MSL_MAXQ], gg[MSL_MAXQ], r, uu[3], t;
    read_cell<S>(tab, g, l ? bh : bl, l, g.idx(x, y, z), f, gg);
    cell_macros(tab->lat[l], g.dim, tab->thermal, tab->cv, f, gg, r, uu, t);
    if (rref) {
      const double d = r - rref[k];
      acc[0] += d * d;
      acc[1] += rref[k] * rref[k];
      acc[2] = red_max(acc[2], fabs(d));
    }
    if (uref) {
      double d2 = 0.0, r2 = 0.0;
      for (int a = 0; a < g.dim; ++a) {
        const double ra = uref[a * g.ncell + k], d = uu[a] - ra;
        d2 += d * d;
        r2 += ra * ra;
      }
      acc[3] += d2;
      acc[4] += r2;
      acc[5] = red_max(acc[5], sqrt(d2));
    }
    if (Tref) {
      const double d = t - Tref[k];
      acc[6] += d * d;
      acc[7] += Tref[k] * Tref[k];
      acc[8] = red_max(acc[8], fabs(d));
    }
  }
  constexpr unsigned MX = (1u << 2) | (1u << 5) | (1u << 8);
  block_reduce<9>(acc, MX);
  if (threadIdx.x == 0)
    for (int m = 0; m < 9; ++m) part[blockIdx.x * 9 + m] = acc[m];
}

// out: relative L2 = sqrt(sum |x - x_ref|^2 / sum |x_ref|^2) (the root mean
// square of the difference where the reference is zero everywhere) and max
__global__ void __launch_bounds__(AUX_BLOCK)
k_errnorm_final(const double *__restrict__ part, int nb, long long ncell, double *__restrict__ out) {
  constexpr unsigned MX = (1u << 2) | (1u << 5) | (1u << 8);
  double a[9];
  reduce_partials<9>(part, nb, MX, a);
  if (threadIdx.x == 0)
    for (int f = 0; f < 3; ++f) {
      const double sd = a[3 * f], sr = a[3 * f + 1];
      out[2 * f] = sr > 0.0 ? sqrt(sd / sr) : sqrt(sd / (double)ncell);
      out[2 * f + 1] = a[3 * f + 2];
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static inline unsigned nblocks(long long n) { return (unsigned)((n + AUX_BLOCK - 1) / AUX_BLOCK); }

#define DISPATCH_STORE(c, KERNEL, grid, block, ...)                                         \
  do {                                                                                      \
    switch ((c)->cfg.store) {                                                               \
      case MSL_FP64: hipLaunchKernelGGL(KERNEL<double>, grid, block, 0, (c)->stream, __VA_ARGS__); break; \
      case MSL_FP32: hipLaunchKernelGGL(KERNEL<float>, grid, block, 0, (c)->stream, __VA_ARGS__); break;  \
      case MSL_FP16_DEV: hipLaunchKernelGGL(KERNEL<_Float16>, grid, block, 0, (c)->stream, __VA_ARGS__); break; \
      case MSL_BF16_DEV: hipLaunchKernelGGL(KERNEL<bf16_t>, grid, block, 0, (c)->stream, __VA_ARGS__); break;  \
      default: return MSL_EINVAL;                                                           \
    }                                                                                       \
  } while (0)

static inline int last_err() { return hipGetLastError() == hipSuccess ? MSL_OK : MSL_EHIP; }

int msl_launch_init_eq(msl_ctx *c, const double *rho, const double *u, const double *T) {
  char *b0 = c->planes[0][c->cur], *b1 = c->nlat > 1 ? c->planes[1][c->cur] : nullptr;
  DISPATCH_STORE(c, k_init_eq, dim3(nblocks(c->ncell)), dim3(AUX_BLOCK), c->dtab, c->geo, b0, b1,
                 c->cls, rho, u, T);
  return last_err();
}

static void bc_args(const msl_ctx *c, BCArgs &b) {
  for (int f = 0; f < 6; ++f) {
    b.bc[f] = c->cfg.bc[f];
    for (int m = 0; m < 5; ++m) {
      b.st[f][m] = c->cfg.bc_state[f][m];
      b.slot_st[f][m] = c->cfg.slot_state[f][m];
    }
    for (int m = 0; m < 4; ++m) b.slot[f][m] = c->cfg.slot[f][m];
    b.slot_edge[f] = c->cfg.slot_edge[f];
  }
}

static long long host_pass_cells(const Geo &g, int ax) {
  const int N[3] = {g.nx, g.ny, g.nz};
  long long tot = 2 * MSL_G;
  for (int a = 0; a < g.dim; ++a)
    if (a != ax) tot *= a < ax ? N[a] + 2 * MSL_G : N[a];
  return tot;
}

// per step: diffuse walls (from interior cells), then the periodic and
// zero-gradient copies: 2D in one launch; 3D x (unless the previous step
// wrote them), y, z
int msl_launch_bc(msl_ctx *c, char *bl, char *bh) {
  BCArgs b;
  bc_args(c, b);
  const Geo &g = c->geo;
  const int np0 = c->Q[0] * (c->cfg.thermal ? 2 : 1);
  const int np1 = c->nlat > 1 ? c->Q[1] * (c->cfg.thermal ? 2 : 1) : 0;
  const int esz = (int)c->esz;
  auto copies = [&](int ax) {
    const int r0 = b.bc[2 * ax], r1 = b.bc[2 * ax + 1];
    return r0 == MSL_BC_PERIODIC || r0 == MSL_BC_OUTFLOW_ZG || r1 == MSL_BC_PERIODIC ||
           r1 == MSL_BC_OUTFLOW_ZG;
  };
  for (int ax = 0; ax < c->D; ++ax) {
    const int r0 = b.bc[2 * ax], r1 = b.bc[2 * ax + 1];
    if (r0 == MSL_BC_DIFFUSE_WALL || r1 == MSL_BC_DIFFUSE_WALL)
      DISPATCH_STORE(c, k_bc_diffuse, dim3(nblocks(host_pass_cells(g, ax))), dim3(AUX_BLOCK), c->dtab,
                     g, ax, b, bl, bh, c->cls);
  }
  const dim3 blk(AUX_BLOCK);
  if (c->D == 2) {
    if (c->zgm) return last_err();   // applied by the stream-collide launches
    long long tot = 0;
    for (int ax = 0; ax < 2; ++ax) tot += host_pass_cells(g, ax);
    if (copies(0) || copies(1))
      DISPATCH_STORE(c, k_bc_copy, dim3(nblocks(tot), np0 + np1), blk, c->dtab, g, b, bl, bh, np0);
    return last_err();
  }
  const int nz = g.nz;
  if (copies(0) && !c->xg_ok)
    DISPATCH_STORE(c, k_bc_xcopy, dim3(nblocks((long long)2 * MSL_G * g.ny * nz), np0 + np1), blk, g, b,
                   bl, bh, np0);
  if (copies(1)) {
    const long long n = (long long)g.pitch * esz / 16 * 2 * MSL_G * nz;
    hipLaunchKernelGGL(k_bc_blocks<1>, dim3(nblocks(n), np0 + np1), blk, 0, c->stream, g, b, bl, bh, np0,
                       esz);
  }
  if (copies(2)) {
    const long long n = (long long)g.rows * g.pitch * esz / 16 * 2 * MSL_G;
    hipLaunchKernelGGL(k_bc_blocks<2>, dim3(nblocks(n), np0 + np1), blk, 0, c->stream, g, b, bl, bh, np0,
                       esz);
  }
  return last_err();
}

// once per state load: the constant fixed-equilibrium ghosts of both buffers
int msl_launch_bc_fixed(msl_ctx *c) {
  BCArgs b;
  bc_args(c, b);
  const Geo &g = c->geo;
  for (int buf = 0; buf < 2; ++buf) {
    char *bl = c->planes[0][buf], *bh = c->nlat > 1 ? c->planes[1][buf] : nullptr;
    for (int ax = 0; ax < c->D; ++ax) {
      if (b.bc[2 * ax] != MSL_BC_FIXED_EQ && b.bc[2 * ax + 1] != MSL_BC_FIXED_EQ) continue;
      DISPATCH_STORE(c, k_bc_fixed, dim3(nblocks(host_pass_cells(g, ax))), dim3(AUX_BLOCK), c->dtab,
                     g, ax, b, bl, bh);
    }
  }
  return last_err();
}

// band conversion and switching with compile-time velocity-set sizes
template <typename S, int D, int NL, int NH, bool TH>
__global__ void __launch_bounds__(AUX_BLOCK)
k_band_convert_t(const Tab *__restrict__ tab, Geo g, char *bl, char *bh,
                 const int *__restrict__ list_lo, const int *__restrict__ list_hi,
                 const int *__restrict__ counts, int skip_lift, int xmir) {
  constexpr int q = Pow<D, NL>::v, Q = Pow<D, NH>::v;
  const int nlo = counts[0], nhi = counts[1];
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < nlo + nhi; t += stride) {
    const bool lift = t < nlo;
    if (lift && skip_lift) continue;   // the learned closure writes those
    const long long k = lift ? list_lo[t] : list_hi[t - nlo];
    int x, y, z;
    cell_coords(g, k, x, y, z);
    const int off = g.idx(x, y, z);
    // periodic-x image of the cell in the ghost columns (3D; cells x < 2 and
    // x >= nx - 2; xmir is set only for nx >= 4)
    const bool img = D == 3 && xmir && (x < MSL_G || x >= g.nx - MSL_G);
    const int ioff = x < MSL_G ? off + g.nx : off - g.nx;
    if (lift) {
      double f[q], gg[TH ? q : 1], fo[Q], go[TH ? Q : 1];
      read_cell_t<S, D, NL, TH>(tab, g, bl, 0, off, f, gg);
      lift_t<D, NL, NH, TH>(tab, f, gg, nullptr, fo, go);
      write_cell_t<S, D, NH, TH>(tab, g, bh, 1, off, fo, go);
      if constexpr (D == 3)
        if (img) write_cell_t<S, D, NH, TH>(tab, g, bh, 1, ioff, fo, go);
    } else {
      double f[Q], gg[TH ? Q : 1], fo[q], go[TH ? q : 1];
      read_cell_t<S, D, NH, TH>(tab, g, bh, 1, off, f, gg);
      project_t<D, NL, NH, TH>(tab, f, gg, fo, go);
      write_cell_t<S, D, NL, TH>(tab, g, bl, 0, off, fo, go);
      if constexpr (D == 3)
        if (img) write_cell_t<S, D, NL, TH>(tab, g, bl, 0, ioff, fo, go);
    }
  }
}

template <typename S, int D, int NL, int NH, bool TH>
__global__ void __launch_bounds__(AUX_BLOCK)
k_switch_t(const Tab *__restrict__ tab, Geo g, char *bl, char *bh, uint8_t *__restrict__ cls,
           const uint8_t *__restrict__ newmask, int convert, int xmir) {
  constexpr int q = Pow<D, NL>::v, Q = Pow<D, NH>::v;
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= g.ncell) return;
  const int from = cls[k] & 1, to = newmask[k] & 1;
  if (from != to && convert) {
    int x, y, z;
    cell_coords(g, k, x, y, z);
    const int off = g.idx(x, y, z);
    // 3D, x periodic: the converted cell's image in the ghost column on the
    // other side (the x ghosts of the current buffer stay current)
    const bool img = D == 3 && xmir && (x < MSL_G || x >= g.nx - MSL_G);
    const int ioff = x < MSL_G ? off + g.nx : off - g.nx;
    if (to == 1) {
      double f[q], gg[TH ? q : 1], fo[Q], go[TH ? Q : 1];
      read_cell_t<S, D, NL, TH>(tab, g, bl, 0, off, f, gg);
      lift_t<D, NL, NH, TH>(tab, f, gg, nullptr, fo, go);
      write_cell_t<S, D, NH, TH>(tab, g, bh, 1, off, fo, go);
      if constexpr (D == 3)
        if (img) write_cell_t<S, D, NH, TH>(tab, g, bh, 1, ioff, fo, go);
    } else {
      double f[Q], gg[TH ? Q : 1], fo[q], go[TH ? q : 1];
      read_cell_t<S, D, NH, TH>(tab, g, bh, 1, off, f, gg);
      project_t<D, NL, NH, TH>(tab, f, gg, fo, go);
      write_cell_t<S, D, NL, TH>(tab, g, bl, 0, off, fo, go);
      if constexpr (D == 3)
        if (img) write_cell_t<S, D, NL, TH>(tab, g, bl, 0, ioff, fo, go);
    }
  }
  cls[k] = (uint8_t)to;
}

template <typename S>
static int band_convert_s(msl_ctx *c, char *bl, char *bh, int skip) {
  return msl_pair_dispatch(c->D, c->htab.lat[0].n, c->htab.lat[1].n, [&]<int D, int NL, int NH>() {
    if (c->cfg.thermal)
      hipLaunchKernelGGL((k_band_convert_t<S, D, NL, NH, true>), dim3(512), dim3(AUX_BLOCK), 0,
                         c->stream, c->dtab, c->geo, bl, bh, c->blist[0], c->blist[1], c->bcount, skip,
                         c->xmir);
    else
      hipLaunchKernelGGL((k_band_convert_t<S, D, NL, NH, false>), dim3(512), dim3(AUX_BLOCK), 0,
                         c->stream, c->dtab, c->geo, bl, bh, c->blist[0], c->blist[1], c->bcount, skip,
                         c->xmir);
    return last_err();
  });
}

template <typename S>
static int switch_s(msl_ctx *c, char *bl, char *bh, const uint8_t *newmask, int convert) {
  return msl_pair_dispatch(c->D, c->htab.lat[0].n, c->htab.lat[1].n, [&]<int D, int NL, int NH>() {
    if (c->cfg.thermal)
      hipLaunchKernelGGL((k_switch_t<S, D, NL, NH, true>), dim3(nblocks(c->ncell)), dim3(AUX_BLOCK),
                         0, c->stream, c->dtab, c->geo, bl, bh, c->cls, newmask, convert, c->xmir);
    else
      hipLaunchKernelGGL((k_switch_t<S, D, NL, NH, false>), dim3(nblocks(c->ncell)), dim3(AUX_BLOCK),
                         0, c->stream, c->dtab, c->geo, bl, bh, c->cls, newmask, convert, c->xmir);
    return last_err();
  });
}

int msl_launch_band_convert(msl_ctx *c, char *bl, char *bh) {
  if (c->nlat < 2) return MSL_OK;
  const int mlp = c->cfg.lift_mode == MSL_LIFT_MLP && c->mlp_on;
  switch (c->cfg.store) {
    case MSL_FP64: return band_convert_s<double>(c, bl, bh, mlp);
    case MSL_FP32: return band_convert_s<float>(c, bl, bh, mlp);
    case MSL_FP16_DEV: return band_convert_s<_Float16>(c, bl, bh, mlp);
    case MSL_BF16_DEV: return band_convert_s<bf16_t>(c, bl, bh, mlp);
  }
  return MSL_EINVAL;
}

__global__ void __launch_bounds__(AUX_BLOCK)
k_copy_bytes(const uint8_t *__restrict__ in, uint8_t *__restrict__ out, long long n) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) out[k] = in[k];
}

// the criterion's margin along one axis: out[k] = max of in over the cells
// within m cells of k along that axis (periodic: wrapped; otherwise the box
// ends at the face)
__global__ void __launch_bounds__(AUX_BLOCK)
k_dilate(Geo g, int ax, int m, int periodic, const uint8_t *__restrict__ in, uint8_t *__restrict__ out) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= g.ncell) return;
  int p[3];
  cell_coords(g, k, p[0], p[1], p[2]);
  const int n = ax == 0 ? g.nx : (ax == 1 ? g.ny : g.nz);
  const long long stride = ax == 0 ? 1 : (ax == 1 ? (long long)g.nx : (long long)g.nx * g.ny);
  uint8_t v = 0;
  for (int d = -m; d <= m && !v; ++d) {
    int q = p[ax] + d;
    if (q < 0 || q >= n) {
      if (!periodic) continue;
      q = ((q % n) + n) % n;
    }
    v = in[k + (long long)(q - p[ax]) * stride] & 1;
  }
  out[k] = v;
}

int msl_launch_dilate(msl_ctx *c) {
  const int m = c->cfg.crit_margin;
  if (m <= 0) return MSL_OK;
  // ping-pong through the first band list's bytes (rebuilt after the switch)
  uint8_t *t[2] = {c->newmask, (uint8_t *)c->blist[0]};
  int cur = 0;
  for (int ax = 0; ax < c->D; ++ax) {
    const int per = c->cfg.bc[2 * ax] == MSL_BC_PERIODIC && c->cfg.bc[2 * ax + 1] == MSL_BC_PERIODIC;
    hipLaunchKernelGGL(k_dilate, dim3(nblocks(c->ncell)), dim3(AUX_BLOCK), 0, c->stream, c->geo, ax, m, per,
                       t[cur], t[cur ^ 1]);
    cur ^= 1;
  }
  if (cur) hipLaunchKernelGGL(k_copy_bytes, dim3(nblocks(c->ncell)), dim3(AUX_BLOCK), 0, c->stream, t[1], t[0],
                              c->ncell);
  return last_err();
}

// Kn > crit_thr from the cell densities and mean free paths in kn_rho, kn_lam
// (written by the previous launch) into newmask
int msl_launch_kn_mask(msl_ctx *c) {
  int per = 0;
  for (int a = 0; a < c->D; ++a)
    if (c->cfg.bc[2 * a] == MSL_BC_PERIODIC && c->cfg.bc[2 * a + 1] == MSL_BC_PERIODIC) per |= 1 << a;
  hipLaunchKernelGGL(k_kn_mask, dim3(nblocks(c->ncell)), dim3(AUX_BLOCK), 0, c->stream, c->geo, c->kn_rho,
                     c->kn_lam, per, c->cfg.crit_thr, c->newmask);
  return last_err();
}

template <typename S>
static int criterion_s(msl_ctx *c) {
  return msl_pair_dispatch(c->D, c->htab.lat[0].n, c->htab.lat[1].n, [&]<int D, int NL, int NH>() {
    const char *bl = c->planes[0][c->cur], *bh = c->planes[1][c->cur];
    if (c->cfg.crit_kind == MSL_CRIT_KN) {
      if (c->cfg.thermal)
        hipLaunchKernelGGL((k_kn_fields<S, D, NL, NH, true>), dim3(nblocks(c->ncell)), dim3(AUX_BLOCK), 0,
                           c->stream, c->dtab, c->geo, bl, bh, c->cls, c->kn_rho, c->kn_lam);
      else
        hipLaunchKernelGGL((k_kn_fields<S, D, NL, NH, false>), dim3(nblocks(c->ncell)), dim3(AUX_BLOCK), 0,
                           c->stream, c->dtab, c->geo, bl, bh, c->cls, c->kn_rho, c->kn_lam);
      return msl_launch_kn_mask(c);
    }
    if (c->cfg.thermal)
      hipLaunchKernelGGL((k_criterion_t<S, D, NL, NH, true>), dim3(nblocks(c->ncell)), dim3(AUX_BLOCK),
                         0, c->stream, c->dtab, c->geo, bl, bh, c->cls, c->newmask,
                         c->cfg.crit_kind, c->cfg.crit_thr);
    else
      hipLaunchKernelGGL((k_criterion_t<S, D, NL, NH, false>), dim3(nblocks(c->ncell)),
                         dim3(AUX_BLOCK), 0, c->stream, c->dtab, c->geo, bl, bh, c->cls, c->newmask,
                         c->cfg.crit_kind, c->cfg.crit_thr);
    return last_err();
  });
}

int msl_launch_criterion(msl_ctx *c) {
  if (c->nlat < 2) return MSL_OK;   // nothing to switch to
  switch (c->cfg.store) {
    case MSL_FP64: return criterion_s<double>(c);
    case MSL_FP32: return criterion_s<float>(c);
    case MSL_FP16_DEV: return criterion_s<_Float16>(c);
    case MSL_BF16_DEV: return criterion_s<bf16_t>(c);
  }
  return MSL_EINVAL;
}

int msl_launch_check_mask(msl_ctx *c, const uint8_t *mask) {
  hipLaunchKernelGGL(k_check_mask, dim3(nblocks(c->ncell)), dim3(AUX_BLOCK), 0, c->stream, mask,
                     c->ncell, c->nlat > 1, c->flag);
  return last_err();
}

int msl_launch_get_mask(msl_ctx *c, uint8_t *mask) {
  hipLaunchKernelGGL(k_mask_out, dim3(nblocks(c->ncell)), dim3(AUX_BLOCK), 0, c->stream, c->cls,
                     c->ncell, mask);
  return last_err();
}

int msl_launch_switch(msl_ctx *c, const uint8_t *newmask) {
  char *bl = c->planes[0][c->cur], *bh = c->nlat > 1 ? c->planes[1][c->cur] : nullptr;
  if (c->nlat < 2) {
    hipLaunchKernelGGL(k_switch_one, dim3(nblocks(c->ncell)), dim3(AUX_BLOCK), 0, c->stream, c->cls,
                       newmask, c->ncell);
    return last_err();
  }
  const int conv = c->initialized;
  switch (c->cfg.store) {
    case MSL_FP64: return switch_s<double>(c, bl, bh, newmask, conv);
    case MSL_FP32: return switch_s<float>(c, bl, bh, newmask, conv);
    case MSL_FP16_DEV: return switch_s<_Float16>(c, bl, bh, newmask, conv);
    case MSL_BF16_DEV: return switch_s<bf16_t>(c, bl, bh, newmask, conv);
  }
  return MSL_EINVAL;
}

int msl_launch_classify(msl_ctx *c) {
  int pm = 0;
  for (int f = 0; f < 2 * c->D; ++f)
    if (c->cfg.bc[f] == MSL_BC_PERIODIC) pm |= 1 << f;
  if (c->nlat < 2) {
    hipLaunchKernelGGL(k_classify, dim3(nblocks(c->ncell)), dim3(AUX_BLOCK), 0, c->stream, c->geo, pm,
                       c->cls);
  } else {
    // separable passes through two byte buffers that are free at this point
    // (the criterion's new mask has been applied; the band lists are rebuilt
    // below)
    uint8_t *t[2] = {c->newmask, (uint8_t *)c->blist[0]};
    const uint8_t *src = c->cls;
    for (int ax = 0; ax < c->D; ++ax) {
      const int last = ax == c->D - 1;
      uint8_t *dst = last ? c->cls : t[ax & 1];
      hipLaunchKernelGGL(k_order_extrema, dim3(nblocks(c->ncell)), dim3(AUX_BLOCK), 0, c->stream,
                         c->geo, ax, pm, src, ax == 0, dst, last);
      src = dst;
    }
  }
  const Geo &g = c->geo;
  const long long nt = (long long)g.ntx * g.nty * g.ntz;
  hipLaunchKernelGGL(k_tileflags, dim3((unsigned)nt), dim3(64), 0, c->stream, g, c->cls, c->tflag);
  c->tl_ok = 0;
  hipLaunchKernelGGL(k_band_count, dim3(c->nblk), dim3(AUX_BLOCK), 0, c->stream, g, c->cls, c->blk,
                     c->nblk);
  hipLaunchKernelGGL(k_band_scan, dim3(3), dim3(1024), 0, c->stream, c->blk, c->nblk, c->bcount);
  hipLaunchKernelGGL(k_band_scatter, dim3(c->nblk), dim3(256), 0, c->stream, g, c->cls, c->blk,
                     c->nblk, c->blist[0], c->blist[1]);
  return last_err();
}

int msl_launch_macros(msl_ctx *c, double *rho, double *u, double *T) {
  DISPATCH_STORE(c, k_macros, dim3(nblocks(c->ncell)), dim3(AUX_BLOCK), c->dtab, c->geo,
                 c->planes[0][c->cur], c->nlat > 1 ? c->planes[1][c->cur] : nullptr, c->cls, rho,
                 u, T);
  return last_err();
}

// plain vectorised copy: the bandwidth reference of the roofline figures
// one 16-byte element per thread, one pass (no grid-stride loop): the
// fastest plain copy measured on this GPU
__global__ void __launch_bounds__(256) k_copy(const uint4 *__restrict__ src, uint4 *__restrict__ dst,
                                              long long n) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) dst[k] = src[k];
}

extern "C" int msl_device_copy(void *dst, const void *src, size_t bytes, void *stream) {
  if (!dst || !src || bytes % 16) return MSL_EINVAL;
  const long long n = (long long)(bytes / 16);
  if (n == 0) return MSL_OK;
  if ((n + 255) / 256 > 0x7fffffffLL) return MSL_EINVAL;
  hipLaunchKernelGGL(k_copy, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                     (const uint4 *)src, (uint4 *)dst, n);
  return last_err();
}

int msl_launch_pops(msl_ctx *c, int which, int fg, double *out, const double *in) {
  DISPATCH_STORE(c, k_pops, dim3(nblocks(c->ncell)), dim3(AUX_BLOCK), c->dtab, c->geo,
                 c->planes[which][c->cur], which, fg, c->cls, out, in);
  return last_err();
}

int msl_launch_error_norms(msl_ctx *c, const double *rref, const double *uref, const double *Tref,
                           double *dev_out6) {
  DISPATCH_STORE(c, k_errnorm_partial, dim3(RED_BLOCKS), dim3(AUX_BLOCK), c->dtab, c->geo,
                 c->planes[0][c->cur], c->nlat > 1 ? c->planes[1][c->cur] : nullptr, c->cls, rref, uref, Tref,
                 c->red);
  hipLaunchKernelGGL(k_errnorm_final, dim3(1), dim3(AUX_BLOCK), 0, c->stream, c->red, RED_BLOCKS, c->ncell,
                     dev_out6);
  return last_err();
}

int msl_launch_conservation(msl_ctx *c, double *dev_out6) {
  DISPATCH_STORE(c, k_conserve_partial, dim3(RED_BLOCKS), dim3(AUX_BLOCK), c->dtab, c->geo,
                 c->planes[0][c->cur], c->nlat > 1 ? c->planes[1][c->cur] : nullptr, c->cls, c->red);
  hipLaunchKernelGGL(k_conserve_final, dim3(1), dim3(AUX_BLOCK), 0, c->stream, c->red, RED_BLOCKS,
                     dev_out6);
  return last_err();
}
