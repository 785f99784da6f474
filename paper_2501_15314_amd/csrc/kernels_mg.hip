// Geometric multigrid V-cycle for the pressure Laplacian L = G^T G, used as
// the preconditioner M^-1 ~ L^+ of the Schur Krylov solve.  The paper applies
// an exact fast-diagonalisation solve of L once per iteration (Sec. 4.2) and
// names a multigrid V-cycle as its linear-time replacement (Sec. 7).
//
// Cycle: red-black Gauss-Seidel smoothing (pre: red then black, post: black
// then red, so the cycle is symmetric), residual restricted by averaging the
// eight children, trilinear cell-centred prolongation, coarse operators
// rediscretised on 2h, and a single-workgroup kernel that runs V-cycles on
// the coarsest grids entirely in LDS.  Kernels are templated on the working
// precision T (float or double) and on the right-hand-side type TB.
#include <hip/hip_ext.h>

#include "internal.h"
#include "march.h"

namespace ibs {

__device__ __forceinline__ bool row_pos1m(const Geo &g, int color, RowPos &p) {
  p.m = blockIdx.x * blockDim.x + threadIdx.x;
  p.j = blockIdx.y * blockDim.y + threadIdx.y;
  p.i = blockIdx.z;
  p.comp = 0;
  p.c = color;
  if (p.m >= g.hn2 || p.j >= g.n1) return false;
  p.k = 2 * p.m + ((p.c + p.i + p.j) & 1);
  p.e = (long long)p.c * g.half + ((long long)p.i * g.n1 + p.j) * g.hn2 + p.m;
  return true;
}

template <typename T>
__device__ __forceinline__ T nb_sum(const Geo &g, const T *x, int i, int j, int k, int c, int m) {
  const T *o = x + (long long)(1 - c) * g.half;
  T s = T(0);
  int t;
  t = nbr(i, -1, g.n0, g.bc0); if (t >= 0) s += o[((long long)t * g.n1 + j) * g.hn2 + m];
  t = nbr(i, 1, g.n0, g.bc0);  if (t >= 0) s += o[((long long)t * g.n1 + j) * g.hn2 + m];
  t = nbr(j, -1, g.n1, g.bc1); if (t >= 0) s += o[((long long)i * g.n1 + t) * g.hn2 + m];
  t = nbr(j, 1, g.n1, g.bc1);  if (t >= 0) s += o[((long long)i * g.n1 + t) * g.hn2 + m];
  long long row = ((long long)i * g.n1 + j) * g.hn2;
  t = nbr(k, -1, g.n2, g.bc2); if (t >= 0) s += o[row + (t >> 1)];
  t = nbr(k, 1, g.n2, g.bc2);  if (t >= 0) s += o[row + (t >> 1)];
  return s;
}

// Coarse right-hand side: the average of the fine residual over the eight
// children.  The last half sweep relaxed the black cells, whose residual is
// therefore zero; only the four red children contribute: in fine planes 2I
// and 2I+1, rows 2J and 2J+1, each at in-row index K of the red plane.
//
// Plane march over the fine grid like the sweeps (register window of black
// planes along axis 0, LDS tile of the current black plane): a thread forms
// the residuals of its two red cells (in-row m0, m0+1 = coarse K, K+1),
// sums them over the plane pair, and the pair of rows is combined through
// LDS; the even-row thread writes the two coarse values (one per colour).
// The chunk of planes per workgroup is even, so a pair never splits.
__host__ __device__ inline int restrict_chunk(const Geo &gf) { return march_chunk(gf) < 2 ? 2 : march_chunk(gf); }

template <typename T, typename TB>
__global__ void __launch_bounds__(256) k_restrict(Geo gf, const T *xf, const TB *bf, Geo gc, T *bc) {
  __shared__ T tile[MARCH_TILE];
  __shared__ T pair[256][2];
  const int BX = blockDim.x, BY = blockDim.y, W2 = 2 * BX + 2;
  const int tx = threadIdx.x, ty = threadIdx.y, tid = tx + BX * ty;
  const int m0 = 2 * (blockIdx.x * BX + tx), j = blockIdx.y * BY + ty;
  const int len = restrict_chunk(gf);
  const int i0 = blockIdx.z * len, i1 = min(i0 + len, gf.n0);
  const T *red = xf, *blk = xf + gf.half;
  const int mbase = blockIdx.x * BX * 2, jbase = blockIdx.y * BY;
  auto row = [&](int i, int jj) { return ((long long)i * gf.n1 + jj) * gf.hn2; };
  auto bval = [&](int i, int jj, int mm) -> T { return blk[row(i, jj) + mm]; };
  auto bwin = [&](int i) -> V2<T> {
    V2<T> v;
    v.x = T(0);
    v.y = T(0);
    const int ii = mwrap(i, gf.n0, gf.bc0);
    if (ii < 0) return v;
    return ld2<T>(blk + row(ii, j) + m0);
  };
  const T ih2 = (T)(1.0 / gf.h2);
  T acc[2] = {T(0), T(0)};
  V2<T> prev = bwin(i0 - 1), cur = bwin(i0);
  for (int i = i0; i < i1; ++i) {
    V2<T> next = bwin(i + 1);
    tile[(ty + 1) * W2 + 2 * tx + 1] = cur.x;
    tile[(ty + 1) * W2 + 2 * tx + 2] = cur.y;
    tile_halo(tile, gf, i, jbase, mbase, BX, BY, bval);
    __syncthreads();
    const long long r = row(i, j) + m0;
    const V2<T> xr = ld2<T>(red + r);
    const V2<T> br = ld2<T>(bf + r);
    const int s = (i + j) & 1;
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int k = 2 * (m0 + u) + s, col = 2 * tx + 1 + u;
      const T *trow = tile + (ty + 1) * W2;
      const T sum = (u ? prev.y : prev.x) + (u ? next.y : next.x) + tile[ty * W2 + col] + tile[(ty + 2) * W2 + col] +
                    trow[col - 1 + s] + trow[col + s];
      const T xv = u ? xr.y : xr.x, bv = u ? br.y : br.x;
      acc[u] += pc_resid(bv, xv, sum, cell_nnb(gf, i, j, k), ih2);
    }
    if (i & 1) {
      // plane pair done: add the partner row and write the coarse values
      pair[tid][0] = acc[0];
      pair[tid][1] = acc[1];
    }
    __syncthreads();
    if ((i & 1) && !(ty & 1)) {
      const T v0 = (acc[0] + pair[tid + BX][0]) * (T)0.125;
      const T v1 = (acc[1] + pair[tid + BX][1]) * (T)0.125;
      const int I = i >> 1, J = j >> 1, K = m0;  // K even: colour of (I, J, K) is (I + J) & 1
      const long long cr = ((long long)I * gc.n1 + J) * gc.hn2 + (K >> 1);
      const int c0 = (I + J) & 1;
      bc[(long long)c0 * gc.half + cr] = v0;
      bc[(long long)(1 - c0) * gc.half + cr] = v1;
    }
    if (i & 1) {
      acc[0] = T(0);
      acc[1] = T(0);
    }
    prev = cur;
    cur = next;
  }
}

// x_f += P x_c on the red fine cells only (the following black half sweep
// overwrites the black cells without reading them).  P is trilinear
// cell-centred interpolation: per axis weight 3/4 on the parent and 1/4 on
// the parent's neighbour on the child's side (past a wall the parent itself,
// periodic axes wrap).
//
// Plane march over the fine grid: a thread owns the red cells at in-row
// m0, m0+1 of fine row (i, j).  Along axis 0 the two coarse planes in use,
// (i-1)>>1 and (i+1)>>1, are held in registers (each coarse plane is read
// once per march); per plane the thread keeps its two coarse rows (parent and
// neighbour along axis 1) at the four coarse K = m0-1 .. m0+2 that both
// parities of the fine row need.
template <typename T>
__global__ void __launch_bounds__(256) k_prolong(Geo gf, T *xf, Geo gc, const T *xc) {
  const int BX = blockDim.x, BY = blockDim.y;
  const int m0 = 2 * (blockIdx.x * BX + threadIdx.x), j = blockIdx.y * BY + threadIdx.y;
  const int len = march_chunk(gf);
  const int i0 = blockIdx.z * len, i1 = min(i0 + len, gf.n0);
  auto side = [](int C, int o, int n, int bc) { return (o < 0 || o >= n) ? (bc ? C : (o < 0 ? o + n : o - n)) : o; };
  const int J = j >> 1, Jo = side(J, J + ((j & 1) ? 1 : -1), gc.n1, gc.bc1);
  int Kq[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int K = m0 - 1 + q;
    Kq[q] = (K < 0) ? (gc.bc2 ? 0 : gc.n2 - 1) : (K >= gc.n2 ? (gc.bc2 ? gc.n2 - 1 : 0) : K);
  }
  // coarse plane P: values at rows J, Jo and K = Kq[0..3]
  auto load_plane = [&](int P, T v[2][4]) {
    const int rows[2] = {J, Jo};
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int q = 0; q < 4; ++q) v[r][q] = xc[sidx(gc, P, rows[r], Kq[q])];
  };
  auto wrapP = [&](int P) { return side(P < 0 ? 0 : gc.n0 - 1, P, gc.n0, gc.bc0); };
  int lo = (i0 - 1) >> 1;
  T vlo[2][4], vhi[2][4], vpre[2][4];
  load_plane(wrapP(lo), vlo);
  load_plane(wrapP(lo + 1), vhi);
  auto xrow = [&](int i) { return xf + ((long long)i * gf.n1 + j) * gf.hn2 + m0; };
  V2<T> xcur = ld2<T>(xrow(i0));
  for (int i = i0; i < i1; ++i) {
    if (((i - 1) >> 1) != lo) {
      // the window moves up one coarse plane (prefetched one fine plane ago)
      ++lo;
#pragma unroll
      for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          vlo[r][q] = vhi[r][q];
          vhi[r][q] = vpre[r][q];
        }
    }
    // software pipeline: the next fine row and, when the window will move at
    // plane i+1, its new coarse plane
    const bool more = i + 1 < i1;
    V2<T> xnext = xcur;
    if (more) {
      xnext = ld2<T>(xrow(i + 1));
      if ((i >> 1) != lo) load_plane(wrapP(lo + 2), vpre);
    }
    // parent plane i>>1 is lo for odd i, hi for even i
    const T wlo = (i & 1) ? (T)0.75 : (T)0.25, whi = (T)1 - wlo;
    const int s = (i + j) & 1;  // fine red cells k = 2 (m0 + u) + s
    T out[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      // parent K = m0 + u (slot u + 1), neighbour K - 1 (slot u) or K + 1 (slot u + 2)
      const int qc = u + 1, qo = s ? u + 2 : u;
      T acc = T(0);
#pragma unroll
      for (int pl = 0; pl < 2; ++pl) {
        const T(*v)[4] = pl ? vhi : vlo;
        const T zJ = blend34(v[0][qc], v[0][qo]);
        const T zO = blend34(v[1][qc], v[1][qo]);
        acc = fma(pl ? whi : wlo, blend34(zJ, zO), acc);
      }
      out[u] = acc;
    }
    st2(xrow(i), xcur.x + out[0], xcur.y + out[1]);
    xcur = xnext;
  }
}

template <typename T, typename TB>
hipError_t mg_smooth_first(const Geo &g, T *x, const TB *b, bool store_red, hipStream_t s) {
  MarchShape M = march_shape(g, 1);
  // launched with the events of an enclosing ProbeExt, if any (as the three below)
  hipEvent_t e0, e1;
  probe_ext_take(&e0, &e1);
  if (store_red)
    hipExtLaunchKernelGGL((k_sweep<T, TB, SW_FIRST>), M.grid, M.block, 0, s, e0, e1, 0, g, x, b, 1, g.h2, 0.0, 0.0,
                          1.0);
  else
    hipExtLaunchKernelGGL((k_sweep<T, TB, SW_FIRST1>), M.grid, M.block, 0, s, e0, e1, 0, g, x, b, 1, g.h2, 0.0, 0.0,
                          1.0);
  return hipGetLastError();
}
template <typename T, typename TB>
hipError_t mg_smooth(const Geo &g, T *x, const TB *b, int color, hipStream_t s) {
  MarchShape M = march_shape(g, 1);
  hipEvent_t e0, e1;
  probe_ext_take(&e0, &e1);
  hipExtLaunchKernelGGL((k_sweep<T, TB, SW_POISSON>), M.grid, M.block, 0, s, e0, e1, 0, g, x, b, color, g.h2, 0.0,
                        0.0, 1.0);
  return hipGetLastError();
}

template <typename T, typename TB>
hipError_t mg_restrict(const Geo &gf, const T *xf, const TB *bf, const Geo &gc, T *bc, hipStream_t s) {
  MarchShape M = march_shape(gf, 1);
  const int len = restrict_chunk(gf);
  M.grid.z = (gf.n0 + len - 1) / len;
  // pairs of planes and rows stay inside one workgroup
  if (gf.n0 % 2 || M.block.y % 2 || len % 2) return hipErrorInvalidValue;
  hipEvent_t e0, e1;
  probe_ext_take(&e0, &e1);
  hipExtLaunchKernelGGL((k_restrict<T, TB>), M.grid, M.block, 0, s, e0, e1, 0, gf, xf, bf, gc, bc);
  return hipGetLastError();
}
template <typename T>
hipError_t mg_prolong(const Geo &gf, T *xf, const Geo &gc, const T *xc, hipStream_t s) {
  MarchShape M = march_shape(gf, 1);
  hipEvent_t e0, e1;
  probe_ext_take(&e0, &e1);
  hipExtLaunchKernelGGL(k_prolong<T>, M.grid, M.block, 0, s, e0, e1, 0, gf, xf, gc, xc);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Tile levels.  On the small levels of the cycle a launch costs more than the
// work it carries (a few microseconds whatever the grid), and the march
// kernels above spend seven launches per level.  A tile level takes two: one
// workgroup per 8^3 tile loads its tile with a halo into LDS and runs the
// tile's whole descent (pre-smoothing, residual, restriction: k_tile_down) or
// whole ascent (prolongation, post-smoothing: k_tile_up), recomputing the
// halo cells that neighbouring tiles own.  A half sweep is exact on a box one
// cell smaller on every side than the box whose values it reads, so the box
// shrinks by one cell per half sweep and a halo of two cells per sweep
// suffices.  Every cell takes the operations of k_sweep, k_restrict and
// k_prolong in the same order (pc_first, pc_relax, pc_resid, blend34), so a
// tile level gives the bits of the march kernels.
//
// Region coordinates r in [0, R) of a tile at grid origin o with halo H stand
// for the unwrapped grid coordinate u = o - H + r.  A wall axis has no cells
// outside [0, n) (their LDS slots hold 0, which a neighbour sum then adds as
// the missing neighbour); a periodic axis wraps.  Origins and halos are even
// and n is even, so the colour of a cell is the parity of r0 + r1 + r2.
constexpr int TL_TS = 8;  // tile edge in cells
constexpr int TL_THREADS = 512;  // at most, per tile workgroup (tile_threads: whole region columns)

struct TileAxes {
  int o[3], n[3], bc[3];
  __device__ __forceinline__ bool inside(int a, int u) const { return (unsigned)u < (unsigned)n[a] || !bc[a]; }
  // the grid coordinate of an unwrapped u in [-n, 2n) (a halo is at most n
  // cells: n is a multiple of 8 on the fine grid and of 4 on the coarse one);
  // inside a wall box u is its own
  __device__ __forceinline__ int wrap(int a, int u) const {
    return u + (u < 0 ? n[a] : 0) - (u >= n[a] ? n[a] : 0);
  }
  // neighbours that a wall removes along axis a
  __device__ __forceinline__ int walls(int a, int u) const {
    return (bc[a] != 0) * ((u == 0) + (u == n[a] - 1));
  }
};
// the tile of this workgroup on grid g (or the matching block of the coarse
// grid gc, whose origin is half the fine one)
__device__ __forceinline__ TileAxes tile_axes(const Geo &g, int scale) {
  TileAxes t;
  const int t1 = g.n1 / TL_TS, t2 = g.n2 / TL_TS, b = blockIdx.x;
  const int tile[3] = {b / (t1 * t2), (b / t2) % t1, b % t2};
  t.n[0] = g.n0 / scale; t.n[1] = g.n1 / scale; t.n[2] = g.n2 / scale;
  t.bc[0] = g.bc0; t.bc[1] = g.bc1; t.bc[2] = g.bc2;
#pragma unroll
  for (int a = 0; a < 3; ++a) t.o[a] = tile[a] * TL_TS / scale;
  return t;
}

// A thread's share of the sweeps over an LDS region of edge R: half a row,
// (r0, r1) = the row, cells r2 in [s0, s0 + R/2) (2 R^2 <= TL_THREADS threads
// take part), with what the row's cells share: whether the row lies in the
// grid, the neighbours its axes 0 and 1 leave (nn01) and its LDS base.  LDS
// rows are R + 1 entries apart, so the rows that the lanes of a wavefront
// work on fall in different banks.
template <int R>
struct TileRow {
  static constexpr int SEG = R / 2;  // even: a segment starts on an even r2
  int r0, r1, s0, u0, u1, nn01, qrow;
  bool live;
};
template <int R>
__device__ __forceinline__ TileRow<R> tile_row(const TileAxes &ax, int H) {
  static_assert(2 * R * R <= TL_THREADS && (R / 2) % 2 == 0, "two threads per row, even segments");
  TileRow<R> w;
  const int tid = threadIdx.x, row = tid >> 1;
  w.r0 = row / R;
  w.r1 = row % R;
  w.s0 = (tid & 1) * TileRow<R>::SEG;
  w.u0 = ax.o[0] - H + w.r0;
  w.u1 = ax.o[1] - H + w.r1;
  w.live = row < R * R && ax.inside(0, w.u0) && ax.inside(1, w.u1);
  w.nn01 = 6 - ax.walls(0, w.u0) - ax.walls(1, w.u1);
  w.qrow = (w.r0 * R + w.r1) * (R + 1);
  return w;
}

// The loads of a region of edge R: a tile kernel runs KP = TL_THREADS / R^2
// threads per column (r1, r2) of the region, thread tid taking planes
// r0 = tid / R^2 + KP m, so that everything but the plane is fixed per
// thread and consecutive threads read consecutive cells of a row.
template <int R>
struct TileCols {
  static constexpr int KP = TL_THREADS / (R * R);
  static constexpr int NT = KP * R * R;  // threads of the launch
  static constexpr int NL = R / KP;      // planes per thread
  static_assert(KP >= 2 && R % KP == 0 && NL <= 32, "whole columns, two threads per sweep row, one bit per plane");
};
__host__ __device__ constexpr int tile_threads(int R) { return (TL_THREADS / (R * R)) * R * R; }
// a thread's column: its region and grid coordinates along axes 1 and 2
struct TileCol {
  int r1, r2, rb, u1, u2, par, w12, plane;
  bool in12;
  long long base0, base1;  // split-layout offset of the column in plane 0, per colour of its cell there
};
template <int R>
__device__ __forceinline__ TileCol tile_col(const Geo &g, const TileAxes &ax, int H) {
  TileCol c;
  const int tid = threadIdx.x;
  c.r2 = tid % R;
  c.r1 = (tid / R) % R;
  c.rb = tid / (R * R);
  c.u1 = ax.o[1] - H + c.r1;
  c.u2 = ax.o[2] - H + c.r2;
  c.in12 = ax.inside(1, c.u1) && ax.inside(2, c.u2);
  const int gj = ax.wrap(1, c.u1), gk = ax.wrap(2, c.u2);
  c.par = (gj + gk) & 1;
  c.w12 = ax.walls(1, c.u1) + ax.walls(2, c.u2);
  c.plane = g.n1 * g.hn2;
  c.base0 = gj * g.hn2 + (gk >> 1);
  c.base1 = c.base0 + g.half;
  return c;
}
// split-layout index of the cell of column c in grid plane gi
__device__ __forceinline__ long long tile_cidx(const TileCol &c, int gi) {
  return (((gi + c.par) & 1) ? c.base1 : c.base0) + gi * c.plane;
}

// one red-black half sweep of colour c over the cells of the box [LO, R-LO)^3
// of an LDS region of edge R (x, b by region index)
template <typename T, int R, int LO>
__device__ __forceinline__ void tile_sweep(T *sx, const T *sb, const TileAxes &ax, const TileRow<R> &w, int H, int c,
                                           T th2) {
  if (w.live && w.r0 >= LO && w.r0 < R - LO && w.r1 >= LO && w.r1 < R - LO) {
    const int p = (c + w.r0 + w.r1) & 1;
#pragma unroll
    for (int m = 0; m < R / 4; ++m) {
      const int r2 = w.s0 + 2 * m + p, u2 = ax.o[2] - H + r2;
      if (r2 < LO || r2 >= R - LO || !ax.inside(2, u2)) continue;
      const int q = w.qrow + r2;
      constexpr int DJ = R + 1, DI = R * (R + 1);
      const T sum = sx[q - DI] + sx[q + DI] + sx[q - DJ] + sx[q + DJ] + sx[q - 1] + sx[q + 1];
      sx[q] = pc_relax(th2, sb[q], sum, w.nn01 - ax.walls(2, u2));
    }
  }
  __syncthreads();
}

// Descent of one tile: PRE red-black sweeps from x = 0 (red then black), x of
// the tile's cells written, and the coarse right-hand side of the tile's
// coarse cells: the average of the residuals of the four red children (the
// black ones were relaxed last and have none).  The halo is 2 PRE: the first
// red values need only their own b, every later half sweep shrinks the box.
template <typename T, typename TB, int PRE>
__global__ void __launch_bounds__(TL_THREADS) k_tile_down(Geo g, T *x, const TB *b, Geo gc, T *bc) {
  constexpr int H = 2 * PRE, R = TL_TS + 2 * H, R3 = R * R * (R + 1);
  constexpr int DJ = R + 1, DI = R * (R + 1);
  constexpr int TC = TL_TS / 2;
  __shared__ T sx[R3];
  __shared__ T sb[R3];
  const TileAxes ax = tile_axes(g, 1);
  const TileRow<R> w = tile_row<R>(ax, H);
  const int tid = threadIdx.x;
  const T th2 = (T)g.h2, ih2 = (T)(1.0 / g.h2);
  // b over the region, column by column (every load of a thread issued
  // before the first is used; a cell outside the grid loads element 0 and
  // keeps 0); the red cells take their first-sweep values on the way
  using CL = TileCols<R>;
  {
    const TileCol c = tile_col<R>(g, ax, H);
    TB bl[CL::NL];
    unsigned ok = 0;
#pragma unroll
    for (int m = 0; m < CL::NL; ++m) {
      const int u0 = ax.o[0] - H + c.rb + CL::KP * m;
      const bool in = c.in12 && ax.inside(0, u0);
      ok |= (unsigned)in << m;
      bl[m] = b[in ? tile_cidx(c, ax.wrap(0, u0)) : 0];
    }
#pragma unroll
    for (int m = 0; m < CL::NL; ++m) {
      const int r0 = c.rb + CL::KP * m, q = (r0 * R + c.r1) * DJ + c.r2;
      const bool in = (ok >> m) & 1u;
      const T bv = in ? (T)bl[m] : T(0);
      sb[q] = bv;
      sx[q] = (in && !((r0 + c.r1 + c.r2) & 1)) ? pc_first(th2, bv, 6 - ax.walls(0, ax.o[0] - H + r0) - c.w12)
                                                : T(0);
    }
  }
  __syncthreads();
  tile_sweep<T, R, 1>(sx, sb, ax, w, H, 1, th2);
  if (PRE == 2) {
    tile_sweep<T, R, 2>(sx, sb, ax, w, H, 0, th2);
    tile_sweep<T, R, 3>(sx, sb, ax, w, H, 1, th2);
  }
  // the tile's cells, both colours
  for (int e = tid; e < TL_TS * TL_TS * TL_TS; e += CL::NT) {
    const int r2 = H + e % TL_TS, r1 = H + (e / TL_TS) % TL_TS, r0 = H + e / (TL_TS * TL_TS);
    x[sidx(g, ax.o[0] - H + r0, ax.o[1] - H + r1, ax.o[2] - H + r2)] = sx[(r0 * R + r1) * (R + 1) + r2];
  }
  // coarse cell (C0, C1, C2) of the tile: the red child of fine row
  // (2 C0 + di, 2 C1 + dj) sits at 2 C2 + ((di + dj) & 1); the residuals are
  // added plane by plane per row, then the two rows, as k_restrict does
  if (tid < TC * TC * TC) {
    const int C2 = tid % TC, C1 = (tid / TC) % TC, C0 = tid / (TC * TC);
    T acc[2];
#pragma unroll
    for (int dj = 0; dj < 2; ++dj) {
      T a = T(0);
#pragma unroll
      for (int di = 0; di < 2; ++di) {
        const int r0 = H + 2 * C0 + di, r1 = H + 2 * C1 + dj, r2 = H + 2 * C2 + ((di + dj) & 1);
        const int q = (r0 * R + r1) * (R + 1) + r2;
        const T sum = sx[q - DI] + sx[q + DI] + sx[q - DJ] + sx[q + DJ] + sx[q - 1] + sx[q + 1];
        const int nn = 6 - ax.walls(0, ax.o[0] - H + r0) - ax.walls(1, ax.o[1] - H + r1) -
                       ax.walls(2, ax.o[2] - H + r2);
        a += pc_resid(sb[q], sx[q], sum, nn, ih2);
      }
      acc[dj] = a;
    }
    bc[sidx(gc, ax.o[0] / 2 + C0, ax.o[1] / 2 + C1, ax.o[2] / 2 + C2)] = (acc[0] + acc[1]) * (T)0.125;
  }
}

// Ascent of one tile: x = xin + P x_c on the red cells (trilinear
// cell-centred, as k_prolong: per axis 3/4 on the parent, 1/4 on the
// parent's neighbour on the child's side, the parent itself past a wall),
// then POST sweeps black then red, and the tile's cells written to xout.
// xout is not xin: neighbouring tiles still read the halo's old values.  The
// halo is 2 POST; the coarse block spans the parents and their neighbours of
// the whole region.
template <typename T, typename TB, int POST>
__global__ void __launch_bounds__(TL_THREADS) k_tile_up(Geo g, const T *xin, T *xout, const TB *b, Geo gc,
                                                            const T *xc) {
  constexpr int H = 2 * POST, R = TL_TS + 2 * H, R3 = R * R * (R + 1), DJ = R + 1;
  constexpr int HC = H / 2 + 1, RC = TL_TS / 2 + 2 * HC, RC3 = RC * RC * RC;
  __shared__ T sx[R3];
  __shared__ T sb[R3];
  __shared__ T sc[RC3];
  const TileAxes ax = tile_axes(g, 1), cx = tile_axes(g, 2);
  const TileRow<R> w = tile_row<R>(ax, H);
  const int tid = threadIdx.x;
  const T th2 = (T)g.h2;
  // the coarse block, then b and the red x of the region column by column,
  // every load of a thread issued before the first is used (slots outside
  // the grid load element 0 and keep 0; black x values are overwritten
  // unread)
  using CL = TileCols<R>;
  constexpr int NC = (RC3 + CL::NT - 1) / CL::NT;
  static_assert(NC <= 32, "one bit per slot");
  {
    T cl[NC];
    unsigned okc = 0;
#pragma unroll
    for (int t = 0; t < NC; ++t) {
      const int e = tid + t * CL::NT;
      const int c2 = e % RC, c1 = (e / RC) % RC, c0 = e / (RC * RC);
      const int U0 = cx.o[0] - HC + c0, U1 = cx.o[1] - HC + c1, U2 = cx.o[2] - HC + c2;
      const bool in = e < RC3 && cx.inside(0, U0) && cx.inside(1, U1) && cx.inside(2, U2);
      okc |= (unsigned)in << t;
      cl[t] = xc[in ? sidx(gc, cx.wrap(0, U0), cx.wrap(1, U1), cx.wrap(2, U2)) : 0];
    }
    const TileCol c = tile_col<R>(g, ax, H);
    TB bl[CL::NL];
    T xl[CL::NL];
    unsigned ok = 0;
#pragma unroll
    for (int m = 0; m < CL::NL; ++m) {
      const int r0 = c.rb + CL::KP * m, u0 = ax.o[0] - H + r0;
      const bool in = c.in12 && ax.inside(0, u0);
      ok |= (unsigned)in << m;
      const long long q = in ? tile_cidx(c, ax.wrap(0, u0)) : 0;
      bl[m] = b[q];
      xl[m] = xin[(in && !((r0 + c.r1 + c.r2) & 1)) ? q : 0];
    }
#pragma unroll
    for (int t = 0; t < NC; ++t) {
      const int e = tid + t * CL::NT;
      if (e < RC3) sc[e] = ((okc >> t) & 1u) ? cl[t] : T(0);
    }
#pragma unroll
    for (int m = 0; m < CL::NL; ++m) {
      const int r0 = c.rb + CL::KP * m, q = (r0 * R + c.r1) * DJ + c.r2;
      const bool in = (ok >> m) & 1u;
      sb[q] = in ? (T)bl[m] : T(0);
      sx[q] = (in && !((r0 + c.r1 + c.r2) & 1)) ? xl[m] : T(0);
    }
  }
  __syncthreads();
  // prolongation onto the red cells of the thread's half row: the planes
  // (u0 - 1) >> 1 and the next with weights by the parity of u0, and the
  // coarse rows J, Jo are the row's; per cell the coarse K and Ko
  if (w.live) {
    auto other = [&](int a, int P, int odd) {
      const int O = P + (odd ? 1 : -1);
      return (cx.bc[a] && (O < 0 || O >= cx.n[a])) ? P : O;
    };
    int lo = (w.u0 - 1) >> 1, hi = lo + 1;
    if (cx.bc[0]) {
      lo = lo < 0 ? 0 : lo;
      hi = hi >= cx.n[0] ? cx.n[0] - 1 : hi;
    }
    const int J = w.u1 >> 1, Jo = other(1, J, w.u1 & 1);
    const int b0 = cx.o[0] - HC, b1 = cx.o[1] - HC, b2 = cx.o[2] - HC;
    const T wlo = (w.u0 & 1) ? (T)0.75 : (T)0.25, whi = (T)1 - wlo;
    const int plo = ((lo - b0) * RC + (J - b1)) * RC - b2, plo_o = ((lo - b0) * RC + (Jo - b1)) * RC - b2;
    const int phi = ((hi - b0) * RC + (J - b1)) * RC - b2, phi_o = ((hi - b0) * RC + (Jo - b1)) * RC - b2;
    const int p = (w.r0 + w.r1) & 1;
#pragma unroll
    for (int m = 0; m < R / 4; ++m) {
      const int r2 = w.s0 + 2 * m + p, u2 = ax.o[2] - H + r2;
      if (!ax.inside(2, u2)) continue;
      const int K = u2 >> 1, Ko = other(2, K, u2 & 1);
      T acc = T(0);
#pragma unroll
      for (int pl = 0; pl < 2; ++pl) {
        const int pJ = pl ? phi : plo, pO = pl ? phi_o : plo_o;
        const T zJ = blend34(sc[pJ + K], sc[pJ + Ko]);
        const T zO = blend34(sc[pO + K], sc[pO + Ko]);
        acc = fma(pl ? whi : wlo, blend34(zJ, zO), acc);
      }
      const int q = w.qrow + r2;
      sx[q] = sx[q] + acc;
    }
  }
  __syncthreads();
  tile_sweep<T, R, 1>(sx, sb, ax, w, H, 1, th2);
  tile_sweep<T, R, 2>(sx, sb, ax, w, H, 0, th2);
  if (POST == 2) {
    tile_sweep<T, R, 3>(sx, sb, ax, w, H, 1, th2);
    tile_sweep<T, R, 4>(sx, sb, ax, w, H, 0, th2);
  }
  for (int e = tid; e < TL_TS * TL_TS * TL_TS; e += CL::NT) {
    const int r2 = H + e % TL_TS, r1 = H + (e / TL_TS) % TL_TS, r0 = H + e / (TL_TS * TL_TS);
    xout[sidx(g, ax.o[0] - H + r0, ax.o[1] - H + r1, ax.o[2] - H + r2)] = sx[(r0 * R + r1) * (R + 1) + r2];
  }
}

bool tile_level_fits(const Geo &g, const Geo &gc, int pre, int post) {
  return g.n0 % TL_TS == 0 && g.n1 % TL_TS == 0 && g.n2 % TL_TS == 0 && gc.n0 * 2 == g.n0 &&
         gc.n1 * 2 == g.n1 && gc.n2 * 2 == g.n2 && (pre == 1 || pre == 2) && (post == 1 || post == 2);
}
static unsigned tile_count(const Geo &g) { return (unsigned)((g.n0 / TL_TS) * (g.n1 / TL_TS) * (g.n2 / TL_TS)); }

template <typename T, typename TB>
hipError_t mg_tile_down(const Geo &g, T *x, const TB *b, const Geo &gc, T *bc, int pre, hipStream_t s) {
  if (!tile_level_fits(g, gc, pre, 1)) return hipErrorInvalidValue;
  hipEvent_t e0, e1;
  probe_ext_take(&e0, &e1);
  if (pre == 2)
    hipExtLaunchKernelGGL((k_tile_down<T, TB, 2>), dim3(tile_count(g)), dim3(tile_threads(TL_TS + 8)), 0, s, e0,
                          e1, 0, g, x, b, gc, bc);
  else
    hipExtLaunchKernelGGL((k_tile_down<T, TB, 1>), dim3(tile_count(g)), dim3(tile_threads(TL_TS + 4)), 0, s, e0,
                          e1, 0, g, x, b, gc, bc);
  return hipGetLastError();
}
template <typename T, typename TB>
hipError_t mg_tile_up(const Geo &g, const T *xin, T *xout, const TB *b, const Geo &gc, const T *xc, int post,
                      hipStream_t s) {
  if (!tile_level_fits(g, gc, 1, post) || xin == xout) return hipErrorInvalidValue;
  hipEvent_t e0, e1;
  probe_ext_take(&e0, &e1);
  if (post == 2)
    hipExtLaunchKernelGGL((k_tile_up<T, TB, 2>), dim3(tile_count(g)), dim3(tile_threads(TL_TS + 8)), 0, s, e0,
                          e1, 0, g, xin, xout, b, gc, xc);
  else
    hipExtLaunchKernelGGL((k_tile_up<T, TB, 1>), dim3(tile_count(g)), dim3(tile_threads(TL_TS + 4)), 0, s, e0,
                          e1, 0, g, xin, xout, b, gc, xc);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Coarse-grid kernel: one workgroup, the whole coarse hierarchy in LDS
// (natural layout).  Projects the right-hand side to mean zero (L is
// singular on constants), then runs `cycles` V-cycles with `sweeps` red-black
// sweeps per level and `bottom` sweeps on the smallest grid.
constexpr int COARSE_MAX = 4096;                 // cells of the coarse grid
constexpr int COARSE_CAP = 4096 + 512 + 64 + 8 + 8;
constexpr int COARSE_THREADS = 1024;
constexpr int COARSE_MAXLEV = 8;
int coarse_max_cells() { return COARSE_MAX; }

struct LvlDim { int n0, n1, n2, off, l1, l2, pow2; };

__device__ __forceinline__ void lds_decode(const LvlDim &d, int e, int &i, int &j, int &k) {
  if (d.pow2) {
    k = e & (d.n2 - 1);
    j = (e >> d.l2) & (d.n1 - 1);
    i = e >> (d.l1 + d.l2);
  } else {
    k = e % d.n2;
    int r = e / d.n2;
    j = r % d.n1;
    i = r / d.n1;
  }
}

template <typename T>
__device__ __forceinline__ T lds_nb(const T *x, LvlDim d, int bc0, int bc1, int bc2, int i, int j, int k, int &nn) {
  T s = T(0);
  int t;
  nn = 0;
  t = nbr(i, -1, d.n0, bc0); if (t >= 0) { s += x[d.off + (t * d.n1 + j) * d.n2 + k]; ++nn; }
  t = nbr(i, 1, d.n0, bc0);  if (t >= 0) { s += x[d.off + (t * d.n1 + j) * d.n2 + k]; ++nn; }
  t = nbr(j, -1, d.n1, bc1); if (t >= 0) { s += x[d.off + (i * d.n1 + t) * d.n2 + k]; ++nn; }
  t = nbr(j, 1, d.n1, bc1);  if (t >= 0) { s += x[d.off + (i * d.n1 + t) * d.n2 + k]; ++nn; }
  t = nbr(k, -1, d.n2, bc2); if (t >= 0) { s += x[d.off + (i * d.n1 + j) * d.n2 + t]; ++nn; }
  t = nbr(k, 1, d.n2, bc2);  if (t >= 0) { s += x[d.off + (i * d.n1 + j) * d.n2 + t]; ++nn; }
  return s;
}

// Sync of the threads that take part in a coarse-kernel phase: the whole
// workgroup, or only wavefront 0 for levels small enough for one wavefront
// (its LDS operations complete in program order, so a compiler-level fence
// between phases suffices).
__device__ __forceinline__ void phase_sync(bool one_wave) {
  if (one_wave) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  } else {
    __syncthreads();
  }
}

// One red-black half sweep over the cells of colour `color` only (the
// in-row index of a colour-c cell of row (i, j) is k = 2 kh + ((i+j+c) & 1);
// every level has an even n2).
template <typename T>
__device__ void lds_smooth(T *x, const T *b, LvlDim d, int bc0, int bc1, int bc2, T h2, int color, int nthr) {
  const int hn2 = d.n2 >> 1;
  const int nc = d.n0 * d.n1 * hn2;
  for (int e = threadIdx.x; e < nc; e += nthr) {
    int kh, r, i, j;
    if (d.pow2) {
      kh = e & (hn2 - 1);
      r = e >> (d.l2 - 1);
      j = r & (d.n1 - 1);
      i = r >> d.l1;
    } else {
      kh = e % hn2;
      r = e / hn2;
      j = r % d.n1;
      i = r / d.n1;
    }
    const int k = 2 * kh + ((i + j + color) & 1);
    int nn;
    T s = lds_nb(x, d, bc0, bc1, bc2, i, j, k, nn);
    const int q = d.off + (i * d.n1 + j) * d.n2 + k;
    x[q] = (h2 * b[q] + s) * inv_nn<T>(nn);
  }
}

template <typename T>
__device__ __forceinline__ T lds_resid(const T *x, const T *b, LvlDim d, int bc0, int bc1, int bc2, T ih2, int i,
                                       int j, int k) {
  int nn;
  T s = lds_nb(x, d, bc0, bc1, bc2, i, j, k, nn);
  int e = d.off + (i * d.n1 + j) * d.n2 + k;
  return b[e] - ((T)nn * x[e] - s) * ih2;
}

template <typename T>
__device__ double block_sum(double v, double *red) {
  v = wave_sum(v);
  int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  if (l == 0) red[w] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0) {
    for (int q = 0; q < COARSE_THREADS / 64; ++q) t += red[q];
    red[COARSE_THREADS / 64] = t;
  }
  __syncthreads();
  t = red[COARSE_THREADS / 64];
  __syncthreads();
  return t;
}

__device__ __forceinline__ int coarse_partner(int C, int odd, int nc, int bc) {
  int o = C + (odd ? 1 : -1);
  if (o < 0 || o >= nc) o = bc ? C : (o < 0 ? o + nc : o - nc);
  return o;
}

template <typename T, typename TB>
__global__ void __launch_bounds__(COARSE_THREADS) k_coarse(Geo g, const TB *bin, T *xout, int cycles, int sweeps,
                                                           int bottom) {
  __shared__ T sx[COARSE_CAP];
  __shared__ T sb[COARSE_CAP];
  __shared__ double red[COARSE_THREADS / 64 + 1];
  __shared__ LvlDim dims[COARSE_MAXLEV];
  __shared__ int s_nl;
  if (threadIdx.x == 0) {
    int nl = 1;
    dims[0].n0 = g.n0; dims[0].n1 = g.n1; dims[0].n2 = g.n2; dims[0].off = 0;
    while (nl < COARSE_MAXLEV) {
      LvlDim q = dims[nl - 1];
      if ((q.n0 & 1) || (q.n1 & 1) || (q.n2 & 1) || q.n0 < 4 || q.n1 < 4 || q.n2 < 4) break;
      LvlDim nx;
      nx.n0 = q.n0 / 2; nx.n1 = q.n1 / 2; nx.n2 = q.n2 / 2;
      nx.off = q.off + q.n0 * q.n1 * q.n2;
      dims[nl] = nx;
      ++nl;
    }
    for (int l = 0; l < nl; ++l) {
      LvlDim &q = dims[l];
      bool p2 = !(q.n0 & (q.n0 - 1)) && !(q.n1 & (q.n1 - 1)) && !(q.n2 & (q.n2 - 1));
      q.pow2 = p2;
      q.l1 = 31 - __clz(q.n1);
      q.l2 = 31 - __clz(q.n2);
    }
    s_nl = nl;
  }
  __syncthreads();
  const int nl = s_nl;
  const int bc0 = g.bc0, bc1 = g.bc1, bc2 = g.bc2;
  const int nc0 = g.n0 * g.n1 * g.n2;
  // load b (split layout -> natural) and project it to mean zero
  double loc = 0.0;
  for (int e = threadIdx.x; e < nc0; e += COARSE_THREADS) {
    int k = e % g.n2, r = e / g.n2, j = r % g.n1, i = r / g.n1;
    T v = (T)bin[sidx(g, i, j, k)];
    sb[e] = v;
    sx[e] = T(0);
    loc += (double)v;
  }
  double mean = block_sum<T>(loc, red) / (double)nc0;
  for (int e = threadIdx.x; e < nc0; e += COARSE_THREADS) sb[e] -= (T)mean;
  __syncthreads();

  // levels of at most 2 x 64 cells run on wavefront 0 alone
  auto small = [&](const LvlDim &q) { return q.n0 * q.n1 * q.n2 <= 128; };
  for (int cyc = 0; cyc < cycles; ++cyc) {
    T h = (T)g.h;
    for (int l = 0; l + 1 < nl; ++l) {
      const LvlDim f = dims[l], c = dims[l + 1];
      const bool one = small(f);
      const int nthr = one ? 64 : COARSE_THREADS;
      if (!one || threadIdx.x < 64) {
        T h2 = h * h;
        for (int s = 0; s < sweeps; ++s) {
          lds_smooth(sx, sb, f, bc0, bc1, bc2, h2, 0, nthr);
          phase_sync(one);
          lds_smooth(sx, sb, f, bc0, bc1, bc2, h2, 1, nthr);
          phase_sync(one);
        }
        int ncc = c.n0 * c.n1 * c.n2;
        T ih2 = T(1) / h2;
        for (int e = threadIdx.x; e < ncc; e += nthr) {
          int i, j, k;
          lds_decode(c, e, i, j, k);
          T acc = T(0);
          for (int q = 0; q < 8; ++q)
            acc += lds_resid(sx, sb, f, bc0, bc1, bc2, ih2, 2 * i + (q >> 2), 2 * j + ((q >> 1) & 1), 2 * k + (q & 1));
          sb[c.off + e] = acc * (T)0.125;
          sx[c.off + e] = T(0);
        }
      }
      if (one) phase_sync(true);
      else __syncthreads();
      h = h * (T)2;
    }
    {
      const LvlDim f = dims[nl - 1];
      const bool one = small(f);
      const int nthr = one ? 64 : COARSE_THREADS;
      if (!one || threadIdx.x < 64) {
        T h2 = h * h;
        for (int s = 0; s < bottom; ++s) {
          lds_smooth(sx, sb, f, bc0, bc1, bc2, h2, 0, nthr);
          phase_sync(one);
          lds_smooth(sx, sb, f, bc0, bc1, bc2, h2, 1, nthr);
          phase_sync(one);
        }
      }
    }
    for (int l = nl - 2; l >= 0; --l) {
      h = h * (T)0.5;
      const LvlDim f = dims[l], c = dims[l + 1];
      const bool one = small(f);
      const int nthr = one ? 64 : COARSE_THREADS;
      // the coarse level was written by all threads (large) or wavefront 0
      if (!small(c) || !one) __syncthreads();
      if (!one || threadIdx.x < 64) {
        int ncf = f.n0 * f.n1 * f.n2;
        for (int e = threadIdx.x; e < ncf; e += nthr) {
          int i, j, k;
          lds_decode(f, e, i, j, k);
          int I0 = i >> 1, J0 = j >> 1, K0 = k >> 1;
          int I1 = coarse_partner(I0, i & 1, c.n0, bc0);
          int J1 = coarse_partner(J0, j & 1, c.n1, bc1);
          int K1 = coarse_partner(K0, k & 1, c.n2, bc2);
          const T *xc = sx + c.off;
#define XC(a, b, cc) xc[((a) * c.n1 + (b)) * c.n2 + (cc)]
          T v0 = (T)0.75 * XC(I0, J0, K0) + (T)0.25 * XC(I1, J0, K0);
          T v1 = (T)0.75 * XC(I0, J1, K0) + (T)0.25 * XC(I1, J1, K0);
          T v2 = (T)0.75 * XC(I0, J0, K1) + (T)0.25 * XC(I1, J0, K1);
          T v3 = (T)0.75 * XC(I0, J1, K1) + (T)0.25 * XC(I1, J1, K1);
#undef XC
          T w0 = (T)0.75 * v0 + (T)0.25 * v1;
          T w1 = (T)0.75 * v2 + (T)0.25 * v3;
          sx[f.off + e] += (T)0.75 * w0 + (T)0.25 * w1;
        }
        phase_sync(one);
        T h2 = h * h;
        for (int s = 0; s < sweeps; ++s) {
          lds_smooth(sx, sb, f, bc0, bc1, bc2, h2, 1, nthr);
          phase_sync(one);
          lds_smooth(sx, sb, f, bc0, bc1, bc2, h2, 0, nthr);
          phase_sync(one);
        }
      }
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < nc0; e += COARSE_THREADS) {
    int k = e % g.n2, r = e / g.n2, j = r % g.n1, i = r / g.n1;
    xout[sidx(g, i, j, k)] = sx[e];
  }
}

template <typename T, typename TB>
hipError_t mg_coarse(const Geo &gc, const TB *b, T *x, int cycles, int sweeps, hipStream_t s) {
  if ((long long)gc.n0 * gc.n1 * gc.n2 > COARSE_MAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_coarse<T, TB>), dim3(1), dim3(COARSE_THREADS), 0, s, gc, b, x, cycles, sweeps, 8);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Exact coarse-grid solve by fast diagonalisation (the direct method of
// Sec. 4.2, here on the coarsest multigrid grid): the rediscretised
// Laplacian of a box with a per-axis boundary type is a Kronecker sum
// L = L0 (+) L1 (+) L2 of 1-D operators with known orthonormal eigenvectors
// Q_a and eigenvalues lam_a, so
//     x = (Q0 x Q1 x Q2) diag(1 / (lam0_i + lam1_j + lam2_k)) (Q0 x Q1 x Q2)^T b,
// the constant mode (all eigenvalues zero) dropped (the pseudo-inverse).
// One workgroup keeps the grid in LDS and applies the six 1-D transforms.
constexpr int FD_MAXN = 32;
constexpr int FD_CELLS = 4096;
constexpr int FD_THREADS = 1024;

template <typename T, typename TB>
__global__ void __launch_bounds__(FD_THREADS) k_coarse_fd(Geo g, const TB *bin, T *xout, const double *fd) {
  __shared__ T bufA[FD_CELLS];
  __shared__ T bufB[FD_CELLS];
  __shared__ T Q[3][FD_MAXN * FD_MAXN];
  __shared__ T lam[3][FD_MAXN];
  const int n[3] = {g.n0, g.n1, g.n2};
  const int nc = g.n0 * g.n1 * g.n2;
  const int tid = threadIdx.x;
  {
    const double *p = fd;
    for (int a = 0; a < 3; ++a) {
      for (int q = tid; q < n[a] * n[a]; q += FD_THREADS) Q[a][q] = (T)p[q];
      p += n[a] * n[a];
    }
    for (int a = 0; a < 3; ++a) {
      for (int q = tid; q < n[a]; q += FD_THREADS) lam[a][q] = (T)p[q];
      p += n[a];
    }
  }
  for (int e = tid; e < nc; e += FD_THREADS) {
    int k = e % g.n2, r = e / g.n2, j = r % g.n1, i = r / g.n1;
    bufA[e] = (T)bin[sidx(g, i, j, k)];
  }
  __syncthreads();
  // one 1-D transform along axis a: out[.., m, ..] = sum_t M[t][m] in[.., t, ..]
  // (forward, coefficients) or sum_t M[m][t] in[.., t, ..] (backward)
  auto pass = [&](const T *in, T *out, int a, bool fwd) {
    const int na = n[a];
    const int stride = a == 2 ? 1 : (a == 1 ? g.n2 : g.n1 * g.n2);
    const T *M = Q[a];
    for (int e = tid; e < nc; e += FD_THREADS) {
      const int ia = (e / stride) % na;
      const int base = e - ia * stride;
      T acc = T(0);
      for (int t = 0; t < na; ++t) acc += (fwd ? M[t * na + ia] : M[ia * na + t]) * in[base + t * stride];
      out[e] = acc;
    }
    __syncthreads();
  };
  pass(bufA, bufB, 2, true);
  pass(bufB, bufA, 1, true);
  pass(bufA, bufB, 0, true);
  for (int e = tid; e < nc; e += FD_THREADS) {
    int k = e % g.n2, r = e / g.n2, j = r % g.n1, i = r / g.n1;
    T d = lam[0][i] + lam[1][j] + lam[2][k];
    bufB[e] = d > T(0) ? bufB[e] / d : T(0);
  }
  __syncthreads();
  pass(bufB, bufA, 0, false);
  pass(bufA, bufB, 1, false);
  pass(bufB, bufA, 2, false);
  for (int e = tid; e < nc; e += FD_THREADS) {
    int k = e % g.n2, r = e / g.n2, j = r % g.n1, i = r / g.n1;
    xout[sidx(g, i, j, k)] = bufA[e];
  }
}

template <typename T, typename TB>
hipError_t mg_coarse_fd(const Geo &gc, const TB *b, T *x, const double *fd, hipStream_t s) {
  if ((long long)gc.n0 * gc.n1 * gc.n2 > FD_CELLS || gc.n0 > FD_MAXN || gc.n1 > FD_MAXN || gc.n2 > FD_MAXN)
    return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_coarse_fd<T, TB>), dim3(1), dim3(FD_THREADS), 0, s, gc, b, x, fd);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// The last two levels of the V-cycle in one workgroup: a fine grid of at most
// SUB_FINE cells (natural layout in LDS) and its coarsest grid, solved exactly
// by fast diagonalisation.  The same cycle as the grid-wide levels: from
// x = 0, `pre` red-black pairs (the first one is the sweep from zero), the
// residual averaged over the eight children, the exact coarse solve (constant
// mode dropped), trilinear prolongation, `post` black-red pairs.  One launch
// replaces the eight of the two levels, which are bound by latency.
constexpr int SUB_FINE = 4096;
constexpr int SUB_COARSE = SUB_FINE / 8;
constexpr int SUB_ZERO = SUB_FINE + SUB_COARSE;  // an LDS slot that always holds 0
constexpr int SUB_SLOTS = SUB_FINE / 2 / COARSE_THREADS;  // fine cells of one colour per thread

// A fine cell of the subcycle with everything its relaxation and residual
// need that does not change during the kernel: its LDS index q, its
// neighbour count nn (meta = q | nn << 16, -1 for an absent slot) and the LDS
// indices of its neighbours in the order -x, +x, -y, +y, -z, +z, two per word
// (a missing neighbour past a wall points at the zero slot, so it adds 0).
// Built once per thread, so a half sweep costs six LDS reads and a few adds
// per cell instead of the index decoding and boundary logic of lds_nb, which
// bound the single workgroup's four SIMDs.
struct SubCell {
  int meta;
  unsigned nb[3];
};
__device__ __forceinline__ SubCell sub_cell(const LvlDim &f, int bc0, int bc1, int bc2, int color, int ec) {
  SubCell r;
  const int hn2 = f.n2 >> 1;
  r.meta = -1;
  r.nb[0] = r.nb[1] = r.nb[2] = 0;
  if (ec >= f.n0 * f.n1 * hn2) return r;
  int kh, rr, i, j;
  if (f.pow2) {
    kh = ec & (hn2 - 1);
    rr = ec >> (f.l2 - 1);
    j = rr & (f.n1 - 1);
    i = rr >> f.l1;
  } else {
    kh = ec % hn2;
    rr = ec / hn2;
    j = rr % f.n1;
    i = rr / f.n1;
  }
  const int k = 2 * kh + ((i + j + color) & 1);
  auto at = [&](int ii, int jj, int kk) { return f.off + (ii * f.n1 + jj) * f.n2 + kk; };
  const int t[6] = {nbr(i, -1, f.n0, bc0), nbr(i, 1, f.n0, bc0), nbr(j, -1, f.n1, bc1),
                    nbr(j, 1, f.n1, bc1),  nbr(k, -1, f.n2, bc2), nbr(k, 1, f.n2, bc2)};
  int id[6], nn = 0;
#pragma unroll
  for (int d = 0; d < 6; ++d) {
    const int a = d >> 1;
    id[d] = t[d] < 0 ? SUB_ZERO : (a == 0 ? at(t[d], j, k) : (a == 1 ? at(i, t[d], k) : at(i, j, t[d])));
    nn += t[d] >= 0;
  }
#pragma unroll
  for (int w = 0; w < 3; ++w) r.nb[w] = (unsigned)id[2 * w] | ((unsigned)id[2 * w + 1] << 16);
  r.meta = at(i, j, k) | (nn << 16);
  return r;
}
template <typename T>
__device__ __forceinline__ T sub_nbsum(const T *x, const SubCell &c) {
  T s = T(0);
#pragma unroll
  for (int w = 0; w < 3; ++w) {
    s += x[c.nb[w] & 0xffffu];
    s += x[c.nb[w] >> 16];
  }
  return s;
}

// The subcycle's per-thread tables, built once per grid (k_subcycle_tables)
// so that a launch reads them instead of forming them: int4 slot s of thread
// tid at tab[s * COARSE_THREADS + tid]; slots 0-3 the SubCell of cell (cc,
// u) = (s >> 1, s & 1), slots 4-7 the prolongation of natural-order fine
// cell e = tid + (s - 4) COARSE_THREADS: the coarse offsets of the parent and
// of its neighbour on the child's side along each axis, two 16-bit offsets
// per word (axis 0 in x, 1 in y, 2 in z; w = 1 for a cell of the grid).
constexpr int SUB_TAB_SLOTS = 8;
int subcycle_table_ints() { return 4 * SUB_TAB_SLOTS * COARSE_THREADS; }
__device__ __forceinline__ int4 sub_prolong_entry(const LvlDim &f, const LvlDim &c, int bc0, int bc1, int bc2, int e) {
  int4 r = make_int4(0, 0, 0, 0);
  if (e >= f.n0 * f.n1 * f.n2) return r;
  int i, j, k;
  lds_decode(f, e, i, j, k);
  const int I0 = i >> 1, J0 = j >> 1, K0 = k >> 1;
  const int I1 = coarse_partner(I0, i & 1, c.n0, bc0);
  const int J1 = coarse_partner(J0, j & 1, c.n1, bc1);
  const int K1 = coarse_partner(K0, k & 1, c.n2, bc2);
  const int s0 = c.n1 * c.n2, s1 = c.n2;
  r.x = (I0 * s0) | ((I1 * s0) << 16);
  r.y = (J0 * s1) | ((J1 * s1) << 16);
  r.z = K0 | (K1 << 16);
  r.w = 1;
  return r;
}
__device__ __forceinline__ LvlDim sub_dims(const Geo &g, int off) {
  LvlDim d;
  d.n0 = g.n0; d.n1 = g.n1; d.n2 = g.n2; d.off = off;
  d.pow2 = !(g.n0 & (g.n0 - 1)) && !(g.n1 & (g.n1 - 1)) && !(g.n2 & (g.n2 - 1));
  d.l1 = 31 - __clz(g.n1);
  d.l2 = 31 - __clz(g.n2);
  return d;
}
__global__ void __launch_bounds__(COARSE_THREADS) k_subcycle_tables(Geo gf, Geo gc, int4 *tab) {
  const int tid = threadIdx.x, nf = gf.n0 * gf.n1 * gf.n2;
  const LvlDim f = sub_dims(gf, 0), c = sub_dims(gc, nf);
#pragma unroll
  for (int cc = 0; cc < 2; ++cc)
#pragma unroll
    for (int u = 0; u < SUB_SLOTS; ++u) {
      const SubCell sc = sub_cell(f, gf.bc0, gf.bc1, gf.bc2, cc, tid + u * COARSE_THREADS);
      tab[(cc * SUB_SLOTS + u) * COARSE_THREADS + tid] = make_int4(sc.meta, (int)sc.nb[0], (int)sc.nb[1], (int)sc.nb[2]);
    }
#pragma unroll
  for (int r = 0; r < SUB_FINE / COARSE_THREADS; ++r)
    tab[(2 * SUB_SLOTS + r) * COARSE_THREADS + tid] =
        sub_prolong_entry(f, c, gf.bc0, gf.bc1, gf.bc2, tid + r * COARSE_THREADS);
}

template <typename T, typename TB>
__global__ void __launch_bounds__(COARSE_THREADS) k_subcycle(Geo gf, Geo gc, const TB *bin, T *xout,
                                                             const double *fd, const int4 *tab, int pre, int post) {
  __shared__ T sx[SUB_FINE + SUB_COARSE + 1];
  __shared__ T sb[SUB_FINE + SUB_COARSE];
  __shared__ T rf[SUB_FINE];  // fine residuals for the restriction
  __shared__ T fa[SUB_COARSE], fb[SUB_COARSE];
  __shared__ T Q[3][FD_MAXN * FD_MAXN];
  __shared__ T lam[3][FD_MAXN];
  const int tid = threadIdx.x;
  const int nf = gf.n0 * gf.n1 * gf.n2, nc = gc.n0 * gc.n1 * gc.n2;
  const LvlDim c = sub_dims(gc, nf);
  // the right-hand side of the thread's cells and its tables, every load
  // issued before any is used; slot (cc, u) is the colour-cc cell with
  // split-layout index cc half + tid + u COARSE_THREADS, so the right-hand
  // side is read and the result written with coalesced accesses and no
  // index arithmetic
  TB bl[2][SUB_SLOTS];
  SubCell cell[2][SUB_SLOTS];
  int4 pe[SUB_FINE / COARSE_THREADS];
#pragma unroll
  for (int cc = 0; cc < 2; ++cc)
#pragma unroll
    for (int u = 0; u < SUB_SLOTS; ++u) {
      const long long ec = tid + u * COARSE_THREADS;
      bl[cc][u] = ec < gf.half ? bin[(long long)cc * gf.half + ec] : TB(0);
      const int4 t = tab[(cc * SUB_SLOTS + u) * COARSE_THREADS + tid];
      cell[cc][u].meta = t.x;
      cell[cc][u].nb[0] = (unsigned)t.y;
      cell[cc][u].nb[1] = (unsigned)t.z;
      cell[cc][u].nb[2] = (unsigned)t.w;
    }
#pragma unroll
  for (int r = 0; r < SUB_FINE / COARSE_THREADS; ++r) pe[r] = tab[(2 * SUB_SLOTS + r) * COARSE_THREADS + tid];
  {
    const int n[3] = {gc.n0, gc.n1, gc.n2};
    const double *p = fd;
    for (int a = 0; a < 3; ++a) {
      for (int q = tid; q < n[a] * n[a]; q += COARSE_THREADS) Q[a][q] = (T)p[q];
      p += n[a] * n[a];
    }
    for (int a = 0; a < 3; ++a) {
      for (int q = tid; q < n[a]; q += COARSE_THREADS) lam[a][q] = (T)p[q];
      p += n[a];
    }
  }
  if (tid == 0) sx[SUB_ZERO] = T(0);
#pragma unroll
  for (int cc = 0; cc < 2; ++cc)
#pragma unroll
    for (int u = 0; u < SUB_SLOTS; ++u)
      if (cell[cc][u].meta >= 0) {
        const int q = cell[cc][u].meta & 0xffff;
        sb[q] = (T)bl[cc][u];
        sx[q] = T(0);
      }
  __syncthreads();
  const T h2 = (T)(gf.h * gf.h), ih2 = T(1) / h2;
  // one half sweep over colour cc (the same operations as lds_smooth)
  auto smooth = [&](int cc) {
#pragma unroll
    for (int u = 0; u < SUB_SLOTS; ++u) {
      const SubCell &cl = cell[cc][u];
      if (cl.meta >= 0) {
        const int q = cl.meta & 0xffff, nn = cl.meta >> 16;
        const T sum = sub_nbsum(sx, cl);
        sx[q] = (h2 * sb[q] + sum) * inv_nn<T>(nn);
      }
    }
  };
  for (int q = 0; q < pre; ++q) {
    smooth(0);
    __syncthreads();
    smooth(1);
    __syncthreads();
  }
  // residual of every fine cell (as lds_resid), then the average over the
  // eight children of each coarse cell
#pragma unroll
  for (int cc = 0; cc < 2; ++cc)
#pragma unroll
    for (int u = 0; u < SUB_SLOTS; ++u) {
      const SubCell &cl = cell[cc][u];
      if (cl.meta >= 0) {
        const int q = cl.meta & 0xffff, nn = cl.meta >> 16;
        const T sum = sub_nbsum(sx, cl);
        rf[q] = sb[q] - ((T)nn * sx[q] - sum) * ih2;
      }
    }
  __syncthreads();
  for (int e = tid; e < nc; e += COARSE_THREADS) {
    int i, j, k;
    lds_decode(c, e, i, j, k);
    T acc = T(0);
    for (int q = 0; q < 8; ++q)
      acc += rf[((2 * i + (q >> 2)) * gf.n1 + 2 * j + ((q >> 1) & 1)) * gf.n2 + 2 * k + (q & 1)];
    fa[e] = acc * (T)0.125;
  }
  __syncthreads();
  // exact coarse solve: the six 1-D eigenbasis transforms and the division;
  // thread tid owns coarse element tid (nc <= SUB_COARSE <= COARSE_THREADS),
  // whose index along each axis and line base are formed once
  static_assert(SUB_COARSE <= COARSE_THREADS, "one coarse element per thread");
  const int n[3] = {gc.n0, gc.n1, gc.n2};
  const int cstride[3] = {gc.n1 * gc.n2, gc.n2, 1};
  int cia[3], cbase[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    cia[a] = (tid / cstride[a]) % n[a];
    cbase[a] = tid - cia[a] * cstride[a];
  }
  auto pass = [&](const T *in, T *out, int a, bool fwd) {
    if (tid < nc) {
      const int na = n[a], stride = cstride[a], ia = cia[a], base = cbase[a];
      const T *M = Q[a];
      T acc = T(0);
#pragma unroll 8
      for (int t = 0; t < na; ++t) acc += (fwd ? M[t * na + ia] : M[ia * na + t]) * in[base + t * stride];
      out[tid] = acc;
    }
    __syncthreads();
  };
  pass(fa, fb, 2, true);
  pass(fb, fa, 1, true);
  pass(fa, fb, 0, true);
  if (tid < nc) {
    T d = lam[0][cia[0]] + lam[1][cia[1]] + lam[2][cia[2]];
    fb[tid] = d > T(0) ? fb[tid] / d : T(0);
  }
  __syncthreads();
  pass(fb, fa, 0, false);
  pass(fa, fb, 1, false);
  pass(fb, sx + nf, 2, false);  // the coarse solution, after the fine cells
  // trilinear prolongation of the coarse solution onto every fine cell (the
  // coarse offsets of each cell's parents from the tables)
#pragma unroll
  for (int r = 0; r < SUB_FINE / COARSE_THREADS; ++r) {
    const int e = tid + r * COARSE_THREADS;
    if (!pe[r].w) continue;
    const int I0 = pe[r].x & 0xffff, I1 = pe[r].x >> 16, J0 = pe[r].y & 0xffff, J1 = pe[r].y >> 16;
    const int K0 = pe[r].z & 0xffff, K1 = pe[r].z >> 16;
    const T *xc = sx + nf;
    auto X = [&](int a, int b, int cc) { return xc[a + b + cc]; };
    const T v0 = (T)0.75 * X(I0, J0, K0) + (T)0.25 * X(I1, J0, K0);
    const T v1 = (T)0.75 * X(I0, J1, K0) + (T)0.25 * X(I1, J1, K0);
    const T v2 = (T)0.75 * X(I0, J0, K1) + (T)0.25 * X(I1, J0, K1);
    const T v3 = (T)0.75 * X(I0, J1, K1) + (T)0.25 * X(I1, J1, K1);
    const T w0 = (T)0.75 * v0 + (T)0.25 * v1;
    const T w1 = (T)0.75 * v2 + (T)0.25 * v3;
    sx[e] += (T)0.75 * w0 + (T)0.25 * w1;
  }
  __syncthreads();
  for (int q = 0; q < post; ++q) {
    smooth(1);
    __syncthreads();
    smooth(0);
    __syncthreads();
  }
#pragma unroll
  for (int cc = 0; cc < 2; ++cc)
#pragma unroll
    for (int u = 0; u < SUB_SLOTS; ++u)
      if (cell[cc][u].meta >= 0)
        xout[(long long)cc * gf.half + tid + u * COARSE_THREADS] = sx[cell[cc][u].meta & 0xffff];
}

bool subcycle_fits(const Geo &gf, const Geo &gc) {
  const long long nf = (long long)gf.n0 * gf.n1 * gf.n2;
  return nf <= SUB_FINE && gc.n0 <= FD_MAXN && gc.n1 <= FD_MAXN && gc.n2 <= FD_MAXN && gc.n0 * 2 == gf.n0 &&
         gc.n1 * 2 == gf.n1 && gc.n2 * 2 == gf.n2;
}

template <typename T, typename TB>
hipError_t mg_subcycle(const Geo &gf, const Geo &gc, const TB *b, T *x, const double *fd, const int *tab, int pre,
                       int post, hipStream_t s) {
  if (!subcycle_fits(gf, gc) || !tab) return hipErrorInvalidValue;
  hipEvent_t e0, e1;
  probe_ext_take(&e0, &e1);
  hipExtLaunchKernelGGL((k_subcycle<T, TB>), dim3(1), dim3(COARSE_THREADS), 0, s, e0, e1, 0, gf, gc, b, x, fd,
                        (const int4 *)tab, pre, post);
  return hipGetLastError();
}
hipError_t mg_subcycle_tables(const Geo &gf, const Geo &gc, int *tab, hipStream_t s) {
  if (!subcycle_fits(gf, gc) || !tab) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_subcycle_tables, dim3(1), dim3(COARSE_THREADS), 0, s, gf, gc, (int4 *)tab);
  return hipGetLastError();
}

// Packed eigen-decompositions of the three 1-D Laplacians of a coarse grid
// (host): Q0 (n0 x n0), Q1, Q2 row-major with the eigenvectors as columns,
// then lam0, lam1, lam2.  No-slip axes: cell-centred Neumann operator,
// eigenvectors cos(pi k (i + 1/2) / n), eigenvalues (4/h^2) sin^2(pi k / 2n).
// Periodic axes: the constant, cos / sin(2 pi k i / n) pairs and, for even n,
// (-1)^i, eigenvalues (4/h^2) sin^2(pi k / n).
int coarse_fd_size(const int n[3]) { return n[0] * n[0] + n[1] * n[1] + n[2] * n[2] + n[0] + n[1] + n[2]; }
void coarse_fd_build(const int n[3], const int bc[3], double h, double *out) {
  const double pi = 3.14159265358979323846;
  double *q = out;
  double *l = out + n[0] * n[0] + n[1] * n[1] + n[2] * n[2];
  for (int a = 0; a < 3; ++a) {
    const int na = n[a];
    const double c = 4.0 / (h * h);
    for (int col = 0; col < na; ++col) {
      double lamv;
      for (int i = 0; i < na; ++i) {
        double v;
        if (bc[a]) {
          const double nrm = col == 0 ? sqrt((double)na) : sqrt(0.5 * na);
          v = cos(pi * col * (i + 0.5) / na) / nrm;
        } else if (col == 0) {
          v = 1.0 / sqrt((double)na);
        } else if ((na % 2 == 0) && col == na - 1) {
          v = ((i & 1) ? -1.0 : 1.0) / sqrt((double)na);
        } else {
          const int k = (col + 1) / 2;  // columns 1, 2 -> k = 1 (cos, sin), 3, 4 -> k = 2 ...
          const double th = 2.0 * pi * k * i / na;
          v = ((col & 1) ? cos(th) : sin(th)) / sqrt(0.5 * na);
        }
        q[i * na + col] = v;
      }
      if (bc[a]) {
        const double sn = sin(pi * col / (2.0 * na));
        lamv = c * sn * sn;
      } else if (col == 0) {
        lamv = 0.0;
      } else if ((na % 2 == 0) && col == na - 1) {
        lamv = c;
      } else {
        const int k = (col + 1) / 2;
        const double sn = sin(pi * k / na);
        lamv = c * sn * sn;
      }
      l[col] = lamv;
    }
    q += na * na;
    l += na;
  }
}

#define INST(T, TB)                                                                                    \
  template hipError_t mg_smooth_first<T, TB>(const Geo &, T *, const TB *, bool, hipStream_t);        \
  template hipError_t mg_smooth<T, TB>(const Geo &, T *, const TB *, int, hipStream_t);               \
  template hipError_t mg_restrict<T, TB>(const Geo &, const T *, const TB *, const Geo &, T *,         \
                                         hipStream_t);                                                 \
  template hipError_t mg_coarse<T, TB>(const Geo &, const TB *, T *, int, int, hipStream_t);                   \
  template hipError_t mg_coarse_fd<T, TB>(const Geo &, const TB *, T *, const double *, hipStream_t);   \
  template hipError_t mg_subcycle<T, TB>(const Geo &, const Geo &, const TB *, T *, const double *, const int *, \
                                         int, int, hipStream_t);                                               \
  template hipError_t mg_tile_down<T, TB>(const Geo &, T *, const TB *, const Geo &, T *, int, hipStream_t);   \
  template hipError_t mg_tile_up<T, TB>(const Geo &, const T *, T *, const TB *, const Geo &, const T *, int, \
                                        hipStream_t);
INST(float, float)
INST(float, double)
INST(double, double)
#undef INST
template hipError_t mg_prolong<float>(const Geo &, float *, const Geo &, const float *, hipStream_t);
template hipError_t mg_prolong<double>(const Geo &, double *, const Geo &, const double *, hipStream_t);

}  // namespace ibs
