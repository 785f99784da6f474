// Plane-marching stencil kernels on the red/black split layout.
//
// A workgroup owns a tile of BY rows (axis 1) x 2*BX in-row indices m
// (axis 2, two per thread, accessed as 2-vectors) and marches over a chunk of
// planes along axis 0 (march_chunk).  The x-neighbours of a cell come from a
// register window over three planes, the y- and z-neighbours from an LDS copy
// of the current plane with a one-cell halo.  BX divides hn2/2 and BY divides
// n1, so no workgroup is partial and every halo cell is loaded.
#pragma once
#include "internal.h"

namespace ibs {

constexpr int MARCH_CH = 8;       // most planes per workgroup
constexpr int MARCH_TILE = 1104;  // >= max (BY+2)(2BX+2) over BX*BY <= 256

struct MarchShape {
  int bx, by;
  dim3 grid, block;
};

__host__ __device__ inline int pow2_divisor(int n, int cap) {
  int p = 1;
  while (p * 2 <= cap && n % (p * 2) == 0) p *= 2;
  return p;
}

// Planes per workgroup: MARCH_CH on large grids (long register-window
// chains, few halo re-reads), halved until the grid has g.march_min_blocks
// workgroups on coarse multigrid levels, where latency rather than bytes
// bounds a sweep.
__host__ __device__ inline int march_chunk(const Geo &g) {
  const int bx = pow2_divisor(g.hn2 / 2, 64);
  const int by = pow2_divisor(g.n1, 256 / bx);
  const long long xy = (long long)(g.hn2 / (2 * bx)) * (g.n1 / by);
  int ch = MARCH_CH;
  while (ch > 1 && xy * ((g.n0 + ch - 1) / ch) < g.march_min_blocks) ch >>= 1;
  return ch;
}

// ncomp stacks independent component grids along grid.z.
inline MarchShape march_shape(const Geo &g, int ncomp) {
  MarchShape s;
  s.bx = pow2_divisor(g.hn2 / 2, 64);
  s.by = pow2_divisor(g.n1, 256 / s.bx);
  s.block = dim3(s.bx, s.by, 1);
  const int ch = march_chunk(g);
  int nch = (g.n0 + ch - 1) / ch;
  s.grid = dim3(g.hn2 / (2 * s.bx), g.n1 / s.by, nch * ncomp);
  return s;
}

template <typename T>
struct V2 {
  T x, y;
};
// 2-vector load of S values converted to R
template <typename R, typename S>
__device__ __forceinline__ V2<R> ld2(const S *p) {
  V2<R> v;
  if (sizeof(S) == 4) {
    float2 f = *(const float2 *)p;
    v.x = (R)f.x;
    v.y = (R)f.y;
  } else {
    double2 f = *(const double2 *)p;
    v.x = (R)f.x;
    v.y = (R)f.y;
  }
  return v;
}
template <typename T>
__device__ __forceinline__ void st2(T *p, T a, T b) {
  if (sizeof(T) == 4) {
    *(float2 *)p = make_float2((float)a, (float)b);
  } else {
    *(double2 *)p = make_double2((double)a, (double)b);
  }
}

// Coordinate wrap for periodic axes; -1 if outside a wall box.
__device__ __forceinline__ int mwrap(int i, int n, int bc) {
  if (i < 0) return bc ? -1 : i + n;
  if (i >= n) return bc ? -1 : i - n;
  return i;
}

// Tile coordinates of this workgroup.  The dispatcher deals consecutive
// workgroups round-robin to the 8 XCDs; with `xcd` set, each XCD walks all
// row tiles of one plane chunk (grid.z) in turn while the other XCDs take the
// seven chunks beside it, so the tiles that share halo rows run on one XCD at
// the same time and those re-reads hit its L2.  Measured, this pays on the
// three-component momentum grids and on the Laplacian of the S~ product, and
// costs time on the single-component multigrid levels, which keep the plain
// order.
struct MarchBlock {
  int x, y, z;
};
__device__ __forceinline__ MarchBlock march_block(bool xcd) {
  const unsigned gx = gridDim.x, gxy = gx * gridDim.y;
  MarchBlock mb;
  if (xcd && gridDim.z % 8 == 0) {
    const unsigned b = blockIdx.x + gx * (blockIdx.y + gridDim.y * blockIdx.z);
    const unsigned slot = b / 8, rem = slot % gxy;
    mb.x = rem % gx;
    mb.y = rem / gx;
    mb.z = (slot / gxy) * 8 + b % 8;
  } else {
    mb.x = blockIdx.x;
    mb.y = blockIdx.y;
    mb.z = blockIdx.z;
  }
  return mb;
}

// Per-block geometry of a march.
struct MarchPos {
  int tx, ty, m0, j, i0, i1, comp, mbase, jbase;
};
__device__ __forceinline__ MarchPos march_pos(const Geo &g, bool xcd) {
  MarchPos p;
  const MarchBlock mb = march_block(xcd);
  p.tx = threadIdx.x;
  p.ty = threadIdx.y;
  p.mbase = mb.x * blockDim.x * 2;
  p.jbase = mb.y * blockDim.y;
  p.m0 = p.mbase + 2 * threadIdx.x;
  p.j = p.jbase + threadIdx.y;
  const int len = march_chunk(g);
  int nch = (g.n0 + len - 1) / len;
  p.comp = mb.z / nch;
  int ch = mb.z - p.comp * nch;
  p.i0 = ch * len;
  p.i1 = min(p.i0 + len, g.n0);
  return p;
}

// Load the one-cell halo of the plane tile (rows ty = -1, BY and columns
// m = -1, 2BX) cooperatively; val(i, j, m) returns the value of a plane at an
// in-domain position (already wrapped), 0 is stored outside a wall box.
template <typename T, class F>
__device__ __forceinline__ void tile_halo(T *tile, const Geo &g, int i, int jbase, int mbase, int BX, int BY,
                                          F val) {
  const int W2 = 2 * BX + 2;
  const int nrow = 2 * (2 * BX), ncol = 2 * BY;
  const int tid = threadIdx.x + blockDim.x * threadIdx.y;
  for (int h = tid; h < nrow + ncol; h += blockDim.x * blockDim.y) {
    int r, cidx;
    if (h < nrow) {
      r = h < 2 * BX ? 0 : BY + 1;
      cidx = 1 + (h % (2 * BX));
    } else {
      int q = h - nrow;
      r = 1 + (q >> 1);
      cidx = (q & 1) ? 2 * BX + 1 : 0;
    }
    int jj = mwrap(jbase + r - 1, g.n1, g.bc1);
    int mm = mwrap(mbase + cidx - 1, g.hn2, g.bc2);
    T v = T(0);
    if (jj >= 0 && mm >= 0 && (unsigned)i < (unsigned)g.n0) v = val(i, jj, mm);
    tile[r * W2 + cidx] = v;
  }
}

// The same halo in two halves, so that the loads of the next plane can be
// issued before the current plane is computed: halo_fetch reads up to
// HALO_REG values per thread into registers, halo_put stores them (and loads
// any remainder of very thin tiles directly).
constexpr int HALO_REG = 2;
template <typename T>
struct Halo {
  T v[HALO_REG];
};
__device__ __forceinline__ void halo_slot(int h, int BX, int BY, int &r, int &cidx) {
  const int nrow = 2 * (2 * BX);
  if (h < nrow) {
    r = h < 2 * BX ? 0 : BY + 1;
    cidx = 1 + (h % (2 * BX));
  } else {
    const int q = h - nrow;
    r = 1 + (q >> 1);
    cidx = (q & 1) ? 2 * BX + 1 : 0;
  }
}
template <typename T, class F>
__device__ __forceinline__ Halo<T> halo_fetch(const Geo &g, int i, int jbase, int mbase, int BX, int BY, F val) {
  Halo<T> hv;
  const int total = 2 * (2 * BX) + 2 * BY, nthr = BX * BY;
  const int tid = threadIdx.x + BX * threadIdx.y;
#pragma unroll
  for (int q = 0; q < HALO_REG; ++q) {
    hv.v[q] = T(0);
    const int h = tid + q * nthr;
    if (h < total) {
      int r, cidx;
      halo_slot(h, BX, BY, r, cidx);
      const int jj = mwrap(jbase + r - 1, g.n1, g.bc1);
      const int mm = mwrap(mbase + cidx - 1, g.hn2, g.bc2);
      if (jj >= 0 && mm >= 0 && (unsigned)i < (unsigned)g.n0) hv.v[q] = val(i, jj, mm);
    }
  }
  return hv;
}
template <typename T, class F>
__device__ __forceinline__ void halo_put(T *tile, const Halo<T> &hv, const Geo &g, int i, int jbase, int mbase,
                                         int BX, int BY, F val) {
  const int total = 2 * (2 * BX) + 2 * BY, nthr = BX * BY, W2 = 2 * BX + 2;
  const int tid = threadIdx.x + BX * threadIdx.y;
#pragma unroll
  for (int q = 0; q < HALO_REG; ++q) {
    const int h = tid + q * nthr;
    if (h < total) {
      int r, cidx;
      halo_slot(h, BX, BY, r, cidx);
      tile[r * W2 + cidx] = hv.v[q];
    }
  }
  for (int h = tid + HALO_REG * nthr; h < total; h += nthr) {
    int r, cidx;
    halo_slot(h, BX, BY, r, cidx);
    const int jj = mwrap(jbase + r - 1, g.n1, g.bc1);
    const int mm = mwrap(mbase + cidx - 1, g.hn2, g.bc2);
    T v = T(0);
    if (jj >= 0 && mm >= 0 && (unsigned)i < (unsigned)g.n0) v = val(i, jj, mm);
    tile[r * W2 + cidx] = v;
  }
}
// halo_put for halos fetched as raw operands: the register part stores
// xf(i, jj, mm, raw) (0 outside a wall box), the remainder val(i, jj, mm).
template <typename T, class F, class X>
__device__ __forceinline__ void halo_put_xf(T *tile, const Halo<T> &hv, const Geo &g, int i, int jbase, int mbase,
                                            int BX, int BY, F val, X xf) {
  const int total = 2 * (2 * BX) + 2 * BY, nthr = BX * BY, W2 = 2 * BX + 2;
  const int tid = threadIdx.x + BX * threadIdx.y;
#pragma unroll
  for (int q = 0; q < HALO_REG; ++q) {
    const int h = tid + q * nthr;
    if (h < total) {
      int r, cidx;
      halo_slot(h, BX, BY, r, cidx);
      const int jj = mwrap(jbase + r - 1, g.n1, g.bc1);
      const int mm = mwrap(mbase + cidx - 1, g.hn2, g.bc2);
      tile[r * W2 + cidx] = (jj >= 0 && mm >= 0 && (unsigned)i < (unsigned)g.n0) ? xf(i, jj, mm, hv.v[q]) : T(0);
    }
  }
  for (int h = tid + HALO_REG * nthr; h < total; h += nthr) {
    int r, cidx;
    halo_slot(h, BX, BY, r, cidx);
    const int jj = mwrap(jbase + r - 1, g.n1, g.bc1);
    const int mm = mwrap(mbase + cidx - 1, g.hn2, g.bc2);
    T v = T(0);
    if (jj >= 0 && mm >= 0 && (unsigned)i < (unsigned)g.n0) v = val(i, jj, mm);
    tile[r * W2 + cidx] = v;
  }
}

}  // namespace ibs

namespace ibs {

// Plane-invariant halo slots of a thread (HALO_REG of them): LDS slot (-1:
// none), in-plane offset (-1: outside a wall box), row and in-row index.
// Thin tiles (more halo cells than HALO_REG per thread) load the rest of
// their halo directly.
struct HaloSlots {
  int slot[HALO_REG], off[HALO_REG], jj[HALO_REG], mm[HALO_REG];
  int total, nthr, tid;
  bool rem;
};
__device__ __forceinline__ HaloSlots halo_slots(const Geo &g, int jbase, int mbase, int BX, int BY) {
  HaloSlots hs;
  const int W2 = 2 * BX + 2;
  hs.total = 2 * (2 * BX) + 2 * BY;
  hs.nthr = BX * BY;
  hs.tid = threadIdx.x + BX * threadIdx.y;
  hs.rem = hs.total > HALO_REG * hs.nthr;
#pragma unroll
  for (int q = 0; q < HALO_REG; ++q) {
    const int h = hs.tid + q * hs.nthr;
    hs.slot[q] = -1;
    hs.off[q] = -1;
    hs.jj[q] = 0;
    hs.mm[q] = 0;
    if (h < hs.total) {
      int r, cidx;
      halo_slot(h, BX, BY, r, cidx);
      hs.slot[q] = r * W2 + cidx;
      const int jj = mwrap(jbase + r - 1, g.n1, g.bc1);
      const int mm = mwrap(mbase + cidx - 1, g.hn2, g.bc2);
      if (jj >= 0 && mm >= 0) {
        hs.off[q] = jj * g.hn2 + mm;
        hs.jj[q] = jj;
        hs.mm[q] = mm;
      }
    }
  }
  return hs;
}

// Stencil diagonal of a thread's two cells k = 2 (m0 + u) + s of row j, split
// into the part of axes 1 and 2 (fixed along a march along axis 0, tabulated
// for both parities s) and the part of axis 0 (per plane).  Pressure
// Laplacian: the number of missing neighbours (the cell has 6 - di - djk);
// momentum operator on component d: the 7-point diagonal count in units of
// 1/h^2 (di + djk) with the tangential wall ghosts, and the wall-face flag.
struct DiagJK {
  int d[2][2];
  bool w[2][2];
  // entries for parity s and (compile-time) cell u, selected without a
  // dynamic index so that the table stays in registers
  __device__ __forceinline__ int dg(int s, int u) const { return s ? d[1][u] : d[0][u]; }
  __device__ __forceinline__ bool wl(int s, int u) const { return s ? w[1][u] : w[0][u]; }
};
__device__ __forceinline__ DiagJK diag_jk(const Geo &g, int j, int m0, bool helm, int d) {
  DiagJK r;
#pragma unroll
  for (int sp = 0; sp < 2; ++sp)
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int k = 2 * (m0 + u) + sp;
      if (helm) {
        int dg = 4;
        if (g.bc1 && d != 1) dg += wall_ghost_diag(g.bc1) * ((j == 0) + (j == g.n1 - 1));
        if (g.bc2 && d != 2) dg += wall_ghost_diag(g.bc2) * ((k == 0) + (k == g.n2 - 1));
        r.d[sp][u] = dg;
        r.w[sp][u] = d == 1 ? (g.bc1 && j == 0) : (d == 2 ? (g.bc2 && k == 0) : false);
      } else {
        r.d[sp][u] = (g.bc1 ? (j == 0) + (j == g.n1 - 1) : 0) + (g.bc2 ? (k == 0) + (k == g.n2 - 1) : 0);
        r.w[sp][u] = false;
      }
    }
  return r;
}
__device__ __forceinline__ int diag_i(const Geo &g, int i, bool helm, int d) {
  const int e = (i == 0) + (i == g.n0 - 1);
  return helm ? 2 + ((g.bc0 && d != 0) ? wall_ghost_diag(g.bc0) * e : 0) : (g.bc0 ? e : 0);
}

// One red-black half sweep of colour `color` on the component grids of x.
//   SW_POISSON: x_c = (h^2 b_c + sum of neighbours) / (number of neighbours)
//               (Gauss-Seidel for L = G^T G);
//   SW_FIRST:   the first pressure sweep from x = 0, colour 1: the colour-0
//               values h^2 b / nnb are formed on the fly from b (and stored),
//               then the colour-1 update as above;
//   SW_HELM:    SOR for A = a0 - nu Delta_h on velocity component `comp`:
//               x_c += omega ((b_c + nu/h^2 sum) / (a0 + nu/h^2 diag) - x_c),
//               wall faces untouched.  Neighbours outside a wall box are 0
//               (normal walls hold 0, tangential ghosts enter the diagonal:
//               -u on a no-slip wall, +u on a free-slip wall).
//   SW_HFIRST:  the first SOR sweep of SW_HELM from x = 0, colour 1: the
//               colour-0 values omega b / (a0 + nu/h^2 diag) are formed on
//               the fly from b (and stored), then the colour-1 update; one
//               pass replaces clearing x and two half sweeps.
//   SW_FIRST1:  SW_FIRST without storing the colour-0 values, for a cycle
//               whose next half sweep recomputes colour 0 from colour 1
//               (a Gauss-Seidel update never reads the old value of its
//               own colour).
enum { SW_POISSON = 0, SW_FIRST = 1, SW_HELM = 2, SW_HFIRST = 3, SW_FIRST1 = 4 };

template <typename T, typename TB, int MODE>
__global__ void __launch_bounds__(256) k_sweep(Geo g, T *x, const TB *b, int color, double h2, double a0,
                                               double nuh2, double omega) {
  __shared__ T tile[MARCH_TILE];
  const MarchPos p = march_pos(g, MODE == SW_HELM || MODE == SW_HFIRST);
  const int BX = blockDim.x, BY = blockDim.y, W2 = 2 * BX + 2;
  const long long N = 2 * g.half;
  const int d = p.comp;
  T *xg = x + d * N;
  const TB *bg = b + d * N;
  const int c = color;
  T *own = xg + (long long)c * g.half;
  T *oth = xg + (long long)(1 - c) * g.half;
  const TB *bown = bg + (long long)c * g.half;
  const TB *both = bg + (long long)(1 - c) * g.half;
  const int mbase = p.mbase, jbase = p.jbase;
  auto row = [&](int i, int jj) { return ((long long)i * g.n1 + jj) * g.hn2; };
  const long long P = (long long)g.n1 * g.hn2;  // one plane of one colour
  const int rw = p.j * g.hn2 + p.m0;            // this thread's two cells within a plane
  const T th2 = (T)h2, ta0 = (T)a0, tnu = (T)nuh2, tom = (T)omega;
  constexpr bool FIRSTM = MODE == SW_FIRST || MODE == SW_HFIRST || MODE == SW_FIRST1;
  constexpr bool HELMM = MODE == SW_HELM || MODE == SW_HFIRST;
  // momentum stencil at face (i, jj, kk) of component d: the diagonal count
  // (2 per axis plus the tangential wall ghosts) and whether it is a wall face
  auto helm_cell = [&](int i, int jj, int kk, bool &wall) -> int {
    const int xs[3] = {i, jj, kk};
    int diag = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      int bca = geo_bc(g, a), na = geo_n(g, a);
      diag += 2;
      if (bca && a != d) diag += wall_ghost_diag(bca) * ((xs[a] == 0) + (xs[a] == na - 1));
    }
    const int xd = d == 0 ? i : (d == 1 ? jj : kk);
    wall = geo_bc(g, d) && xd == 0;
    return diag;
  };
  // In the first-sweep modes the other-colour operand is formed from the
  // right-hand side: the loads of the next plane fetch it raw, oxf turns it
  // into the colour-0 value once the current plane has been computed.
  auto oxf = [&](int i, int jj, int mm, T bv) -> T {
    const int kk = 2 * mm + ((i + jj) & 1);  // colour-0 cell of row (i, jj) at index mm
    if (MODE == SW_FIRST || MODE == SW_FIRST1) return pc_first(th2, bv, cell_nnb(g, i, jj, kk));
    bool wall;
    const int dg = helm_cell(i, jj, kk, wall);
    return wall ? T(0) : tom * (bv / (ta0 + tnu * (T)dg));
  };
  auto oval = [&](int i, int jj, int mm) -> T {
    if (FIRSTM) return oxf(i, jj, mm, (T)both[row(i, jj) + mm]);
    return oth[row(i, jj) + mm];
  };
  // other-colour operand of plane ii (in the domain) at in-plane offset o
  auto oget = [&](int ii, int o) -> T {
    if (FIRSTM) return (T)both[ii * P + o];
    return oth[ii * P + o];
  };
  auto owin_ld = [&](int i) -> V2<T> {
    V2<T> v;
    v.x = T(0);
    v.y = T(0);
    int ii = mwrap(i, g.n0, g.bc0);
    if (ii < 0) return v;
    if (FIRSTM) return ld2<T>(both + ii * P + rw);
    return ld2<T>(oth + ii * P + rw);
  };
  auto owin_xf = [&](int i, V2<T> v) -> V2<T> {
    if (!FIRSTM) return v;
    int ii = mwrap(i, g.n0, g.bc0);
    if (ii < 0) return v;  // zeros from owin_ld
    v.x = oxf(ii, p.j, p.m0, v.x);
    v.y = oxf(ii, p.j, p.m0 + 1, v.y);
    return v;
  };
  const HaloSlots hs = halo_slots(g, jbase, mbase, BX, BY);
  auto hfetch = [&](int i, T *hv) {
#pragma unroll
    for (int q = 0; q < HALO_REG; ++q) hv[q] = hs.off[q] >= 0 ? oget(i, hs.off[q]) : T(0);
  };
  auto hput = [&](int i, const T *hv) {
#pragma unroll
    for (int q = 0; q < HALO_REG; ++q)
      if (hs.slot[q] >= 0) tile[hs.slot[q]] = (FIRSTM && hs.off[q] >= 0) ? oxf(i, hs.jj[q], hs.mm[q], hv[q]) : hv[q];
    if (hs.rem) {
      for (int h = hs.tid + HALO_REG * hs.nthr; h < hs.total; h += hs.nthr) {
        int r, cidx;
        halo_slot(h, BX, BY, r, cidx);
        const int jj = mwrap(jbase + r - 1, g.n1, g.bc1);
        const int mm = mwrap(mbase + cidx - 1, g.hn2, g.bc2);
        tile[r * W2 + cidx] = (jj >= 0 && mm >= 0) ? oval(i, jj, mm) : T(0);
      }
    }
  };
  const DiagJK djk = diag_jk(g, p.j, p.m0, HELMM, d);
  V2<T> prev = owin_xf(p.i0 - 1, owin_ld(p.i0 - 1)), cur = owin_xf(p.i0, owin_ld(p.i0)),
        next = owin_xf(p.i0 + 1, owin_ld(p.i0 + 1));
  T hcur[HALO_REG], hnext[HALO_REG];
  hfetch(p.i0, hcur);
  // software pipeline: the window plane i+2, the halo and the own-colour
  // operands of plane i+1 are loaded while plane i is computed
  auto own_ops = [&](int i, V2<T> &bb, V2<T> &xo) {
    const long long r = i * P + rw;
    bb = ld2<T>(bown + r);
    xo.x = T(0);
    xo.y = T(0);
    if (MODE == SW_HELM) xo = ld2<T>((const T *)own + r);
  };
  V2<T> bb, xo;
  own_ops(p.i0, bb, xo);
  for (int i = p.i0; i < p.i1; ++i) {
    const bool more = i + 1 < p.i1;
    V2<T> nn = more ? owin_ld(i + 2) : next;
    V2<T> bbn = bb, xon = xo;
#pragma unroll
    for (int q = 0; q < HALO_REG; ++q) hnext[q] = hcur[q];
    if (more) {
      hfetch(i + 1, hnext);
      own_ops(i + 1, bbn, xon);
    }
    tile[(p.ty + 1) * W2 + 2 * p.tx + 1] = cur.x;
    tile[(p.ty + 1) * W2 + 2 * p.tx + 2] = cur.y;
    hput(i, hcur);
    __syncthreads();
    T out[2];
    const int s = (c + i + p.j) & 1;
    const int di = diag_i(g, i, HELMM, d);
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int col = 2 * p.tx + 1 + u;
      const T *trow = tile + (p.ty + 1) * W2;
      T sum = (u ? prev.y : prev.x) + (u ? next.y : next.x) + tile[p.ty * W2 + col] + tile[(p.ty + 2) * W2 + col] +
              trow[col - 1 + s] + trow[col + s];
      T bv = u ? bb.y : bb.x;
      if (!HELMM) {
        out[u] = pc_relax(th2, bv, sum, 6 - di - djk.dg(s, u));
      } else {
        const int diag = di + djk.dg(s, u);
        const bool wall = d == 0 ? (g.bc0 && i == 0) : djk.wl(s, u);
        T xv = u ? xo.y : xo.x;  // 0 in SW_HFIRST
        T gs = (bv + tnu * sum) / (ta0 + tnu * (T)diag);
        out[u] = wall ? xv : xv + tom * (gs - xv);
      }
    }
    const long long r = i * P + rw;
    st2(own + r, out[0], out[1]);
    if (MODE == SW_FIRST || MODE == SW_HFIRST) st2(oth + r, cur.x, cur.y);
    __syncthreads();
    prev = cur;
    cur = next;
    next = more ? owin_xf(i + 2, nn) : nn;
#pragma unroll
    for (int q = 0; q < HALO_REG; ++q) hcur[q] = hnext[q];
    bb = bbn;
    xo = xon;
  }
}

}  // namespace ibs

namespace ibs {

// Operators on both colours at once: every thread owns the four cells of
// row (i, j) stored at in-row indices m0, m0+1 of both colour planes.
//   AP_LAP:    y = L x  (x of type T, y double) for the pressure Laplacian;
//   AP_HRESID: r = b - A x on velocity component `comp` (x, b double; r of
//              type TR), plus per-block partial sums of r^2 into part.
enum { AP_LAP = 0, AP_HRESID = 1 };

template <typename T, typename TR, int MODE>
__global__ void __launch_bounds__(256) k_apply2(Geo g, const T *x, const double *b, TR *out, double a0, double nuh2,
                                                double *part) {
  __shared__ T tile[2][MARCH_TILE];
  __shared__ double red[4];
  const MarchPos p = march_pos(g, true);  // chunk-per-XCD order (L z at 256^3: 46.2 -> 42.9 us)
  const int BX = blockDim.x, BY = blockDim.y, W2 = 2 * BX + 2;
  const long long N = 2 * g.half;
  const int d = p.comp;
  const T *xg = x + d * N;
  const double *bg = b ? b + d * N : nullptr;
  TR *og = out + d * N;
  const int mbase = p.mbase, jbase = p.jbase;
  const long long P = (long long)g.n1 * g.hn2;  // one plane of one colour
  const int rw = p.j * g.hn2 + p.m0;            // this thread's cells within a plane
  constexpr bool HELMM = MODE == AP_HRESID;
  auto win = [&](int q, int i) -> V2<T> {
    V2<T> v;
    v.x = T(0);
    v.y = T(0);
    int ii = mwrap(i, g.n0, g.bc0);
    if (ii < 0) return v;
    return ld2<T>(xg + (long long)q * g.half + ii * P + rw);
  };
  // software pipeline as in the sweeps: the window plane i+2, both halos and
  // the right-hand side of plane i+1 are loaded while plane i is computed
  auto plane_val = [&](int q) {
    const T *plane = xg + (long long)q * g.half;
    return [=](int ii, int jj, int mm) -> T { return plane[((long long)ii * g.n1 + jj) * g.hn2 + mm]; };
  };
  const HaloSlots hs = halo_slots(g, jbase, mbase, BX, BY);
  auto hfetch = [&](int q, int i, T *hv) {
    const T *plane = xg + (long long)q * g.half + i * P;
#pragma unroll
    for (int e = 0; e < HALO_REG; ++e) hv[e] = hs.off[e] >= 0 ? plane[hs.off[e]] : T(0);
  };
  auto hput = [&](int q, int i, const T *hv) {
    T *tq = tile[q];
#pragma unroll
    for (int e = 0; e < HALO_REG; ++e)
      if (hs.slot[e] >= 0) tq[hs.slot[e]] = hv[e];
    if (hs.rem) {
      auto val = plane_val(q);
      for (int h = hs.tid + HALO_REG * hs.nthr; h < hs.total; h += hs.nthr) {
        int r, cidx;
        halo_slot(h, BX, BY, r, cidx);
        const int jj = mwrap(jbase + r - 1, g.n1, g.bc1);
        const int mm = mwrap(mbase + cidx - 1, g.hn2, g.bc2);
        tq[r * W2 + cidx] = (jj >= 0 && mm >= 0) ? val(i, jj, mm) : T(0);
      }
    }
  };
  auto rhs = [&](int i, V2<double> *bb) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      bb[q].x = 0.0;
      bb[q].y = 0.0;
      if (MODE == AP_HRESID) bb[q] = ld2<double>(bg + (long long)q * g.half + i * P + rw);
    }
  };
  const DiagJK djk = diag_jk(g, p.j, p.m0, HELMM, d);
  V2<T> prv[2], cur[2], nxt[2];
  T hcur[2][HALO_REG];
  V2<double> bbc[2];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    prv[q] = win(q, p.i0 - 1);
    cur[q] = win(q, p.i0);
    nxt[q] = win(q, p.i0 + 1);
    hfetch(q, p.i0, hcur[q]);
  }
  rhs(p.i0, bbc);
  double acc = 0.0;
  for (int i = p.i0; i < p.i1; ++i) {
    const bool more = i + 1 < p.i1;
    V2<T> nn[2];
    T hnext[2][HALO_REG];
    V2<double> bbn[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      nn[q] = more ? win(q, i + 2) : nxt[q];
      if (more) {
        hfetch(q, i + 1, hnext[q]);
      } else {
#pragma unroll
        for (int e = 0; e < HALO_REG; ++e) hnext[q][e] = hcur[q][e];
      }
    }
    if (more) rhs(i + 1, bbn);
    else {
      bbn[0] = bbc[0];
      bbn[1] = bbc[1];
    }
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      T *tq = tile[q];
      tq[(p.ty + 1) * W2 + 2 * p.tx + 1] = cur[q].x;
      tq[(p.ty + 1) * W2 + 2 * p.tx + 2] = cur[q].y;
      hput(q, i, hcur[q]);
    }
    __syncthreads();
    const long long r = i * P + rw;
    const int di = diag_i(g, i, HELMM, d);
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const T *to = tile[1 - q];
      const int s = (q + i + p.j) & 1;
      const V2<double> bb = bbc[q];
      double o[2];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int col = 2 * p.tx + 1 + u;
        const T *trow = to + (p.ty + 1) * W2;
        double sum = (double)(u ? prv[1 - q].y : prv[1 - q].x) + (double)(u ? nxt[1 - q].y : nxt[1 - q].x) +
                     (double)to[p.ty * W2 + col] + (double)to[(p.ty + 2) * W2 + col] + (double)trow[col - 1 + s] +
                     (double)trow[col + s];
        double xv = (double)(u ? cur[q].y : cur[q].x);
        if (MODE == AP_LAP) {
          o[u] = ((double)(6 - di - djk.dg(s, u)) * xv - sum) / g.h2;
        } else {
          const int diag = di + djk.dg(s, u);
          const bool wall = d == 0 ? (g.bc0 && i == 0) : djk.wl(s, u);
          double rv = (u ? bb.y : bb.x) - ((a0 + nuh2 * diag) * xv - nuh2 * sum);
          o[u] = wall ? 0.0 : rv;
          acc += o[u] * o[u];
        }
      }
      st2(og + (long long)q * g.half + r, (TR)o[0], (TR)o[1]);
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      prv[q] = cur[q];
      cur[q] = nxt[q];
      nxt[q] = nn[q];
#pragma unroll
      for (int e = 0; e < HALO_REG; ++e) hcur[q][e] = hnext[q][e];
      bbc[q] = bbn[q];
    }
  }
  if (MODE == AP_HRESID) {
    const int tid = threadIdx.x + blockDim.x * threadIdx.y;
    acc = wave_sum(acc);
    if ((tid & 63) == 0) red[tid >> 6] = acc;
    __syncthreads();
    if (tid == 0) {
      double t = 0.0;
      const int nw = (blockDim.x * blockDim.y + 63) / 64;
      for (int w = 0; w < nw; ++w) t += red[w];
      part[blockIdx.x + (long long)gridDim.x * (blockIdx.y + (long long)gridDim.y * blockIdx.z)] = t;
    }
  }
}

}  // namespace ibs
