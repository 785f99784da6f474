// Staggered-grid stencil kernels in the red/black split layout: layout
// conversion, the pressure Laplacian L = G^T G, gradient G and divergence
// D = -G^T (paper Sec. 3.1, eq. modified_poisson), the momentum operator
// A = 3/(2 dt) - nu Delta_h and its red-black relaxation (eq. ustar), the
// explicit convection term and the momentum right-hand side.
//
// Boundary rules (MAC grid): on a wall axis d the index-0 face of velocity
// component d is the wall (always 0) and the far wall is implicit; the
// pressure Laplacian is Neumann there; a tangential velocity's neighbour
// beyond a wall is the ghost value -u on a no-slip wall and +u on a
// free-slip wall.
#include <hip/hip_ext.h>

#include "internal.h"
#include "march.h"

namespace ibs {

Geo make_geo(int n0, int n1, int n2, int bc0, int bc1, int bc2, double h) {
  Geo g;
  g.n0 = n0; g.n1 = n1; g.n2 = n2; g.hn2 = n2 / 2;
  g.half = (long long)n0 * n1 * (n2 / 2);
  g.bc0 = bc0; g.bc1 = bc1; g.bc2 = bc2;
  g.march_min_blocks = MARCH_MIN_BLOCKS_DEFAULT;
  g.h = h; g.h2 = h * h;
  return g;
}

RowLaunch row_launch(const Geo &g, int nz) {
  int bx = 1;
  while (bx < g.hn2 && bx < 64) bx <<= 1;
  int by = 256 / bx;
  RowLaunch L;
  L.block = dim3(bx, by, 1);
  L.grid = dim3((g.hn2 + bx - 1) / bx, (g.n1 + by - 1) / by, nz);
  return L;
}

// Value of a split-layout plane at (i,j,k); 0 outside a wall box, wrapped on
// periodic axes.
template <typename T>
__device__ __forceinline__ T fetch(const T *f, const Geo &g, int i, int j, int k) {
  if (i < 0 || i >= g.n0) { if (g.bc0) return T(0); i = wrapi(i, g.n0); }
  if (j < 0 || j >= g.n1) { if (g.bc1) return T(0); j = wrapi(j, g.n1); }
  if (k < 0 || k >= g.n2) { if (g.bc2) return T(0); k = wrapi(k, g.n2); }
  return f[sidx(g, i, j, k)];
}

// Sum of the six neighbours of cell (i,j,k) (colour c, in-row index m) that
// exist; all of them lie in the other colour plane.
template <typename T>
__device__ __forceinline__ T cell_nb_sum(const Geo &g, const T *x, int i, int j, int k, int c, int m) {
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

// ---------------------------------------------------------------------------
__global__ void k_to_split(Geo g, const double *nat, double *spl) {
  RowPos p;
  if (!row_pos(g, p)) return;
  long long N = 2 * g.half;
  long long ni = ((long long)p.i * g.n1 + p.j) * g.n2 + p.k;
  spl[p.comp * N + p.e] = nat[p.comp * N + ni];
}
// nat = spl - mult * sum[0] (sum null: a plain copy)
__global__ void k_to_natural(Geo g, const double *spl, double *nat, const double *sum, double mult) {
  RowPos p;
  if (!row_pos(g, p)) return;
  long long N = 2 * g.half;
  long long ni = ((long long)p.i * g.n1 + p.j) * g.n2 + p.k;
  const double v = spl[p.comp * N + p.e];
  // separately rounded product and difference (no fused multiply-add), as
  // in the paired form below, so both give the same bits
  nat[p.comp * N + ni] = sum ? __dsub_rn(v, __dmul_rn(mult, sum[0])) : v;
}

// The same conversions a cell pair per thread: cells k = 2m and 2m + 1 of
// row (i, j) are adjacent in natural order (one 16-byte access) and sit at
// in-row index m of the two colours (grid.z = plane x component).
__device__ __forceinline__ bool pair_pos(const Geo &g, long long &ni, long long &e0, long long &e1, int &comp) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y * blockDim.y + threadIdx.y;
  comp = blockIdx.z / g.n0;
  const int i = blockIdx.z - comp * g.n0;
  if (m >= g.hn2 || j >= g.n1) return false;
  const long long row = (long long)i * g.n1 + j;
  const int c0 = (i + j) & 1;  // colour of cell k = 2m
  ni = row * g.n2 + 2 * m;
  e0 = (long long)c0 * g.half + row * g.hn2 + m;
  e1 = (long long)(1 - c0) * g.half + row * g.hn2 + m;
  return true;
}
__global__ void k_to_split2(Geo g, const double *nat, double *spl) {
  long long ni, e0, e1;
  int comp;
  if (!pair_pos(g, ni, e0, e1, comp)) return;
  const long long N = 2 * g.half;
  const double2 v = *(const double2 *)(nat + comp * N + ni);
  spl[comp * N + e0] = v.x;
  spl[comp * N + e1] = v.y;
}
__global__ void k_to_natural2(Geo g, const double *spl, double *nat, const double *sum, double mult) {
  long long ni, e0, e1;
  int comp;
  if (!pair_pos(g, ni, e0, e1, comp)) return;
  const long long N = 2 * g.half;
  const double sh = sum ? __dmul_rn(mult, sum[0]) : 0.0;
  const double a = spl[comp * N + e0], b = spl[comp * N + e1];
  *(double2 *)(nat + comp * N + ni) = sum ? make_double2(__dsub_rn(a, sh), __dsub_rn(b, sh)) : make_double2(a, b);
}

hipError_t to_split(const Geo &g, int ncomp, const double *nat, double *spl, hipStream_t s) {
  if ((uintptr_t)nat % 16 == 0) {
    RowLaunch L = row_launch(g, g.n0 * ncomp);
    hipLaunchKernelGGL(k_to_split2, L.grid, L.block, 0, s, g, nat, spl);
  } else {
    RowLaunch L = row_launch(g, 2 * g.n0 * ncomp);
    hipLaunchKernelGGL(k_to_split, L.grid, L.block, 0, s, g, nat, spl);
  }
  return hipGetLastError();
}
hipError_t to_natural(const Geo &g, int ncomp, const double *spl, double *nat, hipStream_t s, const double *sum,
                      double mult) {
  if ((uintptr_t)nat % 16 == 0) {
    RowLaunch L = row_launch(g, g.n0 * ncomp);
    hipLaunchKernelGGL(k_to_natural2, L.grid, L.block, 0, s, g, spl, nat, sum, mult);
  } else {
    RowLaunch L = row_launch(g, 2 * g.n0 * ncomp);
    hipLaunchKernelGGL(k_to_natural, L.grid, L.block, 0, s, g, spl, nat, sum, mult);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// y = L x, L = G^T G: (L x)_c = sum over existing neighbours (x_c - x_nb) / h^2
// (formed in float64, stored as TY)
template <typename T, typename TY>
hipError_t lap_apply(const Geo &g, const T *x, TY *y, hipStream_t s) {
  MarchShape M = march_shape(g, 1);
  hipEvent_t e0, e1;
  probe_ext_take(&e0, &e1);  // the events of an enclosing ProbeExt, if any
  hipExtLaunchKernelGGL((k_apply2<T, TY, AP_LAP>), M.grid, M.block, 0, s, e0, e1, 0, g, x, nullptr, y, 0.0, 0.0,
                        (double *)nullptr);
  return hipGetLastError();
}
template hipError_t lap_apply<float, double>(const Geo &, const float *, double *, hipStream_t);
template hipError_t lap_apply<double, double>(const Geo &, const double *, double *, hipStream_t);
template hipError_t lap_apply<float, float>(const Geo &, const float *, float *, hipStream_t);

// f3 = add3 + alpha G p ; (G p)_d(idx) = (p(idx) - p(idx - e_d)) / h, zero on wall faces.
// One thread per cell writes the cell's lower face along every axis, so p is
// read once for the three components.
__global__ void k_grad(Geo g, const double *p_, double *f3, double alpha, const double *add3) {
  RowPos p;
  if (!row_pos(g, p)) return;
  long long N = 2 * g.half;
  const double pc = p_[p.e];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    int bcd = geo_bc(g, d);
    int xd = d == 0 ? p.i : (d == 1 ? p.j : p.k);
    double v = 0.0;
    if (!(bcd && xd == 0)) {
      int i = p.i - (d == 0), j = p.j - (d == 1), k = p.k - (d == 2);
      double lo = fetch(p_, g, i, j, k);
      v = alpha * (pc - lo) / g.h;
      if (add3) v += add3[d * N + p.e];
    }
    f3[d * N + p.e] = v;
  }
}
hipError_t grad_apply(const Geo &g, const double *p, double *f3, double alpha, const double *add3,
                      hipStream_t s) {
  RowLaunch L = row_launch(g, 2 * g.n0);
  hipLaunchKernelGGL(k_grad, L.grid, L.block, 0, s, g, p, f3, alpha, add3);
  return hipGetLastError();
}

// y = alpha D u ; (D u)_c = sum_d (u_d(c + e_d) - u_d(c)) / h with wall faces = 0
__global__ void k_div(Geo g, const double *u3, double *y, double alpha) {
  RowPos p;
  if (!row_pos(g, p)) return;
  long long N = 2 * g.half;
  double acc = 0.0;
  for (int d = 0; d < 3; ++d) {
    const double *ud = u3 + d * N;
    int bcd = geo_bc(g, d);
    int xd = d == 0 ? p.i : (d == 1 ? p.j : p.k);
    double lo = (bcd && xd == 0) ? 0.0 : ud[p.e];
    double hi = fetch(ud, g, p.i + (d == 0), p.j + (d == 1), p.k + (d == 2));
    acc += hi - lo;
  }
  y[p.e] = alpha * acc / g.h;
}
hipError_t div_apply(const Geo &g, const double *u3, double *y, double alpha, hipStream_t s) {
  RowLaunch L = row_launch(g, 2 * g.n0);
  hipLaunchKernelGGL(k_div, L.grid, L.block, 0, s, g, u3, y, alpha);
  return hipGetLastError();
}

__global__ void k_fill(double *x, long long n, double v) {
  long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  long long st = (long long)gridDim.x * blockDim.x;
  for (; t < n; t += st) x[t] = v;
}
__global__ void k_fill_i32(int *x, long long n, int v) {
  long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  long long st = (long long)gridDim.x * blockDim.x;
  for (; t < n; t += st) x[t] = v;
}
static int stream_blocks(long long n) {
  long long b = (n + 255) / 256;
  return (int)(b < 8192 ? (b < 1 ? 1 : b) : 8192);
}
hipError_t fill(double *x, long long n, double v, hipStream_t s) {
  hipLaunchKernelGGL(k_fill, dim3(stream_blocks(n)), dim3(256), 0, s, x, n, v);
  return hipGetLastError();
}
hipError_t fill_i32(int *x, long long n, int v, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_i32, dim3(stream_blocks(n)), dim3(256), 0, s, x, n, v);
  return hipGetLastError();
}

__global__ void k_zero_wall(Geo g, double *u3) {
  RowPos p;
  if (!row_pos(g, p)) return;
  int d = p.comp;
  int xd = d == 0 ? p.i : (d == 1 ? p.j : p.k);
  if (geo_bc(g, d) && xd == 0) u3[d * 2 * g.half + p.e] = 0.0;
}
hipError_t zero_wall_faces(const Geo &g, double *u3, hipStream_t s) {
  RowLaunch L = row_launch(g, 2 * g.n0 * 3);
  hipLaunchKernelGGL(k_zero_wall, L.grid, L.block, 0, s, g, u3);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Momentum operator on the component-d face grid.  Per axis a the second
// difference has diagonal weight 2 (periodic, or normal-to-wall where the
// wall faces 0 and n hold 0); for a tangential wall each missing neighbour
// adds 1 (no-slip, ghost value -u) or removes 1 (free-slip, ghost value +u).
// nb = sum of the existing neighbours.
template <typename T>
__device__ __forceinline__ void helm_stencil(const Geo &g, const T *ud, int d, int i, int j, int k,
                                             T &nb, int &diag) {
  nb = T(0);
  diag = 0;
  const int xs[3] = {i, j, k};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    int n = geo_n(g, a), bc = geo_bc(g, a);
#pragma unroll
    for (int s = -1; s <= 1; s += 2) {
      int y = xs[a] + s;
      bool valid;
      if (!bc) {
        y = y < 0 ? y + n : (y >= n ? y - n : y);
        valid = true;
        diag += 1;
      } else if (a == d) {
        valid = (y >= 1) && (y <= n - 1);
        diag += 1;
      } else {
        valid = (y >= 0) && (y <= n - 1);
        diag += valid ? 1 : 1 + wall_ghost_diag(bc);
      }
      if (valid) {
        int ii = a == 0 ? y : i, jj = a == 1 ? y : j, kk = a == 2 ? y : k;
        nb += ud[sidx(g, ii, jj, kk)];
      }
    }
  }
}

__global__ void k_helm_apply(Geo g, double a0, double nu, const double *u3, double *y3) {
  RowPos p;
  if (!row_pos(g, p)) return;
  long long N = 2 * g.half;
  int d = p.comp;
  int xd = d == 0 ? p.i : (d == 1 ? p.j : p.k);
  double out = 0.0;
  if (!(geo_bc(g, d) && xd == 0)) {
    const double *ud = u3 + d * N;
    double nb;
    int diag;
    helm_stencil(g, ud, d, p.i, p.j, p.k, nb, diag);
    out = (a0 + nu * diag / g.h2) * ud[p.e] - nu / g.h2 * nb;
  }
  y3[d * N + p.e] = out;
}
hipError_t helm_apply(const Geo &g, double a0, double nu, const double *u3, double *y3, hipStream_t s) {
  RowLaunch L = row_launch(g, 2 * g.n0 * 3);
  hipLaunchKernelGGL(k_helm_apply, L.grid, L.block, 0, s, g, a0, nu, u3, y3);
  return hipGetLastError();
}

template <typename TR>
hipError_t helm_resid(const Geo &g, double a0, double nu, const double *x3, const double *b3, TR *r3,
                      double *part, int *nblocks, hipStream_t s) {
  MarchShape M = march_shape(g, 3);
  hipLaunchKernelGGL((k_apply2<double, TR, AP_HRESID>), M.grid, M.block, 0, s, g, x3, b3, r3, a0, nu / g.h2, part);
  *nblocks = (int)(M.grid.x * M.grid.y * M.grid.z);
  return hipGetLastError();
}
template hipError_t helm_resid<float>(const Geo &, double, double, const double *, const double *, float *,
                                      double *, int *, hipStream_t);
template hipError_t helm_resid<double>(const Geo &, double, double, const double *, const double *, double *,
                                       double *, int *, hipStream_t);
int helm_resid_blocks(const Geo &g) {
  MarchShape M = march_shape(g, 3);
  return (int)(M.grid.x * M.grid.y * M.grid.z);
}

// Red-black SOR half sweep for A e = r on all three face grids.
template <typename T, typename TB>
hipError_t helm_sor(const Geo &g, double a0, double nu, double omega, T *x3, const TB *b3, int color,
                    hipStream_t s) {
  MarchShape M = march_shape(g, 3);
  hipLaunchKernelGGL((k_sweep<T, TB, SW_HELM>), M.grid, M.block, 0, s, g, x3, b3, color, g.h2, a0, nu / g.h2,
                     omega);
  return hipGetLastError();
}
template hipError_t helm_sor<float, float>(const Geo &, double, double, double, float *, const float *, int,
                                           hipStream_t);
template hipError_t helm_sor<double, double>(const Geo &, double, double, double, double *, const double *, int,
                                             hipStream_t);

// The first SOR sweep of a correction solve A e = r from e = 0 (both colours
// written, so e need not be cleared beforehand).
template <typename T>
hipError_t helm_sor_first(const Geo &g, double a0, double nu, double omega, T *x3, const T *b3, hipStream_t s) {
  MarchShape M = march_shape(g, 3);
  hipLaunchKernelGGL((k_sweep<T, T, SW_HFIRST>), M.grid, M.block, 0, s, g, x3, b3, 1, g.h2, a0, nu / g.h2, omega);
  return hipGetLastError();
}
template hipError_t helm_sor_first<float>(const Geo &, double, double, double, float *, const float *, hipStream_t);
template hipError_t helm_sor_first<double>(const Geo &, double, double, double, double *, const double *,
                                           hipStream_t);

template <typename T>
__global__ void k_fill_t(T *x, long long n) {
  long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  long long st = (long long)gridDim.x * blockDim.x;
  for (; t < n; t += st) x[t] = T(0);
}
template <typename T>
hipError_t zero_t(T *x, long long n, hipStream_t s) {
  long long b = (n + 255) / 256;
  int nb = (int)(b < 8192 ? (b < 1 ? 1 : b) : 8192);
  hipLaunchKernelGGL(k_fill_t<T>, dim3(nb), dim3(256), 0, s, x, n);
  return hipGetLastError();
}
template hipError_t zero_t<float>(float *, long long, hipStream_t);
template hipError_t zero_t<double>(double *, long long, hipStream_t);

template <typename T>
__global__ void k_add_cast(double *y, const T *x, long long n) {
  long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  long long st = (long long)gridDim.x * blockDim.x;
  for (; t < n; t += st) y[t] += (double)x[t];
}
template <typename T>
hipError_t add_cast(double *y, const T *x, long long n, hipStream_t s) {
  hipLaunchKernelGGL(k_add_cast<T>, dim3(stream_blocks(n)), dim3(256), 0, s, y, x, n);
  return hipGetLastError();
}
template hipError_t add_cast<float>(double *, const float *, long long, hipStream_t);
template hipError_t add_cast<double>(double *, const double *, long long, hipStream_t);

template <typename T>
__global__ void k_cast_copy(T *y, const double *x, long long n) {
  long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  long long st = (long long)gridDim.x * blockDim.x;
  for (; t < n; t += st) y[t] = (T)x[t];
}
template <typename T>
hipError_t cast_copy(T *y, const double *x, long long n, hipStream_t s) {
  hipLaunchKernelGGL(k_cast_copy<T>, dim3(stream_blocks(n)), dim3(256), 0, s, y, x, n);
  return hipGetLastError();
}
template hipError_t cast_copy<float>(float *, const double *, long long, hipStream_t);
template hipError_t cast_copy<double>(double *, const double *, long long, hipStream_t);

// ---------------------------------------------------------------------------
// Convection div(u u) at a component-d face, divergence form with arithmetic
// averages; fluxes through walls (either kind) vanish.
__device__ double conv_at(const Geo &g, const double *u3, int d, int i, int j, int k) {
  long long N = 2 * g.half;
  const double *ud = u3 + d * N;
  double acc = 0.0;
  const int x0[3] = {i, j, k};
  for (int a = 0; a < 3; ++a) {
    int ea[3] = {a == 0, a == 1, a == 2};
    if (a == d) {
      double u0 = fetch(ud, g, i, j, k);
      double up = fetch(ud, g, i + ea[0], j + ea[1], k + ea[2]);
      double um = fetch(ud, g, i - ea[0], j - ea[1], k - ea[2]);
      double cp = 0.5 * (u0 + up), cm = 0.5 * (um + u0);
      acc += (cp * cp - cm * cm) / g.h;
    } else {
      const double *ua = u3 + a * N;
      int ed[3] = {d == 0, d == 1, d == 2};
      int na = geo_n(g, a), bca = geo_bc(g, a);
      double fp = 0.0, fm = 0.0;
      if (!(bca && x0[a] == na - 1)) {
        double udm = 0.5 * (fetch(ud, g, i, j, k) + fetch(ud, g, i + ea[0], j + ea[1], k + ea[2]));
        double uam = 0.5 * (fetch(ua, g, i + ea[0], j + ea[1], k + ea[2]) +
                            fetch(ua, g, i + ea[0] - ed[0], j + ea[1] - ed[1], k + ea[2] - ed[2]));
        fp = udm * uam;
      }
      if (!(bca && x0[a] == 0)) {
        double udm = 0.5 * (fetch(ud, g, i - ea[0], j - ea[1], k - ea[2]) + fetch(ud, g, i, j, k));
        double uam = 0.5 * (fetch(ua, g, i, j, k) + fetch(ua, g, i - ed[0], j - ed[1], k - ed[2]));
        fm = udm * uam;
      }
      acc += (fp - fm) / g.h;
    }
  }
  return acc;
}

__global__ void k_convection(Geo g, const double *u3, double *out3) {
  RowPos p;
  if (!row_pos(g, p)) return;
  long long N = 2 * g.half;
  int d = p.comp;
  int xd = d == 0 ? p.i : (d == 1 ? p.j : p.k);
  double v = 0.0;
  if (!(geo_bc(g, d) && xd == 0)) v = conv_at(g, u3, d, p.i, p.j, p.k);
  out3[d * N + p.e] = v;
}
hipError_t convection(const Geo &g, const double *u3, double *out3, hipStream_t s) {
  RowLaunch L = row_launch(g, 2 * g.n0 * 3);
  hipLaunchKernelGGL(k_convection, L.grid, L.block, 0, s, g, u3, out3);
  return hipGetLastError();
}

// rhs = (4 u^n - u^{n-1}) / (2 dt) - G p^n - N(u^n)     (eq. ustar; W Phi^n is
// added afterwards by the band kernel), and optionally the extrapolated
// initial guess 2 u^n - u^{n-1} of the momentum solve (0 on wall faces).
//
// Plane march along axis 0: a workgroup owns MQ_BY rows (axis 1) x MQ_BK
// cells (axis 2, natural order) and a chunk of MQ_CH planes.  LDS holds a
// ring of three planes (i-1, i, i+1) of the three velocity components with a
// one-cell halo in axes 1 and 2 (every value the divergence-form convection
// of a face needs), and the current plane of p with its lower halo; plane
// i+2 is fetched into registers while plane i is computed.  Each thread
// computes two neighbouring cells of a row, whose split-layout addresses lie
// in the two colour planes at the same in-row index, so the stores of a wave
// are two contiguous runs.  Tiles are handed out XCD-major (consecutive tiles
// go to the same XCD), so halos shared by neighbouring tiles come from its L2.
constexpr int MQ_BY = 8, MQ_BK = 64, MQ_CH = 16, MQ_T = 256;
constexpr int MQ_RY = MQ_BY + 2, MQ_RK = MQ_BK + 2, MQ_PL = MQ_RY * MQ_RK;  // 660 cells per plane
constexpr int MQ_PY = MQ_BY + 1, MQ_PK = MQ_BK + 1, MQ_PP = MQ_PY * MQ_PK;  // p: lower halo only
constexpr int MQ_NU = (MQ_PL + MQ_T - 1) / MQ_T;                            // plane loads per thread
constexpr int MQ_NP = (MQ_PP + MQ_T - 1) / MQ_T;

// Split-layout index of a (possibly outside) cell, or -1 outside a wall box.
__device__ __forceinline__ long long mq_index(const Geo &g, int i, int j, int k) {
  if (i < 0 || i >= g.n0) { if (g.bc0) return -1; i = wrapi(i, g.n0); }
  if (j < 0 || j >= g.n1) { if (g.bc1) return -1; j = wrapi(j, g.n1); }
  if (k < 0 || k >= g.n2) { if (g.bc2) return -1; k = wrapi(k, g.n2); }
  return sidx(g, i, j, k);
}

__global__ void __launch_bounds__(MQ_T) k_mom_rhs(Geo g, double dt, const double *u3, const double *um3,
                                                  const double *p_, double *out3, double *guess3, int ntk, int ntj,
                                                  int ntiles) {
  __shared__ double su[3][3][MQ_PL];  // [ring slot][component][cell]
  __shared__ double sp[MQ_PP];
  const long long N = 2 * g.half;
  const int b = blockIdx.x;
  const int per = ntiles / 8;
  const int tile = (ntiles % 8 == 0) ? (b % 8) * per + b / 8 : b;
  const int tk = tile % ntk, r0 = tile / ntk, tj = r0 % ntj, tc = r0 / ntj;
  const int j0 = tj * MQ_BY, k0 = tk * MQ_BK, i0 = tc * MQ_CH;
  const int i1 = min(i0 + MQ_CH, g.n0);
  const int tid = threadIdx.x;
  const int cj = tid / (MQ_BK / 2), ck = 2 * (tid % (MQ_BK / 2));
  const int j = j0 + cj, k = k0 + ck;
  const bool act = j < g.n1 && k < g.n2;  // n2 is even, so k + 1 < n2 too
  const double ih = 1.0 / g.h, i2dt = 1.0 / (2.0 * dt);
  // plane loads: register staging of plane `pl` of the velocity components
  double ru[MQ_NU][3];
  auto fetch_u = [&](int pl) {
#pragma unroll
    for (int t = 0; t < MQ_NU; ++t) {
      const int q = tid + t * MQ_T;
      const int yy = q / MQ_RK, kk = q - yy * MQ_RK;
      const long long e = q < MQ_PL ? mq_index(g, pl, j0 - 1 + yy, k0 - 1 + kk) : -1;
#pragma unroll
      for (int c = 0; c < 3; ++c) ru[t][c] = e >= 0 ? u3[c * N + e] : 0.0;
    }
  };
  auto store_u = [&](int slot) {
#pragma unroll
    for (int t = 0; t < MQ_NU; ++t) {
      const int q = tid + t * MQ_T;
      if (q < MQ_PL)
#pragma unroll
        for (int c = 0; c < 3; ++c) su[slot][c][q] = ru[t][c];
    }
  };
  double rp[MQ_NP];
  auto fetch_p = [&](int pl) {
#pragma unroll
    for (int t = 0; t < MQ_NP; ++t) {
      const int q = tid + t * MQ_T;
      const int yy = q / MQ_PK, kk = q - yy * MQ_PK;
      const long long e = q < MQ_PP ? mq_index(g, pl, j0 - 1 + yy, k0 - 1 + kk) : -1;
      rp[t] = e >= 0 ? p_[e] : 0.0;
    }
  };
  auto store_p = [&]() {
#pragma unroll
    for (int t = 0; t < MQ_NP; ++t) {
      const int q = tid + t * MQ_T;
      if (q < MQ_PP) sp[q] = rp[t];
    }
  };
  // the ring starts with planes i0 - 1 and i0; p of plane i0 - 1 at the own cells
  double pprev[2] = {0.0, 0.0};
  if (act) {
    const long long e0 = mq_index(g, i0 - 1, j, k), e1 = mq_index(g, i0 - 1, j, k + 1);
    pprev[0] = e0 >= 0 ? p_[e0] : 0.0;
    pprev[1] = e1 >= 0 ? p_[e1] : 0.0;
  }
  fetch_u(i0 - 1);
  store_u((i0 + 2) % 3);
  fetch_u(i0);
  store_u(i0 % 3);
  fetch_u(i0 + 1);
  fetch_p(i0);
  for (int i = i0; i < i1; ++i) {
    const int sm = (i + 2) % 3, s0 = i % 3, s1 = (i + 1) % 3;
    __syncthreads();  // the previous plane's readers are done with slot s1 and sp
    store_u(s1);
    store_p();
    __syncthreads();
    if (i + 1 < i1) {
      fetch_u(i + 2);  // in flight while this plane is computed
      fetch_p(i + 1);
    }
    if (act) {
      const int x0[2][3] = {{i, j, k}, {i, j, k + 1}};
#pragma unroll
      for (int h2 = 0; h2 < 2; ++h2) {
        const int cy = cj + 1, cz = ck + 1 + h2;
        // component c at offset (dx, dy, dz) from this cell
        auto U = [&](int c, int dx, int dy, int dz) -> double {
          const int sl = dx < 0 ? sm : (dx > 0 ? s1 : s0);
          return su[sl][c][(cy + dy) * MQ_RK + cz + dz];
        };
        const double pv = sp[(cj + 1) * MQ_PK + ck + 1 + h2];
        const double plo[3] = {pprev[h2], sp[cj * MQ_PK + ck + 1 + h2], sp[(cj + 1) * MQ_PK + ck + h2]};
        const long long e = sidx(g, x0[h2][0], x0[h2][1], x0[h2][2]);
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          double v = 0.0, gv = 0.0;
          if (!(geo_bc(g, d) && x0[h2][d] == 0)) {
            const int ed0 = d == 0, ed1 = d == 1, ed2 = d == 2;
            double acc = 0.0;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
              const int ea0 = a == 0, ea1 = a == 1, ea2 = a == 2;
              if (a == d) {
                const double u0 = U(d, 0, 0, 0);
                const double cp = 0.5 * (u0 + U(d, ea0, ea1, ea2)), cm = 0.5 * (U(d, -ea0, -ea1, -ea2) + u0);
                acc += (cp * cp - cm * cm) * ih;
              } else {
                const int na = geo_n(g, a), bca = geo_bc(g, a);
                double fp = 0.0, fm = 0.0;
                if (!(bca && x0[h2][a] == na - 1))
                  fp = 0.5 * (U(d, 0, 0, 0) + U(d, ea0, ea1, ea2)) * 0.5 *
                       (U(a, ea0, ea1, ea2) + U(a, ea0 - ed0, ea1 - ed1, ea2 - ed2));
                if (!(bca && x0[h2][a] == 0))
                  fm = 0.5 * (U(d, -ea0, -ea1, -ea2) + U(d, 0, 0, 0)) * 0.5 * (U(a, 0, 0, 0) + U(a, -ed0, -ed1, -ed2));
                acc += (fp - fm) * ih;
              }
            }
            const double gp = (pv - plo[d]) * ih;
            const double umv = um3[d * N + e];
            const double u0 = U(d, 0, 0, 0);
            v = (4.0 * u0 - umv) * i2dt - gp - acc;
            gv = 2.0 * u0 - umv;
          }
          out3[d * N + e] = v;
          if (guess3) guess3[d * N + e] = gv;
        }
        pprev[h2] = pv;
      }
    }
  }
}
hipError_t mom_rhs(const Geo &g, double dt, const double *u3, const double *um3, const double *p,
                   double *out3, double *guess3, hipStream_t s) {
  const int ntj = (g.n1 + MQ_BY - 1) / MQ_BY, ntk = (g.n2 + MQ_BK - 1) / MQ_BK;
  const int nch = (g.n0 + MQ_CH - 1) / MQ_CH;
  const int ntiles = ntj * ntk * nch;
  hipLaunchKernelGGL(k_mom_rhs, dim3(ntiles), dim3(MQ_T), 0, s, g, dt, u3, um3, p, out3, guess3, ntk, ntj, ntiles);
  return hipGetLastError();
}

}  // namespace ibs
