// Device-side helpers shared by the HIP kernels: grid geometry in the
// red/black split layout, boundary handling, the discrete delta kernels and
// deterministic wavefront reductions.
//
// Split layout.  A grid array of n0 x n1 x n2 entries (cells or the faces of
// one velocity component) is stored as two colour planes,
//     element (i,j,k)  ->  c*half + (i*n1 + j)*hn2 + (k >> 1),
// c = (i+j+k) & 1, hn2 = n2/2, half = n0*n1*hn2.  Red (c = 0) and black
// (c = 1) entries of a row are contiguous, so a red-black Gauss-Seidel half
// sweep streams one colour plane and reads only the other.  The six
// neighbours of (i,j,k) all have the other colour; the x- and y-neighbours sit
// at the same in-row index m = k>>1, the z-neighbours at m - 1 + s and m + s
// with s = k & 1.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ibs {

// Plane-marching kernels shorten their chunks of planes until a grid has at
// least this many workgroups (coarse multigrid levels); 0 keeps full chunks
// on every grid.  1024 gives the 128^3 level of a 256^3 grid 2-plane chunks
// (2048 gave it 1-plane chunks, 512 4-plane ones: both slower).
constexpr int MARCH_MIN_BLOCKS_DEFAULT = 1024;

struct Geo {
  int n0, n1, n2, hn2;
  long long half;   // n0*n1*hn2
  int bc0, bc1, bc2;  // 0 periodic, 1 no-slip wall, 2 free-slip wall (Neumann for cell fields)
  int march_min_blocks;  // see MARCH_MIN_BLOCKS_DEFAULT
  double h, h2;     // cell width and its square
};

__host__ __device__ inline int geo_n(const Geo &g, int a) { return a == 0 ? g.n0 : (a == 1 ? g.n1 : g.n2); }
__host__ __device__ inline int geo_bc(const Geo &g, int a) { return a == 0 ? g.bc0 : (a == 1 ? g.bc1 : g.bc2); }

// Change of the viscous 7-point diagonal (in units of 1/h^2, on top of the
// centre's 2 per axis) for each missing tangential neighbour beyond a wall:
// the ghost value is -u on a no-slip wall (+1) and +u on a free-slip wall
// (-1).  Both wall kinds hold zero normal velocity, so every other operator
// only asks whether an axis is a wall (bc != 0).
__host__ __device__ inline int wall_ghost_diag(int bc) { return bc == 1 ? 1 : -1; }

__device__ __forceinline__ long long sidx(const Geo &g, int i, int j, int k) {
  return (long long)((i + j + k) & 1) * g.half + ((long long)i * g.n1 + j) * g.hn2 + (k >> 1);
}

// Neighbour coordinate along an axis with wrap (periodic) or -1 (outside a wall box).
__device__ __forceinline__ int nbr(int i, int s, int n, int bc) {
  int r = i + s;
  if (r < 0) return bc ? -1 : r + n;
  if (r >= n) return bc ? -1 : r - n;
  return r;
}

__device__ __forceinline__ int wrapi(int i, int n) {
  i %= n;
  return i < 0 ? i + n : i;
}

// Coordinates of the thread in a "row launch": block (bx, by), grid
// (ceil(hn2/bx), ceil(n1/by), 2*n0*ncomp).  Returns false for padding threads.
struct RowPos { int i, j, k, m, c, comp; long long e; };

__device__ __forceinline__ bool row_pos(const Geo &g, RowPos &p) {
  p.m = blockIdx.x * blockDim.x + threadIdx.x;
  p.j = blockIdx.y * blockDim.y + threadIdx.y;
  int z = blockIdx.z;
  p.c = z & 1;
  int r = z >> 1;
  p.comp = r / g.n0;
  p.i = r - p.comp * g.n0;
  if (p.m >= g.hn2 || p.j >= g.n1) return false;
  p.k = 2 * p.m + ((p.c + p.i + p.j) & 1);
  p.e = (long long)p.c * g.half + ((long long)p.i * g.n1 + p.j) * g.hn2 + p.m;
  return true;
}

// 1 / (number of neighbours), rounded once: the pressure relaxations
// multiply by it instead of dividing.  Selects among constants (no division,
// no branch); a cell has 1..6 neighbours.
template <typename T>
__device__ __forceinline__ T inv_nn(int nn) {
  T r = nn >= 6 ? T(1) / T(6) : T(1) / T(5);
  r = nn == 4 ? T(0.25) : r;
  r = nn == 3 ? T(1) / T(3) : r;
  r = nn == 2 ? T(0.5) : r;
  r = nn <= 1 ? T(1) : r;
  return r;
}

// Number of neighbours of a cell that exist (walls remove one per side); the
// diagonal of L = G^T G is nnb / h^2.
__device__ __forceinline__ int cell_nnb(const Geo &g, int i, int j, int k) {
  int n = 6;
  if (g.bc0) n -= (i == 0) + (i == g.n0 - 1);
  if (g.bc1) n -= (j == 0) + (j == g.n1 - 1);
  if (g.bc2) n -= (k == 0) + (k == g.n2 - 1);
  return n;
}

// Pressure-cell arithmetic of the multigrid cycle, with its fused
// multiply-adds written out so that the plane-march kernels and the
// tile-level kernels round every cell the same way:
//   pc_first:  the Gauss-Seidel value h^2 b / nn of a first sweep from
//              x = 0 (products rounded one at a time, never fused into a
//              later sum);
//   pc_relax:  Gauss-Seidel value (h^2 b + sum of neighbours) / nn;
//   pc_resid:  residual b - (nn x - sum of neighbours) / h^2;
//   blend34:   3/4 near + 1/4 far, one axis of cell-centred trilinear
//              interpolation.
__device__ __forceinline__ float mul_rn(float a, float b) { return __fmul_rn(a, b); }
__device__ __forceinline__ double mul_rn(double a, double b) { return __dmul_rn(a, b); }
template <typename T>
__device__ __forceinline__ T pc_first(T h2, T b, int nn) {
  return mul_rn(mul_rn(h2, b), inv_nn<T>(nn));
}
template <typename T>
__device__ __forceinline__ T pc_relax(T h2, T b, T sum, int nn) {
  return fma(h2, b, sum) * inv_nn<T>(nn);
}
template <typename T>
__device__ __forceinline__ T pc_resid(T b, T x, T sum, int nn, T ih2) {
  return fma(-fma((T)nn, x, -sum), ih2, b);
}
template <typename T>
__device__ __forceinline__ T blend34(T near, T far) {
  return fma((T)0.75, near, (T)0.25 * far);
}

// ---------------------------------------------------------------------------
// Discrete delta kernels (argument in cell widths).  ROMA3 is the 3-point
// kernel of the paper (Sec. 2.3, eq. delta); PESKIN4 the standard 4-point one.
enum { KER_PESKIN4 = 0, KER_ROMA3 = 1 };

__device__ __forceinline__ double phi_peskin4(double r) {
  double a = fabs(r);
  if (a <= 1.0) return (3.0 - 2.0 * a + sqrt(1.0 + 4.0 * a - 4.0 * a * a)) * 0.125;
  if (a < 2.0) return (5.0 - 2.0 * a - sqrt(fmax(0.0, -7.0 + 12.0 * a - 4.0 * a * a))) * 0.125;
  return 0.0;
}
__device__ __forceinline__ double dphi_peskin4(double r) {
  double a = fabs(r), s = r < 0.0 ? -1.0 : 1.0;
  if (a <= 1.0) return s * (-2.0 + (2.0 - 4.0 * a) / sqrt(1.0 + 4.0 * a - 4.0 * a * a)) * 0.125;
  if (a < 2.0) return s * (-2.0 - (6.0 - 4.0 * a) / sqrt(fmax(1e-300, -7.0 + 12.0 * a - 4.0 * a * a))) * 0.125;
  return 0.0;
}
__device__ __forceinline__ double phi_roma3(double r) {
  double a = fabs(r);
  if (a <= 0.5) return (1.0 + sqrt(1.0 - 3.0 * a * a)) * (1.0 / 3.0);
  if (a <= 1.5) {
    double t = 1.0 - a;
    return (5.0 - 3.0 * a - sqrt(fmax(0.0, 1.0 - 3.0 * t * t))) * (1.0 / 6.0);
  }
  return 0.0;
}
__device__ __forceinline__ double dphi_roma3(double r) {
  double a = fabs(r), s = r < 0.0 ? -1.0 : 1.0;
  if (a <= 0.5) return -s * a / sqrt(fmax(1e-300, 1.0 - 3.0 * a * a));
  if (a < 1.5) {
    double t = 1.0 - a;
    return s * (-3.0 - 3.0 * t / sqrt(fmax(1e-300, 1.0 - 3.0 * t * t))) * (1.0 / 6.0);
  }
  return 0.0;
}

template <int KER> __device__ __forceinline__ double phi(double r) {
  return KER == KER_PESKIN4 ? phi_peskin4(r) : phi_roma3(r);
}
template <int KER> __device__ __forceinline__ double dphi(double r) {
  return KER == KER_PESKIN4 ? dphi_peskin4(r) : dphi_roma3(r);
}
template <int KER> struct KerWidth { static constexpr int W = (KER == KER_PESKIN4) ? 4 : 3; };

// First node index and offset of a point's support along one axis.  Nodes of
// a velocity component along its own axis are faces (offset 0), otherwise
// cell centres (offset 1/2).  r_t = s - (i0 + t) is the distance to node t in
// cell widths.
template <int KER> __device__ __forceinline__ int support_start(double x, double inv_h, bool face, double &s) {
  s = x * inv_h - (face ? 0.0 : 0.5);
  return KER == KER_PESKIN4 ? (int)floor(s) - 1 : (int)floor(s + 0.5) - 1;
}

// All weights of a point along one axis from one square root.  With
// s = x/h - offset (offset 0 for face nodes, 1/2 for centre nodes):
//   4-point: nodes floor(s)-1 .. floor(s)+2, f = s - floor(s),
//            q = sqrt(1 + 4f - 4f^2) (the same radicand for all four nodes),
//            w = ((3-2f-q)/8, (3-2f+q)/8, (1+2f+q)/8, (1+2f-q)/8);
//   3-point: nodes round(s)-1 .. round(s)+1, f = s - round(s),
//            q = sqrt(1 - 3f^2), w = ((2-3f-q)/6, (1+q)/3, (2+3f-q)/6, 0).
// The node index and f come from s in float64 (positions reach n h); the
// weights are formed in TA: float64, or float32 where they are rounded to
// float32 anyway (the products of the float32 Krylov cycle), which spares
// the float64 square root and its refinement.
template <int KER, typename TA = double>
__device__ __forceinline__ int axis_weights(double x, double inv_h, bool face, TA w[4]) {
  double s = x * inv_h - (face ? 0.0 : 0.5);
  if (KER == KER_PESKIN4) {
    double fl = floor(s);
    TA f = (TA)(s - fl);
    TA q = sqrt(fmax(TA(0), TA(1) + TA(4) * f - TA(4) * f * f));
    w[0] = (TA(3) - TA(2) * f - q) * TA(0.125);
    w[1] = (TA(3) - TA(2) * f + q) * TA(0.125);
    w[2] = (TA(1) + TA(2) * f + q) * TA(0.125);
    w[3] = (TA(1) + TA(2) * f - q) * TA(0.125);
    return (int)fl - 1;
  } else {
    double rd = floor(s + 0.5);
    TA f = (TA)(s - rd);
    TA q = sqrt(fmax(TA(0), TA(1) - TA(3) * f * f));
    w[0] = (TA(2) - TA(3) * f - q) * TA(1.0 / 6.0);
    w[1] = (TA(1) + q) * TA(1.0 / 3.0);
    w[2] = (TA(2) + TA(3) * f - q) * TA(1.0 / 6.0);
    w[3] = TA(0);
    return (int)rd - 1;
  }
}

// ---------------------------------------------------------------------------
// Deterministic reductions: fixed butterfly order within a wavefront.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
// Sum over groups of 16 lanes (lanes 16q .. 16q+15), fixed order.
template <typename TA>
__device__ __forceinline__ TA sum16(TA v) {
#pragma unroll
  for (int o = 8; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

}  // namespace ibs
