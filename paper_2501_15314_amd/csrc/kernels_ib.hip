// Lagrangian-point kernels: placement of the body points, binning into 4^3-
// cell tiles, interpolation W^T (paper Sec. 2.3, eq. interpolation) and
// spreading W (eq. regularization), optionally followed by the divergence
// (B^T = D W, eq. modified_poisson).
//
// Determinism.  No floating-point atomics are used.  Points are sorted into
// tiles in canonical order (tile, original index).  Interpolation reduces
// each point's stencil in a fixed butterfly order.  Spreading is done per
// active tile by one workgroup: a wavefront per velocity component walks the
// candidate points of the 27 neighbouring tiles in a fixed order, and for
// each point its 64 stencil nodes are 64 distinct lanes adding into distinct
// LDS cells, so every grid value is summed in the same order on every run.
#include <hip/hip_ext.h>

#include "internal.h"

namespace ibs {

static int nblk(long long n, int bs) { return (int)((n + bs - 1) / bs); }

__global__ void k_points(Geo g, int K, const BodyDev *bodies, const int *body_of, const double *off,
                         double *X, double *U, int *tile, int nt0, int nt1, int nt2) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;
  const BodyDev &b = bodies[body_of[k]];
  double o0 = off[3 * k], o1 = off[3 * k + 1], o2 = off[3 * k + 2];
  double l0 = b.R[0] * o0 + b.R[1] * o1 + b.R[2] * o2;
  double l1 = b.R[3] * o0 + b.R[4] * o1 + b.R[5] * o2;
  double l2 = b.R[6] * o0 + b.R[7] * o1 + b.R[8] * o2;
  double x0 = b.c[0] + l0, x1 = b.c[1] + l1, x2 = b.c[2] + l2;
  X[3 * k] = x0; X[3 * k + 1] = x1; X[3 * k + 2] = x2;
  // U = u_s + omega x L~
  U[3 * k] = b.v[0] + (b.w[1] * l2 - b.w[2] * l1);
  U[3 * k + 1] = b.v[1] + (b.w[2] * l0 - b.w[0] * l2);
  U[3 * k + 2] = b.v[2] + (b.w[0] * l1 - b.w[1] * l0);
  double ih = 1.0 / g.h;
  int c0 = (int)floor(x0 * ih), c1 = (int)floor(x1 * ih), c2 = (int)floor(x2 * ih);
  c0 = g.bc0 ? min(max(c0, 0), g.n0 - 1) : wrapi(c0, g.n0);
  c1 = g.bc1 ? min(max(c1, 0), g.n1 - 1) : wrapi(c1, g.n1);
  c2 = g.bc2 ? min(max(c2, 0), g.n2 - 1) : wrapi(c2, g.n2);
  tile[k] = ((c0 >> 2) * nt1 + (c1 >> 2)) * nt2 + (c2 >> 2);
}
hipError_t points_place(const Geo &g, int K, const BodyDev *bodies, const int *body_of, const double *off,
                        double *X, double *U, int *tile, int nt0, int nt1, int nt2, hipStream_t s) {
  if (K == 0) return hipSuccess;
  hipLaunchKernelGGL(k_points, dim3(nblk(K, 256)), dim3(256), 0, s, g, K, bodies, body_of, off, X, U, tile,
                     nt0, nt1, nt2);
  return hipGetLastError();
}

__global__ void k_count(int K, const int *tile, int *counts) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < K) atomicAdd(&counts[tile[k]], 1);
}
hipError_t bin_count(int K, const int *tile, int *counts, hipStream_t s) {
  if (K == 0) return hipSuccess;
  hipLaunchKernelGGL(k_count, dim3(nblk(K, 256)), dim3(256), 0, s, K, tile, counts);
  return hipGetLastError();
}

// ---- exclusive scan: 1024 items per block, then the block totals ----------
constexpr int SCAN_T = 256, SCAN_ITEMS = 4, SCAN_CHUNK = SCAN_T * SCAN_ITEMS;

__device__ int block_excl_scan(int v, int *sh) {
  int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int o = 1; o < SCAN_T; o <<= 1) {
    int a = t >= o ? sh[t - o] : 0;
    __syncthreads();
    sh[t] += a;
    __syncthreads();
  }
  int incl = sh[t];
  int tot = sh[SCAN_T - 1];
  __syncthreads();
  sh[SCAN_T] = tot;
  return incl - v;
}

__global__ void k_scan1(const int *in, int *out, int n, int *bsum) {
  __shared__ int sh[SCAN_T + 1];
  long long base = (long long)blockIdx.x * SCAN_CHUNK + threadIdx.x * SCAN_ITEMS;
  int v[SCAN_ITEMS], s = 0;
  for (int q = 0; q < SCAN_ITEMS; ++q) {
    long long i = base + q;
    v[q] = i < n ? in[i] : 0;
    s += v[q];
  }
  int ex = block_excl_scan(s, sh);
  for (int q = 0; q < SCAN_ITEMS; ++q) {
    long long i = base + q;
    if (i < n) out[i] = ex;
    ex += v[q];
  }
  if (threadIdx.x == 0) bsum[blockIdx.x] = sh[SCAN_T];
}
// single block: exclusive scan of the block sums in place (any count), total at bsum[nb]
__global__ void k_scan2(int *bsum, int nb) {
  __shared__ int sh[SCAN_T + 1];
  int carry = 0;
  for (int base = 0; base < nb; base += SCAN_T) {
    int i = base + threadIdx.x;
    int v = i < nb ? bsum[i] : 0;
    int ex = block_excl_scan(v, sh);
    int tot = sh[SCAN_T];
    if (i < nb) bsum[i] = ex + carry;
    carry += tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) bsum[nb] = carry;
}
__global__ void k_scan3(int *out, int n, const int *bsum, int nb) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] += bsum[i / SCAN_CHUNK];
  if (i == 0) out[n] = bsum[nb];
}
hipError_t scan_exclusive(const int *in, int *out, int n, int *tmp, hipStream_t s) {
  int nb = nblk(n, SCAN_CHUNK);
  hipLaunchKernelGGL(k_scan1, dim3(nb), dim3(SCAN_T), 0, s, in, out, n, tmp);
  hipLaunchKernelGGL(k_scan2, dim3(1), dim3(SCAN_T), 0, s, tmp, nb);
  hipLaunchKernelGGL(k_scan3, dim3(nblk(n, 256)), dim3(256), 0, s, out, n, tmp, nb);
  return hipGetLastError();
}

__global__ void k_scatter(int K, const int *tile, const int *start, int *fillc, int *perm_tmp) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;
  int t = tile[k];
  perm_tmp[start[t] + atomicAdd(&fillc[t], 1)] = k;
}
hipError_t bin_scatter(int K, const int *tile, const int *start, int *fillc, int *perm_tmp, hipStream_t s) {
  if (K == 0) return hipSuccess;
  hipLaunchKernelGGL(k_scatter, dim3(nblk(K, 256)), dim3(256), 0, s, K, tile, start, fillc, perm_tmp);
  return hipGetLastError();
}

// Canonical order inside each tile: rank by original index.
__global__ void k_canon(int K, const int *tile, const int *start, const int *perm_tmp, int *perm) {
  int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= K) return;
  int k = perm_tmp[q];
  int t = tile[k];
  int s0 = start[t], s1 = start[t + 1];
  int r = 0;
  for (int p = s0; p < s1; ++p) r += perm_tmp[p] < k;
  perm[s0 + r] = k;
}
hipError_t bin_canon(int K, const int *tile, const int *start, const int *perm_tmp, int *perm, hipStream_t s) {
  if (K == 0) return hipSuccess;
  hipLaunchKernelGGL(k_canon, dim3(nblk(K, 256)), dim3(256), 0, s, K, tile, start, perm_tmp, perm);
  return hipGetLastError();
}

__global__ void k_compact(int n, const int *flags, const int *pos, int *list) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n && flags[t]) list[pos[t]] = t;
}
hipError_t compact(int n, const int *flags, const int *pos, int *list, hipStream_t s) {
  hipLaunchKernelGGL(k_compact, dim3(nblk(n, 256)), dim3(256), 0, s, n, flags, pos, list);
  return hipGetLastError();
}

__global__ void k_gather3(int K, const int *perm, const double *src, double *dst) {
  int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= 3 * K) return;
  int s = q / 3, d = q - 3 * s;
  dst[q] = src[3 * perm[s] + d];
}
__global__ void k_scatter3(int K, const int *perm, const double *src, double *dst) {
  int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= 3 * K) return;
  int s = q / 3, d = q - 3 * s;
  dst[3 * perm[s] + d] = src[q];
}
__global__ void k_scale3(int n, const double *x, double a, const double *y, double b, double *out) {
  int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  out[q] = a * x[q] + (y ? b * y[q] : 0.0);
}
hipError_t gather3(int K, const int *perm, const double *src, double *dst, hipStream_t s) {
  if (K == 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather3, dim3(nblk(3LL * K, 256)), dim3(256), 0, s, K, perm, src, dst);
  return hipGetLastError();
}
hipError_t scatter3(int K, const int *perm, const double *src, double *dst, hipStream_t s) {
  if (K == 0) return hipSuccess;
  hipLaunchKernelGGL(k_scatter3, dim3(nblk(3LL * K, 256)), dim3(256), 0, s, K, perm, src, dst);
  return hipGetLastError();
}
hipError_t scale3(int K, const double *x, double alpha, const double *y, double beta, double *out,
                  hipStream_t s) {
  if (K == 0) return hipSuccess;
  hipLaunchKernelGGL(k_scale3, dim3(nblk(3LL * K, 256)), dim3(256), 0, s, 3 * K, x, alpha, y, beta, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Interpolation, one workgroup per non-empty point tile.  The points of tile
// T (cells 4T..4T+3 per axis) only reach nodes 4T-2 .. 4T+5 per axis, so the
// workgroup first stages that 8^3 region of the source in LDS (MODE 0: the
// three face fields; MODE 1: the cell field, whose face gradients are formed
// from LDS) together with the 1-D weights of its points (face and centre
// nodes per axis), then gathers every point's stencil from LDS: 16 lanes per
// point (node offsets (a, b)), z nodes summed in order, the 16 partial sums
// reduced by a fixed butterfly.
constexpr int IREG = 8;   // region width per axis
// region stride between x planes: 2 more than IREG^2, so the 16 lanes of a
// point (x offsets a, y offsets b) fall on 16 distinct LDS banks
constexpr int IRS = IREG * IREG + 2;
constexpr int IPTS = 64;  // points staged per pass

template <int KER, int MODE, typename T, typename TA>
__global__ void __launch_bounds__(256) k_interp(Geo g, int nt1, int nt2, const int *tiles, const int *tstart,
                                                const double *X, const T *src, double alpha, const double *y,
                                                double beta, double *out) {
  constexpr int W = KerWidth<KER>::W;
  constexpr int NC = MODE == 0 ? 3 : 1;
  // TA: the arithmetic type (float64, or float32 for the gradient of a
  // float32 cell field in the float32 Krylov cycle, weights rounded to it)
  __shared__ TA reg[NC][IREG * IRS];
  __shared__ TA pw[IPTS][3][2][4];   // [point][axis][face/centre][node]
  __shared__ int pb[IPTS][3][2];         // local start of the support
  const int tile = tiles[blockIdx.x];
  if (tile < 0) return;  // a hole of the launch order
  const int T2 = tile % nt2, r = tile / nt2, T1 = r % nt1, T0 = r / nt1;
  const int o0 = 4 * T0 - 2, o1 = 4 * T1 - 2, o2 = 4 * T2 - 2;  // region origin
  const long long N = 2 * g.half;
  const int s0 = tstart[tile], s1 = tstart[tile + 1];
  // the coordinates of this thread's staging tasks in the first chunk
  // (task t: point t / 6, axis (t % 6) / 2), loaded before the region so
  // that both sets of loads are in flight together
  double xpre[2];
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int task = threadIdx.x + 256 * u, pt = task / 6;
    xpre[u] = s0 + pt < s1 && pt < IPTS ? X[3 * (s0 + pt) + ((task - 6 * pt) >> 1)] : 0.0;
  }
  for (int e = threadIdx.x; e < NC * IREG * IREG * IREG; e += 256) {
    int comp = e / (IREG * IREG * IREG), l = e % (IREG * IREG * IREG);
    int li = l / (IREG * IREG), lj = (l / IREG) % IREG, lk = l % IREG;
    int i = o0 + li, j = o1 + lj, k = o2 + lk;
    bool ok = true;
    if (g.bc0) ok = ok && i >= 0 && i < g.n0; else i = wrapi(i, g.n0);
    if (g.bc1) ok = ok && j >= 0 && j < g.n1; else j = wrapi(j, g.n1);
    if (g.bc2) ok = ok && k >= 0 && k < g.n2; else k = wrapi(k, g.n2);
    reg[comp][li * IRS + lj * IREG + lk] = ok ? (TA)src[comp * N + sidx(g, i, j, k)] : TA(0);
  }
  const int lane = threadIdx.x & 15, ta = lane >> 2, tb = lane & 3;
  const double ih = 1.0 / g.h;
  const int org[3] = {o0, o1, o2};
  const int nn[3] = {g.n0, g.n1, g.n2};
  const int bcs[3] = {g.bc0, g.bc1, g.bc2};
  for (int c0 = s0; c0 < s1; c0 += IPTS) {
    const int np = min(IPTS, s1 - c0);
    __syncthreads();
    // stage weights: one task per (point, axis, staggering)
    static_assert(6 * IPTS <= 2 * 256, "two staging tasks per thread");
    for (int task = threadIdx.x; task < np * 6; task += 256) {
      int pt = task / 6, rem = task - 6 * pt, ax = rem >> 1, st = rem & 1;
      TA wv[4];
      const double xv = c0 == s0 ? (task < 256 ? xpre[0] : xpre[1]) : X[3 * (c0 + pt) + ax];
      int i0 = axis_weights<KER, TA>(xv, ih, st == 0, wv);
      int l0 = i0 - org[ax];
      if (!bcs[ax]) l0 = wrapi(l0 + nn[ax] / 2, nn[ax]) - nn[ax] / 2;
      pb[pt][ax][st] = l0;
      // a wall face (index 0 along a wall axis) carries no gradient: zero its weight
#pragma unroll
      for (int t = 0; t < 4; ++t)
        pw[pt][ax][st][t] = (MODE == 1 && st == 0 && bcs[ax] && i0 + t == 0) ? TA(0) : wv[t];
    }
    __syncthreads();
    for (int pb0 = 0; pb0 < np; pb0 += 16) {
      int pt = pb0 + (threadIdx.x >> 4);
      bool active = pt < np;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        TA acc = TA(0);
        if (active && ta < W && tb < W) {
          const int sx = d == 0 ? 0 : 1, sy = d == 1 ? 0 : 1, sz = d == 2 ? 0 : 1;
          int li = pb[pt][0][sx] + ta, lj = pb[pt][1][sy] + tb, lk0 = pb[pt][2][sz];
          TA wab = pw[pt][0][sx][ta] * pw[pt][1][sy][tb];
#pragma unroll
          for (int c = 0; c < W; ++c) {
            int lk = lk0 + c;
            TA v = TA(0);
            bool in = (unsigned)li < IREG && (unsigned)lj < IREG && (unsigned)lk < IREG;
            if (MODE == 0) {
              if (in) v = reg[d][li * IRS + lj * IREG + lk];
            } else {
              int mi = li - (d == 0), mj = lj - (d == 1), mk = lk - (d == 2);
              bool inm = (unsigned)mi < IREG && (unsigned)mj < IREG && (unsigned)mk < IREG;
              if (in && inm) v = (reg[0][li * IRS + lj * IREG + lk] - reg[0][mi * IRS + mj * IREG + mk]) * (TA)ih;
            }
            acc += (wab * pw[pt][2][sz][c]) * v;
          }
        }
        acc = sum16(acc);
        if (active && lane == 0) {
          long long o = 3LL * (c0 + pt) + d;
          out[o] = alpha * (double)acc + (y ? beta * y[o] : 0.0);
        }
      }
    }
  }
}

template <typename T>
hipError_t interp_grad(int ker, const Geo &g, int nt1, int nt2, int ntiles_nz, const int *tiles, const int *tstart,
                       const double *X, const T *z, double alpha, const double *y, double beta, double *out,
                       hipStream_t s, bool f32) {
  // positions read, results written (and y read), the cells of the support band (T each)
  ProbeExt probe_(PR_INTERP_GRAD, s,
                    (double)probe_points() * (beta != 0.0 ? 72 : 48) + (double)probe_band_cells() * sizeof(T));
  if (ntiles_nz == 0) return hipSuccess;
  if (f32 && sizeof(T) != sizeof(float)) return hipErrorInvalidValue;
  dim3 gr(ntiles_nz), bl(256);
  hipEvent_t e0, e1;
  probe_ext_take(&e0, &e1);
#define INTERP(K_, A_)                                                                                             \
  hipExtLaunchKernelGGL((k_interp<K_, 1, T, A_>), gr, bl, 0, s, e0, e1, 0, g, nt1, nt2, tiles, tstart, X, z, alpha, y, \
                        beta, out)
  if (ker == KER_PESKIN4) {
    if (f32) INTERP(KER_PESKIN4, float);
    else INTERP(KER_PESKIN4, double);
  } else {
    if (f32) INTERP(KER_ROMA3, float);
    else INTERP(KER_ROMA3, double);
  }
#undef INTERP
  return hipGetLastError();
}
template hipError_t interp_grad<float>(int, const Geo &, int, int, int, const int *, const int *, const double *,
                                       const float *, double, const double *, double, double *, hipStream_t, bool);
template hipError_t interp_grad<double>(int, const Geo &, int, int, int, const int *, const int *, const double *,
                                        const double *, double, const double *, double, double *, hipStream_t, bool);

hipError_t interp_face(int ker, const Geo &g, int nt1, int nt2, int ntiles_nz, const int *tiles, const int *tstart,
                       const double *X, const double *u3, double alpha, const double *y, double beta, double *out,
                       hipStream_t s) {
  // positions read, results written (and y read), three face components of the support band
  ProbeScope probe_(PR_INTERP_FACE, s,
                    (double)probe_points() * (beta != 0.0 ? 72 : 48) + (double)probe_band_cells() * 3 * 8);
  if (ntiles_nz == 0) return hipSuccess;
  dim3 gr(ntiles_nz), bl(256);
  if (ker == KER_PESKIN4)
    hipLaunchKernelGGL((k_interp<KER_PESKIN4, 0, double, double>), gr, bl, 0, s, g, nt1, nt2, tiles, tstart, X, u3, alpha,
                       y, beta, out);
  else
    hipLaunchKernelGGL((k_interp<KER_ROMA3, 0, double, double>), gr, bl, 0, s, g, nt1, nt2, tiles, tstart, X, u3, alpha, y,
                       beta, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Touch lists.  Tile T owns the cells 4T..4T+3 per axis; for velocity
// component d its face box also holds the upper face 4T+4 along d (needed by
// the divergence of its last cell).  A point touches T when its support meets
// that box for some component.  Lists are built once per placement: count
// per tile, scan, then fill per tile.

// Range of tiles touched along one axis (union over the components).
template <int KER>
__device__ __forceinline__ void touch_range(double x, double ih, int &lo, int &hi) {
  constexpr int W = KerWidth<KER>::W;
  double s;
  int f0 = support_start<KER>(x, ih, true, s);   // face nodes along this axis
  int c0 = support_start<KER>(x, ih, false, s);  // centre nodes
  auto fdiv = [](int a) { return a >= 0 ? a / 4 : -((-a + 3) / 4); };
  lo = min(fdiv(f0 - 1), fdiv(c0));
  hi = max(fdiv(f0 + W - 1), fdiv(c0 + W - 1));
}

// Touch lists built tile by tile, without atomics: the 64 lanes of a
// wavefront walk the points of the neighbouring point tiles of tile t (home
// tiles within one tile along each axis, wrapped on periodic axes; a point's
// support never reaches further) in a fixed order (neighbour offsets in
// lexicographic order, sorted points within a tile) and keep those whose
// support touches t.  PASS 0 writes the count of every tile; PASS 1 writes the
// lists of the active tiles by ordered wavefront compaction, so every list
// has the same order on every run.
template <int KER, int PASS>
__global__ void __launch_bounds__(256) k_touch_tile(Geo g, int nt0, int nt1, int nt2, int ntl, const int *ntl_dev,
                                                    const int *tiles, const int *tstart, const double *X,
                                                    int *counts, const int *lstart, int *list) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int w = blockIdx.x * 4 + wave;
  if (w >= ntl || (ntl_dev && w >= *ntl_dev)) return;
  const int t = tiles ? tiles[w] : w;
  const int nt[3] = {nt0, nt1, nt2}, bc[3] = {g.bc0, g.bc1, g.bc2};
  const int tc[3] = {t / (nt1 * nt2), (t / nt2) % nt1, t % nt2};
  int nb[3][3], nn[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    nn[a] = 0;
    for (int sft = -1; sft <= 1; ++sft) {
      int v = tc[a] + sft;
      if (v < 0 || v >= nt[a]) {
        if (bc[a]) continue;
        v = wrapi(v, nt[a]);
      }
      bool dup = false;
      for (int q = 0; q < nn[a]; ++q) dup = dup || nb[a][q] == v;
      if (!dup) nb[a][nn[a]++] = v;
    }
  }
  const double ih = 1.0 / g.h;
  const unsigned long long below = (1ull << lane) - 1ull;
  const int base = PASS ? lstart[t] : 0;
  int cnt = 0;
  for (int q0 = 0; q0 < nn[0]; ++q0)
    for (int q1 = 0; q1 < nn[1]; ++q1)
      for (int q2 = 0; q2 < nn[2]; ++q2) {
        const int n = (nb[0][q0] * nt1 + nb[1][q1]) * nt2 + nb[2][q2];
        const int p0 = tstart[n], p1 = tstart[n + 1];
        for (int pb = p0; pb < p1; pb += 64) {
          const int p = pb + lane;
          bool hit = false;
          if (p < p1) {
            hit = true;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
              int lo, hi;
              touch_range<KER>(X[3 * p + a], ih, lo, hi);
              bool in = false;
              for (int v = lo; v <= hi; ++v) {
                int u = v;
                if (u < 0 || u >= nt[a]) {
                  if (bc[a]) continue;
                  u = wrapi(u, nt[a]);
                }
                in = in || u == tc[a];
              }
              hit = hit && in;
            }
          }
          const unsigned long long m = __ballot(hit);
          if (PASS == 1 && hit) list[base + cnt + __popcll(m & below)] = p;
          cnt += __popcll(m);
        }
      }
  if (PASS == 0 && lane == 0) counts[t] = cnt;
}

hipError_t touch_tiles(int ker, const Geo &g, int nt0, int nt1, int nt2, int ntl, const int *ntl_dev,
                       const int *tiles, const int *tstart, const double *X, int *counts, const int *lstart,
                       int *list, hipStream_t s) {
  if (ntl == 0) return hipSuccess;
  const dim3 gr((ntl + 3) / 4), bl(256);
  if (list == nullptr) {
    if (ker == KER_PESKIN4)
      hipLaunchKernelGGL((k_touch_tile<KER_PESKIN4, 0>), gr, bl, 0, s, g, nt0, nt1, nt2, ntl, ntl_dev, tiles,
                         tstart, X, counts, lstart, list);
    else
      hipLaunchKernelGGL((k_touch_tile<KER_ROMA3, 0>), gr, bl, 0, s, g, nt0, nt1, nt2, ntl, ntl_dev, tiles, tstart,
                         X, counts, lstart, list);
  } else {
    if (ker == KER_PESKIN4)
      hipLaunchKernelGGL((k_touch_tile<KER_PESKIN4, 1>), gr, bl, 0, s, g, nt0, nt1, nt2, ntl, ntl_dev, tiles,
                         tstart, X, counts, lstart, list);
    else
      hipLaunchKernelGGL((k_touch_tile<KER_ROMA3, 1>), gr, bl, 0, s, g, nt0, nt1, nt2, ntl, ntl_dev, tiles, tstart,
                         X, counts, lstart, list);
  }
  return hipGetLastError();
}

// Flag the tiles within one tile (per axis, wrapped on periodic axes) of the
// n non-empty point tiles: the only tiles a point's support can reach.  Every
// writer stores the same value 1.
__global__ void k_mark_near(Geo g, int nt0, int nt1, int nt2, int n, const int *nz, int *flags) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= 27 * n) return;
  const int t = nz[q / 27], o = q % 27;
  const int nt[3] = {nt0, nt1, nt2}, bc[3] = {g.bc0, g.bc1, g.bc2};
  const int tc[3] = {t / (nt1 * nt2), (t / nt2) % nt1, t % nt2};
  const int off[3] = {o / 9 - 1, (o / 3) % 3 - 1, o % 3 - 1};
  int v[3];
  for (int a = 0; a < 3; ++a) {
    v[a] = tc[a] + off[a];
    if (v[a] < 0 || v[a] >= nt[a]) {
      if (bc[a]) return;
      v[a] = wrapi(v[a], nt[a]);
    }
  }
  flags[(v[0] * nt1 + v[1]) * nt2 + v[2]] = 1;
}
hipError_t mark_near(const Geo &g, int nt0, int nt1, int nt2, int n, const int *nz, int *flags, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_mark_near, dim3(nblk(27LL * n, 256)), dim3(256), 0, s, g, nt0, nt1, nt2, n, nz, flags);
  return hipGetLastError();
}

// Launch order of a tile list (one workgroup, counting sort).  The
// dispatcher deals consecutive workgroups round-robin to the 8 XCDs, each
// with its own L2: the list (in tile-index order, i.e. spatially sorted) is
// cut into ORD_X contiguous chunks and chunk c is dealt to the workgroups
// c, c + 8, c + 16, ..., so the neighbouring tiles that share points and
// halo cells run on one XCD and find them in its L2.  Within a chunk the
// tiles go in order of decreasing list length (the workgroups with the most
// work start first, which shortens the tail).  out has ORD_X * ceil(n /
// ORD_X) entries; -1 marks the holes of a short last chunk (those
// workgroups exit).  Each tile's result does not depend on the order, which
// within a length bucket is arbitrary.
constexpr int ORD_T = 1024, ORD_B = 256, ORD_X = 8;
__global__ void __launch_bounds__(ORD_T) k_order_active(int n, const int *active, const int *lstart, int *out) {
  __shared__ int cnt[ORD_X * ORD_B], base[ORD_X * ORD_B];
  const int t = threadIdx.x;
  const int cs = (n + ORD_X - 1) / ORD_X;
  for (int b = t; b < ORD_X * ORD_B; b += ORD_T) cnt[b] = 0;
  for (int i = t; i < ORD_X * cs; i += ORD_T) out[i] = -1;
  __syncthreads();
  auto key = [&](int i) {
    const int a = active[i];
    return (i / cs) * ORD_B + ORD_B - 1 - min(lstart[a + 1] - lstart[a], ORD_B - 1);
  };
  for (int i = t; i < n; i += ORD_T) atomicAdd(&cnt[key(i)], 1);
  __syncthreads();
  if (t < ORD_X) {
    int acc = 0;  // position within chunk t
    for (int b = 0; b < ORD_B; ++b) {
      base[t * ORD_B + b] = acc;
      acc += cnt[t * ORD_B + b];
    }
  }
  __syncthreads();
  for (int i = t; i < n; i += ORD_T) out[atomicAdd(&base[key(i)], 1) * ORD_X + i / cs] = active[i];
}
int order_launch_count(int n) { return ORD_X * ((n + ORD_X - 1) / ORD_X); }
hipError_t order_active(int n, const int *active, const int *lstart, int *out, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_order_active, dim3(1), dim3(ORD_T), 0, s, n, active, lstart, out);
  return hipGetLastError();
}

__global__ void k_positive(int n, const int *counts, int *flags) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) flags[t] = counts[t] > 0;
}
hipError_t positive_flags(int n, const int *counts, int *flags, hipStream_t s) {
  hipLaunchKernelGGL(k_positive, dim3(nblk(n, 256)), dim3(256), 0, s, n, counts, flags);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Spreading on one active tile from its touch list.
//
// Staging: up to BAND_CH listed points at a time, one task per (point, axis)
// computing the face- and centre-node weights of that axis (one square root
// each) and laying them out over the tile's own positions along the axis
// (5 face / 4 centre positions per component, zero outside the point's
// support; the x weights of component d carry q_d).
//
// Accumulation: lane l < 30 of every half-wavefront owns two neighbouring
// z-columns (same x, consecutive y) of a face box (component 0: 5 x 4
// columns of 4 faces, component 1: 4 x 5 columns of 4 faces, component 2:
// 4 x 4 columns of 5 faces).  Half-wavefront h (0..7) adds the listed points
// h, h+8, h+16, ... in list order into registers, with no branch:
// w_x[ci] w_y[cj] times the five z weights of the column (zeros add
// nothing); the x and z weights serve both columns, so a lane reads 8 LDS
// values per point for 10 products.  The eight partial sums of a face are
// added in a fixed order, so every grid value is summed in the same order
// on every run.
constexpr int BAND_CH = 64;
// doubles per point: x[comp][5], y[comp][5], z[comp][5].  The point stride
// is odd in 8-byte units, so staging writes of consecutive points spread
// over the LDS banks, and the three components' 5-double blocks of one axis
// fall on distinct banks for the accumulation reads.
constexpr int BAND_WS = 45;

template <int KER, bool DIV, typename TA, typename TO>
__global__ void __launch_bounds__(256) k_band(Geo g, int nt1, int nt2, const int *active, const int *lstart,
                                              const int *list, const double *X, const double *q, double alpha,
                                              TO *out) {
  // [cand][axis a * 15 + comp * 5 + position]; after the last chunk the same
  // LDS holds the per-half-wavefront face sums part[8][3][80]
  static_assert(8 * 3 * 80 <= BAND_CH * BAND_WS, "face sums must fit the weight buffer");
  // TA: the weights' and sums' type (float64, or float32 for the S~ products
  // of the float32 Krylov cycle)
  __shared__ TA wts[BAND_CH][BAND_WS];
  TA(*part)[3][80] = reinterpret_cast<TA(*)[3][80]>(&wts[0][0]);
  const int tile = active[blockIdx.x];
  if (tile < 0) return;  // a hole of the launch order
  const int T2 = tile % nt2, r = tile / nt2, T1 = r % nt1, T0 = r / nt1;
  const int tid = threadIdx.x;
  const int s0 = lstart[tile], s1 = lstart[tile + 1];
  const double ih = 1.0 / g.h;
  const int org[3] = {4 * T0, 4 * T1, 4 * T2};
  const int nn[3] = {g.n0, g.n1, g.n2};
  const int bcs[3] = {g.bc0, g.bc1, g.bc2};
  // Accumulation: each half-wavefront takes every 8th listed point; lane hl
  // of a half owns, for component cd, the x position ci and the two y
  // positions cj0, cj0 + 1 (the second absent at the odd end of a 5-wide box)
  // of a pair of face columns, nf faces along z: 30 of the 32 lanes, 4 LDS
  // reads per (point, tile) pair and lane instead of 7 with one column each.
  const int wv = tid >> 6, lane = tid & 63, half = lane >> 5, hl = lane & 31;
  const int cd = hl < 10 ? 0 : (hl < 22 ? 1 : 2);
  const int cl = hl - (cd == 0 ? 0 : (cd == 1 ? 10 : 22));
  const int npair = cd == 1 ? 3 : 2;  // column pairs along y
  const int cby = cd == 1 ? 5 : 4;    // columns along y in this component's box
  const int ci = min(cl / npair, 4), cj0 = 2 * (cl % npair);
  const bool has1 = cj0 + 1 < cby;
  const int nf = cd == 2 ? 5 : 4;
  const bool owner = hl < 30;
  TA acc0[5] = {TA(0), TA(0), TA(0), TA(0), TA(0)}, acc1[5] = {TA(0), TA(0), TA(0), TA(0), TA(0)};
  // Staging task of this thread in every chunk (3 BAND_CH <= 256 tasks: at
  // most one per thread): axis a of listed point cand.  Its operands are
  // loaded one chunk ahead and its list entry two chunks ahead, so the
  // dependent loads (list entry, then position and value) of the next chunk
  // are in flight while the current one is accumulated.
  static_assert(3 * BAND_CH <= 256, "one staging task per thread");
  const int cand = tid / 3, a = tid - 3 * cand;
  const bool stager = tid < 3 * BAND_CH;
  auto entry = [&](int c0) { return (stager && c0 + cand < s1) ? list[c0 + cand] : -1; };
  int p_cur = entry(s0);
  double xa, qv[3];
  auto operands = [&](int p, double &x, double (&qq)[3]) {
    const int pc = p >= 0 ? p : 0;  // every list here is non-empty, so point 0 exists
    x = X[3 * pc + a];
#pragma unroll
    for (int d = 0; d < 3; ++d) qq[d] = a == 0 ? q[3 * pc + d] : 1.0;
  };
  operands(p_cur, xa, qv);
  int p_nxt = entry(s0 + BAND_CH);
  for (int c0 = s0; c0 < s1; c0 += BAND_CH) {
    const int nc = min(BAND_CH, s1 - c0);
    __syncthreads();
    if (p_cur >= 0) {
      TA wf[4], wc[4];
      int f0 = axis_weights<KER, TA>(xa, ih, true, wf);
      int e0 = axis_weights<KER, TA>(xa, ih, false, wc);
      int lf = f0 - org[a], lc = e0 - org[a];
      if (!bcs[a]) {
        // periodic image of the support start in [-4, n - 4): every offset
        // that reaches the box (-3 .. its last position) keeps its value,
        // and no image of another can reach it, for any n >= 16
        lf = wrapi(lf + 4, nn[a]) - 4;
        lc = wrapi(lc + 4, nn[a]) - 4;
      }
      // the weights over the box positions along this axis: faces (5) and
      // centres (4), zero outside the support (select chains: no dynamic
      // index into a register array, no branch)
      TA F[5], C[4];
#pragma unroll
      for (int t = 0; t < 5; ++t) {
        const int i_f = t - lf, i_c = t - lc;
        TA v = i_f == 0 ? wf[0] : TA(0);
        v = i_f == 1 ? wf[1] : v;
        v = i_f == 2 ? wf[2] : v;
        v = i_f == 3 ? wf[3] : v;
        F[t] = v;
        if (t < 4) {
          TA u = i_c == 0 ? wc[0] : TA(0);
          u = i_c == 1 ? wc[1] : u;
          u = i_c == 2 ? wc[2] : u;
          u = i_c == 3 ? wc[3] : u;
          C[t] = u;
        }
      }
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const TA qd = (TA)qv[d];
#pragma unroll
        for (int t = 0; t < 5; ++t) {
          // position t exists for the faces of axis d (5) and the cells of the others (4)
          const TA v = d == a ? F[t] : (t < 4 ? C[t] : TA(0));
          wts[cand][15 * a + 5 * d + t] = v * qd;
        }
      }
    }
    // the next chunk's operands and the list entries of the one after it
    p_cur = p_nxt;
    operands(p_cur, xa, qv);
    p_nxt = entry(c0 + 2 * BAND_CH);
    __syncthreads();
    if (owner) {
#pragma unroll 2
      for (int c = 2 * wv + half; c < nc; c += 8) {
        const TA *W = wts[c] + 5 * cd;
        const TA wx = W[ci];
        const TA wab0 = wx * W[15 + cj0];
        // without a second column (has1 false) the lane reads the next
        // block's first y weight, inside the point's row, and acc1 is
        // never stored
        const TA wab1 = wx * W[16 + cj0];
#pragma unroll
        for (int fk = 0; fk < 5; ++fk) {
          const TA wz = W[30 + fk];
          acc0[fk] += wab0 * wz;
          acc1[fk] += wab1 * wz;
        }
      }
    }
  }
  __syncthreads();
  if (owner) {
    // face box index: (ci * by + cj) * bz + fk with by = 4 or 5, bz = 4 or 5
    const int bz = cd == 2 ? 5 : 4, slot = 2 * wv + half;
#pragma unroll
    for (int fk = 0; fk < 5; ++fk) {
      if (fk < nf) {
        part[slot][cd][(ci * cby + cj0) * bz + fk] = acc0[fk];
        if (has1) part[slot][cd][(ci * cby + cj0 + 1) * bz + fk] = acc1[fk];
      }
    }
  }
  __syncthreads();
  long long N = 2 * g.half;
  auto face = [&](int d, int idx) {
    TA f = part[0][d][idx];
#pragma unroll
    for (int q = 1; q < 8; ++q) f += part[q][d][idx];
    return f;
  };
  if (DIV) {
    if (tid < 64) {
      int ci2 = tid >> 4, cj2 = (tid >> 2) & 3, ck = tid & 3;
      TA dv = TA(0);
      dv += face(0, ((ci2 + 1) * 4 + cj2) * 4 + ck) - face(0, (ci2 * 4 + cj2) * 4 + ck);
      dv += face(1, (ci2 * 5 + cj2 + 1) * 4 + ck) - face(1, (ci2 * 5 + cj2) * 4 + ck);
      dv += face(2, (ci2 * 4 + cj2) * 5 + ck + 1) - face(2, (ci2 * 4 + cj2) * 5 + ck);
      int gi = 4 * T0 + ci2, gj = 4 * T1 + cj2, gk = 4 * T2 + ck;
      const long long o = sidx(g, gi, gj, gk);
      out[o] = (TO)((double)out[o] + alpha * (double)dv * ih);
    }
  } else {
    if (tid < 192) {
      int d = tid >> 6, t = tid & 63;
      int fi = t >> 4, fj = (t >> 2) & 3, fk = t & 3;
      int by = 4 + (d == 1), bz = 4 + (d == 2);
      int gi = 4 * T0 + fi, gj = 4 * T1 + fj, gk = 4 * T2 + fk;
      const long long o = d * N + sidx(g, gi, gj, gk);
      out[o] = (TO)((double)out[o] + alpha * (double)face(d, (fi * by + fj) * bz + fk));
    }
  }
}

template <typename TO>
static hipError_t band_launch(int ker, bool div, const Geo &g, int nt1, int nt2, int nactive, const int *active,
                              const int *lstart, const int *list, const double *X, const double *q, double alpha,
                              TO *out, hipStream_t s, bool f32) {
  // positions and values read, the active tiles' cells (div) or faces read and written
  ProbeExt probe_(div ? PR_BAND_DIV : PR_BAND_FACE, s,
                    (double)probe_points() * 48 + (double)probe_band_cells() * (div ? 1 : 3) * 2 * sizeof(TO));
  if (nactive == 0) return hipSuccess;
  dim3 gr(nactive), bl(256);
  hipEvent_t e0, e1;
  probe_ext_take(&e0, &e1);
#define BAND(K_, D_, A_)                                                                                           \
  hipExtLaunchKernelGGL((k_band<K_, D_, A_, TO>), gr, bl, 0, s, e0, e1, 0, g, nt1, nt2, active, lstart, list, X, q, \
                        alpha, out)
  if (f32) {
    if (!div) return hipErrorInvalidValue;  // float32 sums serve the S~ products only
    if (ker == KER_PESKIN4) BAND(KER_PESKIN4, true, float);
    else BAND(KER_ROMA3, true, float);
  } else if constexpr (sizeof(TO) == sizeof(double)) {
    if (ker == KER_PESKIN4) {
      if (div) BAND(KER_PESKIN4, true, double);
      else BAND(KER_PESKIN4, false, double);
    } else {
      if (div) BAND(KER_ROMA3, true, double);
      else BAND(KER_ROMA3, false, double);
    }
  } else {
    return hipErrorInvalidValue;  // a float32 output takes float32 sums
  }
#undef BAND
  return hipGetLastError();
}
hipError_t band_apply(int ker, bool div, const Geo &g, int nt1, int nt2, int nactive, const int *active,
                      const int *lstart, const int *list, const double *X, const double *q, double alpha,
                      double *out, hipStream_t s, bool f32) {
  return band_launch(ker, div, g, nt1, nt2, nactive, active, lstart, list, X, q, alpha, out, s, f32);
}
hipError_t band_apply(int ker, bool div, const Geo &g, int nt1, int nt2, int nactive, const int *active,
                      const int *lstart, const int *list, const double *X, const double *q, double alpha,
                      float *out, hipStream_t s, bool f32) {
  return band_launch(ker, div, g, nt1, nt2, nactive, active, lstart, list, X, q, alpha, out, s, f32);
}

}  // namespace ibs
