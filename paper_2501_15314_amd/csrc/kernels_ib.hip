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

// A tile is active when it or one of its 26 neighbours holds points: only
// those tiles can receive spread values.
__global__ void k_active(int nt0, int nt1, int nt2, int bc0, int bc1, int bc2, const int *counts, int *flags) {
  long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  long long nt = (long long)nt0 * nt1 * nt2;
  if (t >= nt) return;
  int t2 = (int)(t % nt2), r = (int)(t / nt2), t1 = r % nt1, t0 = r / nt1;
  int f = 0;
  for (int a = -1; a <= 1 && !f; ++a) {
    int u0 = nbr(t0, a, nt0, bc0);
    if (u0 < 0) continue;
    for (int b = -1; b <= 1 && !f; ++b) {
      int u1 = nbr(t1, b, nt1, bc1);
      if (u1 < 0) continue;
      for (int c = -1; c <= 1; ++c) {
        int u2 = nbr(t2, c, nt2, bc2);
        if (u2 < 0) continue;
        if (counts[((long long)u0 * nt1 + u1) * nt2 + u2] > 0) { f = 1; break; }
      }
    }
  }
  flags[t] = f;
}
hipError_t active_flags(int nt0, int nt1, int nt2, int bc0, int bc1, int bc2, const int *counts, int *flags,
                        hipStream_t s) {
  long long nt = (long long)nt0 * nt1 * nt2;
  hipLaunchKernelGGL(k_active, dim3(nblk(nt, 256)), dim3(256), 0, s, nt0, nt1, nt2, bc0, bc1, bc2, counts,
                     flags);
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
// Interpolation.  16 lanes per point (node offsets (a, b) of the x-y
// support), each summing the z nodes in order; the 16 partial sums are then
// reduced by a fixed butterfly.  MODE 0: face field u3; MODE 1: G z of a cell
// field z, (G z)_d(idx) = (z(idx) - z(idx - e_d)) / h.
template <int KER, int MODE, typename T>
__global__ void __launch_bounds__(256) k_interp(Geo g, int K, const double *X, const T *src, double alpha,
                                                const double *y, double beta, double *out) {
  constexpr int W = KerWidth<KER>::W;
  int lane = threadIdx.x & 15;
  int pnt = blockIdx.x * 16 + (threadIdx.x >> 4);
  bool active = pnt < K;
  int ta = lane >> 2, tb = lane & 3;
  double xp0 = 0, xp1 = 0, xp2 = 0;
  if (active) { xp0 = X[3 * pnt]; xp1 = X[3 * pnt + 1]; xp2 = X[3 * pnt + 2]; }
  double ih = 1.0 / g.h;
  long long N = 2 * g.half;
  for (int d = 0; d < 3; ++d) {
    double acc = 0.0;
    if (active && ta < W && tb < W) {
      double s0, s1, s2;
      int i0 = support_start<KER>(xp0, ih, d == 0, s0);
      int j0 = support_start<KER>(xp1, ih, d == 1, s1);
      int k0 = support_start<KER>(xp2, ih, d == 2, s2);
      int i = i0 + ta, j = j0 + tb;
      bool ok = true;
      if (g.bc0) ok = ok && i >= 0 && i < g.n0; else i = wrapi(i, g.n0);
      if (g.bc1) ok = ok && j >= 0 && j < g.n1; else j = wrapi(j, g.n1);
      double wab = phi<KER>(s0 - (double)(i0 + ta)) * phi<KER>(s1 - (double)(j0 + tb));
      if (ok) {
        for (int c = 0; c < W; ++c) {
          int k = k0 + c;
          if (g.bc2) { if (k < 0 || k >= g.n2) continue; } else k = wrapi(k, g.n2);
          double wgt = wab * phi<KER>(s2 - (double)(k0 + c));
          double v = 0.0;
          if (MODE == 0) {
            v = (double)src[d * N + sidx(g, i, j, k)];
          } else {
            int im = i - (d == 0), jm = j - (d == 1), km = k - (d == 2);
            int bcd = geo_bc(g, d), nd = geo_n(g, d);
            int xm = d == 0 ? im : (d == 1 ? jm : km);
            bool wall_face = xm < 0 && bcd;  // the wall face carries no gradient
            if (xm < 0 && !bcd) {
              if (d == 0) im += nd; else if (d == 1) jm += nd; else km += nd;
            }
            if (!wall_face)
              v = ((double)src[sidx(g, i, j, k)] - (double)src[sidx(g, im, jm, km)]) * ih;
          }
          acc += wgt * v;
        }
      }
    }
    acc = sum16(acc);
    if (active && lane == 0) out[3 * pnt + d] = alpha * acc + (y ? beta * y[3 * pnt + d] : 0.0);
  }
}

template <typename T>
hipError_t interp_grad(int ker, const Geo &g, int K, const double *X, const T *z, double alpha, const double *y,
                       double beta, double *out, hipStream_t s) {
  if (K == 0) return hipSuccess;
  dim3 gr(nblk(K, 16)), bl(256);
  if (ker == KER_PESKIN4)
    hipLaunchKernelGGL((k_interp<KER_PESKIN4, 1, T>), gr, bl, 0, s, g, K, X, z, alpha, y, beta, out);
  else
    hipLaunchKernelGGL((k_interp<KER_ROMA3, 1, T>), gr, bl, 0, s, g, K, X, z, alpha, y, beta, out);
  return hipGetLastError();
}
template hipError_t interp_grad<float>(int, const Geo &, int, const double *, const float *, double,
                                       const double *, double, double *, hipStream_t);
template hipError_t interp_grad<double>(int, const Geo &, int, const double *, const double *, double,
                                        const double *, double, double *, hipStream_t);

hipError_t interp_face(int ker, const Geo &g, int K, const double *X, const double *u3, double alpha,
                       const double *y, double beta, double *out, hipStream_t s) {
  if (K == 0) return hipSuccess;
  dim3 gr(nblk(K, 16)), bl(256);
  if (ker == KER_PESKIN4)
    hipLaunchKernelGGL((k_interp<KER_PESKIN4, 0, double>), gr, bl, 0, s, g, K, X, u3, alpha, y, beta, out);
  else
    hipLaunchKernelGGL((k_interp<KER_ROMA3, 0, double>), gr, bl, 0, s, g, K, X, u3, alpha, y, beta, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Spreading on one active tile.  Local face box of component d: 4 cells per
// axis plus the upper face along d (5 x 4 x 4 with the 5 along d).
template <int KER, bool DIV>
__global__ void __launch_bounds__(256) k_band(Geo g, int nt0, int nt1, int nt2, const int *active,
                                              const int *tstart, const double *X, const double *q,
                                              double alpha, double *out) {
  constexpr int W = KerWidth<KER>::W;
  __shared__ double acc[3][80];
  int tile = active[blockIdx.x];
  int T2 = tile % nt2, r = tile / nt2, T1 = r % nt1, T0 = r / nt1;
  for (int t = threadIdx.x; t < 240; t += blockDim.x) (&acc[0][0])[t] = 0.0;
  __syncthreads();
  int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double ih = 1.0 / g.h;
  if (wave < 3) {
    const int d = wave;
    const int bx = 4 + (d == 0), by = 4 + (d == 1), bz = 4 + (d == 2);
    const int la = lane >> 4, lb = (lane >> 2) & 3, lc = lane & 3;
    const bool lane_ok = la < W && lb < W && lc < W;
    for (int a = -1; a <= 1; ++a) {
      int u0 = nbr(T0, a, nt0, g.bc0);
      if (u0 < 0) continue;
      for (int b = -1; b <= 1; ++b) {
        int u1 = nbr(T1, b, nt1, g.bc1);
        if (u1 < 0) continue;
        for (int c = -1; c <= 1; ++c) {
          int u2 = nbr(T2, c, nt2, g.bc2);
          if (u2 < 0) continue;
          int nt = (u0 * nt1 + u1) * nt2 + u2;
          int s0 = tstart[nt], s1 = tstart[nt + 1];
          for (int p = s0; p < s1; ++p) {
            double x0 = X[3 * p], x1 = X[3 * p + 1], x2 = X[3 * p + 2];
            double f0, f1, f2;
            int i0 = support_start<KER>(x0, ih, d == 0, f0);
            int j0 = support_start<KER>(x1, ih, d == 1, f1);
            int k0 = support_start<KER>(x2, ih, d == 2, f2);
            // stencil start relative to the tile origin (minimum image on periodic axes)
            int li0 = i0 - 4 * T0, lj0 = j0 - 4 * T1, lk0 = k0 - 4 * T2;
            if (!g.bc0) li0 = wrapi(li0 + g.n0 / 2, g.n0) - g.n0 / 2;
            if (!g.bc1) lj0 = wrapi(lj0 + g.n1 / 2, g.n1) - g.n1 / 2;
            if (!g.bc2) lk0 = wrapi(lk0 + g.n2 / 2, g.n2) - g.n2 / 2;
            if (li0 + W <= 0 || li0 >= bx || lj0 + W <= 0 || lj0 >= by || lk0 + W <= 0 || lk0 >= bz) continue;
            int li = li0 + la, lj = lj0 + lb, lk = lk0 + lc;
            if (lane_ok && li >= 0 && li < bx && lj >= 0 && lj < by && lk >= 0 && lk < bz) {
              double w = phi<KER>(f0 - (double)(i0 + la)) * phi<KER>(f1 - (double)(j0 + lb)) *
                         phi<KER>(f2 - (double)(k0 + lc));
              acc[d][(li * by + lj) * bz + lk] += w * q[3 * p + d];
            }
          }
        }
      }
    }
  }
  __syncthreads();
  long long N = 2 * g.half;
  if (DIV) {
    if (threadIdx.x < 64) {
      int ci = threadIdx.x >> 4, cj = (threadIdx.x >> 2) & 3, ck = threadIdx.x & 3;
      double dv = 0.0;
      // component 0: box 5x4x4
      dv += acc[0][((ci + 1) * 4 + cj) * 4 + ck] - acc[0][(ci * 4 + cj) * 4 + ck];
      // component 1: box 4x5x4
      dv += acc[1][(ci * 5 + cj + 1) * 4 + ck] - acc[1][(ci * 5 + cj) * 4 + ck];
      // component 2: box 4x4x5
      dv += acc[2][(ci * 4 + cj) * 5 + ck + 1] - acc[2][(ci * 4 + cj) * 5 + ck];
      int gi = 4 * T0 + ci, gj = 4 * T1 + cj, gk = 4 * T2 + ck;
      out[sidx(g, gi, gj, gk)] += alpha * dv * ih;
    }
  } else {
    if (threadIdx.x < 192) {
      int d = threadIdx.x >> 6, t = threadIdx.x & 63;
      int ci = t >> 4, cj = (t >> 2) & 3, ck = t & 3;
      int by = 4 + (d == 1), bz = 4 + (d == 2);
      int gi = 4 * T0 + ci, gj = 4 * T1 + cj, gk = 4 * T2 + ck;
      out[d * N + sidx(g, gi, gj, gk)] += alpha * acc[d][(ci * by + cj) * bz + ck];
    }
  }
}

hipError_t band_apply(int ker, bool div, const Geo &g, int nt0, int nt1, int nt2, int nactive, const int *active,
                      const int *tstart, const double *X, const double *q, double alpha, double *out,
                      hipStream_t s) {
  if (nactive == 0) return hipSuccess;
  dim3 gr(nactive), bl(256);
  if (ker == KER_PESKIN4) {
    if (div)
      hipLaunchKernelGGL((k_band<KER_PESKIN4, true>), gr, bl, 0, s, g, nt0, nt1, nt2, active, tstart, X, q, alpha, out);
    else
      hipLaunchKernelGGL((k_band<KER_PESKIN4, false>), gr, bl, 0, s, g, nt0, nt1, nt2, active, tstart, X, q, alpha, out);
  } else {
    if (div)
      hipLaunchKernelGGL((k_band<KER_ROMA3, true>), gr, bl, 0, s, g, nt0, nt1, nt2, active, tstart, X, q, alpha, out);
    else
      hipLaunchKernelGGL((k_band<KER_ROMA3, false>), gr, bl, 0, s, g, nt0, nt1, nt2, active, tstart, X, q, alpha, out);
  }
  return hipGetLastError();
}

}  // namespace ibs
