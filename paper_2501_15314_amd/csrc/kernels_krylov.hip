// Vector kernels of the flexible GMRES outer loop: fused multi-dot products
// (classical Gram-Schmidt), fused orthogonalisation update with the norm of
// the result, the solution update x += Z y, and small helpers.  All
// reductions are deterministic: per-thread partials in a fixed grid-stride
// order, fixed butterfly inside the wavefront, fixed order across the
// wavefronts of a block, then a second kernel that sums the per-block
// partials in a fixed order.
#include <hip/hip_ext.h>

#include "internal.h"

namespace ibs {

constexpr int RED_BLOCKS = 1024;
constexpr int RED_T = 256;
constexpr int MD_MAX = 24;  // dot products per multidot pass
int red_blocks() { return RED_BLOCKS; }

__device__ __forceinline__ double block_reduce(double v, double *sh) {
  v = wave_sum(v);
  int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) sh[w] = v;
  __syncthreads();
  double r = ((sh[0] + sh[1]) + sh[2]) + sh[3];
  __syncthreads();
  return r;
}

// Two consecutive entries per thread per grid-stride step (n is even: every
// vector here is a whole split-layout grid array); the basis V may be stored
// in float32 (the FP32-MG form) or float64, products accumulate in float64.
template <typename TV>
__device__ __forceinline__ void ld_pair(const TV *p, double &a, double &b) {
  if (sizeof(TV) == 4) {
    float2 f = *(const float2 *)p;
    a = f.x;
    b = f.y;
  } else {
    double2 f = *(const double2 *)p;
    a = f.x;
    b = f.y;
  }
}

// The number of vectors is a template parameter (1 .. MD_MAX): the loop over
// them unrolls completely, so every load of a grid-stride step is issued
// before the first product waits on one
template <typename TV, typename TW, int NV>
__global__ void __launch_bounds__(RED_T) k_multidot(const TW *w, const TV *V, long long stride, long long n,
                                                    double *part) {
  double acc[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) acc[i] = 0.0;
  const long long n2 = n >> 1;
  for (long long t = (long long)blockIdx.x * RED_T + threadIdx.x; t < n2; t += (long long)gridDim.x * RED_T) {
    double2 wv;
    ld_pair(w + 2 * t, wv.x, wv.y);
    double a[NV], b[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) ld_pair(V + i * stride + 2 * t, a[i], b[i]);
#pragma unroll
    for (int i = 0; i < NV; ++i) acc[i] += wv.x * a[i] + wv.y * b[i];
  }
  __shared__ double sh[4][NV];
  int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    double v = wave_sum(acc[i]);
    if (ln == 0) sh[wv][i] = v;
  }
  __syncthreads();
  if (threadIdx.x < NV)
    part[(long long)blockIdx.x * NV + threadIdx.x] =
        ((sh[0][threadIdx.x] + sh[1][threadIdx.x]) + sh[2][threadIdx.x]) + sh[3][threadIdx.x];
}

template <typename TV, typename TW, int NV>
static void launch_multidot(const TW *w, const TV *V, long long stride, int nv, long long n, double *part,
                            hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  if constexpr (NV > 1) {
    if (nv < NV) return launch_multidot<TV, TW, NV - 1>(w, V, stride, nv, n, part, s, e0, e1);
  }
  hipExtLaunchKernelGGL((k_multidot<TV, TW, NV>), dim3(RED_BLOCKS), dim3(RED_T), 0, s, e0, e1, 0, w, V, stride, n,
                        part);
}

template <typename TV, typename TW>
hipError_t multidot(const TW *w, const TV *V, long long stride, int nv, long long n, double *part,
                    hipStream_t s) {
  // the events of an enclosing ProbeExt, if any: stamped by the one launch,
  // or recorded around the launches when there are several
  hipEvent_t e0, e1;
  probe_ext_take(&e0, &e1);
  if ((n & 1) || (stride & 1)) return hipErrorInvalidValue;
  const bool one = nv <= MD_MAX;
  if (!one && e0) hipEventRecord(e0, s);
  // part layout: [blk][nv]; chunks of MD_MAX vectors write consecutive column groups
  for (int c0 = 0; c0 < nv; c0 += MD_MAX) {
    int nc = nv - c0 < MD_MAX ? nv - c0 : MD_MAX;
    launch_multidot<TV, TW, MD_MAX>(w, V + c0 * stride, stride, nc, n, part + (long long)c0 * RED_BLOCKS, s,
                                    one ? e0 : nullptr, one ? e1 : nullptr);
  }
  if (!one && e1) hipEventRecord(e1, s);
  return hipGetLastError();
}

// vout = (TV)(w - sum_i sig2_i g_i V_i) and partial |vout|^2 (vout may alias
// w when TV is double): the next unnormalised basis vector in one pass
// NV > 0: that many vectors, unrolled (all loads of a step issued together);
// NV = 0: nv vectors in a runtime loop
template <typename TV, typename TW, int NV>
__global__ void __launch_bounds__(RED_T) k_update_cast_norm(TV *vout, const TW *w, const TV *V, long long stride,
                                                            int nv, const double *g, KCoef sig2, long long n,
                                                            double *part) {
  __shared__ double hs[64];
  __shared__ double sh[4];
  for (int i = threadIdx.x; i < nv; i += RED_T) hs[i] = sig2.v[i] * g[i];
  __syncthreads();
  double acc = 0.0;
  const long long n2 = n >> 1;
  for (long long t = (long long)blockIdx.x * RED_T + threadIdx.x; t < n2; t += (long long)gridDim.x * RED_T) {
    double2 v;
    ld_pair(w + 2 * t, v.x, v.y);
    if constexpr (NV > 0) {
      double a[NV], b[NV];
#pragma unroll
      for (int i = 0; i < NV; ++i) ld_pair(V + i * stride + 2 * t, a[i], b[i]);
#pragma unroll
      for (int i = 0; i < NV; ++i) {
        v.x -= hs[i] * a[i];
        v.y -= hs[i] * b[i];
      }
    } else {
      for (int i = 0; i < nv; ++i) {
        double a, b;
        ld_pair(V + i * stride + 2 * t, a, b);
        v.x -= hs[i] * a;
        v.y -= hs[i] * b;
      }
    }
    if (sizeof(TV) == 4) {
      const float2 f = make_float2((float)v.x, (float)v.y);
      *(float2 *)(vout + 2 * t) = f;
      acc += (double)f.x * (double)f.x + (double)f.y * (double)f.y;
    } else {
      *(double2 *)(vout + 2 * t) = v;
      acc += v.x * v.x + v.y * v.y;
    }
  }
  acc = block_reduce(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

template <typename TV, typename TW, int NV>
static void launch_update(TV *vout, const TW *w, const TV *V, long long stride, int nv, const double *g,
                          const KCoef &sig2, long long n, double *part, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  if constexpr (NV > 1) {
    if (nv < NV) return launch_update<TV, TW, NV - 1>(vout, w, V, stride, nv, g, sig2, n, part, s, e0, e1);
  }
  hipExtLaunchKernelGGL((k_update_cast_norm<TV, TW, NV>), dim3(RED_BLOCKS), dim3(RED_T), 0, s, e0, e1, 0, vout, w,
                        V, stride, nv, g, sig2, n, part);
}

template <typename TV, typename TW>
hipError_t update_cast_norm(TV *vout, const TW *w, const TV *V, long long stride, int nv, const double *g,
                            const KCoef &sig2, long long n, double *part, hipStream_t s) {
  hipEvent_t e0, e1;
  probe_ext_take(&e0, &e1);  // the events of an enclosing ProbeExt, if any
  if (nv < 1 || nv > 64 || (n & 1) || (stride & 1)) return hipErrorInvalidValue;
  if (nv <= MD_MAX)
    launch_update<TV, TW, MD_MAX>(vout, w, V, stride, nv, g, sig2, n, part, s, e0, e1);
  else
    hipExtLaunchKernelGGL((k_update_cast_norm<TV, TW, 0>), dim3(RED_BLOCKS), dim3(RED_T), 0, s, e0, e1, 0, vout, w, V,
                          stride, nv, g, sig2, n, part);
  return hipGetLastError();
}
template hipError_t update_cast_norm<float, double>(float *, const double *, const float *, long long, int,
                                                    const double *, const KCoef &, long long, double *, hipStream_t);
template hipError_t update_cast_norm<float, float>(float *, const float *, const float *, long long, int,
                                                   const double *, const KCoef &, long long, double *, hipStream_t);
template hipError_t update_cast_norm<double, double>(double *, const double *, const double *, long long, int,
                                                     const double *, const KCoef &, long long, double *, hipStream_t);
template hipError_t multidot<float, double>(const double *, const float *, long long, int, long long, double *,
                                            hipStream_t);
template hipError_t multidot<float, float>(const float *, const float *, long long, int, long long, double *,
                                           hipStream_t);
template hipError_t multidot<double, double>(const double *, const double *, long long, int, long long, double *,
                                             hipStream_t);

// out[i] = sum_b part[b][i] over nblk blocks (chunked layout of multidot);
// with host != null the sums are also written to that pinned host buffer
// (read by the host after the stream is synchronised, no separate copy)
__global__ void __launch_bounds__(RED_T) k_finalize(const double *part, int nblk, int nv, double *out,
                                                    double *host) {
  int i = blockIdx.x;
  int c0 = (i / MD_MAX) * MD_MAX;
  int nc = nv - c0 < MD_MAX ? nv - c0 : MD_MAX;
  const double *pc = part + (long long)c0 * nblk;
  int col = i - c0;
  double v = 0.0;
  for (int b = threadIdx.x; b < nblk; b += RED_T) v += pc[(long long)b * nc + col];
  __shared__ double sh[4];
  v = block_reduce(v, sh);
  if (threadIdx.x == 0) {
    out[i] = v;
    if (host) {
      host[i] = v;
      __threadfence_system();
    }
  }
}
hipError_t finalize(const double *part, int nblk, int nv, double *out, hipStream_t s, double *host) {
  hipLaunchKernelGGL(k_finalize, dim3(nv), dim3(RED_T), 0, s, part, nblk, nv, out, host);
  return hipGetLastError();
}

// w -= sum_i h_i V_i ; partial |w|^2
template <typename TV>
__global__ void __launch_bounds__(RED_T) k_update_norm(double *w, const TV *V, long long stride, int nv,
                                                       const double *hcoef, long long n, double *part) {
  __shared__ double hs[64];
  __shared__ double sh[4];
  for (int i = threadIdx.x; i < nv; i += RED_T) hs[i] = hcoef[i];
  __syncthreads();
  double acc = 0.0;
  const long long n2 = n >> 1;
  for (long long t = (long long)blockIdx.x * RED_T + threadIdx.x; t < n2; t += (long long)gridDim.x * RED_T) {
    double2 v = *(double2 *)(w + 2 * t);
    for (int i = 0; i < nv; ++i) {
      double a, b;
      ld_pair(V + i * stride + 2 * t, a, b);
      v.x -= hs[i] * a;
      v.y -= hs[i] * b;
    }
    *(double2 *)(w + 2 * t) = v;
    acc += v.x * v.x + v.y * v.y;
  }
  acc = block_reduce(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = acc;
}
template <typename TV>
hipError_t update_norm(double *w, const TV *V, long long stride, int nv, const double *hcoef, long long n,
                       double *part, hipStream_t s) {
  if (nv > 64 || (n & 1) || (stride & 1)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_update_norm<TV>, dim3(RED_BLOCKS), dim3(RED_T), 0, s, w, V, stride, nv, hcoef, n, part);
  return hipGetLastError();
}
template hipError_t update_norm<float>(double *, const float *, long long, int, const double *, long long,
                                       double *, hipStream_t);
template hipError_t update_norm<double>(double *, const double *, long long, int, const double *, long long,
                                        double *, hipStream_t);

__global__ void k_scale_copy(double *y, const double *x, long long n, double a) {
  for (long long t = (long long)blockIdx.x * RED_T + threadIdx.x; t < n; t += (long long)gridDim.x * RED_T)
    y[t] = a * x[t];
}
hipError_t scale_inplace(double *x, long long n, double alpha, hipStream_t s) {
  hipLaunchKernelGGL(k_scale_copy, dim3(RED_BLOCKS * 4), dim3(RED_T), 0, s, x, x, n, alpha);
  return hipGetLastError();
}
hipError_t scale_copy(double *y, const double *x, long long n, double alpha, hipStream_t s) {
  hipLaunchKernelGGL(k_scale_copy, dim3(RED_BLOCKS * 4), dim3(RED_T), 0, s, y, x, n, alpha);
  return hipGetLastError();
}

// x = (first ? 0 : x) + sum_j y_j Z_j; with part != null also the per-block
// partial sums of the new x (part[blockIdx.x], SOL_BLOCKS blocks), from
// which the mean of the final solution is formed without another pass
constexpr int SOL_BLOCKS = RED_BLOCKS * 4;
int sol_blocks() { return SOL_BLOCKS; }
template <typename T>
__global__ void __launch_bounds__(RED_T) k_sol_update(double *x, const T *Z, long long stride, int nz, KCoef y,
                                                      long long n, bool first, double *part) {
  __shared__ double ys[64];
  __shared__ double sh[4];
  for (int i = threadIdx.x; i < nz; i += RED_T) ys[i] = y.v[i];
  __syncthreads();
  double acc = 0.0;
  for (long long t = (long long)blockIdx.x * RED_T + threadIdx.x; t < n; t += (long long)gridDim.x * RED_T) {
    double v = first ? 0.0 : x[t];
    for (int j = 0; j < nz; ++j) v += ys[j] * (double)Z[j * stride + t];
    x[t] = v;
    acc += v;
  }
  if (part) {
    acc = block_reduce(acc, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = acc;
  }
}
template <typename T>
hipError_t sol_update(double *x, const T *Z, long long stride, int nz, const KCoef &y, long long n,
                      hipStream_t s, bool first, double *part) {
  if (nz > 64) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_sol_update<T>, dim3(SOL_BLOCKS), dim3(RED_T), 0, s, x, Z, stride, nz, y, n, first, part);
  return hipGetLastError();
}
template hipError_t sol_update<float>(double *, const float *, long long, int, const KCoef &, long long,
                                      hipStream_t, bool, double *);
template hipError_t sol_update<double>(double *, const double *, long long, int, const KCoef &, long long,
                                       hipStream_t, bool, double *);

__global__ void k_axpby(double *y, const double *x, long long n, double a, double b) {
  for (long long t = (long long)blockIdx.x * RED_T + threadIdx.x; t < n; t += (long long)gridDim.x * RED_T)
    y[t] = a * x[t] + b * y[t];
}
hipError_t axpby(double *y, const double *x, long long n, double a, double b, hipStream_t s) {
  hipLaunchKernelGGL(k_axpby, dim3(RED_BLOCKS * 4), dim3(RED_T), 0, s, y, x, n, a, b);
  return hipGetLastError();
}

__global__ void k_add_scalar(double *x, long long n, const double *ds, double mult) {
  double a = mult * ds[0];
  for (long long t = (long long)blockIdx.x * RED_T + threadIdx.x; t < n; t += (long long)gridDim.x * RED_T)
    x[t] += a;
}
hipError_t add_scalar_dev(double *x, long long n, const double *dscalar, double mult, hipStream_t s) {
  hipLaunchKernelGGL(k_add_scalar, dim3(RED_BLOCKS * 4), dim3(RED_T), 0, s, x, n, dscalar, mult);
  return hipGetLastError();
}

// r = b - ax ; partial |r|^2
__global__ void __launch_bounds__(RED_T) k_sub_norm(double *r, const double *b, const double *ax, long long n,
                                                    double *part) {
  __shared__ double sh[4];
  double acc = 0.0;
  for (long long t = (long long)blockIdx.x * RED_T + threadIdx.x; t < n; t += (long long)gridDim.x * RED_T) {
    double v = b[t] - ax[t];
    r[t] = v;
    acc += v * v;
  }
  acc = block_reduce(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = acc;
}
hipError_t sub_mul(double *r, const double *b, const double *ax, long long n, double *part, hipStream_t s) {
  hipLaunchKernelGGL(k_sub_norm, dim3(RED_BLOCKS), dim3(RED_T), 0, s, r, b, ax, n, part);
  return hipGetLastError();
}

// y = (TV)(b - mult bsum[0] - ax) (ax or bsum null: that term absent) ;
// partial |.|^2 of the float64 value: a Krylov cycle's first (unnormalised)
// basis vector together with the norm of the residual it stands for (bsum:
// the sum of a right-hand side whose mean is removed on the fly)
template <typename TV>
__global__ void __launch_bounds__(RED_T) k_sub_cast_norm(TV *y, const double *b, const double *ax, long long n,
                                                         double *part, const double *bsum, double mult) {
  __shared__ double sh[4];
  const double shift = bsum ? mult * bsum[0] : 0.0;
  double acc = 0.0;
  // two consecutive entries per thread and step (16-byte loads), as in the
  // Gram-Schmidt kernels; an odd last entry is taken by thread 0 of block 0
  const long long n2 = n >> 1;
  for (long long t = (long long)blockIdx.x * RED_T + threadIdx.x; t < n2; t += (long long)gridDim.x * RED_T) {
    const double2 bv = *(const double2 *)(b + 2 * t);
    double v0 = bv.x - shift, v1 = bv.y - shift;
    if (ax) {
      const double2 av = *(const double2 *)(ax + 2 * t);
      v0 -= av.x;
      v1 -= av.y;
    }
    if (sizeof(TV) == 4) {
      *(float2 *)(y + 2 * t) = make_float2((float)v0, (float)v1);
    } else {
      *(double2 *)(y + 2 * t) = make_double2(v0, v1);
    }
    acc += v0 * v0;
    acc += v1 * v1;
  }
  if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
    double v = b[n - 1] - shift;
    if (ax) v -= ax[n - 1];
    y[n - 1] = (TV)v;
    acc += v * v;
  }
  acc = block_reduce(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = acc;
}
template <typename TV>
hipError_t sub_cast_norm(TV *y, const double *b, const double *ax, long long n, double *part, hipStream_t s,
                         const double *bsum, double mult) {
  // the paired accesses need 16-byte aligned vectors (8-byte for a float32 y)
  if (((uintptr_t)b | (uintptr_t)ax) % 16 || (uintptr_t)y % (2 * sizeof(TV))) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_sub_cast_norm<TV>, dim3(RED_BLOCKS), dim3(RED_T), 0, s, y, b, ax, n, part, bsum, mult);
  return hipGetLastError();
}
template hipError_t sub_cast_norm<float>(float *, const double *, const double *, long long, double *, hipStream_t,
                                         const double *, double);
template hipError_t sub_cast_norm<double>(double *, const double *, const double *, long long, double *,
                                          hipStream_t, const double *, double);

__global__ void __launch_bounds__(RED_T) k_dot2(const double *a, const double *b, long long n, double *part) {
  __shared__ double sh[4];
  double acc = 0.0;
  for (long long t = (long long)blockIdx.x * RED_T + threadIdx.x; t < n; t += (long long)gridDim.x * RED_T)
    acc += b ? a[t] * b[t] : a[t];
  acc = block_reduce(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = acc;
}
// the same with two consecutive entries per thread and step (16-byte loads;
// an odd last entry is taken by thread 0 of block 0)
__global__ void __launch_bounds__(RED_T) k_dot2_pairs(const double *a, const double *b, long long n, double *part) {
  __shared__ double sh[4];
  double acc = 0.0;
  const long long n2 = n >> 1;
  for (long long t = (long long)blockIdx.x * RED_T + threadIdx.x; t < n2; t += (long long)gridDim.x * RED_T) {
    const double2 av = *(const double2 *)(a + 2 * t);
    if (b) {
      const double2 bv = *(const double2 *)(b + 2 * t);
      acc += av.x * bv.x;
      acc += av.y * bv.y;
    } else {
      acc += av.x;
      acc += av.y;
    }
  }
  if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) acc += b ? a[n - 1] * b[n - 1] : a[n - 1];
  acc = block_reduce(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = acc;
}
hipError_t dot2(const double *a, const double *b, long long n, double *part, hipStream_t s) {
  if (((uintptr_t)a | (uintptr_t)b) % 16 == 0)
    hipLaunchKernelGGL(k_dot2_pairs, dim3(RED_BLOCKS), dim3(RED_T), 0, s, a, b, n, part);
  else
    hipLaunchKernelGGL(k_dot2, dim3(RED_BLOCKS), dim3(RED_T), 0, s, a, b, n, part);
  return hipGetLastError();
}

// BiCGStab vector updates: y = ca a + cb b (+ cc c), with per-block partial
// sums of y.y (nd >= 1) and y.d (nd = 2), two per block in part.  y may
// alias a, b or c (elementwise).
__global__ void __launch_bounds__(RED_T) k_lincomb(double *y, const double *a, double ca, const double *b, double cb,
                                                   const double *c, double cc, const double *d, int nd, long long n,
                                                   double *part) {
  __shared__ double sh[4];
  double s0 = 0.0, s1 = 0.0;
  for (long long t = (long long)blockIdx.x * RED_T + threadIdx.x; t < n; t += (long long)gridDim.x * RED_T) {
    double v = ca * a[t] + cb * b[t];
    if (c) v += cc * c[t];
    y[t] = v;
    s0 += v * v;
    if (nd == 2) s1 += v * d[t];
  }
  if (nd == 0) return;
  s0 = block_reduce(s0, sh);
  s1 = block_reduce(s1, sh);
  if (threadIdx.x == 0) {
    part[2LL * blockIdx.x] = s0;
    part[2LL * blockIdx.x + 1] = s1;
  }
}
hipError_t lincomb(double *y, const double *a, double ca, const double *b, double cb, const double *c, double cc,
                   const double *d, int nd, long long n, double *part, hipStream_t s) {
  hipLaunchKernelGGL(k_lincomb, dim3(RED_BLOCKS), dim3(RED_T), 0, s, y, a, ca, b, cb, c, cc, d, nd, n, part);
  return hipGetLastError();
}

// a.b0 and a.b1, two partial sums per block in part
__global__ void __launch_bounds__(RED_T) k_dots2(const double *a, const double *b0, const double *b1, long long n,
                                                 double *part) {
  __shared__ double sh[4];
  double s0 = 0.0, s1 = 0.0;
  for (long long t = (long long)blockIdx.x * RED_T + threadIdx.x; t < n; t += (long long)gridDim.x * RED_T) {
    const double av = a[t];
    s0 += av * b0[t];
    s1 += av * b1[t];
  }
  s0 = block_reduce(s0, sh);
  s1 = block_reduce(s1, sh);
  if (threadIdx.x == 0) {
    part[2LL * blockIdx.x] = s0;
    part[2LL * blockIdx.x + 1] = s1;
  }
}
hipError_t dots2(const double *a, const double *b0, const double *b1, long long n, double *part, hipStream_t s) {
  hipLaunchKernelGGL(k_dots2, dim3(RED_BLOCKS), dim3(RED_T), 0, s, a, b0, b1, n, part);
  return hipGetLastError();
}

// Step diagnostics in one pass each: sum |a| and sum |b| (two per block), and
// the sums of squares of up to three vectors of different lengths (three per
// block; a null vector contributes 0).
__global__ void __launch_bounds__(RED_T) k_abs_sums(const double *a, const double *b, long long n, double *part) {
  __shared__ double sh[4];
  double s0 = 0.0, s1 = 0.0;
  for (long long t = (long long)blockIdx.x * RED_T + threadIdx.x; t < n; t += (long long)gridDim.x * RED_T) {
    s0 += fabs(a[t]);
    s1 += fabs(b[t]);
  }
  s0 = block_reduce(s0, sh);
  s1 = block_reduce(s1, sh);
  if (threadIdx.x == 0) {
    part[2LL * blockIdx.x] = s0;
    part[2LL * blockIdx.x + 1] = s1;
  }
}
hipError_t abs_sums(const double *a, const double *b, long long n, double *part, hipStream_t s) {
  hipLaunchKernelGGL(k_abs_sums, dim3(RED_BLOCKS), dim3(RED_T), 0, s, a, b, n, part);
  return hipGetLastError();
}

__global__ void __launch_bounds__(RED_T) k_sumsq3(const double *a, long long na, const double *b, long long nb,
                                                  const double *c, long long nc, double *part) {
  __shared__ double sh[4];
  double s[3] = {0.0, 0.0, 0.0};
  const double *v[3] = {a, b, c};
  const long long nn[3] = {a ? na : 0, b ? nb : 0, c ? nc : 0};
#pragma unroll
  for (int q = 0; q < 3; ++q)
    for (long long t = (long long)blockIdx.x * RED_T + threadIdx.x; t < nn[q]; t += (long long)gridDim.x * RED_T)
      s[q] += v[q][t] * v[q][t];
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const double r = block_reduce(s[q], sh);
    if (threadIdx.x == 0) part[3LL * blockIdx.x + q] = r;
  }
}
hipError_t sumsq3(const double *a, long long na, const double *b, long long nb, const double *c, long long nc,
                  double *part, hipStream_t s) {
  hipLaunchKernelGGL(k_sumsq3, dim3(RED_BLOCKS), dim3(RED_T), 0, s, a, na, b, nb, c, nc, part);
  return hipGetLastError();
}

}  // namespace ibs
