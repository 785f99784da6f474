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
// therefore zero; only the four red children contribute.
template <typename T, typename TB>
__global__ void k_restrict(Geo gf, const T *xf, const TB *bf, Geo gc, T *bc) {
  RowPos p;
  if (!row_pos(gc, p)) return;
  const int ch[4][3] = {{0, 0, 0}, {0, 1, 1}, {1, 0, 1}, {1, 1, 0}};
  T acc = T(0);
  T ih2 = (T)(1.0 / gf.h2);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    int i = 2 * p.i + ch[q][0], j = 2 * p.j + ch[q][1], k = 2 * p.k + ch[q][2];
    int m = k >> 1;
    long long e = ((long long)i * gf.n1 + j) * gf.hn2 + m;  // red plane
    T s = nb_sum(gf, xf, i, j, k, 0, m);
    int nn = cell_nnb(gf, i, j, k);
    acc += (T)bf[e] - ((T)nn * xf[e] - s) * ih2;
  }
  bc[p.e] = acc * (T)0.125;
}

// x_f += P x_c on the red fine cells only (the following black half sweep
// overwrites the black cells without reading them).
template <typename T>
__global__ void k_prolong(Geo gf, T *xf, Geo gc, const T *xc) {
  RowPos p;
  if (!row_pos1m(gf, 0, p)) return;
  int I[3][2];
  T w[3][2];
  const int xs[3] = {p.i, p.j, p.k};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    int C = xs[a] >> 1;
    int s = (xs[a] & 1) ? 1 : -1;
    int nc = geo_n(gc, a), bc = geo_bc(gc, a);
    int o = C + s;
    if (o < 0 || o >= nc) o = bc ? C : (o < 0 ? o + nc : o - nc);
    I[a][0] = C;
    I[a][1] = o;
    w[a][0] = (T)0.75;
    w[a][1] = (T)0.25;
  }
  T acc = T(0);
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int c = 0; c < 2; ++c)
        acc += w[0][a] * w[1][b] * w[2][c] * xc[sidx(gc, I[0][a], I[1][b], I[2][c])];
  xf[p.e] += acc;
}

template <typename T, typename TB>
hipError_t mg_smooth_first(const Geo &g, T *x, const TB *b, hipStream_t s) {
  MarchShape M = march_shape(g, 1);
  hipLaunchKernelGGL((k_sweep<T, TB, SW_FIRST>), M.grid, M.block, 0, s, g, x, b, 1, g.h2, 0.0, 0.0, 1.0);
  return hipGetLastError();
}
template <typename T, typename TB>
hipError_t mg_smooth(const Geo &g, T *x, const TB *b, int color, hipStream_t s) {
  MarchShape M = march_shape(g, 1);
  hipLaunchKernelGGL((k_sweep<T, TB, SW_POISSON>), M.grid, M.block, 0, s, g, x, b, color, g.h2, 0.0, 0.0, 1.0);
  return hipGetLastError();
}
template <typename T, typename TB>
hipError_t mg_restrict(const Geo &gf, const T *xf, const TB *bf, const Geo &gc, T *bc, hipStream_t s) {
  RowLaunch L = row_launch(gc, 2 * gc.n0);
  hipLaunchKernelGGL((k_restrict<T, TB>), L.grid, L.block, 0, s, gf, xf, bf, gc, bc);
  return hipGetLastError();
}
template <typename T>
hipError_t mg_prolong(const Geo &gf, T *xf, const Geo &gc, const T *xc, hipStream_t s) {
  RowLaunch L = row_launch(gf, gf.n0);
  hipLaunchKernelGGL(k_prolong<T>, L.grid, L.block, 0, s, gf, xf, gc, xc);
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

// 1 / (number of neighbours) for 0..6 neighbours
template <typename T>
__device__ __forceinline__ T inv_nn(int nn) {
  return nn == 6 ? T(1) / T(6) : nn == 5 ? T(1) / T(5) : nn == 4 ? T(0.25) : nn == 3 ? T(1) / T(3) : T(1) / T(nn);
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
  template hipError_t mg_smooth_first<T, TB>(const Geo &, T *, const TB *, hipStream_t);              \
  template hipError_t mg_smooth<T, TB>(const Geo &, T *, const TB *, int, hipStream_t);               \
  template hipError_t mg_restrict<T, TB>(const Geo &, const T *, const TB *, const Geo &, T *,         \
                                         hipStream_t);                                                 \
  template hipError_t mg_coarse<T, TB>(const Geo &, const TB *, T *, int, int, hipStream_t);                   \
  template hipError_t mg_coarse_fd<T, TB>(const Geo &, const TB *, T *, const double *, hipStream_t);
INST(float, float)
INST(float, double)
INST(double, double)
#undef INST
template hipError_t mg_prolong<float>(const Geo &, float *, const Geo &, const float *, hipStream_t);
template hipError_t mg_prolong<double>(const Geo &, double *, const Geo &, const double *, hipStream_t);

}  // namespace ibs
