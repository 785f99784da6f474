// Exact pseudo-inverse of the pressure Laplacian by fast diagonalisation in
// float64: the direct solve of paper Sec. 4.2 (Lynch et al.), which factors
// L once and applies L^-1 exactly in every Krylov iteration.
//
// L = Lx (x) I (x) I + I (x) Ly (x) I + I (x) I (x) Lz is a Kronecker sum of
// 1-D second-difference matrices, each diagonalised by an orthonormal
// eigenbasis Q_a (DCT-II vectors on a wall axis, the real Fourier basis on a
// periodic one, eigenvalues lambda_a).  So
//     L^+ v = Q diag(1 / (lx + ly + lz)) Q^T v,   Q = Qx (x) Qy (x) Qz,
// with the constant mode (all three eigenvalues zero) mapped to zero.  Q^T v
// and Q w are three mode products each: the n x n matrix applied along one
// axis of the n0 x n1 x n2 array.  A mode product is a (batched) dense
// matrix product, computed here in float64 on the vector units from LDS
// tiles (2 n N flops per product, 12 n N per application).
#include "internal.h"

namespace ibs {

constexpr int MP_T = 64;  // output tile: 64 values of the transformed index x 64 lines
constexpr int MP_K = 16;  // summation step

// Mode product along one axis of an array viewed as [P][n][R]:
//     out[p][k][r] = sum_m M[k][m] in[p][m][r],   M row-major n x n.
// LAST (R == 1, the contiguous axis): the lines are the rows in[p][0..n) and
// the tile runs over 64 of them.  With lam (x transform only, P == 1) the
// result is scaled by 1 / (lx[k] + ly[j] + lz[i]) for r = j n2 + i, and the
// all-zero mode set to 0.
template <bool LAST>
__global__ void __launch_bounds__(256) k_mode(const double *__restrict__ M, const double *__restrict__ in,
                                              double *__restrict__ out, int n, long long P, long long R,
                                              const double *__restrict__ lx, const double *__restrict__ ly,
                                              const double *__restrict__ lz, int n1, int n2) {
  __shared__ double Ms[MP_K][MP_T + 1];  // [m][k]
  __shared__ double Xs[MP_K][MP_T + 1];  // [m][line]
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  const int k0 = blockIdx.y * MP_T;
  const long long l0 = (long long)blockIdx.x * MP_T;  // first line (r, or p when LAST)
  const long long p = LAST ? 0 : blockIdx.z;
  double acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
  const long long nlines = LAST ? P : R;
  for (int m0 = 0; m0 < n; m0 += MP_K) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + 256 * q;
      const int kk = e >> 4, mm = e & 15;
      const int k = k0 + kk, m = m0 + mm;
      Ms[mm][kk] = (k < n && m < n) ? M[(long long)k * n + m] : 0.0;
      if (LAST) {
        const long long pp = l0 + kk;  // 64 lines x 16 m, m fastest
        Xs[mm][kk] = (pp < P && m < n) ? in[pp * n + m] : 0.0;
      } else {
        const int mr = e >> 6, rr = e & 63;  // 16 m x 64 r, r fastest
        const long long r = l0 + rr;
        const int mx = m0 + mr;
        Xs[mr][rr] = (r < R && mx < n) ? in[(p * n + mx) * R + r] : 0.0;
      }
    }
    __syncthreads();
#pragma unroll
    for (int mm = 0; mm < MP_K; ++mm) {
      double a[4], b[4];
      if (LAST) {
        // thread: k = k0 + tx + 16 j, line = l0 + 4 ty + i
#pragma unroll
        for (int j = 0; j < 4; ++j) a[j] = Ms[mm][tx + 16 * j];
#pragma unroll
        for (int i = 0; i < 4; ++i) b[i] = Xs[mm][4 * ty + i];
      } else {
        // thread: k = k0 + 4 ty + i, line r = l0 + tx + 16 j
#pragma unroll
        for (int i = 0; i < 4; ++i) a[i] = Ms[mm][4 * ty + i];
#pragma unroll
        for (int j = 0; j < 4; ++j) b[j] = Xs[mm][tx + 16 * j];
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fma(LAST ? a[j] : a[i], LAST ? b[i] : b[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (LAST) {
        const int k = k0 + tx + 16 * j;
        const long long pp = l0 + 4 * ty + i;
        if (k < n && pp < nlines) out[pp * n + k] = acc[i][j];
      } else {
        const int k = k0 + 4 * ty + i;
        const long long r = l0 + tx + 16 * j;
        if (k < n && r < nlines) {
          double v = acc[i][j];
          if (lx) {
            const int jj = (int)(r / n2), ii = (int)(r - (long long)jj * n2);
            const double lam = lx[k] + ly[jj] + lz[ii];
            v = lam > 0.0 ? v / lam : 0.0;
          }
          out[(p * n + k) * R + r] = v;
        }
      }
    }
  (void)n1;
}

namespace {
hipError_t mode(bool last, const double *M, const double *in, double *out, int n, long long P, long long R,
                const double *lx, const double *ly, const double *lz, int n1, int n2, hipStream_t s) {
  const long long lines = last ? P : R;
  dim3 grid((unsigned)((lines + MP_T - 1) / MP_T), (unsigned)((n + MP_T - 1) / MP_T), last ? 1u : (unsigned)P);
  if (last)
    hipLaunchKernelGGL(k_mode<true>, grid, dim3(256), 0, s, M, in, out, n, P, R, lx, ly, lz, n1, n2);
  else
    hipLaunchKernelGGL(k_mode<false>, grid, dim3(256), 0, s, M, in, out, n, P, R, lx, ly, lz, n1, n2);
  return hipGetLastError();
}
}  // namespace

size_t fdx_blob_doubles(const int n[3]) {
  return 2 * ((size_t)n[0] * n[0] + (size_t)n[1] * n[1] + (size_t)n[2] * n[2]) + n[0] + n[1] + n[2];
}

// blob = [Qx^T, Qy^T, Qz^T, Qx, Qy, Qz, lx, ly, lz] (row-major) from the
// eigen-decomposition q = [Qx, Qy, Qz, lx, ly, lz] of coarse_fd_build, whose
// Q_a[i][c] is eigenvector c at grid index i.
void fdx_blob_pack(const int n[3], const double *q, double *blob) {
  const double *qa = q;
  double *fwd = blob;
  double *bwd = blob + (size_t)n[0] * n[0] + (size_t)n[1] * n[1] + (size_t)n[2] * n[2];
  for (int a = 0; a < 3; ++a) {
    const int na = n[a];
    for (int i = 0; i < na; ++i)
      for (int c = 0; c < na; ++c) {
        fwd[(size_t)c * na + i] = qa[(size_t)i * na + c];  // M[k = c][m = i] = Q[i][c]
        bwd[(size_t)i * na + c] = qa[(size_t)i * na + c];  // M[k = i][m = c] = Q[i][c]
      }
    qa += (size_t)na * na;
    fwd += (size_t)na * na;
    bwd += (size_t)na * na;
  }
  const double *lam = q + (size_t)n[0] * n[0] + (size_t)n[1] * n[1] + (size_t)n[2] * n[2];
  for (int a = 0; a < n[0] + n[1] + n[2]; ++a) bwd[a] = lam[a];
}

hipError_t fdx_precond(const Geo &g, const double *v, double *z, double *w1, double *w2, const double *blob,
                       hipStream_t s) {
  const int n0 = g.n0, n1 = g.n1, n2 = g.n2;
  const double *Qxt = blob, *Qyt = Qxt + (size_t)n0 * n0, *Qzt = Qyt + (size_t)n1 * n1;
  const double *Qx = Qzt + (size_t)n2 * n2, *Qy = Qx + (size_t)n0 * n0, *Qz = Qy + (size_t)n1 * n1;
  const double *lx = Qz + (size_t)n2 * n2, *ly = lx + n0, *lz = ly + n1;
  const long long rows = (long long)n0 * n1;
  hipError_t e;
  if ((e = to_natural(g, 1, v, w1, s))) return e;
  // forward: z, y, then x with the division by the eigenvalues
  if ((e = mode(true, Qzt, w1, w2, n2, rows, 1, nullptr, nullptr, nullptr, n1, n2, s))) return e;
  if ((e = mode(false, Qyt, w2, w1, n1, n0, n2, nullptr, nullptr, nullptr, n1, n2, s))) return e;
  if ((e = mode(false, Qxt, w1, w2, n0, 1, (long long)n1 * n2, lx, ly, lz, n1, n2, s))) return e;
  // back: x, y, z
  if ((e = mode(false, Qx, w2, w1, n0, 1, (long long)n1 * n2, nullptr, nullptr, nullptr, n1, n2, s))) return e;
  if ((e = mode(false, Qy, w1, w2, n1, n0, n2, nullptr, nullptr, nullptr, n1, n2, s))) return e;
  if ((e = mode(true, Qz, w2, w1, n2, rows, 1, nullptr, nullptr, nullptr, n1, n2, s))) return e;
  return to_split(g, 1, w1, z, s);
}

}  // namespace ibs
