// Fast-diagonalisation preconditioner: z = L^+ v on the whole grid, the
// direct solver the paper applies once per Krylov iteration (Sec. 4.1-4.2).
// On a box with one boundary type per axis, L is the Kronecker sum of three
// 1-D Laplacians with orthonormal eigenvectors Q_a and eigenvalues lam_a, so
//     z = (Qx (x) Qy (x) Qz) diag(1 / (lam_x + lam_y + lam_z)) (Qx (x) Qy (x) Qz)^T v,
// the constant mode dropped.  Each 1-D transform along an axis is a dense
// product of an n x n matrix with every grid line along that axis: six
// batched GEMMs per application, run on the matrix cores (bfloat16 operands,
// float32 accumulation; the preconditioner only has to be spectrally close to
// L^+, and FGMRES accepts its bfloat16 rounding).
//
// Each pass is C = A D with A an n x n eigenvector matrix (Q or Q^T, bfloat16,
// rows contiguous along the reduction index, read from L2) and D the grid
// lines of the pass: a workgroup stages 64 lines (n x 64, bfloat16) in LDS
// and its four wavefronts produce all n outputs of them with
// v_mfma_f32_16x16x16_bf16 (16 x 16 tiles, float32 accumulation).  The first
// and the last pass read / write the solver's red/black split layout directly.
#include <string.h>

#include "internal.h"

namespace ibs {

namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int FD_COLS = 64;  // grid lines per workgroup
constexpr int FD_T = 256;

__device__ __forceinline__ unsigned short to_bf16(float x) {
  unsigned int u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float from_bf16(unsigned short h) { return __uint_as_float((unsigned int)h << 16); }

// where the n x ncols operand D of a pass lives
enum { SRC_SPLIT = 0,  // line r = i n1 + j of a split-layout field, element k (first pass)
       SRC_LINES = 1,  // element (k, col) = src[col n + k]
       SRC_ROWS = 2 }; // element (k, col) = src[b bstride + k ld + col]
enum { DST_SPLIT = 0, DST_LINES = 1, DST_ROWS = 2, DST_ROWS_SCALED = 3 };

struct FdPass {
  int n, ncols;
  long long bstride, ld;
  const unsigned short *A;  // n x n, row-major
  const unsigned short *src;
  unsigned short *dst;
  Geo g;
  float scale;                // input scale (SRC_SPLIT) or output scale (DST_SPLIT)
  const float *lx, *ly, *lz;  // eigenvalues (DST_ROWS_SCALED)
};

template <int SRC, int DST, int MAXT, typename TI, typename TO>
__global__ void __launch_bounds__(FD_T) k_fd_pass(FdPass P, const TI *vsplit, TO *zsplit) {
  extern __shared__ unsigned short Ds[];  // [FD_COLS][ldsk]
  const int n = P.n, n16 = (n + 15) & ~15, ldsk = n16 + 4;
  const int b = blockIdx.z, col0 = blockIdx.x * FD_COLS;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  // stage D (n16 x 64, zero padded) as Ds[col][k]
  if (SRC == SRC_ROWS) {
    for (int e = tid; e < n16 * FD_COLS; e += FD_T) {
      const int k = e / FD_COLS, cc = e - k * FD_COLS, col = col0 + cc;
      unsigned short v = 0;
      if (k < n && col < P.ncols) v = P.src[b * P.bstride + (long long)k * P.ld + col];
      Ds[cc * ldsk + k] = v;
    }
  } else {
    for (int e = tid; e < n16 * FD_COLS; e += FD_T) {
      const int cc = e / n16, k = e - cc * n16, col = col0 + cc;
      unsigned short v = 0;
      if (k < n && col < P.ncols) {
        if (SRC == SRC_LINES) {
          v = P.src[(long long)col * n + k];
        } else {
          const int i = col / P.g.n1, j = col - i * P.g.n1;
          v = to_bf16(P.scale * (float)vsplit[sidx(P.g, i, j, k)]);
        }
      }
      Ds[cc * ldsk + k] = v;
    }
  }
  __syncthreads();
  const int ntiles = n16 >> 4;
  f32x4 acc[MAXT][4];
#pragma unroll
  for (int q = 0; q < MAXT; ++q)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[q][c] = f32x4{0.f, 0.f, 0.f, 0.f};
  const bf16x4 zero4 = {0, 0, 0, 0};
  for (int k0 = 0; k0 < n16; k0 += 16) {
    const int kq = k0 + 4 * (lane >> 4);
    bf16x4 bb[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) bb[c] = *(const bf16x4 *)&Ds[(16 * c + (lane & 15)) * ldsk + kq];
#pragma unroll
    for (int q = 0; q < MAXT; ++q) {
      const int t = wv + 4 * q;
      if (t < ntiles) {
        const int row = 16 * t + (lane & 15);
        const bf16x4 a = (row < n && kq < n) ? *(const bf16x4 *)&P.A[(long long)row * n + kq] : zero4;
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[q][c] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bb[c], acc[q][c], 0, 0, 0);
      }
    }
  }
  // output tile layout: lane holds column lane % 16 and rows 4 (lane / 16) + i
#pragma unroll
  for (int q = 0; q < MAXT; ++q) {
    const int t = wv + 4 * q;
    if (t >= ntiles) continue;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int col = col0 + 16 * c + (lane & 15);
      if (col >= P.ncols) continue;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int m = 16 * t + 4 * (lane >> 4) + i;
        if (m >= n) continue;
        float x = acc[q][c][i];
        if (DST == DST_LINES) {
          P.dst[(long long)col * n + m] = to_bf16(x);
        } else if (DST == DST_ROWS || DST == DST_ROWS_SCALED) {
          if (DST == DST_ROWS_SCALED) {
            const int jj = col / P.g.n2, kk = col - jj * P.g.n2;
            const float d = P.lx[m] + P.ly[jj] + P.lz[kk];
            x = d > 0.f ? x / d : 0.f;
          }
          P.dst[b * P.bstride + (long long)m * P.ld + col] = to_bf16(x);
        } else {
          const int i0 = col / P.g.n1, j0 = col - i0 * P.g.n1;
          zsplit[sidx(P.g, i0, j0, m)] = (TO)(P.scale * x);
        }
      }
    }
  }
}

template <int SRC, int DST, typename TI, typename TO>
hipError_t run_pass(const FdPass &P, int batch, const TI *v, TO *z, hipStream_t s) {
  // each of the four wavefronts owns every fourth 16-row output tile: up to
  // 4 tiles (64 float32 accumulators per lane) for n <= 256, 8 for n <= 512
  const int n16 = (P.n + 15) & ~15;
  if (P.n % 4 || n16 > 512) return hipErrorInvalidValue;
  const size_t lds = sizeof(unsigned short) * FD_COLS * (n16 + 4);
  dim3 grid((P.ncols + FD_COLS - 1) / FD_COLS, 1, batch);
  if (n16 <= 256)
    hipLaunchKernelGGL((k_fd_pass<SRC, DST, 4, TI, TO>), grid, dim3(FD_T), lds, s, P, v, z);
  else
    hipLaunchKernelGGL((k_fd_pass<SRC, DST, 8, TI, TO>), grid, dim3(FD_T), lds, s, P, v, z);
  return hipGetLastError();
}

}  // namespace

// Packed eigenbases of the three axes (device blob): float lam_x, lam_y,
// lam_z (n0 + n1 + n2), then bfloat16 Q_x, Q_x^T, Q_y, Q_y^T, Q_z, Q_z^T.
size_t fd_blob_bytes(const int n[3]) {
  size_t f = sizeof(float) * (size_t)(n[0] + n[1] + n[2]);
  f = (f + 15) & ~(size_t)15;
  return f + sizeof(unsigned short) * 2 * (size_t)(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
}
void fd_blob_pack(const int n[3], const double *qd, unsigned char *out) {
  // qd: Q0, Q1, Q2 (double, row-major) then lam0, lam1, lam2 (coarse_fd_build)
  const double *lam = qd + n[0] * n[0] + n[1] * n[1] + n[2] * n[2];
  float *lf = (float *)out;
  for (int q = 0; q < n[0] + n[1] + n[2]; ++q) lf[q] = (float)lam[q];
  size_t f = sizeof(float) * (size_t)(n[0] + n[1] + n[2]);
  f = (f + 15) & ~(size_t)15;
  unsigned short *qb = (unsigned short *)(out + f);
  auto bf = [](double x) {
    float v = (float)x;
    unsigned int u;
    memcpy(&u, &v, 4);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
  };
  const double *Q = qd;
  for (int a = 0; a < 3; ++a) {
    const int na = n[a];
    for (int r = 0; r < na; ++r)
      for (int c = 0; c < na; ++c) {
        qb[r * na + c] = bf(Q[r * na + c]);            // Q
        qb[na * na + r * na + c] = bf(Q[c * na + r]);  // Q^T
      }
    qb += 2 * na * na;
    Q += na * na;
  }
}

// z = L^+ v (split layout); w1, w2: two bfloat16 scratch grids (natural
// layout); blob from fd_blob_pack.  The input is scaled by vscale (to keep it
// O(1)) and the result by 1 / vscale.
template <typename TI, typename T>
hipError_t fd_precond(const Geo &g, const TI *v, T *z, unsigned short *w1, unsigned short *w2, const void *blob,
                      float vscale, hipStream_t s) {
  const int n0 = g.n0, n1 = g.n1, n2 = g.n2;
  const long long plane = (long long)n1 * n2;
  const float *lx = (const float *)blob, *ly = lx + n0, *lz = ly + n1;
  size_t f = sizeof(float) * (size_t)(n0 + n1 + n2);
  f = (f + 15) & ~(size_t)15;
  const unsigned short *Qx = (const unsigned short *)((const unsigned char *)blob + f);
  const unsigned short *QxT = Qx + n0 * n0, *Qy = QxT + n0 * n0, *QyT = Qy + n1 * n1, *Qz = QyT + n1 * n1,
                       *QzT = Qz + n2 * n2;
  hipError_t e;
  FdPass P{};
  P.g = g;
  P.lx = lx; P.ly = ly; P.lz = lz;
  // forward along z: w1[r][m] = sum_k Qz[k][m] v[r][k]
  P.n = n2; P.ncols = n0 * n1; P.A = QzT; P.dst = w1; P.scale = vscale;
  if ((e = run_pass<SRC_SPLIT, DST_LINES, TI, T>(P, 1, v, z, s))) return e;
  // forward along y, per plane i: w2[i][m][k] = sum_j Qy[j][m] w1[i][j][k]
  P.n = n1; P.ncols = n2; P.bstride = plane; P.ld = n2; P.A = QyT; P.src = w1; P.dst = w2;
  if ((e = run_pass<SRC_ROWS, DST_ROWS, TI, T>(P, n0, v, z, s))) return e;
  // forward along x and the scaling: w1[m][c] = sum_i Qx[i][m] w2[i][c] / lam
  P.n = n0; P.ncols = (int)plane; P.bstride = 0; P.ld = plane; P.A = QxT; P.src = w2; P.dst = w1;
  if ((e = run_pass<SRC_ROWS, DST_ROWS_SCALED, TI, T>(P, 1, v, z, s))) return e;
  // back along x: w2[i][c] = sum_m Qx[i][m] w1[m][c]
  P.A = Qx; P.src = w1; P.dst = w2;
  if ((e = run_pass<SRC_ROWS, DST_ROWS, TI, T>(P, 1, v, z, s))) return e;
  // back along y: w1[i][j][k] = sum_m Qy[j][m] w2[i][m][k]
  P.n = n1; P.ncols = n2; P.bstride = plane; P.ld = n2; P.A = Qy; P.src = w2; P.dst = w1;
  if ((e = run_pass<SRC_ROWS, DST_ROWS, TI, T>(P, n0, v, z, s))) return e;
  // back along z into the split layout: z[r][k] = sum_m Qz[k][m] w1[r][m]
  P.n = n2; P.ncols = n0 * n1; P.bstride = 0; P.ld = 0; P.A = Qz; P.src = w1; P.dst = nullptr; P.scale = 1.0f / vscale;
  return run_pass<SRC_LINES, DST_SPLIT, TI, T>(P, 1, v, z, s);
}
template hipError_t fd_precond<float, float>(const Geo &, const float *, float *, unsigned short *, unsigned short *,
                                             const void *, float, hipStream_t);
template hipError_t fd_precond<double, double>(const Geo &, const double *, double *, unsigned short *,
                                               unsigned short *, const void *, float, hipStream_t);
template hipError_t fd_precond<double, float>(const Geo &, const double *, float *, unsigned short *,
                                              unsigned short *, const void *, float, hipStream_t);

}  // namespace ibs
