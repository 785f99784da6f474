// Fast-diagonalisation preconditioner: z = L^+ v on the whole grid, the
// direct solver the paper applies once per Krylov iteration (Sec. 4.1-4.2).
// On a box with one boundary type per axis, L is the Kronecker sum of three
// 1-D Laplacians with orthonormal eigenvectors Q_a and eigenvalues lam_a, so
//     z = (Qx (x) Qy (x) Qz) diag(1 / (lam_x + lam_y + lam_z)) (Qx (x) Qy (x) Qz)^T v,
// the constant mode dropped.  Each 1-D transform along an axis is a dense
// product of an n x n matrix with every grid line along that axis, run on the
// matrix cores (bfloat16 operands, float32 accumulation; the preconditioner
// only has to be spectrally close to L^+, and FGMRES accepts its bfloat16
// rounding).  Five passes over the grid: z and y forward, x forward + scaling
// + x back in one pass (a workgroup holds every mode of its x lines), y and z
// back.
//
// A pass is C = A D with A an n x n eigenvector matrix (Q or Q^T, bfloat16,
// rows contiguous along the reduction index, read from L2) and D the grid
// lines of the pass: a workgroup stages 64 lines (n x 64, bfloat16) in LDS
// and its four wavefronts produce all n outputs of them with
// v_mfma_f32_16x16x32_bf16 (16 x 16 tiles, float32 accumulation), written
// back through LDS in 16-byte pieces.  The first and the last pass read /
// write the solver's red/black split layout directly.
#include <string.h>

#include <algorithm>
#include <type_traits>

#include "internal.h"

namespace ibs {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int FD_COLS = 64;  // grid lines per workgroup
constexpr int FD_T = 256;    // four wavefronts

__device__ __forceinline__ unsigned int to_bf16(float x) {
  unsigned int u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even
  return u >> 16;
}
__device__ __forceinline__ unsigned int pack_bf16(float lo, float hi) { return to_bf16(lo) | (to_bf16(hi) << 16); }

// where the n x ncols operand D of a pass lives (element (k, col))
enum { SRC_SPLIT = 0,   // k-th cell of line col = i n1 + j of a split-layout field (first pass)
       SRC_LINES = 1,   // src[col n + k]
       SRC_ROWS = 2 };  // src[b bstride + k ld + col]
// where the n x ncols result (element (m, col)) goes
enum { DST_SPLIT = 0, DST_LINES = 1, DST_ROWS = 2, DST_ROWS_FUSED = 3 };

struct FdPass {
  int n, ncols;
  long long bstride, ld;
  const unsigned short *A;  // n x n, row-major
  const unsigned short *A2; // second product of DST_ROWS_FUSED
  const unsigned short *src;
  unsigned short *dst;
  Geo g;
  float scale;                // input scale (SRC_SPLIT) or output scale (DST_SPLIT)
  const float *lx, *ly, *lz;  // eigenvalues (DST_ROWS_FUSED)
};

template <typename T> struct Vec4;
template <> struct Vec4<float> { typedef float4 type; };
template <> struct Vec4<double> { typedef double4 type; };
template <typename T> struct Vec2;
template <> struct Vec2<float> { typedef float2 type; };
template <> struct Vec2<double> { typedef double2 type; };

// Stage the 64 lines of this workgroup as Ds[col][k] (k contiguous, rows of
// ldsk bfloat16, zero padded up to nk) with 16-byte global reads, issued in
// batches so that one workgroup has many reads in flight.
template <int SRC, typename TI>
__device__ __forceinline__ void stage(const FdPass &P, const TI *vsplit, unsigned short *Ds, int ldsk, int nk,
                                      int b, int col0) {
  const int n = P.n, tid = threadIdx.x;
  if (SRC == SRC_ROWS) {
    // task: 8 columns x 4 rows; four 16-byte row reads, transposed into eight
    // 8-byte LDS writes
    constexpr int BT = 2;
    const int ntask = 8 * (nk >> 2);
    for (int e0 = 0; e0 < ntask; e0 += BT * FD_T) {
      uint4 r[BT][4];
#pragma unroll
      for (int u = 0; u < BT; ++u) {
        const int e = e0 + u * FD_T + tid;
        const int cg = e & 7, k0 = 4 * (e >> 3), col = col0 + 8 * cg;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          r[u][q] = make_uint4(0, 0, 0, 0);
          if (e < ntask && k0 + q < n && col < P.ncols)
            r[u][q] = *(const uint4 *)&P.src[b * P.bstride + (long long)(k0 + q) * P.ld + col];
        }
      }
#pragma unroll
      for (int u = 0; u < BT; ++u) {
        const int e = e0 + u * FD_T + tid;
        if (e >= ntask) continue;
        const int cg = e & 7, k0 = 4 * (e >> 3);
        const unsigned int *w0 = (const unsigned int *)&r[u][0], *w1 = (const unsigned int *)&r[u][1],
                           *w2 = (const unsigned int *)&r[u][2], *w3 = (const unsigned int *)&r[u][3];
#pragma unroll
        for (int c = 0; c < 8; ++c) {
          const int sh = (c & 1) * 16, wi = c >> 1;
          const unsigned int e0v = (w0[wi] >> sh) & 0xFFFFu, e1v = (w1[wi] >> sh) & 0xFFFFu;
          const unsigned int e2v = (w2[wi] >> sh) & 0xFFFFu, e3v = (w3[wi] >> sh) & 0xFFFFu;
          *(uint2 *)&Ds[(8 * cg + c) * ldsk + k0] = make_uint2(e0v | (e1v << 16), e2v | (e3v << 16));
        }
      }
    }
  } else if (SRC == SRC_LINES) {
    constexpr int BT = 8;
    const int n8 = nk >> 3, nr = n >> 3, ntask = FD_COLS * n8;
    for (int e0 = 0; e0 < ntask; e0 += BT * FD_T) {
      uint4 v[BT];
#pragma unroll
      for (int u = 0; u < BT; ++u) {
        const int e = e0 + u * FD_T + tid;
        const int cc = e / n8, part = e - cc * n8, col = col0 + cc;
        v[u] = make_uint4(0, 0, 0, 0);
        if (e < ntask && part < nr && col < P.ncols) v[u] = *(const uint4 *)&P.src[(long long)col * n + 8 * part];
      }
#pragma unroll
      for (int u = 0; u < BT; ++u) {
        const int e = e0 + u * FD_T + tid;
        const int cc = e / n8, part = e - cc * n8;
        if (e < ntask) *(uint4 *)&Ds[cc * ldsk + 8 * part] = v[u];
      }
    }
  } else {
    // split layout: cells k = 8p .. 8p+7 of line (i, j) are four consecutive
    // values of each colour half; interleave them into one 16-byte LDS write
    typedef typename Vec4<TI>::type V4;
    constexpr int BT = sizeof(TI) == 4 ? 4 : 2;
    const int n8 = nk >> 3, nr = n >> 3, ntask = FD_COLS * n8;
    const float s = P.scale;
    for (int e0 = 0; e0 < ntask; e0 += BT * FD_T) {
      V4 ev[BT], od[BT];
#pragma unroll
      for (int u = 0; u < BT; ++u) {
        const int e = e0 + u * FD_T + tid;
        const int cc = e / n8, part = e - cc * n8, col = col0 + cc;
        if (e < ntask && part < nr && col < P.ncols) {
          const int i = col / P.g.n1, j = col - i * P.g.n1;
          const int ce = (i + j) & 1;  // colour of the even cells of this line
          const long long base = (long long)col * P.g.hn2 + 4 * part;
          ev[u] = *(const V4 *)&vsplit[ce * P.g.half + base];
          od[u] = *(const V4 *)&vsplit[(1 - ce) * P.g.half + base];
        } else {
          ev[u].x = ev[u].y = ev[u].z = ev[u].w = TI(0);
          od[u] = ev[u];
        }
      }
#pragma unroll
      for (int u = 0; u < BT; ++u) {
        const int e = e0 + u * FD_T + tid;
        const int cc = e / n8, part = e - cc * n8;
        if (e >= ntask) continue;
        uint4 o;
        o.x = pack_bf16(s * (float)ev[u].x, s * (float)od[u].x);
        o.y = pack_bf16(s * (float)ev[u].y, s * (float)od[u].y);
        o.z = pack_bf16(s * (float)ev[u].z, s * (float)od[u].z);
        o.w = pack_bf16(s * (float)ev[u].w, s * (float)od[u].w);
        *(uint4 *)&Ds[cc * ldsk + 8 * part] = o;
      }
    }
  }
}

// One pass.  ORIENT_C swaps the MFMA operands so that a lane ends up with
// four consecutive columns of one output row (8-byte stores along rows);
// otherwise a lane holds four consecutive rows of one column (stores along
// lines).  DST_ROWS_FUSED runs the whole x stage in one pass: forward
// transform, scaling by 1 / (lam_x + lam_y + lam_z) and back transform, the
// scaled modes going through LDS between the two products.
template <int SRC, int DST, int MAXT, typename TI, typename TO>
__global__ void __launch_bounds__(FD_T, MAXT == 4 ? 4 : 2) k_fd_pass(FdPass P, const TI *vsplit, TO *zsplit) {
  constexpr bool ORIENT_C = DST == DST_ROWS || DST == DST_ROWS_FUSED;
  extern __shared__ unsigned short Ds[];  // [FD_COLS][ldsk]
  // k is zero padded to nk (a multiple of 64: the k loop takes two steps of
  // 32 per trip); output rows to n16
  const int n = P.n, n16 = (n + 15) & ~15, nk = (n + 63) & ~63, ldsk = nk + 8;
  const int b = blockIdx.z, col0 = blockIdx.x * FD_COLS;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  stage<SRC, TI>(P, vsplit, Ds, ldsk, nk, b, col0);
  __syncthreads();
  const int ntiles = n16 >> 4;
  const int l16 = lane & 15, lq = lane >> 4;
  f32x4 acc[MAXT][4];
  // acc = A Ds (n16 x 64).  Eigenvector fragments (16 rows x 32 k per tile)
  // are read from L2 two k steps ahead of their use; lane l holds row l % 16,
  // k = 8 (l / 16) .. + 7 (the same k for both operands of
  // v_mfma_f32_16x16x32_bf16).
  auto gemm = [&](const unsigned short *A, auto orient_c) {
    constexpr bool OC = decltype(orient_c)::value;
#pragma unroll
    for (int q = 0; q < MAXT; ++q)
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[q][c] = f32x4{0.f, 0.f, 0.f, 0.f};
    auto load_a = [&](bf16x8 *dst, int k0) {
#pragma unroll
      for (int q = 0; q < MAXT; ++q) {
        // clamped addresses instead of a condition, so that the wait for these
        // loads falls at their use: rows beyond n produce outputs that are
        // dropped, and k beyond n meets the zero padding of Ds
        const int row = 16 * (wv + 4 * q) + l16, kq = k0 + 8 * lq;
        dst[q] = *(const bf16x8 *)&A[(long long)min(row, n - 1) * n + min(kq, n - 8)];
      }
    };
    auto step = [&](const bf16x8 *a, int k0) {
      const int kq = k0 + 8 * lq;
      bf16x8 bb[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) bb[c] = *(const bf16x8 *)&Ds[(16 * c + l16) * ldsk + kq];
#pragma unroll
      for (int q = 0; q < MAXT; ++q) {
#pragma unroll
        for (int c = 0; c < 4; ++c)
          acc[q][c] = OC ? __builtin_amdgcn_mfma_f32_16x16x32_bf16(bb[c], a[q], acc[q][c], 0, 0, 0)
                         : __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[q], bb[c], acc[q][c], 0, 0, 0);
      }
    };
    bf16x8 a0[MAXT], a1[MAXT];
    load_a(a0, 0);
    load_a(a1, 32);
    for (int k0 = 0; k0 < nk; k0 += 64) {
      step(a0, k0);
      load_a(a0, k0 + 64);
      step(a1, k0 + 32);
      load_a(a1, k0 + 96);
    }
  };
  if (DST == DST_ROWS_FUSED) {
    gemm(P.A, std::false_type());
    __syncthreads();
    // scaled modes back into Ds as the operand of the second product: lane
    // holds column cc, modes m .. m+3; modes n .. n16-1 are zeroed (n16 .. nk
    // still hold the zero padding of the staging)
#pragma unroll
    for (int q = 0; q < MAXT; ++q) {
      const int t = wv + 4 * q;
      if (t >= ntiles) continue;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int cc = 16 * c + l16, m = 16 * t + 4 * lq, col = col0 + cc;
        const int cl = min(col, P.ncols - 1);
        const int jj = cl / P.g.n2, kk = cl - jj * P.g.n2;
        const float lyz = P.ly[jj] + P.lz[kk];
        float y[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const float d = P.lx[min(m + i, n - 1)] + lyz;
          y[i] = (m + i < n && d > 0.f) ? acc[q][c][i] * __builtin_amdgcn_rcpf(d) : 0.f;
        }
        *(uint2 *)&Ds[cc * ldsk + m] = make_uint2(pack_bf16(y[0], y[1]), pack_bf16(y[2], y[3]));
      }
    }
    __syncthreads();
    gemm(P.A2, std::true_type());
  } else {
    gemm(P.A, std::integral_constant<bool, ORIENT_C>());
  }
  // Epilogue through LDS, so that global writes are whole 16-byte pieces of
  // contiguous rows / lines: the result tile goes to Os as bfloat16, rows
  // [m][col] (ORIENT_C, ldo = 72) or lines [col][m] (ldo = n16 + 8).
  __syncthreads();
  unsigned short *Os = Ds;
  const int ldo = ORIENT_C ? FD_COLS + 8 : n16 + 8;
#pragma unroll
  for (int q = 0; q < MAXT; ++q) {
    const int t = wv + 4 * q;
    if (t >= ntiles) continue;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const f32x4 x = acc[q][c];
      if (ORIENT_C) {
        // row m, columns cc .. cc+3
        const int m = 16 * t + l16, cc = 16 * c + 4 * lq;
        const float y0 = x[0], y1 = x[1], y2 = x[2], y3 = x[3];
        *(uint2 *)&Os[m * ldo + cc] = make_uint2(pack_bf16(y0, y1), pack_bf16(y2, y3));
      } else {
        // column cc, rows m .. m+3
        const int cc = 16 * c + l16, m = 16 * t + 4 * lq;
        *(uint2 *)&Os[cc * ldo + m] = make_uint2(pack_bf16(x[0], x[1]), pack_bf16(x[2], x[3]));
      }
    }
  }
  __syncthreads();
  if (ORIENT_C) {
    // row m of the block: 64 contiguous columns, eight 16-byte pieces
    for (int e = tid; e < n * 8; e += FD_T) {
      const int m = e >> 3, p8 = e & 7, col = col0 + 8 * p8;
      if (col < P.ncols)
        *(uint4 *)&P.dst[b * P.bstride + (long long)m * P.ld + col] = *(const uint4 *)&Os[m * ldo + 8 * p8];
    }
  } else if (DST == DST_LINES) {
    // the 64 lines of the block are contiguous in the destination
    const int n8 = n >> 3;
    for (int e = tid; e < FD_COLS * n8; e += FD_T) {
      const int cc = e / n8, p8 = e - cc * n8, col = col0 + cc;
      if (col < P.ncols) *(uint4 *)&P.dst[(long long)col * n + 8 * p8] = *(const uint4 *)&Os[cc * ldo + 8 * p8];
    }
  } else {
    // cells 8p .. 8p+7 of line (i, j): four consecutive values in each colour half
    typedef typename Vec4<TO>::type V4;
    const int n8 = n >> 3;
    const float s = P.scale;
    for (int e = tid; e < FD_COLS * n8; e += FD_T) {
      const int cc = e / n8, p8 = e - cc * n8, col = col0 + cc;
      if (col >= P.ncols) continue;
      const uint4 v = *(const uint4 *)&Os[cc * ldo + 8 * p8];
      const int i0 = col / P.g.n1, j0 = col - i0 * P.g.n1;
      const int ce = (i0 + j0) & 1;
      const long long base = (long long)col * P.g.hn2 + 4 * p8;
      auto lo = [](unsigned int w) { return __uint_as_float(w << 16); };
      auto hi = [](unsigned int w) { return __uint_as_float(w & 0xFFFF0000u); };
      V4 ev, od;
      ev.x = (TO)(s * lo(v.x)); od.x = (TO)(s * hi(v.x));
      ev.y = (TO)(s * lo(v.y)); od.y = (TO)(s * hi(v.y));
      ev.z = (TO)(s * lo(v.z)); od.z = (TO)(s * hi(v.z));
      ev.w = (TO)(s * lo(v.w)); od.w = (TO)(s * hi(v.w));
      *(V4 *)&zsplit[ce * P.g.half + base] = ev;
      *(V4 *)&zsplit[(1 - ce) * P.g.half + base] = od;
    }
  }
}

template <int SRC, int DST, typename TI, typename TO>
hipError_t run_pass(const FdPass &P, int batch, const TI *v, TO *z, hipStream_t s) {
  // each of the four wavefronts owns every fourth 16-row output tile: up to
  // 4 tiles (64 float32 accumulators per lane) for n <= 256, 8 for n <= 512
  const int n16 = (P.n + 15) & ~15, nk = (P.n + 63) & ~63;
  if (P.n % 8 || P.ncols % 8 || n16 > 512) return hipErrorInvalidValue;
  // staging [64][nk + 8]; epilogue [n16][72] (rows) or [64][n16 + 8] (lines)
  const size_t lds = sizeof(unsigned short) *
                     std::max<size_t>((size_t)FD_COLS * (nk + 8),
                                      (DST == DST_ROWS || DST == DST_ROWS_FUSED) ? (size_t)n16 * (FD_COLS + 8)
                                                                                  : (size_t)FD_COLS * (n16 + 8));
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
  // along x, all in one pass: w1[i][c] = sum_m Qx[i][m] (sum_i' Qx[i'][m] w2[i'][c]) / lam
  P.n = n0; P.ncols = (int)plane; P.bstride = 0; P.ld = plane; P.A = QxT; P.A2 = Qx; P.src = w2; P.dst = w1;
  if ((e = run_pass<SRC_ROWS, DST_ROWS_FUSED, TI, T>(P, 1, v, z, s))) return e;
  // back along y: w2[i][j][k] = sum_m Qy[j][m] w1[i][m][k]
  P.n = n1; P.ncols = n2; P.bstride = plane; P.ld = n2; P.A = Qy; P.src = w1; P.dst = w2;
  if ((e = run_pass<SRC_ROWS, DST_ROWS, TI, T>(P, n0, v, z, s))) return e;
  // back along z into the split layout: z[r][k] = sum_m Qz[k][m] w2[r][m]
  P.n = n2; P.ncols = n0 * n1; P.bstride = 0; P.ld = 0; P.A = Qz; P.src = w2; P.dst = nullptr; P.scale = 1.0f / vscale;
  return run_pass<SRC_LINES, DST_SPLIT, TI, T>(P, 1, v, z, s);
}
template hipError_t fd_precond<float, float>(const Geo &, const float *, float *, unsigned short *, unsigned short *,
                                             const void *, float, hipStream_t);
template hipError_t fd_precond<double, double>(const Geo &, const double *, double *, unsigned short *,
                                               unsigned short *, const void *, float, hipStream_t);
template hipError_t fd_precond<double, float>(const Geo &, const double *, float *, unsigned short *,
                                              unsigned short *, const void *, float, hipStream_t);

}  // namespace ibs
