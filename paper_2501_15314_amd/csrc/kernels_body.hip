// Per-body sums of the two-way coupling (paper Sec. 3.2, eq. volume_integrals;
// Sec. 3.2.1 Step 3, eqs. bdy_linear_vel_iter and bdy_angular_vel_iter):
//   * the total force h^3 sum Phi_k and torque h^3 sum L~_k x Phi_k of each
//     body's Lagrangian forces, L~_k = R X~_k (one workgroup per body);
//   * the volume integrals sum alpha u h^3 and sum alpha r x u h^3 of the fluid
//     velocity over the velocity nodes near each sphere, with the volume
//     fraction alpha of the cell-sized box around a node taken from the signed
//     distances s = |x - X_c| - a at its 8 corners (Kempe & Uhlmann):
//     alpha = sum(-s, s < 0) / sum |s|.
// A node farther than a + h sqrt(3)/2 from the centre has alpha = 0, so each
// body only visits the nodes of a box of about (2a/h + 5)^3 around it.  All
// sums are in a fixed order, so the results are bitwise repeatable.
#include "internal.h"

namespace ibs {

namespace {

constexpr int BT = 256;  // threads per workgroup

// fixed-order sum of NV values over the workgroup; result valid in thread 0
template <int NV>
__device__ void block_sums(double (&v)[NV], double (*sh)[NV]) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < NV; ++q) v[q] = wave_sum(v[q]);
  if (lane == 0)
#pragma unroll
    for (int q = 0; q < NV; ++q) sh[wv][q] = v[q];
  __syncthreads();
  if (threadIdx.x == 0)
#pragma unroll
    for (int q = 0; q < NV; ++q) v[q] = sh[0][q] + sh[1][q] + sh[2][q] + sh[3][q];
}

__global__ void __launch_bounds__(BT) k_body_ft(const BodyDev *bodies, const BodySpan *span,
                                                 const double *off, const double *phi, double h3,
                                                 double *out) {
  const int b = blockIdx.x;
  const BodyDev B = bodies[b];
  const int k0 = span[b].k0, kn = span[b].kn;
  double v[6] = {0, 0, 0, 0, 0, 0};
  for (int k = k0 + threadIdx.x; k < k0 + kn; k += BT) {
    const double o0 = off[3 * k], o1 = off[3 * k + 1], o2 = off[3 * k + 2];
    const double l0 = B.R[0] * o0 + B.R[1] * o1 + B.R[2] * o2;
    const double l1 = B.R[3] * o0 + B.R[4] * o1 + B.R[5] * o2;
    const double l2 = B.R[6] * o0 + B.R[7] * o1 + B.R[8] * o2;
    const double f0 = phi[3 * k], f1 = phi[3 * k + 1], f2 = phi[3 * k + 2];
    v[0] += f0;
    v[1] += f1;
    v[2] += f2;
    v[3] += l1 * f2 - l2 * f1;
    v[4] += l2 * f0 - l0 * f2;
    v[5] += l0 * f1 - l1 * f0;
  }
  __shared__ double sh[4][6];
  block_sums<6>(v, sh);
  if (threadIdx.x == 0)
    for (int q = 0; q < 6; ++q) out[12 * b + q] = h3 * v[q];
}

// Partial volume integrals of body blockIdx.z, velocity component
// d = blockIdx.y, chunk blockIdx.x of its node box.  Three sums per
// (body, d): alpha u_d h^3 (linear component d) and the two terms u_d adds to
// r x u: +r_{d+2} alpha u_d h^3 in component d+1, -r_{d+1} alpha u_d h^3 in
// component d+2.
__global__ void __launch_bounds__(BT) k_vol_part(Geo g, const BodySpan *span, const double *u,
                                                  double *part) {
  const int b = blockIdx.z, d = blockIdx.y, ch = blockIdx.x, nch = gridDim.x;
  const BodySpan S = span[b];
  const long long total = (long long)S.dim[0] * S.dim[1] * S.dim[2];
  const double h = g.h, h3 = g.h * g.h * g.h, a = S.radius;
  const int e1 = d == 2 ? 0 : d + 1, e2 = d == 0 ? 2 : d - 1;
  const long long N = 2 * g.half;
  const double *ud = u + d * N;
  double v[3] = {0, 0, 0};
  for (long long t = (long long)ch * BT + threadIdx.x; t < total; t += (long long)nch * BT) {
    int li = (int)(t / ((long long)S.dim[1] * S.dim[2]));
    int rem = (int)(t - (long long)li * S.dim[1] * S.dim[2]);
    int lj = rem / S.dim[2], lk = rem - lj * S.dim[2];
    int idx[3] = {S.lo[0] + li, S.lo[1] + lj, S.lo[2] + lk};
    double r[3];
    bool inside = true;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const int n = geo_n(g, q);
      if (geo_bc(g, q)) {
        inside = inside && idx[q] >= 0 && idx[q] < n;
      } else {
        idx[q] = wrapi(idx[q], n);
      }
      double pos = ((double)idx[q] + 0.5) * h;
      if (q == d) pos -= 0.5 * h;
      double rq = pos - S.c[q];
      if (!geo_bc(g, q)) {
        const double L = n * h;
        rq -= L * rint(rq / L);
      }
      r[q] = rq;
    }
    if (!inside) continue;
    double num = 0.0, den = 0.0;
#pragma unroll
    for (int cc = 0; cc < 8; ++cc) {
      const double cx = r[0] + ((cc & 4) ? 0.5 : -0.5) * h;
      const double cy = r[1] + ((cc & 2) ? 0.5 : -0.5) * h;
      const double cz = r[2] + ((cc & 1) ? 0.5 : -0.5) * h;
      const double sd = sqrt(cx * cx + cy * cy + cz * cz) - a;
      num += sd < 0.0 ? -sd : 0.0;
      den += fabs(sd);
    }
    if (!(num > 0.0)) continue;
    const double alpha = num / den;
    const double au = alpha * ud[sidx(g, idx[0], idx[1], idx[2])] * h3;
    v[0] += au;
    v[1] += r[e2] * au;
    v[2] -= r[e1] * au;
  }
  __shared__ double sh[4][3];
  block_sums<3>(v, sh);
  if (threadIdx.x == 0) {
    double *p = part + (((long long)b * 3 + d) * nch + ch) * 3;
    p[0] = v[0];
    p[1] = v[1];
    p[2] = v[2];
  }
}

// out[12 b + 6 + q], q = 0..2: sum alpha u h^3; q = 3..5: sum alpha r x u h^3
__global__ void k_vol_fin(int nb, int nch, const double *part, double *out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 6 * nb) return;
  const int b = t / 6, q = t % 6;
  double acc = 0.0;
  for (int d = 0; d < 3; ++d) {
    int slot = -1;
    if (q < 3) {
      if (d == q) slot = 0;
    } else {
      const int e = q - 3;
      if ((d + 1) % 3 == e) slot = 1;
      if ((d + 2) % 3 == e) slot = 2;
    }
    if (slot < 0) continue;
    const double *p = part + ((long long)b * 3 + d) * nch * 3;
    for (int ch = 0; ch < nch; ++ch) acc += p[3 * ch + slot];
  }
  out[12 * b + 6 + q] = acc;
}

// Transposed volume integrals of one body (reverse-mode step): with the
// cotangents (Ib, Jb) of (sum alpha u h^3, sum alpha r x u h^3), every node of
// component d = blockIdx.y in the body's box gets
//     ubar_d += alpha h^3 (Ib_d + (Jb x r)_d),
// and the centre cotangent collects, per (d, chunk), the partial sums of
//     d alpha / d X_c * u_d h^3 (Ib_d + (Jb x r)_d) + alpha h^3 u_d (Jb x e_d)
// (r = x - X_c, d s / d X_c = -(corner - X_c) / |corner - X_c| for each
// corner's signed distance s).  One launch per body, so that no node is
// written by two workgroups.
struct VolCot {
  double ib[3], jb[3];
};

__global__ void __launch_bounds__(BT) k_vol_adj(Geo g, BodySpan S, VolCot cot, const double *u, double *ubar,
                                                 double *part) {
  const int d = blockIdx.y, ch = blockIdx.x, nch = gridDim.x;
  const long long total = (long long)S.dim[0] * S.dim[1] * S.dim[2];
  const double h = g.h, h3 = g.h * g.h * g.h, a = S.radius;
  const int e1 = d == 2 ? 0 : d + 1, e2 = d == 0 ? 2 : d - 1;
  const long long N = 2 * g.half;
  const double *ud = u + d * N;
  double *bd = ubar + d * N;
  // Jb x e_d
  double jxe[3];
  jxe[d] = 0.0;
  jxe[e1] = cot.jb[e2];
  jxe[e2] = -cot.jb[e1];
  double v[3] = {0, 0, 0};
  for (long long t = (long long)ch * BT + threadIdx.x; t < total; t += (long long)nch * BT) {
    int li = (int)(t / ((long long)S.dim[1] * S.dim[2]));
    int rem = (int)(t - (long long)li * S.dim[1] * S.dim[2]);
    int lj = rem / S.dim[2], lk = rem - lj * S.dim[2];
    int idx[3] = {S.lo[0] + li, S.lo[1] + lj, S.lo[2] + lk};
    double r[3];
    bool inside = true;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const int n = geo_n(g, q);
      if (geo_bc(g, q)) {
        inside = inside && idx[q] >= 0 && idx[q] < n;
      } else {
        idx[q] = wrapi(idx[q], n);
      }
      double pos = ((double)idx[q] + 0.5) * h;
      if (q == d) pos -= 0.5 * h;
      double rq = pos - S.c[q];
      if (!geo_bc(g, q)) {
        const double L = n * h;
        rq -= L * rint(rq / L);
      }
      r[q] = rq;
    }
    if (!inside) continue;
    double num = 0.0, den = 0.0, dnum[3] = {0, 0, 0}, dden[3] = {0, 0, 0};
#pragma unroll
    for (int cc = 0; cc < 8; ++cc) {
      const double cx = r[0] + ((cc & 4) ? 0.5 : -0.5) * h;
      const double cy = r[1] + ((cc & 2) ? 0.5 : -0.5) * h;
      const double cz = r[2] + ((cc & 1) ? 0.5 : -0.5) * h;
      const double dist = sqrt(cx * cx + cy * cy + cz * cz);
      const double sd = dist - a;
      const double inv = dist > 0.0 ? 1.0 / dist : 0.0;
      const double ds0 = -cx * inv, ds1 = -cy * inv, ds2 = -cz * inv;
      if (sd < 0.0) {
        num -= sd;
        dnum[0] -= ds0;
        dnum[1] -= ds1;
        dnum[2] -= ds2;
      }
      den += fabs(sd);
      const double sg = sd > 0.0 ? 1.0 : (sd < 0.0 ? -1.0 : 0.0);
      dden[0] += sg * ds0;
      dden[1] += sg * ds1;
      dden[2] += sg * ds2;
    }
    if (!(num > 0.0)) continue;
    const double alpha = num / den;
    const long long e = sidx(g, idx[0], idx[1], idx[2]);
    const double wgt = h3 * (cot.ib[d] + cot.jb[e1] * r[e2] - cot.jb[e2] * r[e1]);
    bd[e] += alpha * wgt;
    const double uv = ud[e];
    const double id2 = 1.0 / (den * den);
#pragma unroll
    for (int q = 0; q < 3; ++q) v[q] += (dnum[q] * den - num * dden[q]) * id2 * uv * wgt + alpha * h3 * uv * jxe[q];
  }
  __shared__ double sh[4][3];
  block_sums<3>(v, sh);
  if (threadIdx.x == 0) {
    double *p = part + ((long long)d * nch + ch) * 3;
    p[0] = v[0];
    p[1] = v[1];
    p[2] = v[2];
  }
}

// Per-point transposes of one outer pass (natural order), L~_k = R_b X~_k:
//   phibar_k += h^3 (Fb_b + Tb_b x L~_k)        (F = h^3 sum Phi, T = h^3 sum L~ x Phi)
//   lbar_k   += h^3 (phi_k x Tb_b) + Ubar_k x w_b   (and U = u_s + w x L~)
// coef[9 b + 0..8] = (Fb, Tb, w) of body b.
__global__ void k_point_adj(int K, const int *bodyof, const double *off, const BodyDev *bodies,
                            const double *coef, double h3, const double *phi, const double *ubar, double *phibar,
                            double *lbar) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;
  const int b = bodyof[k];
  const double *R = bodies[b].R;
  const double *cf = coef + 9 * b;
  const double o0 = off[3 * k], o1 = off[3 * k + 1], o2 = off[3 * k + 2];
  const double l[3] = {R[0] * o0 + R[1] * o1 + R[2] * o2, R[3] * o0 + R[4] * o1 + R[5] * o2,
                       R[6] * o0 + R[7] * o1 + R[8] * o2};
  const double *tb = cf + 3, *w = cf + 6;
  const double f[3] = {phi[3 * k], phi[3 * k + 1], phi[3 * k + 2]};
  const double ub[3] = {ubar[3 * k], ubar[3 * k + 1], ubar[3 * k + 2]};
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const int q1 = (q + 1) % 3, q2 = (q + 2) % 3;
    phibar[3 * k + q] += h3 * (cf[q] + tb[q1] * l[q2] - tb[q2] * l[q1]);
    lbar[3 * k + q] += h3 * (f[q1] * tb[q2] - f[q2] * tb[q1]) + (ub[q1] * w[q2] - ub[q2] * w[q1]);
  }
}

}  // namespace

hipError_t body_force_torque(int nb, const BodyDev *bodies, const BodySpan *span, const double *off,
                             const double *phi, double h3, double *out, hipStream_t s) {
  if (nb == 0) return hipSuccess;
  hipLaunchKernelGGL(k_body_ft, dim3(nb), dim3(BT), 0, s, bodies, span, off, phi, h3, out);
  return hipGetLastError();
}

hipError_t body_volume_integrals(const Geo &g, int nb, const BodySpan *span, const double *u, double *part,
                                 double *out, hipStream_t s) {
  if (nb == 0) return hipSuccess;
  hipLaunchKernelGGL(k_vol_part, dim3(VOL_CHUNKS, 3, nb), dim3(BT), 0, s, g, span, u, part);
  hipLaunchKernelGGL(k_vol_fin, dim3((6 * nb + 63) / 64), dim3(64), 0, s, nb, VOL_CHUNKS, part, out);
  return hipGetLastError();
}

}  // namespace ibs

namespace ibs {

hipError_t body_volume_adjoint(const Geo &g, const BodySpan &span, const double ib[3], const double jb[3],
                               const double *u, double *ubar, double *part, hipStream_t s) {
  VolCot cot;
  for (int q = 0; q < 3; ++q) {
    cot.ib[q] = ib[q];
    cot.jb[q] = jb[q];
  }
  hipLaunchKernelGGL(k_vol_adj, dim3(VOL_CHUNKS, 3, 1), dim3(BT), 0, s, g, span, cot, u, ubar, part);
  return hipGetLastError();
}

hipError_t point_adjoint(int K, const int *bodyof, const double *off, const BodyDev *bodies, const double *coef,
                         double h3, const double *phi, const double *ubar, double *phibar, double *lbar,
                         hipStream_t s) {
  if (K == 0) return hipSuccess;
  hipLaunchKernelGGL(k_point_adj, dim3((K + 255) / 256), dim3(256), 0, s, K, bodyof, off, bodies, coef, h3, phi,
                     ubar, phibar, lbar);
  return hipGetLastError();
}

}  // namespace ibs
