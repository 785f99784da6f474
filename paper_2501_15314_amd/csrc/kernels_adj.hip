// Kernels of the reverse-mode step that have no forward counterpart:
//   * interp_dx: gradient with respect to the point coordinates of the
//     bilinear form a^T W(X) b (a a face field, b point values):
//       out_{k,e} += scale sum_d b_{k,d} sum_i a_d(x_i) dw_ik/dX_{k,e},
//     dw/dX_e = phi'(r_e)/h phi(r_f) phi(r_g) (Sec. 2.3 weights, r in cells);
//   * convection_adjoint: J_N(u)^T r for the flux form of N(u) = div(u u)
//     (arithmetic averages, no flux through walls of either kind), written as a
//     gather: after summation by parts r^T N = sum over flux points of
//     F(x) psi(x), psi the difference of r across the flux point, and each
//     face collects dF/du psi from the flux points whose averages contain it.
#include "internal.h"

namespace ibs {

namespace {

template <typename T>
__device__ __forceinline__ T fetch3(const T *f, const Geo &g, const int x[3]) {
  int i = x[0], j = x[1], k = x[2];
  if (i < 0 || i >= g.n0) { if (g.bc0) return T(0); i = wrapi(i, g.n0); }
  if (j < 0 || j >= g.n1) { if (g.bc1) return T(0); j = wrapi(j, g.n1); }
  if (k < 0 || k >= g.n2) { if (g.bc2) return T(0); k = wrapi(k, g.n2); }
  return f[sidx(g, i, j, k)];
}

// Whether x is a grid index (after wrapping periodic axes).
__device__ __forceinline__ bool in_box(const Geo &g, const int x[3]) {
  for (int a = 0; a < 3; ++a)
    if (geo_bc(g, a) && (x[a] < 0 || x[a] >= geo_n(g, a))) return false;
  return true;
}

template <int KER>
__global__ void k_interp_dx(Geo g, int K, const double *X, const double *a3, const double *b, double scale,
                            double *out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;
  constexpr int W = KerWidth<KER>::W;
  const double inv_h = 1.0 / g.h;
  const long long N = 2 * g.half;
  const double x[3] = {X[3 * k], X[3 * k + 1], X[3 * k + 2]};
  double ge[3] = {0.0, 0.0, 0.0};
  for (int d = 0; d < 3; ++d) {
    double w[3][4], dw[3][4];
    int i0[3];
    for (int a = 0; a < 3; ++a) {
      double s;
      i0[a] = support_start<KER>(x[a], inv_h, a == d, s);
      for (int t = 0; t < W; ++t) {
        const double r = s - (double)(i0[a] + t);
        w[a][t] = phi<KER>(r);
        dw[a][t] = dphi<KER>(r) * inv_h;
      }
    }
    const double *ad = a3 + d * N;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int t0 = 0; t0 < W; ++t0) {
      const int i = wrapi(i0[0] + t0, g.n0);
      for (int t1 = 0; t1 < W; ++t1) {
        const int j = wrapi(i0[1] + t1, g.n1);
        for (int t2 = 0; t2 < W; ++t2) {
          const int kk = wrapi(i0[2] + t2, g.n2);
          const double v = ad[sidx(g, i, j, kk)];
          s0 += v * dw[0][t0] * w[1][t1] * w[2][t2];
          s1 += v * w[0][t0] * dw[1][t1] * w[2][t2];
          s2 += v * w[0][t0] * w[1][t1] * dw[2][t2];
        }
      }
    }
    const double bd = b[3 * k + d];
    ge[0] += bd * s0;
    ge[1] += bd * s1;
    ge[2] += bd * s2;
  }
  for (int e = 0; e < 3; ++e) out[3 * k + e] += scale * ge[e];
}

// F_{a,d}(x) is zero through a wall: x_a = n_a - 1 on a wall axis a.
__device__ __forceinline__ bool flux_open(const Geo &g, int a, const int x[3]) {
  return !(geo_bc(g, a) && x[a] == geo_n(g, a) - 1);
}

__global__ void k_conv_adj(Geo g, const double *u3, const double *r3, double *out3) {
  RowPos p;
  if (!row_pos(g, p)) return;
  const long long N = 2 * g.half;
  const int m = p.comp;
  const int y[3] = {p.i, p.j, p.k};
  double acc = 0.0;
  if (!(geo_bc(g, m) && y[m] == 0)) {
    const double h = g.h;
    const double *um = u3 + m * N, *rm = r3 + m * N;
    // (1) a = d = m: F = C^2, C(x) = (u_m(x) + u_m(x + e_m)) / 2,
    //     psi(x) = (r_m(x) - r_m(x + e_m)) / h; u_m(y) enters C(y), C(y - e_m)
    for (int q = 0; q < 2; ++q) {
      int x[3] = {y[0], y[1], y[2]};
      x[m] -= q;
      if (!in_box(g, x)) continue;
      int xp[3] = {x[0], x[1], x[2]};
      xp[m] += 1;
      const double C = 0.5 * (fetch3(um, g, x) + fetch3(um, g, xp));
      const double psi = (fetch3(rm, g, x) - fetch3(rm, g, xp)) / h;
      acc += 2.0 * C * 0.5 * psi;
    }
    for (int o = 1; o < 3; ++o) {
      const int a = (m + o) % 3;
      // (2) d = m, flux along a: F = E1 E2, E1(x) = (u_m(x) + u_m(x + e_a)) / 2,
      //     E2(x) = (u_a(x + e_a) + u_a(x + e_a - e_m)) / 2,
      //     psi(x) = (r_m(x) - r_m(x + e_a)) / h; u_m(y) enters E1(y), E1(y - e_a)
      const double *ua = u3 + a * N;
      for (int q = 0; q < 2; ++q) {
        int x[3] = {y[0], y[1], y[2]};
        x[a] -= q;
        if (!in_box(g, x) || !flux_open(g, a, x)) continue;
        int xa[3] = {x[0], x[1], x[2]};
        xa[a] += 1;
        int xam[3] = {xa[0], xa[1], xa[2]};
        xam[m] -= 1;
        const double E2 = 0.5 * (fetch3(ua, g, xa) + fetch3(ua, g, xam));
        const double psi = (fetch3(rm, g, x) - fetch3(rm, g, xa)) / h;
        acc += 0.5 * E2 * psi;
      }
      // (3) component d = a, flux along m: F = E1 E2 with E1(x) = (u_d(x) + u_d(x + e_m)) / 2,
      //     E2(x) = (u_m(x + e_m) + u_m(x + e_m - e_d)) / 2,
      //     psi(x) = (r_d(x) - r_d(x + e_m)) / h; u_m(y) enters E2 at
      //     x = y - e_m and x = y - e_m + e_d
      const int d = a;
      const double *ud = u3 + d * N, *rd = r3 + d * N;
      for (int q = 0; q < 2; ++q) {
        int x[3] = {y[0], y[1], y[2]};
        x[m] -= 1;
        x[d] += q;
        if (!in_box(g, x) || !flux_open(g, m, x)) continue;
        int xm[3] = {x[0], x[1], x[2]};
        xm[m] += 1;
        const double E1 = 0.5 * (fetch3(ud, g, x) + fetch3(ud, g, xm));
        const double psi = (fetch3(rd, g, x) - fetch3(rd, g, xm)) / h;
        acc += 0.5 * E1 * psi;
      }
    }
  }
  out3[m * N + p.e] = acc;
}

}  // namespace

hipError_t interp_dx(int ker, const Geo &g, int K, const double *X, const double *a3, const double *b, double scale,
                     double *out, hipStream_t s) {
  if (K == 0) return hipSuccess;
  dim3 grid((K + 127) / 128), block(128);
  if (ker == KER_PESKIN4)
    hipLaunchKernelGGL(k_interp_dx<KER_PESKIN4>, grid, block, 0, s, g, K, X, a3, b, scale, out);
  else
    hipLaunchKernelGGL(k_interp_dx<KER_ROMA3>, grid, block, 0, s, g, K, X, a3, b, scale, out);
  return hipGetLastError();
}

hipError_t convection_adjoint(const Geo &g, const double *u3, const double *r3, double *out3, hipStream_t s) {
  RowLaunch L = row_launch(g, 2 * g.n0 * 3);
  hipLaunchKernelGGL(k_conv_adj, L.grid, L.block, 0, s, g, u3, r3, out3);
  return hipGetLastError();
}

}  // namespace ibs
