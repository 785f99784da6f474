// Host-side declarations shared between the kernel translation units and the
// solver driver.  Every launcher enqueues on the given stream and returns the
// launch status; none of them synchronises.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dev.h"

namespace ibs {

// ---- kernel timing probes (probe.hip) --------------------------------------
enum ProbeId {
  PR_SMOOTH = 0, PR_SMOOTH_FIRST, PR_RESTRICT, PR_PROLONG, PR_LAP, PR_BAND_DIV,
  PR_BAND_FACE, PR_INTERP_GRAD, PR_INTERP_FACE, PR_MULTIDOT, PR_UPDATE_NORM, PR_COARSE, PR_HELM_SWEEP,
  PR_HELM_RESID, PR_VCYCLE, PR_MOM_RHS, PR_HELM_FIRST, PR_TILE_DOWN, PR_TILE_UP, PR_COUNT
};
struct ProbeState;  // per handle
ProbeState *probe_new();
void probe_free(ProbeState *ps);
ProbeState *probe_bind(ProbeState *ps);  // binds ps to the calling thread, returns the previous binding
struct ProbeBind {
  ProbeState *prev;
  explicit ProbeBind(ProbeState *ps) : prev(probe_bind(ps)) {}
  ~ProbeBind() { probe_bind(prev); }
};
// Launches made while a handle's state is bound are timed if their probe is
// on; each probed launch also records its algorithmic bytes (every operand
// read once, every result written once), given by the launch site.
int probe_begin(int id, hipStream_t s, double bytes);
void probe_end(int id, int slot, hipStream_t s);
void probe_enable(ProbeState *ps, int id, bool on);
hipError_t probe_read(ProbeState *ps, int id, long long *count, double *ms, double *bytes, bool reset);
// Lagrangian point count and the cells of the active (support-reached) band
// tiles of the bound handle, for the byte models of the spreading and
// interpolation launches; set by the handle whenever it bins its points.
void probe_set_points(ProbeState *ps, long long K, long long band_cells);
long long probe_points();
long long probe_band_cells();
struct ProbeScope {
  int id, slot;
  hipStream_t s;
  ProbeScope(int id_, hipStream_t s_, double bytes = 0.0) : id(id_), slot(probe_begin(id_, s_, bytes)), s(s_) {}
  ~ProbeScope() { probe_end(id, slot, s); }
};
// A probe stamped by the kernel itself: the one launch inside the scope must
// be made with hipExtLaunchKernelGGL and the events of probe_ext_take (null
// when the probe is off).
int probe_ext_begin(int id, double bytes);
void probe_ext_take(hipEvent_t *start, hipEvent_t *stop);
void probe_ext_end(int id, int slot, hipStream_t s);
struct ProbeExt {
  int id, slot;
  hipStream_t s;
  ProbeExt(int id_, hipStream_t s_, double bytes = 0.0) : id(id_), slot(probe_ext_begin(id_, bytes)), s(s_) {}
  ~ProbeExt() { probe_ext_end(id, slot, s); }
};

// ---- launch shapes ---------------------------------------------------------
struct RowLaunch {
  dim3 grid, block;
};
RowLaunch row_launch(const Geo &g, int nz);  // nz = grid.z (2*n0*ncomp, or n0 for one colour)

Geo make_geo(int n0, int n1, int n2, int bc0, int bc1, int bc2, double h);
inline long long geo_cells(const Geo &g) { return 2 * g.half; }

// ---- grid kernels (kernels_grid.hip) ---------------------------------------
hipError_t to_split(const Geo &g, int ncomp, const double *nat, double *spl, hipStream_t s);
// nat = spl - mult * sum[0] with sum on the device (null: a plain copy)
hipError_t to_natural(const Geo &g, int ncomp, const double *spl, double *nat, hipStream_t s,
                      const double *sum = nullptr, double mult = 0.0);
template <typename T, typename TY = double>
hipError_t lap_apply(const Geo &g, const T *x, TY *y, hipStream_t s);  // y = L x
hipError_t grad_apply(const Geo &g, const double *p, double *f3, double alpha, const double *add3,
                      hipStream_t s);  // f3 = add3 + alpha G p   (add3 may be null)
hipError_t div_apply(const Geo &g, const double *u3, double *y, double alpha,
                     hipStream_t s);  // y = alpha D u
hipError_t fill(double *x, long long n, double v, hipStream_t s);
hipError_t fill_i32(int *x, long long n, int v, hipStream_t s);
hipError_t zero_wall_faces(const Geo &g, double *u3, hipStream_t s);
hipError_t helm_apply(const Geo &g, double a0, double nu, const double *u3, double *y3,
                      hipStream_t s);
hipError_t mom_rhs(const Geo &g, double dt, const double *u3, const double *um3, const double *p,
                   double *out3, double *guess3, hipStream_t s);  // guess3 (may be null) = 2u - um
hipError_t convection(const Geo &g, const double *u3, double *out3, hipStream_t s);
// helm_resid: r = b - A x (in precision TR), per-block partial sums of |r|^2
template <typename TR>
hipError_t helm_resid(const Geo &g, double a0, double nu, const double *x3, const double *b3,
                      TR *r3, double *part, int *nblocks, hipStream_t s);
int helm_resid_blocks(const Geo &g);
template <typename T>
hipError_t zero_t(T *x, long long n, hipStream_t s);
// red-black SOR half sweep for A e = r on the three face grids (plane march)
template <typename T, typename TB>
hipError_t helm_sor(const Geo &g, double a0, double nu, double omega, T *x3, const TB *b3, int color,
                    hipStream_t s);
template <typename T>
hipError_t helm_sor_first(const Geo &g, double a0, double nu, double omega, T *x3, const T *b3, hipStream_t s);
template <typename T>
hipError_t add_cast(double *y, const T *x, long long n, hipStream_t s);  // y += x
template <typename T>
hipError_t cast_copy(T *y, const double *x, long long n, hipStream_t s);

// ---- multigrid (kernels_mg.hip) --------------------------------------------
// first sweep from x = 0 (red from b, then black); the red values are
// stored only with store_red (else a following half sweep overwrites them)
template <typename T, typename TB>
hipError_t mg_smooth_first(const Geo &g, T *x, const TB *b, bool store_red, hipStream_t s);
template <typename T, typename TB>
hipError_t mg_smooth(const Geo &g, T *x, const TB *b, int color, hipStream_t s);
template <typename T, typename TB>
hipError_t mg_restrict(const Geo &gf, const T *xf, const TB *bf, const Geo &gc, T *bc, hipStream_t s);
template <typename T>
hipError_t mg_prolong(const Geo &gf, T *xf, const Geo &gc, const T *xc, hipStream_t s);
// tile levels: the descent of a level (pre sweeps from x = 0, x written, the
// coarse right-hand side bc) and its ascent (xout = xin + P xc, then post
// sweeps) in one launch each, for 8^3-divisible grids with gc = g / 2 and
// 1 or 2 pre / post sweeps (tile_level_fits)
bool tile_level_fits(const Geo &g, const Geo &gc, int pre, int post);
template <typename T, typename TB>
hipError_t mg_tile_down(const Geo &g, T *x, const TB *b, const Geo &gc, T *bc, int pre, hipStream_t s);
template <typename T, typename TB>
hipError_t mg_tile_up(const Geo &g, const T *xin, T *xout, const TB *b, const Geo &gc, const T *xc, int post,
                      hipStream_t s);

template <typename T, typename TB>
hipError_t mg_coarse(const Geo &gc, const TB *b, T *x, int cycles, int sweeps, hipStream_t s);
int coarse_max_cells();
// exact coarse solve by fast diagonalisation; fd from coarse_fd_build (device copy)
template <typename T, typename TB>
hipError_t mg_coarse_fd(const Geo &gc, const TB *b, T *x, const double *fd, hipStream_t s);
int coarse_fd_size(const int n[3]);  // doubles
// the last two levels (fine grid gf of at most 4096 cells and its coarsest
// grid gc, solved exactly with fd from coarse_fd_build) in one LDS workgroup:
// x = the V-cycle of those two levels applied to b, from x = 0
// (tab: the per-thread tables from mg_subcycle_tables, subcycle_table_ints()
// ints, built once per grid pair)
bool subcycle_fits(const Geo &gf, const Geo &gc);
int subcycle_table_ints();
hipError_t mg_subcycle_tables(const Geo &gf, const Geo &gc, int *tab, hipStream_t s);
template <typename T, typename TB>
hipError_t mg_subcycle(const Geo &gf, const Geo &gc, const TB *b, T *x, const double *fd, const int *tab, int pre,
                       int post, hipStream_t s);
// z = L^+ v on a grid by fast diagonalisation (bfloat16 matrix-core
// transforms); w1, w2: bfloat16 scratch grids; blob: eigenbases packed by
// fd_blob_pack from coarse_fd_build's output (device copy)
template <typename TI, typename T>
hipError_t fd_precond(const Geo &g, const TI *v, T *z, unsigned short *w1, unsigned short *w2, const void *blob,
                      float vscale, hipStream_t s);
size_t fd_blob_bytes(const int n[3]);
// z = L^+ v exactly by fast diagonalisation in float64 (split layout in and
// out); w1, w2: natural-layout float64 scratch grids; blob: fdx_blob_pack of
// coarse_fd_build's eigen-decomposition of the grid (device copy)
hipError_t fdx_precond(const Geo &g, const double *v, double *z, double *w1, double *w2, const double *blob,
                       hipStream_t s);
size_t fdx_blob_doubles(const int n[3]);
void fdx_blob_pack(const int n[3], const double *q, double *blob);
void fd_blob_pack(const int n[3], const double *qd, unsigned char *out);

void coarse_fd_build(const int n[3], const int bc[3], double h, double *out);
constexpr int COARSE_FD_MAXN = 32;
// whether the single-workgroup exact coarse solver takes this grid
inline bool coarse_lds_fits(int n0, int n1, int n2) {
  return n0 <= COARSE_FD_MAXN && n1 <= COARSE_FD_MAXN && n2 <= COARSE_FD_MAXN && n0 * n1 * n2 <= 4096;
}

// ---- Lagrangian points (kernels_ib.hip) ------------------------------------
struct BodyDev {
  double c[3];
  double R[9];
  double v[3];
  double w[3];
};
// ---- two-way coupling sums (kernels_body.hip) ------------------------------
// Per body: its point range in natural order and the node box that holds
// every velocity node with a non-zero volume fraction (lo may lie outside the
// grid; periodic axes wrap, wall axes clip).
struct BodySpan {
  int k0, kn;
  double c[3];
  double radius;
  int lo[3], dim[3];
};
constexpr int VOL_CHUNKS = 16;  // workgroups per (body, velocity component)
// Reverse mode of the volume integrals of one body: ubar += alpha h^3 (ib + jb x r)
// on the body's node box and part[(d * VOL_CHUNKS + chunk) * 3 + q] the partial
// centre cotangents (summed on the host)
hipError_t body_volume_adjoint(const Geo &g, const BodySpan &span, const double ib[3], const double jb[3],
                               const double *u, double *ubar, double *part, hipStream_t s);
// Per-point transposes of the force / torque sums and of U = u_s + w x L~
// (natural order; coef[9 b ..] = (Fbar, Tbar, w) of body b)
hipError_t point_adjoint(int K, const int *bodyof, const double *off, const BodyDev *bodies, const double *coef,
                         double h3, const double *phi, const double *ubar, double *phibar, double *lbar,
                         hipStream_t s);
// out[12 b + 0..5] = (h^3 sum Phi, h^3 sum L~ x Phi) of body b (phi in natural order)
hipError_t body_force_torque(int nb, const BodyDev *bodies, const BodySpan *span, const double *off,
                             const double *phi, double h3, double *out, hipStream_t s);
// out[12 b + 6..11] = (sum alpha u h^3, sum alpha r x u h^3); part holds
// nb * 3 * VOL_CHUNKS * 3 doubles
hipError_t body_volume_integrals(const Geo &g, int nb, const BodySpan *span, const double *u, double *part,
                                 double *out, hipStream_t s);
hipError_t points_place(const Geo &g, int K, const BodyDev *bodies, const int *body_of,
                        const double *off, double *X, double *U, int *tile, int nt0, int nt1,
                        int nt2, hipStream_t s);
hipError_t bin_count(int K, const int *tile, int *counts, hipStream_t s);
hipError_t scan_exclusive(const int *in, int *out, int n, int *tmp, hipStream_t s);  // out has n+1 entries
hipError_t bin_scatter(int K, const int *tile, const int *start, int *fillc, int *perm_tmp,
                       hipStream_t s);
hipError_t bin_canon(int K, const int *tile, const int *start, const int *perm_tmp, int *perm,
                     hipStream_t s);
hipError_t compact(int n, const int *flags, const int *pos, int *list, hipStream_t s);
hipError_t gather3(int K, const int *perm, const double *src, double *dst, hipStream_t s);
hipError_t scatter3(int K, const int *perm, const double *src, double *dst, hipStream_t s);
hipError_t scale3(int K, const double *x, double alpha, const double *y, double beta, double *out,
                  hipStream_t s);  // out = alpha x + beta y (y may be null)

// interp: out[p][d] = alpha * (W^T src)[p][d] + beta * y[p][d] for the points
// of the ntiles_nz non-empty tiles listed in tiles (points sorted by tile,
// tstart = tile offsets; -1 entries of the list are holes); src is a face
// field (interp_face) or the gradient of a cell field (interp_grad).
template <typename T>
hipError_t interp_grad(int ker, const Geo &g, int nt1, int nt2, int ntiles_nz, const int *tiles,
                       const int *tstart, const double *X, const T *z, double alpha, const double *y,
                       double beta, double *out, hipStream_t s, bool f32 = false);
hipError_t interp_face(int ker, const Geo &g, int nt1, int nt2, int ntiles_nz, const int *tiles,
                       const int *tstart, const double *X, const double *u3, double alpha, const double *y,
                       double beta, double *out, hipStream_t s);
// Band tiles: R x R x R point tiles (4R cells per axis, R = 1 or 2), the
// units of the spreading kernels; nt* count point tiles.
// Touch lists (the band tiles whose face boxes a point's support meets),
// band tile by band tile (no atomics, fixed order): with list == nullptr the
// counts of the listed band tiles (tiles == nullptr: 0..ntl-1), else their
// lists at lstart; ntl bounds the launch, *ntl_dev (if given) is the count
hipError_t touch_tiles(int ker, const Geo &g, int nt0, int nt1, int nt2, int ntl, const int *ntl_dev,
                       const int *tiles, const int *tstart, const double *X, int *counts, const int *lstart,
                       int *list, hipStream_t s);
// flags[b] = 1 for the band tiles holding a point tile within one point tile of
// the n point tiles nz[0..n)
hipError_t mark_near(const Geo &g, int nt0, int nt1, int nt2, int n, const int *nz, int *flags,
                     hipStream_t s);
// launch order of the n tiles of a list (XCD-chunked, longest lists first in
// each chunk): order_launch_count(n) entries, -1 in the holes
hipError_t order_active(int n, const int *active, const int *lstart, int *out, hipStream_t s);
int order_launch_count(int n);
hipError_t positive_flags(int n, const int *counts, int *flags, hipStream_t s);
// band: for the active band tiles, out += alpha D (W q)   (div = true, cell field)
//                          or out += alpha W q       (div = false, face field)
hipError_t band_apply(int ker, bool div, const Geo &g, int nt1, int nt2, int nactive, const int *active,
                      const int *lstart, const int *list, const double *X, const double *q, double alpha,
                      double *out, hipStream_t s, bool f32 = false);
hipError_t band_apply(int ker, bool div, const Geo &g, int nt1, int nt2, int nactive, const int *active,
                      const int *lstart, const int *list, const double *X, const double *q, double alpha,
                      float *out, hipStream_t s, bool f32 = true);

// ---- reductions / Krylov vector kernels (kernels_krylov.hip) ---------------
int red_blocks();
// basis V of type TV (float32 in the FP32-MG form, float64 otherwise); n, stride even
template <typename TV, typename TW = double>  // w in TW (float64, or float32 in the float32 FGMRES cycle)
hipError_t multidot(const TW *w, const TV *V, long long stride, int nv, long long n,
                    double *part, hipStream_t s);  // part[blk*nv + i]
hipError_t finalize(const double *part, int nblk, int nv, double *out, hipStream_t s,
                    double *host = nullptr);  // host: optional pinned mirror of out
template <typename TV>
hipError_t update_norm(double *w, const TV *V, long long stride, int nv, const double *hcoef,
                       long long n, double *part, hipStream_t s);
// Krylov coefficients passed by value to a kernel: one per basis vector of
// a restart cycle of up to 64 iterations, plus the new vector's (65)
constexpr int KCOEF_MAX = 65;
struct KCoef {
  double v[KCOEF_MAX];
};
// vout = (TV)(w - sum_i sig2_i g_i V_i), partial |vout|^2 per block (g on the device)
template <typename TV, typename TW = double>
hipError_t update_cast_norm(TV *vout, const TW *w, const TV *V, long long stride, int nv, const double *g,
                            const KCoef &sig2, long long n, double *part, hipStream_t s);  // w -= sum h_i V_i ; |w|^2
hipError_t scale_inplace(double *x, long long n, double alpha, hipStream_t s);
// ---- reverse-mode step (kernels_adj.hip) ------------------------------------
// out[k][e] += scale * d/dX_{k,e} (a^T W(X) b), a a face field, b [K][3]
hipError_t interp_dx(int ker, const Geo &g, int K, const double *X, const double *a3, const double *b, double scale,
                     double *out, hipStream_t s);
// out3 = J_N(u)^T r (wall faces 0)
hipError_t convection_adjoint(const Geo &g, const double *u3, const double *r3, double *out3, hipStream_t s);

hipError_t scale_copy(double *y, const double *x, long long n, double alpha, hipStream_t s);
// x = (first ? 0 : x) + sum_j y_j Z_j; part (optional): sol_blocks() partial
// sums of the new x
int sol_blocks();
template <typename T>
hipError_t sol_update(double *x, const T *Z, long long stride, int nz, const KCoef &y, long long n,
                      hipStream_t s, bool first = false, double *part = nullptr);
hipError_t axpby(double *y, const double *x, long long n, double a, double b,
                 hipStream_t s);  // y = a x + b y
hipError_t add_scalar_dev(double *x, long long n, const double *dscalar, double mult,
                          hipStream_t s);  // x += mult * (*dscalar)
hipError_t sub_mul(double *r, const double *b, const double *ax, long long n, double *part,
                   hipStream_t s);  // r = b - ax, partial |r|^2
// y = (TV)(b - mult * bsum[0] - ax) (ax, bsum optional), partial |.|^2 of the float64 value
template <typename TV>
hipError_t sub_cast_norm(TV *y, const double *b, const double *ax, long long n, double *part, hipStream_t s,
                         const double *bsum = nullptr, double mult = 0.0);
hipError_t dot2(const double *a, const double *b, long long n, double *part,
                hipStream_t s);
hipError_t lincomb(double *y, const double *a, double ca, const double *b, double cb, const double *c, double cc,
                   const double *d, int nd, long long n, double *part, hipStream_t s);
hipError_t dots2(const double *a, const double *b0, const double *b1, long long n, double *part, hipStream_t s);
hipError_t abs_sums(const double *a, const double *b, long long n, double *part, hipStream_t s);
hipError_t sumsq3(const double *a, long long na, const double *b, long long nb, const double *c, long long nc,
                  double *part, hipStream_t s);  // partial a.b (sum of a when b is null)

}  // namespace ibs
