// Host driver and C ABI of the coupled immersed-boundary solver.
//
//   * workspace: every device array is carved from the caller's buffer;
//   * bodies: rigid-sphere kinematics on the host (paper Sec. 2.1-2.2), point
//     placement and tile binning on the device;
//   * V-cycle driver (FP32 or FP64) approximating L^+ (Sec. 4.1-4.2, Sec. 7);
//   * flexible GMRES(m) on S~ = L + c^-1 B^T B, right-preconditioned by the
//     V-cycle, classical Gram-Schmidt with fused multi-dot / update kernels,
//     Hessenberg least squares with Givens rotations on the host (one
//     device-to-host copy of j+2 doubles per iteration);
//   * the pressure-force correction (Sec. 3.1 eq. Saddle, Sec. 4.1 eqs.
//     ApproxSchurPrimalP/F) and the one-way / two-way time steps (Sec. 3.1,
//     Sec. 3.2.1);
//   * momentum solve (eq. ustar) by defect correction with red-black SOR
//     relaxations at the optimal factor for the constant-coefficient A.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/ibschur.h"
#include "internal.h"

using namespace ibs;

// Static scratch of sim_solve_schur_noalloc (callers that cannot allocate):
// the work arrays of one Schur solve, one copy per device for the life of
// the process.  In host code `scratch` only names the symbol; its device
// address comes from hipGetSymbolAddress (noalloc_scratch_setup).
constexpr size_t NOALLOC_SCRATCH_BYTES = 64ull << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int MAX_BODIES = 4096;
constexpr int MAX_RESTART = 64;
static_assert(KCOEF_MAX >= MAX_RESTART + 1, "FGMRES writes sig_{j+1}^2 for j < MAX_RESTART");
// A float32 FGMRES cycle restarts from the float64 true residual once its
// residual estimate has dropped by this factor: two cycles reach 1e-11.
// Measured on the 256^3 benchmark system at rtol 3e-9 (12 iterations in
// every case): 1e-5 and 3e-6 7.05 ms, 1e-6 7.15, 3e-7 7.28, 1e-7 7.48 ms per
// solve (a longer first cycle orthogonalises against more vectors).
constexpr double FP32_CYCLE_DROP = 3e-6;

struct HostBody {
  sim_body b;
  int k0 = 0, kn = 0;
  double rmax = 0.0;
  // free-motion state (inertial frame)
  double xc[3], xc_m[3], us[3], us_m[3], w[3], w_m[3], R[9];
  double I_n[3], I_m[3], J_n[3], J_m[3];
  double xc1[3], R1[9];  // predicted centre and orientation of the step in progress
};

struct Level {
  Geo g;
  void *x = nullptr;
  void *b = nullptr;
  void *xs = nullptr;  // a tile level's pre-smoothed x (null: the level runs the march kernels)
};

}  // namespace

struct sim_s {
  sim_config cfg;
  hipStream_t st = nullptr;
  std::string err;
  Geo g;
  long long N = 0;  // cells
  int nt0 = 0, nt1 = 0, nt2 = 0;
  long long ntiles = 0;
  int Kmax = 0, K = 0, nb = 0;
  bool fp32 = false;
  int ker = 0;
  double c = 0.5;
  double t = 0.0;
  long long nstep = 0;
  // fields (double, split layout)
  double *U = nullptr, *UM = nullptr, *USTAR = nullptr, *RHSU = nullptr, *TMP3 = nullptr;
  double *P = nullptr, *RHSP = nullptr, *BVEC = nullptr, *PP = nullptr, *TMPC = nullptr;
  // Krylov basis and preconditioned vectors (float32 in the FP32-MG form)
  void *V = nullptr;
  void *Z = nullptr;
  // momentum relaxation work (T precision)
  void *HR = nullptr, *HE0 = nullptr;
  std::vector<Level> lv;  // lv[0] is the finest grid (x, b supplied per call)
  // points
  double *OFF = nullptr, *XN = nullptr, *UN = nullptr, *PHIN = nullptr;
  int *BODYOF = nullptr, *TILE = nullptr, *PERM = nullptr, *PERMTMP = nullptr;
  double *XS = nullptr, *US = nullptr, *Q = nullptr, *RF = nullptr, *PHIP = nullptr, *PHIS = nullptr,
         *PT3 = nullptr;
  int *COUNTS = nullptr, *TSTART = nullptr, *FILLC = nullptr, *FLAGS = nullptr, *FPOS = nullptr,
      *ACTIVE = nullptr, *SCANTMP = nullptr;
  int *TCOUNT = nullptr, *TLSTART = nullptr, *TLIST = nullptr;
  long long tl_cap = 0;  // capacity of the touch lists
  int nactive = 0;       // launch count of ACTIVE (active tiles in launch order)
  int *NZT = nullptr;    // non-empty point tiles in launch order (-1: hole)
  int nnz = 0;           // launch count of NZT
  int ntouch = 0;
  BodyDev *BODIES = nullptr;
  std::vector<HostBody> bodies;
  bool any_free = false;
  // two-way sums: node boxes, per-body results [nb][12], volume-integral partials
  BodySpan *SPAN = nullptr;
  double *BSUM = nullptr, *VPART = nullptr;
  bool vol_init = false;
  std::vector<BodySpan> hspan;  // host copy (kept alive for the asynchronous upload)
  // reverse mode: point cotangent work arrays [5][K][3]; the last step can be
  // transposed while adj_ready (a one-way step with one correction)
  double *ADJ = nullptr;
  bool adj_ready = false;
  // reverse mode of a two-way step (cfg.record_two_way): per outer pass k the
  // velocity u^k before the correction, p'_k, and in tile order Phi^(k),
  // Phi'_k and RHS_F; the pass count, the body velocities of every pass
  // (6 per body and pass) and the body state before the step (18 per body);
  // ADJ2 holds natural-order point work and the per-body coefficients.
  double *REC_U = nullptr, *REC_PP = nullptr, *REC_PHI = nullptr, *REC_PHIP = nullptr, *REC_RF = nullptr;
  double *ADJ2 = nullptr;
  int rec_passes = 0;
  bool adj2_ready = false;
  std::vector<double> rec_body, rec_pre;
  // reductions
  double *PART = nullptr, *RED = nullptr;
  double *COARSEFD = nullptr;  // eigen-decomposition of the coarsest grid (exact coarse solve)
  int *SUBTAB = nullptr;       // the subcycle's per-thread cell tables (built at sim_create)
  // whole-grid fast-diagonalisation preconditioner: eigenbases (float) and two
  // bfloat16 scratch grids
  bool fastdiag = false;
  bool fdx = false;                // exact float64 fast diagonalisation (preconditioner)
  double *FDXQ = nullptr;          // its eigenbases and eigenvalues (fdx_blob_pack)
  double *FDX1 = nullptr, *FDX2 = nullptr;  // two natural-layout float64 work grids
  bool coarse_mfma = false;  // exact coarse solve on the matrix cores
  unsigned char *FDQ = nullptr;  // packed eigenbases (fd_blob_pack)
  double *BCG = nullptr;  // BiCGStab vectors r, r^, p, v, s, t (float64)
  unsigned short *FDW1 = nullptr, *FDW2 = nullptr;
  double *hpin = nullptr;
  double *hpin_dev = nullptr;  // device address of hpin
  // kernel timing probes of this handle; the timing events of a Schur solve
  ProbeState *probes = nullptr;
  hipEvent_t ev_solve[2] = {nullptr, nullptr};
  hipEvent_t ev_iter = nullptr;  // end of an FGMRES iteration's coefficients (pipelined wait)
  // multigrid level sizes (3 per level, finest first)
  std::vector<int> dims;
  // the device address of this device's static scratch (sim_solve_schur_noalloc)
  void *noalloc_scratch = nullptr;
  // last-step statistics
  sim_step_stats last{};
  bool have_bodies = false;
};

namespace {

// ---------------------------------------------------------------------------
// error plumbing
#define CKH(call)                                                                     \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess) return fail(s, SIM_EDEVICE, std::string(#call) + ": " +     \
                                                      hipGetErrorString(e_));         \
  } while (0)

sim_status fail(sim_t s, sim_status code, const std::string &msg) {
  if (s) s->err = msg;
  return code;
}

// bump allocator over the workspace (base may be null for sizing)
struct Carver {
  char *base;
  size_t off = 0;
  explicit Carver(void *b) : base((char *)b) {}
  void *take(size_t bytes) {
    off = (off + 255) & ~(size_t)255;
    void *p = base ? base + off : nullptr;
    off += bytes;
    return p;
  }
  template <typename T>
  T *arr(long long n) { return (T *)take(sizeof(T) * (size_t)(n > 0 ? n : 1)); }
};

bool is_even(int x) { return (x & 1) == 0; }

// IBSCHUR_MARCH_FULL_CHUNKS=1 in the environment at sim_create: every grid,
// however small, runs the plane-marching kernels with their full chunk of
// planes per workgroup, the launch shape of the large grids (so that small
// test problems exercise the same register-window code paths).
int march_min_blocks_setting() {
  const char *e = getenv("IBSCHUR_MARCH_FULL_CHUNKS");
  return (e && e[0] == '1' && e[1] == '\0') ? 0 : MARCH_MIN_BLOCKS_DEFAULT;
}

// Multigrid levels of at most this many cells run as tile levels (two
// launches per level instead of seven: k_tile_down, k_tile_up).  On a 256^3
// grid that is the 64^3 and 32^3 levels: 10.0 + 7.5 us and 6.8 + 6.2 us per
// level against seven launches of about 4.5 us (142.5 -> 149.0 solves/s);
// with the 128^3 level too, the tiles' redundant halo work (an 8^3 tile loads
// 16^3 cells) outweighs the launches saved there (143.5 solves/s), and the
// finest levels stream through the march kernels near the bandwidth bound.
// IBSCHUR_MG_TILE_CELLS in the environment at sim_create overrides it
// (0: no tile levels).
constexpr long long MG_TILE_CELLS_DEFAULT = 64LL * 64 * 64;
long long mg_tile_cells_setting() {
  const char *e = getenv("IBSCHUR_MG_TILE_CELLS");
  if (!e || !e[0]) return MG_TILE_CELLS_DEFAULT;
  char *end = nullptr;
  const long long v = strtoll(e, &end, 10);
  return (end && *end == '\0' && v >= 0) ? v : MG_TILE_CELLS_DEFAULT;
}
// Whether level l of the hierarchy dims (3 entries per level) runs as a tile
// level: a V-cycle preconditioner, a next level of half the edges, edges that
// are multiples of the 8-cell tile, 1 or 2 pre- and post-sweeps, and at most
// mg_tile_cells_setting() cells.
bool tile_level(const sim_config *c, const std::vector<int> &dims, size_t l) {
  if (c->precond != SIM_PRECOND_VCYCLE || 3 * l + 5 >= dims.size()) return false;
  if (c->mg_pre < 1 || c->mg_pre > 2 || c->mg_post < 1 || c->mg_post > 2) return false;
  long long cells = 1;
  for (int a = 0; a < 3; ++a) {
    const int n = dims[3 * l + a];
    if (n % 8 != 0 || dims[3 * l + 3 + a] * 2 != n) return false;
    cells *= n;
  }
  return cells <= mg_tile_cells_setting();
}

// Validate the configuration; fills the level dimensions. Returns "" if ok.
std::string validate(const sim_config *c, std::vector<int> *dims) {
  if (!c) return "null config";
  for (int a = 0; a < 3; ++a) {
    if (c->n[a] < 16 || c->n[a] % 4) return "every n must be a multiple of 4 and >= 16";
    if (c->bc[a] != SIM_BC_PERIODIC && c->bc[a] != SIM_BC_NOSLIP && c->bc[a] != SIM_BC_FREESLIP)
      return "bad bc";
    if (!(c->len[a] > 0)) return "len must be positive";
  }
  double h0 = c->len[0] / c->n[0];
  for (int a = 1; a < 3; ++a)
    if (fabs(c->len[a] / c->n[a] - h0) > 1e-12 * h0) return "cells must be cubic";
  if (!(c->dt > 0) || !(c->nu >= 0)) return "dt must be > 0 and nu >= 0";
  if (!(c->lump_c > 0)) return "lump_c must be > 0";
  if (c->delta != SIM_DELTA_PESKIN4 && c->delta != SIM_DELTA_ROMA3) return "bad delta kernel";
  if (c->precision != SIM_PREC_FP64 && c->precision != SIM_PREC_FP32MG) return "bad precision";
  if (c->krylov_restart < 1 || c->krylov_restart > MAX_RESTART) return "krylov_restart must be 1..64";
  if (c->krylov_maxit < 1) return "krylov_maxit must be >= 1";
  if (!(c->krylov_rtol > 0)) return "krylov_rtol must be > 0";
  if (c->mg_pre < 1 || c->mg_post < 0 || c->mg_coarse_sweeps < 0) return "mg_pre >= 1, mg_coarse_sweeps >= 0";
  if (c->precond != SIM_PRECOND_VCYCLE && c->precond != SIM_PRECOND_FASTDIAG &&
      c->precond != SIM_PRECOND_FASTDIAG_EXACT)
    return "bad precond";
  if (c->precond == SIM_PRECOND_FASTDIAG_EXACT && c->precision != SIM_PREC_FP64)
    return "the exact fast-diagonalisation preconditioner runs in float64: precision must be FP64";
  if (c->krylov != SIM_KRYLOV_FGMRES && c->krylov != SIM_KRYLOV_BICGSTAB) return "bad krylov method";
  if (c->outer_iters < 1) return "outer_iters must be >= 1";
  if (c->helm_maxit < 1 || !(c->helm_rtol > 0)) return "helm_maxit >= 1 and helm_rtol > 0";
  // multigrid hierarchy: halve while above mg_coarsest or too big for the
  // coarse kernel.  The fast-diagonalisation preconditioner never runs a
  // V-cycle, so it keeps the fine level only and takes no multigrid limits.
  int n0 = c->n[0], n1 = c->n[1], n2 = c->n[2];
  if (dims) dims->clear();
  if (dims) { dims->push_back(n0); dims->push_back(n1); dims->push_back(n2); }
  // exact coarse solves (mg_coarse_sweeps = 0) take any coarsest grid: small
  // ones in one LDS workgroup, larger ones on the matrix cores
  const bool fdg = c->precond == SIM_PRECOND_FASTDIAG || c->precond == SIM_PRECOND_FASTDIAG_EXACT;
  const bool exact = fdg || c->mg_coarse_sweeps == 0;
  while (!fdg && (std::max(n0, std::max(n1, n2)) > c->mg_coarsest ||
                  (!exact && (long long)n0 * n1 * n2 > coarse_max_cells()))) {
    if (!is_even(n0) || !is_even(n1) || !is_even(n2) || n0 < 4 || n1 < 4 || n2 < 4) break;
    n0 /= 2; n1 /= 2; n2 /= 2;
    if (dims) { dims->push_back(n0); dims->push_back(n1); dims->push_back(n2); }
  }
  if (!exact && (long long)n0 * n1 * n2 > coarse_max_cells()) return "grid cannot be coarsened to the coarse-kernel size";
  if (!exact && (!is_even(n0) || !is_even(n1) || !is_even(n2))) return "coarsest multigrid grid must have even sizes";
  // the matrix-core fast diagonalisation takes sizes that are multiples of 8, up to 512
  auto mfma_fd_ok = [](int a, int b, int d) { return a % 8 == 0 && b % 8 == 0 && d % 8 == 0 && a <= 512 && b <= 512 && d <= 512; };
  if (c->precond == SIM_PRECOND_FASTDIAG && !mfma_fd_ok(c->n[0], c->n[1], c->n[2]))
    return "the fast-diagonalisation preconditioner takes axis sizes that are multiples of 8, up to 512";
  if (exact && c->precond == SIM_PRECOND_VCYCLE && !coarse_lds_fits(n0, n1, n2) && !mfma_fd_ok(n0, n1, n2))
    return "an exact coarse solve above the single-workgroup size needs coarsest sizes that are multiples of 8, up to 512";
  // the plane-marching kernels handle two in-row values per thread on every grid-wide level
  if (dims)
    for (size_t l = 0; l + 3 < dims->size(); l += 3)
      if ((*dims)[l + 2] % 4) return "axis-2 size of every multigrid level above the coarsest must be a multiple of 4";
  return "";
}

// The arrays a pressure-force Schur solve works in besides the handle's
// state (points, tiles, touch lists, eigenbases): staged right-hand sides,
// the Krylov basis and preconditioned vectors, BiCGStab vectors, the
// multigrid levels below the finest, the point work vector of S~, the
// fast-diagonalisation work grids and the reduction partials.
struct SolveScratch {
  double *RHSP = nullptr, *BVEC = nullptr, *PP = nullptr, *TMPC = nullptr, *BCG = nullptr;
  void *V = nullptr, *Z = nullptr;
  static constexpr int MAX_LEVELS = 24;
  int nlv = 0;                       // levels below the finest
  void *lvx[MAX_LEVELS] = {}, *lvb[MAX_LEVELS] = {};
  void *lvs[MAX_LEVELS + 1] = {};    // pre-smoothed x of the tile levels, from the finest
  double *Q = nullptr, *RF = nullptr, *PHIP = nullptr, *PART = nullptr, *RED = nullptr;
  unsigned short *FDW1 = nullptr, *FDW2 = nullptr;
  double *FDX1 = nullptr, *FDX2 = nullptr;
};

void put_solve_scratch(sim_s *s, const SolveScratch &q) {
  s->RHSP = q.RHSP; s->BVEC = q.BVEC; s->PP = q.PP; s->TMPC = q.TMPC; s->BCG = q.BCG;
  s->V = q.V; s->Z = q.Z;
  for (int l = 0; l < q.nlv; ++l) {
    s->lv[l + 1].x = q.lvx[l];
    s->lv[l + 1].b = q.lvb[l];
  }
  for (size_t l = 0; l < s->lv.size() && l <= (size_t)SolveScratch::MAX_LEVELS; ++l) s->lv[l].xs = q.lvs[l];
  s->Q = q.Q; s->RF = q.RF; s->PHIP = q.PHIP; s->PART = q.PART; s->RED = q.RED;
  s->FDW1 = q.FDW1; s->FDW2 = q.FDW2;
  s->FDX1 = q.FDX1; s->FDX2 = q.FDX2;
}

SolveScratch get_solve_scratch(const sim_s *s) {
  SolveScratch q;
  q.RHSP = s->RHSP; q.BVEC = s->BVEC; q.PP = s->PP; q.TMPC = s->TMPC; q.BCG = s->BCG;
  q.V = s->V; q.Z = s->Z;
  for (size_t l = 1; l < s->lv.size() && q.nlv < SolveScratch::MAX_LEVELS; ++l) {
    q.lvx[q.nlv] = s->lv[l].x;
    q.lvb[q.nlv] = s->lv[l].b;
    ++q.nlv;
  }
  for (size_t l = 0; l < s->lv.size() && l <= (size_t)SolveScratch::MAX_LEVELS; ++l) q.lvs[l] = s->lv[l].xs;
  q.Q = s->Q; q.RF = s->RF; q.PHIP = s->PHIP; q.PART = s->PART; q.RED = s->RED;
  q.FDW1 = s->FDW1; q.FDW2 = s->FDW2;
  q.FDX1 = s->FDX1; q.FDX2 = s->FDX2;
  return q;
}

// Whether the configuration runs a fast diagonalisation on the matrix cores
// (whole-grid preconditioner, or a coarsest grid too large for the LDS solver).
void fd_flags(const sim_config *c, const std::vector<int> &dims, bool &fdg, bool &fdc, int fdn[3]) {
  const int cdims[3] = {dims[dims.size() - 3], dims[dims.size() - 2], dims[dims.size() - 1]};
  fdg = c->precond == SIM_PRECOND_FASTDIAG;
  fdc = !fdg && c->precond == SIM_PRECOND_VCYCLE && c->mg_coarse_sweeps == 0 &&
        !coarse_lds_fits(cdims[0], cdims[1], cdims[2]);
  for (int a = 0; a < 3; ++a) fdn[a] = fdg ? c->n[a] : cdims[a];
}

SolveScratch carve_solve(Carver &cv, const sim_config *c, long long K, long long hparts,
                         const std::vector<int> &dims) {
  SolveScratch q;
  const long long N = (long long)c->n[0] * c->n[1] * c->n[2];
  const size_t ts = c->precision == SIM_PREC_FP32MG ? sizeof(float) : sizeof(double);
  const int m = c->krylov_restart;
  q.RHSP = cv.arr<double>(N);
  q.BVEC = cv.arr<double>(N);
  q.PP = cv.arr<double>(N);
  q.TMPC = cv.arr<double>(N);
  q.V = cv.take(ts * (size_t)(m + 1) * N);
  q.Z = cv.take(ts * (size_t)std::max(m, 2) * N);  // BiCGStab keeps p^, s^ in Z[0], Z[1]
  q.BCG = c->krylov == SIM_KRYLOV_BICGSTAB ? cv.arr<double>(6 * N) : nullptr;
  for (size_t l = 3; l < dims.size() && q.nlv < SolveScratch::MAX_LEVELS; l += 3) {
    const long long nl = (long long)dims[l] * dims[l + 1] * dims[l + 2];
    q.lvx[q.nlv] = cv.take(ts * nl);
    q.lvb[q.nlv] = cv.take(ts * nl);
    ++q.nlv;
  }
  for (size_t l = 0; 3 * l < dims.size() && l <= (size_t)SolveScratch::MAX_LEVELS; ++l)
    if (tile_level(c, dims, l))
      q.lvs[l] = cv.take(ts * (size_t)dims[3 * l] * dims[3 * l + 1] * dims[3 * l + 2]);
  q.Q = cv.arr<double>(3 * K);
  q.RF = cv.arr<double>(3 * K);
  q.PHIP = cv.arr<double>(3 * K);
  const int rb = std::max(red_blocks(), 1);
  q.PART = cv.arr<double>(std::max((long long)rb * (MAX_RESTART + 2), hparts));
  q.RED = cv.arr<double>(4 * (MAX_RESTART + 2));
  bool fdg, fdc;
  int fdn[3];
  fd_flags(c, dims, fdg, fdc, fdn);
  const long long fdcells = (long long)fdn[0] * fdn[1] * fdn[2];
  q.FDW1 = (fdg || fdc) ? cv.arr<unsigned short>(fdcells) : nullptr;
  q.FDW2 = (fdg || fdc) ? cv.arr<unsigned short>(fdcells) : nullptr;
  const bool fdx = c->precond == SIM_PRECOND_FASTDIAG_EXACT;
  q.FDX1 = fdx ? cv.arr<double>(N) : nullptr;
  q.FDX2 = fdx ? cv.arr<double>(N) : nullptr;
  return q;
}

// Lay out every array; with base == nullptr only the size is computed.
size_t layout(sim_s *s, const sim_config *c, int64_t kmax, void *base, const std::vector<int> &dims) {
  Carver cv(base);
  long long N = (long long)c->n[0] * c->n[1] * c->n[2];
  bool f32 = c->precision == SIM_PREC_FP32MG;
  size_t ts = f32 ? sizeof(float) : sizeof(double);
  long long K = kmax > 0 ? kmax : 1;
  long long nt = (long long)(c->n[0] / 4) * (c->n[1] / 4) * (c->n[2] / 4);
  double *U = cv.arr<double>(3 * N), *UM = cv.arr<double>(3 * N), *USTAR = cv.arr<double>(3 * N);
  double *RHSU = cv.arr<double>(3 * N), *TMP3 = cv.arr<double>(3 * N);
  double *P = cv.arr<double>(N);
  void *HR = cv.take(ts * 3 * N), *HE0 = cv.take(ts * 3 * N);
  std::vector<Level> lv;
  int nlev = (int)dims.size() / 3;
  for (int l = 0; l < nlev; ++l) {
    Level L;
    double h = c->len[0] / c->n[0] * (double)(1 << l);
    L.g = make_geo(dims[3 * l], dims[3 * l + 1], dims[3 * l + 2], c->bc[0], c->bc[1], c->bc[2], h);
    L.g.march_min_blocks = march_min_blocks_setting();
    lv.push_back(L);
  }
  // the momentum residual writes one partial per plane-march workgroup
  const long long hparts = helm_resid_blocks(lv[0].g);
  SolveScratch sq = carve_solve(cv, c, K, hparts, dims);
  double *OFF = cv.arr<double>(3 * K), *XN = cv.arr<double>(3 * K), *UN = cv.arr<double>(3 * K);
  double *PHIN = cv.arr<double>(3 * K);
  int *BODYOF = cv.arr<int>(K), *TILE = cv.arr<int>(K), *PERM = cv.arr<int>(K), *PERMTMP = cv.arr<int>(K);
  double *XS = cv.arr<double>(3 * K), *US = cv.arr<double>(3 * K);
  double *PHIS = cv.arr<double>(3 * K);
  double *PT3 = cv.arr<double>(3 * K);
  double *ADJ = cv.arr<double>(15 * K);
  const long long npass = c->record_two_way ? c->outer_iters : 0;
  double *REC_U = npass ? cv.arr<double>(npass * 3 * N) : nullptr;
  double *REC_PP = npass ? cv.arr<double>(npass * N) : nullptr;
  double *REC_PHI = npass ? cv.arr<double>(npass * 3 * K) : nullptr;
  double *REC_PHIP = npass ? cv.arr<double>(npass * 3 * K) : nullptr;
  double *REC_RF = npass ? cv.arr<double>(npass * 3 * K) : nullptr;
  double *ADJ2 = npass ? cv.arr<double>(15 * K + 9 * MAX_BODIES + 9 * VOL_CHUNKS) : nullptr;
  int *COUNTS = cv.arr<int>(nt), *TSTART = cv.arr<int>(nt + 1), *FILLC = cv.arr<int>(nt);
  // FLAGS and ACTIVE swap roles and take launch orders with holes (nt + 8)
  int *FLAGS = cv.arr<int>(nt + 8), *FPOS = cv.arr<int>(nt + 1), *ACTIVE = cv.arr<int>(nt + 8);
  int *SCANTMP = cv.arr<int>(nt / 1024 + 16);
  long long tl_cap = 27 * K;  // a point touches at most 3 x 3 x 3 tiles
  int *TCOUNT = cv.arr<int>(nt), *TLSTART = cv.arr<int>(nt + 1), *TLIST = cv.arr<int>(tl_cap);
  int *NZT = cv.arr<int>(nt + 8);
  BodyDev *BODIES = (BodyDev *)cv.take(sizeof(BodyDev) * MAX_BODIES);
  BodySpan *SPAN = (BodySpan *)cv.take(sizeof(BodySpan) * MAX_BODIES);
  double *BSUM = cv.arr<double>(12LL * MAX_BODIES);
  double *VPART = cv.arr<double>(9LL * VOL_CHUNKS * MAX_BODIES);
  const int cdims[3] = {dims[dims.size() - 3], dims[dims.size() - 2], dims[dims.size() - 1]};
  double *COARSEFD = cv.arr<double>(coarse_fd_size(cdims));
  int *SUBTAB = cv.arr<int>(subcycle_table_ints());
  // matrix-core fast diagonalisation: of the whole grid (FASTDIAG
  // preconditioner) or of a coarsest grid too large for the LDS solver
  bool fdg, fdc;
  int fdn[3];
  fd_flags(c, dims, fdg, fdc, fdn);
  unsigned char *FDQ = (fdg || fdc) ? cv.arr<unsigned char>((long long)fd_blob_bytes(fdn)) : nullptr;
  const bool fdx = c->precond == SIM_PRECOND_FASTDIAG_EXACT;
  double *FDXQ = fdx ? cv.arr<double>((long long)fdx_blob_doubles(c->n)) : nullptr;
  if (s) {
    s->U = U; s->UM = UM; s->USTAR = USTAR; s->RHSU = RHSU; s->TMP3 = TMP3;
    s->P = P; s->HR = HR; s->HE0 = HE0;
    s->lv = lv;
    put_solve_scratch(s, sq);
    s->OFF = OFF; s->XN = XN; s->UN = UN; s->PHIN = PHIN;
    s->BODYOF = BODYOF; s->TILE = TILE; s->PERM = PERM; s->PERMTMP = PERMTMP;
    s->XS = XS; s->US = US; s->PHIS = PHIS; s->PT3 = PT3;
    s->ADJ = ADJ;
    s->REC_U = REC_U; s->REC_PP = REC_PP; s->REC_PHI = REC_PHI; s->REC_PHIP = REC_PHIP; s->REC_RF = REC_RF;
    s->ADJ2 = ADJ2;
    s->COUNTS = COUNTS; s->TSTART = TSTART; s->FILLC = FILLC; s->FLAGS = FLAGS; s->FPOS = FPOS;
    s->ACTIVE = ACTIVE; s->SCANTMP = SCANTMP; s->BODIES = BODIES;
    s->SPAN = SPAN; s->BSUM = BSUM; s->VPART = VPART;
    s->TCOUNT = TCOUNT; s->TLSTART = TLSTART; s->TLIST = TLIST;
    s->tl_cap = tl_cap; s->NZT = NZT;
    s->COARSEFD = COARSEFD;
    s->SUBTAB = SUBTAB;
    s->fastdiag = fdg;
    s->coarse_mfma = fdc;
    s->FDQ = FDQ;
    s->fdx = fdx;
    s->FDXQ = FDXQ;
  }
  return cv.off + 256;
}

// ---------------------------------------------------------------------------
// small host helpers
sim_status sync(sim_t s) {
  CKH(hipStreamSynchronize(s->st));
  return SIM_OK;
}

// values that finalize mirrored into the pinned buffer at offset 0 -> host
// (synchronises)
sim_status read_mirror(sim_t s, int n, double *out) {
  CKH(hipStreamSynchronize(s->st));
  memcpy(out, s->hpin, sizeof(double) * n);
  return SIM_OK;
}


sim_status dev_norm2(sim_t s, const double *x, long long n, double *out) {
  CKH(dot2(x, x, n, s->PART, s->st));
  CKH(finalize(s->PART, red_blocks(), 1, s->RED, s->st, s->hpin_dev));
  return read_mirror(s, 1, out);
}

// subtract the mean of a cell field (enqueued only; mean left in RED[0])
sim_status project_mean(sim_t s, double *x) {
  CKH(dot2(x, nullptr, s->N, s->PART, s->st));
  CKH(finalize(s->PART, red_blocks(), 1, s->RED, s->st));
  CKH(add_scalar_dev(x, s->N, s->RED, -1.0 / (double)s->N, s->st));
  return SIM_OK;
}

void mat_rodrigues(const double axis[3], double gamma, double R[9]) {
  double W[9] = {0, -axis[2], axis[1], axis[2], 0, -axis[0], -axis[1], axis[0], 0};
  double W2[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double v = 0;
      for (int k = 0; k < 3; ++k) v += W[3 * i + k] * W[3 * k + j];
      W2[3 * i + j] = v;
    }
  double sg = sin(gamma), cg = 1.0 - cos(gamma);
  for (int q = 0; q < 9; ++q) R[q] = (q % 4 == 0 ? 1.0 : 0.0) + sg * W[q] + cg * W2[q];
}
void mat_mul(const double A[9], const double B[9], double C[9]) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double v = 0;
      for (int k = 0; k < 3; ++k) v += A[3 * i + k] * B[3 * k + j];
      C[3 * i + j] = v;
    }
}

// kinematic state of a prescribed body at time t
void prescribed_state(const sim_body &b, double t, double c[3], double v[3], double R[9]) {
  double cw = cos(b.osc_omega * t), sw = sin(b.osc_omega * t);
  for (int a = 0; a < 3; ++a) {
    c[a] = b.center[a] + b.vel[a] * t - b.osc_amp[a] * cw;
    v[a] = b.vel[a] + b.osc_amp[a] * b.osc_omega * sw;
  }
  double wn = sqrt(b.omega[0] * b.omega[0] + b.omega[1] * b.omega[1] + b.omega[2] * b.omega[2]);
  if (wn == 0.0) {
    for (int q = 0; q < 9; ++q) R[q] = (q % 4 == 0) ? 1.0 : 0.0;
  } else {
    double ax[3] = {b.omega[0] / wn, b.omega[1] / wn, b.omega[2] / wn};
    mat_rodrigues(ax, wn * t, R);
  }
}

// The support of every point stays on interior nodes of wall axes of either
// kind (Appendix B); checked with each body's bounding sphere.
bool supports_inside(sim_t s, const std::vector<BodyDev> &bd) {
  double margin = (s->ker == SIM_DELTA_PESKIN4 ? 2.0 : 1.5) * s->g.h;
  for (size_t i = 0; i < bd.size(); ++i) {
    for (int a = 0; a < 3; ++a) {
      if (s->cfg.bc[a] == SIM_BC_PERIODIC) continue;
      double lo = bd[i].c[a] - s->bodies[i].rmax, hi = bd[i].c[a] + s->bodies[i].rmax;
      if (lo < margin || hi > s->cfg.len[a] - margin) return false;
    }
  }
  return true;
}

// Place the points of all bodies from the given body states and bin them.
sim_status place_and_bin(sim_t s, const std::vector<BodyDev> &bd) {
  if (!supports_inside(s, bd))
    return fail(s, SIM_EINVAL, "delta-kernel support of a body crosses a wall");
  hipStream_t st = s->st;
  CKH(hipMemcpyAsync(s->BODIES, bd.data(), sizeof(BodyDev) * bd.size(), hipMemcpyHostToDevice, st));
  CKH(points_place(s->g, s->K, s->BODIES, s->BODYOF, s->OFF, s->XN, s->UN, s->TILE, s->nt0, s->nt1, s->nt2, st));
  int nt = (int)s->ntiles;
  CKH(fill_i32(s->COUNTS, nt, 0, st));
  CKH(fill_i32(s->FILLC, nt, 0, st));
  CKH(bin_count(s->K, s->TILE, s->COUNTS, st));
  CKH(scan_exclusive(s->COUNTS, s->TSTART, nt, s->SCANTMP, st));
  CKH(bin_scatter(s->K, s->TILE, s->TSTART, s->FILLC, s->PERMTMP, st));
  CKH(bin_canon(s->K, s->TILE, s->TSTART, s->PERMTMP, s->PERM, st));
  CKH(gather3(s->K, s->PERM, s->XN, s->XS, st));
  CKH(gather3(s->K, s->PERM, s->UN, s->US, st));
  // non-empty point tiles (the interpolation work list; their neighbourhoods hold the touch-list candidates)
  CKH(positive_flags(nt, s->COUNTS, s->FLAGS, st));
  CKH(scan_exclusive(s->FLAGS, s->FPOS, nt, s->SCANTMP, st));
  CKH(compact(nt, s->FLAGS, s->FPOS, s->ACTIVE, st));
  int nz = 0;
  CKH(hipMemcpyAsync(s->hpin, s->FPOS + nt, sizeof(int), hipMemcpyDeviceToHost, st));
  CKH(hipStreamSynchronize(st));
  memcpy(&nz, s->hpin, sizeof(int));
  s->nnz = order_launch_count(nz);  // launch count of NZT (holes included)
  // interpolation launch order of the non-empty point tiles: XCD chunks, fullest first
  CKH(order_active(nz, s->ACTIVE, s->TSTART, s->NZT, st));
  // touch lists of the active tiles (tiles reached by some point's support),
  // counted and filled tile by tile in a fixed order; only the tiles within
  // one tile of a non-empty point tile can be reached (candidates, compacted
  // into ACTIVE; their number stays on the device)
  CKH(fill_i32(s->FLAGS, nt, 0, st));
  CKH(mark_near(s->g, s->nt0, s->nt1, s->nt2, nz, s->ACTIVE, s->FLAGS, st));
  CKH(scan_exclusive(s->FLAGS, s->FPOS, nt, s->SCANTMP, st));
  CKH(compact(nt, s->FLAGS, s->FPOS, s->ACTIVE, st));
  CKH(fill_i32(s->TCOUNT, nt, 0, st));
  CKH(touch_tiles(s->ker, s->g, s->nt0, s->nt1, s->nt2, (int)std::min<long long>(nt, 27LL * nz), s->FPOS + nt,
                  s->ACTIVE, s->TSTART, s->XS, s->TCOUNT, nullptr, nullptr, st));
  CKH(scan_exclusive(s->TCOUNT, s->TLSTART, nt, s->SCANTMP, st));
  CKH(positive_flags(nt, s->TCOUNT, s->FLAGS, st));
  CKH(scan_exclusive(s->FLAGS, s->FPOS, nt, s->SCANTMP, st));
  CKH(compact(nt, s->FLAGS, s->FPOS, s->ACTIVE, st));
  int na = 0, M = 0;
  CKH(hipMemcpyAsync(s->hpin, s->FPOS + nt, sizeof(int), hipMemcpyDeviceToHost, st));
  CKH(hipMemcpyAsync((int *)s->hpin + 1, s->TLSTART + nt, sizeof(int), hipMemcpyDeviceToHost, st));
  CKH(hipStreamSynchronize(st));
  memcpy(&na, s->hpin, sizeof(int));
  memcpy(&M, (int *)s->hpin + 1, sizeof(int));
  if (M > s->tl_cap) return fail(s, SIM_EDEVICE, "touch list overflow");
  CKH(touch_tiles(s->ker, s->g, s->nt0, s->nt1, s->nt2, na, nullptr, s->ACTIVE, s->TSTART, s->XS, nullptr,
                  s->TLSTART, s->TLIST, st));
  // launch order of the active tiles: XCD chunks, longest touch lists first
  // (FLAGS, no longer needed, takes the order)
  CKH(order_active(na, s->ACTIVE, s->TLSTART, s->FLAGS, st));
  std::swap(s->ACTIVE, s->FLAGS);
  s->ntouch = M;
  s->nactive = order_launch_count(na);  // launch count of ACTIVE (holes included)
  probe_set_points(s->probes, s->K, 64LL * na);
  return SIM_OK;
}

std::vector<BodyDev> body_states_at(sim_t s, double t) {
  std::vector<BodyDev> out(s->bodies.size());
  for (size_t i = 0; i < s->bodies.size(); ++i) {
    const HostBody &hb = s->bodies[i];
    BodyDev &d = out[i];
    if (hb.b.motion == SIM_MOTION_PRESCRIBED) {
      prescribed_state(hb.b, t, d.c, d.v, d.R);
      for (int a = 0; a < 3; ++a) d.w[a] = hb.b.omega[a];
    } else {
      for (int a = 0; a < 3; ++a) { d.c[a] = hb.xc[a]; d.v[a] = hb.us[a]; d.w[a] = hb.w[a]; }
      for (int q = 0; q < 9; ++q) d.R[q] = hb.R[q];
    }
  }
  return out;
}

// ---------------------------------------------------------------------------
// Operators on the split layout

// Algorithmic bytes of one whole-grid fast-diagonalisation solve: the input
// (ti bytes per cell) read and bfloat16 lines written, three bfloat16 passes
// (y forward, x forward + scale + back, y back), bfloat16 lines read and the
// output (to bytes per cell) written.
double fd_bytes(const sim_s *s, size_t ti, size_t to) { return (double)s->N * (ti + 2 + 3 * 4 + 2 + to); }

// Algorithmic bytes of one exact float64 fast-diagonalisation solve: the
// split-layout input read and written in natural order, six mode products
// each reading and writing the grid, the natural-order result read and
// written in split order (16 passes of 8 bytes per cell).
double fdx_bytes(const sim_s *s) { return (double)s->N * 16 * 8; }

// w = S~ z = L z + c^-1 G^T W W^T G z  (= L z - c^-1 D W (W^T G z)), in
// float64.  With TW = float (the products of the float32 FGMRES cycle, z in
// float32 too) w is stored in float32 and its coupling term is formed in
// float32 arithmetic; the cycle's restarts from the float64 true residual
// absorb their rounding.  Every other product is float64.
template <typename T, typename TW = double>
sim_status schur_matvec(sim_t s, const T *z, TW *w) {
  constexpr bool f32 = std::is_same<TW, float>::value;
  static_assert(!f32 || std::is_same<T, float>::value, "a float32 product takes a float32 z");
  {
    ProbeExt pr(PR_LAP, s->st, (double)s->N * (sizeof(T) + sizeof(TW)));  // z read, w written
    CKH((lap_apply<T, TW>(s->g, z, w, s->st)));
  }
  CKH(interp_grad<T>(s->ker, s->g, s->nt1, s->nt2, s->nnz, s->NZT, s->TSTART, s->XS, z, 1.0, nullptr, 0.0, s->Q,
                     s->st, f32));
  CKH(band_apply(s->ker, true, s->g, s->nt1, s->nt2, s->nactive, s->ACTIVE, s->TLSTART, s->TLIST, s->XS, s->Q,
                 -1.0 / s->c, w, s->st, f32));
  return SIM_OK;
}

// z ~ L^+ v by one V-cycle (v in precision TV: float64, or float32 for the
// FP32-MG basis).  Every kernel launch is probed with its algorithmic bytes
// (each operand read once, each result written once; T-typed values of the
// level, the finest level's right-hand side in TV).
template <typename T, typename TV>
sim_status vcycle(sim_t s, const TV *v, T *z) {
  hipStream_t st = s->st;
  const sim_config &c = s->cfg;
  const int nl = (int)s->lv.size();
  const int cyc = c.mg_coarse_sweeps;
  const double t = sizeof(T);
  auto cells = [&](int l) { return (double)geo_cells(s->lv[l].g); };
  auto tb = [&](int l) { return l == 0 ? (double)sizeof(TV) : t; };  // right-hand-side bytes of level l
  auto coarse_bytes = [&](int l) { return cells(l) * (tb(l) + t); };  // b read, x written
  auto first_bytes = [&](int l, bool store_red) { return cells(l) * (tb(l) + (store_red ? t : 0.5 * t)); };
  auto half_bytes = [&](int l) { return cells(l) * (0.5 * t + 0.5 * tb(l) + 0.5 * t); };
  auto restrict_bytes = [&](int l) { return cells(l) * (t + 0.5 * tb(l)) + cells(l + 1) * t; };
  auto prolong_bytes = [&](int l) { return cells(l) * t + cells(l + 1) * t; };
  // tile levels: b read, x written, the coarse b written; the red half of x,
  // b and the coarse x read, x written
  auto tile_down_bytes = [&](int l) { return cells(l) * (tb(l) + t) + cells(l + 1) * t; };
  auto tile_up_bytes = [&](int l) { return cells(l) * (0.5 * t + tb(l) + t) + cells(l + 1) * t; };

  // the last two levels run in one LDS workgroup when they fit (an exact
  // coarse solve below a fine level of at most 4096 cells); grid-wide levels
  // run above level lsub
  const bool sub = nl >= 2 && cyc == 0 && !s->coarse_mfma && subcycle_fits(s->lv[nl - 2].g, s->lv[nl - 1].g);
  const int lsub = sub ? nl - 2 : nl - 1;
  auto tiled = [&](int l) { return l < lsub && s->lv[l].xs != nullptr; };
  // the whole cycle: the sum of the per-launch models below
  ProbeScope whole(PR_VCYCLE, st, [&] {
    double b = nl == 1 ? coarse_bytes(0) : coarse_bytes(lsub);
    for (int l = 0; l < lsub; ++l)
      b += tiled(l) ? tile_down_bytes(l) + tile_up_bytes(l)
                    : first_bytes(l, c.mg_pre == 1) + 2.0 * (c.mg_pre - 1) * half_bytes(l) + restrict_bytes(l) +
                          prolong_bytes(l) + 2.0 * c.mg_post * half_bytes(l);
    return b;
  }());
  auto coarse_solve = [&](const Geo &g, auto *b, T *x) -> sim_status {
    using TBc = std::remove_const_t<std::remove_pointer_t<decltype(b)>>;
    ProbeScope pr(PR_COARSE, st, (double)geo_cells(g) * (sizeof(TBc) + t));
    if (cyc == 0 && s->coarse_mfma) CKH((fd_precond<TBc, T>(g, b, x, s->FDW1, s->FDW2, s->FDQ, 1.0f, st)));
    else if (cyc == 0) CKH((mg_coarse_fd<T, TBc>(g, b, x, s->COARSEFD, st)));
    else CKH((mg_coarse<T, TBc>(g, b, x, cyc, 1, st)));
    return SIM_OK;
  };
  if (nl == 1) return coarse_solve(s->lv[0].g, v, z);
  auto subcycle = [&](auto *b, T *x) -> sim_status {
    using TBs = std::remove_const_t<std::remove_pointer_t<decltype(b)>>;
    const Geo &gf = s->lv[nl - 2].g;
    ProbeExt pr(PR_COARSE, st, (double)geo_cells(gf) * (sizeof(TBs) + t));
    CKH((mg_subcycle<T, TBs>(gf, s->lv[nl - 1].g, b, x, s->COARSEFD, s->SUBTAB, c.mg_pre, c.mg_post, st)));
    return SIM_OK;
  };
  if (sub && lsub == 0) return subcycle(v, z);
  // descend: pre-smoothing red then black, the first sweep from zero (which
  // stores the red values only when no further half sweep overwrites them);
  // a tile level runs its sweeps, residual and restriction in one launch and
  // keeps its pre-smoothed x apart (xs), since its ascent reads the old
  // values of neighbouring tiles while writing x
  const bool store_red = c.mg_pre == 1;
  for (int l = 0; l < lsub; ++l) {
    const Geo &g = s->lv[l].g;
    T *x = l == 0 ? z : (T *)s->lv[l].x;
    auto pre = [&](auto *b) -> sim_status {
      using TBl = std::remove_const_t<std::remove_pointer_t<decltype(b)>>;
      if (tiled(l)) {
        ProbeExt pr(PR_TILE_DOWN, st, tile_down_bytes(l));
        CKH((mg_tile_down<T, TBl>(g, (T *)s->lv[l].xs, b, s->lv[l + 1].g, (T *)s->lv[l + 1].b, c.mg_pre, st)));
        return SIM_OK;
      }
      {
        ProbeExt pr(PR_SMOOTH_FIRST, st, first_bytes(l, store_red));
        CKH((mg_smooth_first<T, TBl>(g, x, b, store_red, st)));
      }
      for (int q = 1; q < c.mg_pre; ++q)
        for (int color = 0; color < 2; ++color) {
          ProbeExt pr(PR_SMOOTH, st, half_bytes(l));
          CKH((mg_smooth<T, TBl>(g, x, b, color, st)));
        }
      T *bnext = (T *)s->lv[l + 1].b;
      ProbeExt pr(PR_RESTRICT, st, restrict_bytes(l));
      CKH((mg_restrict<T, TBl>(g, x, b, s->lv[l + 1].g, bnext, st)));
      return SIM_OK;
    };
    sim_status rc = l == 0 ? pre(v) : pre((const T *)s->lv[l].b);
    if (rc) return rc;
  }
  {
    sim_status rc = sub ? subcycle((const T *)s->lv[lsub].b, (T *)s->lv[lsub].x)
                        : coarse_solve(s->lv[nl - 1].g, (const T *)s->lv[nl - 1].b, (T *)s->lv[nl - 1].x);
    if (rc) return rc;
  }
  // ascend: prolongation onto the red cells, post-smoothing black then red
  // (a tile level: both in one launch, from its pre-smoothed x)
  for (int l = lsub - 1; l >= 0; --l) {
    const Geo &g = s->lv[l].g;
    T *x = l == 0 ? z : (T *)s->lv[l].x;
    auto post = [&](auto *b) -> sim_status {
      using TBl = std::remove_const_t<std::remove_pointer_t<decltype(b)>>;
      if (tiled(l)) {
        ProbeExt pr(PR_TILE_UP, st, tile_up_bytes(l));
        CKH((mg_tile_up<T, TBl>(g, (const T *)s->lv[l].xs, x, b, s->lv[l + 1].g, (const T *)s->lv[l + 1].x,
                                c.mg_post, st)));
        return SIM_OK;
      }
      {
        ProbeExt pr(PR_PROLONG, st, prolong_bytes(l));
        CKH(mg_prolong<T>(g, x, s->lv[l + 1].g, (const T *)s->lv[l + 1].x, st));
      }
      for (int q = 0; q < c.mg_post; ++q)
        for (int color = 1; color >= 0; --color) {
          ProbeExt pr(PR_SMOOTH, st, half_bytes(l));
          CKH((mg_smooth<T, TBl>(g, x, b, color, st)));
        }
      return SIM_OK;
    };
    sim_status rc = l == 0 ? post(v) : post((const T *)s->lv[l].b);
    if (rc) return rc;
  }
  return SIM_OK;
}

// Flexible GMRES(m), right preconditioned: solves S~ x = b (b mean-zero).
// T: precision of the preconditioned vectors Z and of the V-cycle; the basis
// V has the same precision (a float32 basis in the FP32-MG form: each cycle
// only has to gain FP32_CYCLE_DROP before the float64 true residual restarts
// it).  w = S~ z_j is stored in T too (in the float32 form its coupling term
// is float32 arithmetic); the Gram-Schmidt products, the update and every
// norm are float64 arithmetic.
//
// Pipelining: the preconditioner of iteration j + 1 applies to the
// unnormalised basis vector V'_{j+1}, which is complete once the update of
// iteration j has run, and it does not need the norm the host is waiting
// for.  So after enqueuing iteration j's update, the preconditioner, S~
// product and Gram-Schmidt products of iteration j + 1 are enqueued before
// the host waits (on an event, not the whole stream) for iteration j's
// coefficients, and the device never idles during the host's Givens step.
// This is done when the iteration count and residual trend predict that
// iteration j + 1 will run; a mispredicted last iteration is discarded
// (its only outputs are z_{j+1}, w and the products, all overwritten).
// The host mirror alternates between two slots so that the products of
// iteration j + 1 never overwrite those of iteration j before they are read.
//
// bsum (optional, on the device): the sum of b, whose mean the solver then
// removes on the fly (b itself is left as it is).  xsum (optional): the
// solver leaves the sum of x there instead of subtracting x's mean; the
// caller removes it.
template <typename T>
sim_status fgmres(sim_t s, const double *b, double *x, sim_solve_stats *stt, const double *bsum = nullptr,
                  double *xsum = nullptr) {
  hipStream_t st = s->st;
  const sim_config &c = s->cfg;
  const long long N = s->N;
  const int m = c.krylov_restart;
  T *V = (T *)s->V;
  T *Z = (T *)s->Z;
  // w = S~ z_j: in the basis vector V_{j+1} itself (float64 basis), or in a
  // float32 scratch vector (float32 basis) that the products and the update read
  using TW = T;
  TW *const wsep = sizeof(T) != sizeof(double) ? (TW *)s->TMPC : nullptr;
  // the bfloat16 fast diagonalisation scales its input by sig_j, known only
  // after the wait: no pipelining with it
  const bool can_pipe = !s->fastdiag;
  sim_solve_stats loc{};
  sim_solve_stats &S = stt ? *stt : loc;
  S.iters = 0;
  S.nhist = 0;
  sim_status rc;
  // Hessenberg matrix, Givens rotations and scales on the host stack (no
  // allocation inside a solve)
  double H[(MAX_RESTART + 1) * MAX_RESTART], cs[MAX_RESTART], sn[MAX_RESTART], gv[MAX_RESTART + 1],
      y[MAX_RESTART], sig[MAX_RESTART + 1];
  KCoef sig2{};  // sig_i^2, passed by value to the update kernel
  auto Hij = [&](int i, int j) -> double & { return H[(size_t)i * m + j]; };
  // host-mirror slots of iteration j: products at slot(j) + 0..j, the norm at slot(j) + MIRROR_NORM
  constexpr int MIRROR_SLOT = 80, MIRROR_NORM = 70;
  auto slot = [&](int j) { return (j & 1) * MIRROR_SLOT; };
  double *const part_dots = s->PART, *const part_norm = s->PART + (long long)(MAX_RESTART + 1) * red_blocks();
  double *const red_norm = s->RED + 2 * (MAX_RESTART + 2);  // device copy of the norm (unused by kernels)
  // preconditioner, S~ product, Gram-Schmidt products of iteration j
  auto front = [&](int j) -> sim_status {
    T *zj = Z + (long long)j * N;
    T *vj = V + (long long)j * N;
    TW *w = wsep ? wsep : V + (long long)(j + 1) * N;
    if (s->fastdiag) {
      ProbeScope pr(PR_VCYCLE, st, fd_bytes(s, sizeof(T), sizeof(T)));
      CKH((fd_precond<T, T>(s->g, vj, zj, s->FDW1, s->FDW2, s->FDQ, (float)sig[j], st)));
    } else if (s->fdx) {
      if constexpr (std::is_same<T, double>::value) {
        ProbeScope pr(PR_VCYCLE, st, fdx_bytes(s));
        CKH(fdx_precond(s->g, vj, zj, s->FDX1, s->FDX2, s->FDXQ, st));
      }
    } else {
      sim_status r = vcycle<T, T>(s, vj, zj);
      if (r) return r;
    }
    sim_status r = schur_matvec<T, TW>(s, zj, w);
    if (r) return r;
    {
      ProbeExt pr(PR_MULTIDOT, st, (double)N * (sizeof(TW) + (j + 1) * sizeof(T)));  // w, V_0..V_j
      CKH((multidot<T, TW>(w, V, N, j + 1, N, part_dots, st)));
    }
    CKH(finalize(part_dots, red_blocks(), j + 1, s->RED, st, s->hpin_dev + slot(j)));
    return SIM_OK;
  };
  // A cycle starts from V'_0 = r, the residual itself (sig_0 = 1 / |r|):
  // the pass that casts r into the basis also forms |r|^2, and since the
  // front of iteration 0 needs no norm, it is enqueued before the host waits
  // for that norm whenever the cycle is expected to run.  The host mirror
  // slot of these norms is apart from the products' slots.
  double *const mirror_res = s->hpin + 2 * MIRROR_SLOT;
  auto cycle_start = [&](const double *ax, bool speculate, double &r2) -> sim_status {
    CKH(sub_cast_norm<T>(V, b, ax, N, s->PART, st, bsum, 1.0 / (double)N));
    CKH(finalize(s->PART, red_blocks(), 1, s->RED, st, s->hpin_dev + 2 * MIRROR_SLOT));
    CKH(hipEventRecord(s->ev_iter, st));
    if (speculate && can_pipe) {
      sim_status r = front(0);
      if (r) return r;
    }
    CKH(hipEventSynchronize(s->ev_iter));
    r2 = mirror_res[0];
    return SIM_OK;
  };
  double bn2;
  if ((rc = cycle_start(nullptr, c.krylov_maxit > 0, bn2))) return rc;
  bool front0 = c.krylov_maxit > 0 && can_pipe;  // the next cycle's front(0) already enqueued
  const double bnorm = sqrt(bn2);
  if (!(bnorm > 0)) {
    CKH(fill(x, N, 0.0, st));
    if (xsum) CKH(fill(xsum, 1, 0.0, st));
    S.rel_res = 0;
    return isfinite(bn2) ? SIM_OK : fail(s, SIM_ENONFINITE, "non-finite right-hand side");
  }
  // the solution: written by the first cycle's update (x = Z y), accumulated
  // by the later ones; the update's per-block sums of x give its mean
  bool xset = false;
  double *const part_x = s->PART + red_blocks();
  double beta = bnorm;
  int total = 0;
  double rel = 1.0;
  while (true) {
    rel = beta / bnorm;
    if (rel <= c.krylov_rtol || total >= c.krylov_maxit) break;
    sig[0] = 1.0 / beta;
    sig2.v[0] = sig[0] * sig[0];
    std::fill(gv, gv + m + 1, 0.0);
    gv[0] = beta;
    int jd = 0;
    bool have_front = front0;  // iteration j's front already enqueued
    front0 = false;
    for (int j = 0; j < m; ++j) {
      T *vnext = V + (long long)(j + 1) * N;
      TW *w = wsep ? wsep : vnext;
      if (!have_front && (rc = front(j))) return rc;
      have_front = false;
      // classical Gram-Schmidt on the unnormalised basis (v_i = sig_i V'_i):
      // g_i = <w', V'_i>, V'_{j+1} = w' - sum_i sig_i^2 g_i V'_i and its norm
      // in one pass; with w' = S~ z'_j = S~ z_j / sig_j the Hessenberg column
      // is h_ij = sig_j sig_i g_i, h_{j+1,j} = sig_j |V'_{j+1}|.
      {
        // w, V_0..V_j read, V_{j+1} written
        ProbeExt pr(PR_UPDATE_NORM, st, (double)N * (sizeof(TW) + (j + 2) * sizeof(T)));
        CKH((update_cast_norm<T, TW>(vnext, w, V, N, j + 1, s->RED, sig2, N, part_norm, st)));
      }
      CKH(finalize(part_norm, red_blocks(), 1, red_norm, st, s->hpin_dev + slot(j) + MIRROR_NORM));
      CKH(hipEventRecord(s->ev_iter, st));
      // iteration j + 1 will run unless this one converges, hits a limit or
      // (float32 basis) the cycle's gain: predicted from the residual trend
      if (can_pipe && j + 1 < m && total + 1 < c.krylov_maxit) {
        const double g0 = fabs(gv[j]), gm = j > 0 ? fabs(gv[j - 1]) : 0.0;
        const double pred = (j > 0 && gm > 0.0) ? g0 * (g0 / gm) : 0.5 * g0;  // |g_{j+1}| expected
        const bool go = pred > 2.0 * c.krylov_rtol * bnorm && (!s->fp32 || pred > 2.0 * FP32_CYCLE_DROP * beta);
        if (go) {
          if ((rc = front(j + 1))) return rc;
          have_front = true;
        }
      }
      CKH(hipEventSynchronize(s->ev_iter));
      double hc[MAX_RESTART + 2];
      memcpy(hc, s->hpin + slot(j), sizeof(double) * (j + 1));
      hc[j + 1] = s->hpin[slot(j) + MIRROR_NORM];
      const double nrm = sqrt(std::max(hc[j + 1], 0.0));
      if (!isfinite(nrm)) return fail(s, SIM_ENONFINITE, "non-finite Krylov norm");
      for (int i = 0; i <= j; ++i) Hij(i, j) = sig[j] * sig[i] * hc[i];
      const double hn = sig[j] * nrm;
      Hij(j + 1, j) = hn;
      if (nrm > 0) {
        sig[j + 1] = 1.0 / nrm;
        sig2.v[j + 1] = sig[j + 1] * sig[j + 1];
      }
      for (int i = 0; i < j; ++i) {
        double t0 = cs[i] * Hij(i, j) + sn[i] * Hij(i + 1, j);
        Hij(i + 1, j) = -sn[i] * Hij(i, j) + cs[i] * Hij(i + 1, j);
        Hij(i, j) = t0;
      }
      double den = hypot(Hij(j, j), Hij(j + 1, j));
      cs[j] = den > 0 ? Hij(j, j) / den : 1.0;
      sn[j] = den > 0 ? Hij(j + 1, j) / den : 0.0;
      Hij(j, j) = den;
      Hij(j + 1, j) = 0.0;
      gv[j + 1] = -sn[j] * gv[j];
      gv[j] = cs[j] * gv[j];
      ++total;
      jd = j + 1;
      double est = fabs(gv[j + 1]) / bnorm;
      if (S.nhist < 64) S.hist[S.nhist++] = est;
      if (est <= c.krylov_rtol || total >= c.krylov_maxit || hn == 0.0) break;
      // FP32 preconditioner: restart from the FP64 true residual before the
      // cycle reaches the float32 accuracy floor of its directions
      if (s->fp32 && fabs(gv[j + 1]) <= FP32_CYCLE_DROP * beta) break;
    }
    // y = H^-1 g (upper triangular)
    for (int i = jd - 1; i >= 0; --i) {
      double v = gv[i];
      for (int k = i + 1; k < jd; ++k) v -= Hij(i, k) * y[k];
      y[i] = v / Hij(i, i);
    }
    KCoef yc{};
    for (int i = 0; i < jd; ++i) yc.v[i] = y[i] * sig[i];  // z_i = sig_i z'_i
    CKH(sol_update<T>(x, Z, N, jd, yc, N, st, !xset, part_x));
    xset = true;
    // true residual r = b - S~ x (S~ x in TMPC), cast into V'_0 of the next
    // cycle; its front is enqueued ahead of the norm when the cycle's
    // residual estimate says another cycle follows
    if ((rc = schur_matvec<double>(s, x, s->TMPC))) return rc;
    const bool more = fabs(gv[jd]) > 10.0 * c.krylov_rtol * bnorm && total < c.krylov_maxit;
    double r2;
    if ((rc = cycle_start(s->TMPC, more, r2))) return rc;
    front0 = more && can_pipe;
    if (!isfinite(r2)) return fail(s, SIM_ENONFINITE, "non-finite residual");
    beta = sqrt(r2);
  }
  S.iters = total;
  S.rel_res = rel;
  if (xset) {
    // the mean of x (its sum from the last update's block sums): subtracted
    // here, or left to the caller in xsum
    CKH(finalize(part_x, sol_blocks(), 1, xsum ? xsum : s->RED, st));
    if (!xsum) CKH(add_scalar_dev(x, N, s->RED, -1.0 / (double)N, st));
  } else {
    CKH(fill(x, N, 0.0, st));
    if (xsum) CKH(fill(xsum, 1, 0.0, st));
  }
  if (rel > c.krylov_rtol) return fail(s, SIM_ENOTCONV, "Krylov iteration limit reached");
  return SIM_OK;
}

// Right-preconditioned BiCGStab (van der Vorst) on S~ x = b: vectors and
// recurrences in float64, the preconditioner (V-cycle or fast
// diagonalisation) in precision T.  Three host synchronisations per
// iteration: (r^, v); |s|, (t, s), (t, t); |r|, (r, r^).  The loop restarts
// from the float64 true residual when the recursive one meets the tolerance
// (or on a breakdown), so the reported residual is the true one.
template <typename T>
sim_status bicgstab(sim_t s, const double *b, double *x, sim_solve_stats *stt) {
  hipStream_t st = s->st;
  const sim_config &c = s->cfg;
  const long long N = s->N;
  double *R = s->BCG, *RH = R + N, *P = RH + N, *Vv = P + N, *Sv = Vv + N, *Tv = Sv + N;
  T *PH = (T *)s->Z, *SH = PH + N;
  sim_solve_stats loc{};
  sim_solve_stats &S = stt ? *stt : loc;
  S.iters = 0;
  S.nhist = 0;
  sim_status rc;
  auto precond = [&](const double *in, T *out) -> sim_status {
    if (s->fastdiag) {
      ProbeScope pr(PR_VCYCLE, st, fd_bytes(s, sizeof(double), sizeof(T)));
      CKH((fd_precond<double, T>(s->g, in, out, s->FDW1, s->FDW2, s->FDQ, 1.0f, st)));
      return SIM_OK;
    }
    if (s->fdx) {
      if constexpr (std::is_same<T, double>::value) {
        ProbeScope pr(PR_VCYCLE, st, fdx_bytes(s));
        CKH(fdx_precond(s->g, in, out, s->FDX1, s->FDX2, s->FDXQ, st));
      }
      return SIM_OK;
    }
    return vcycle<T, double>(s, in, out);
  };
  auto reduce = [&](int nv, double *out) -> sim_status {
    CKH(finalize(s->PART, red_blocks(), nv, s->RED, st, s->hpin_dev));
    return read_mirror(s, nv, out);
  };
  double bn2;
  if ((rc = dev_norm2(s, b, N, &bn2))) return rc;
  const double bnorm = sqrt(bn2);
  CKH(fill(x, N, 0.0, st));
  if (!(bnorm > 0)) {
    S.rel_res = 0;
    return isfinite(bn2) ? SIM_OK : fail(s, SIM_ENONFINITE, "non-finite right-hand side");
  }
  const int rb = red_blocks();
  int total = 0;
  double rel = 1.0;
  double r2 = bn2;
  CKH(scale_copy(R, b, N, 1.0, st));  // x = 0: r = b
  while (true) {
    // (re)start: r^ = r
    CKH(scale_copy(RH, R, N, 1.0, st));
    double rho = r2, rho_old = 1.0, alpha = 1.0, omega = 1.0;
    int since = 0;
    bool breakdown = false;
    while (sqrt(r2) / bnorm > c.krylov_rtol && total < c.krylov_maxit) {
      // p = r + beta (p - omega v); p = r on the first iteration
      if (since == 0) {
        CKH(scale_copy(P, R, N, 1.0, st));
      } else {
        const double beta = (rho / rho_old) * (alpha / omega);
        CKH(lincomb(P, R, 1.0, P, beta, Vv, -beta * omega, nullptr, 0, N, nullptr, st));
      }
      if ((rc = precond(P, PH))) return rc;
      if ((rc = schur_matvec<T>(s, PH, Vv))) return rc;
      CKH(dot2(RH, Vv, N, s->PART, st));
      double rv;
      if ((rc = reduce(1, &rv))) return rc;
      if (!isfinite(rv)) return fail(s, SIM_ENONFINITE, "non-finite Krylov product");
      if (rv == 0.0) {
        breakdown = true;
        break;
      }
      alpha = rho / rv;
      // s = r - alpha v with |s|^2; then (t, s), (t, t) for t = S~ M^-1 s
      CKH(lincomb(Sv, R, 1.0, Vv, -alpha, nullptr, 0.0, nullptr, 1, N, s->PART, st));
      if ((rc = precond(Sv, SH))) return rc;
      if ((rc = schur_matvec<T>(s, SH, Tv))) return rc;
      CKH(dots2(Tv, Sv, Tv, N, s->PART + 2LL * rb, st));
      CKH(finalize(s->PART, rb, 2, s->RED, st, s->hpin_dev));
      CKH(finalize(s->PART + 2LL * rb, rb, 2, s->RED + 2, st, s->hpin_dev + 2));
      double q[4];
      if ((rc = read_mirror(s, 4, q))) return rc;
      const double ss = q[0], ts = q[2], tt = q[3];
      if (!isfinite(ss) || !isfinite(ts) || !isfinite(tt)) return fail(s, SIM_ENONFINITE, "non-finite Krylov norm");
      ++total;
      ++since;
      if (sqrt(ss) / bnorm <= c.krylov_rtol || !(tt > 0.0)) {
        // converged (or t = 0) at the half step: x += alpha p^, r = s
        KCoef y1{};
        y1.v[0] = alpha;
        CKH(sol_update<T>(x, PH, N, 1, y1, N, st));
        CKH(scale_copy(R, Sv, N, 1.0, st));
        r2 = ss;
        if (S.nhist < 64) S.hist[S.nhist++] = sqrt(r2) / bnorm;
        breakdown = !(tt > 0.0) && sqrt(ss) / bnorm > c.krylov_rtol;
        break;
      }
      omega = ts / tt;
      // x += alpha p^ + omega s^ (p^, s^ adjacent in Z); r = s - omega t with |r|^2, (r, r^)
      KCoef y2{};
      y2.v[0] = alpha;
      y2.v[1] = omega;
      CKH(sol_update<T>(x, PH, N, 2, y2, N, st));
      CKH(lincomb(R, Sv, 1.0, Tv, -omega, nullptr, 0.0, RH, 2, N, s->PART, st));
      double rr[2];
      if ((rc = reduce(2, rr))) return rc;
      if (!isfinite(rr[0]) || !isfinite(rr[1])) return fail(s, SIM_ENONFINITE, "non-finite Krylov norm");
      r2 = rr[0];
      rho_old = rho;
      rho = rr[1];
      if (S.nhist < 64) S.hist[S.nhist++] = sqrt(r2) / bnorm;
      if (omega == 0.0 || rho == 0.0) {
        breakdown = true;
        break;
      }
    }
    // the true residual decides; a drifted recursion or a breakdown restarts
    if ((rc = schur_matvec<double>(s, x, s->TMPC))) return rc;
    CKH(sub_mul(R, b, s->TMPC, N, s->PART, st));
    if ((rc = reduce(1, &r2))) return rc;
    if (!isfinite(r2)) return fail(s, SIM_ENONFINITE, "non-finite residual");
    rel = sqrt(r2) / bnorm;
    if (rel <= c.krylov_rtol || total >= c.krylov_maxit) break;
    if (breakdown && since == 0) break;  // no progress since the last restart
  }
  S.iters = total;
  S.rel_res = rel;
  if ((rc = project_mean(s, x))) return rc;
  if (rel > c.krylov_rtol) return fail(s, SIM_ENOTCONV, "Krylov iteration limit reached or breakdown");
  return SIM_OK;
}

sim_status fgmres_any(sim_t s, const double *b, double *x, sim_solve_stats *stt) {
  if (s->cfg.krylov == SIM_KRYLOV_BICGSTAB)
    return s->fp32 ? bicgstab<float>(s, b, x, stt) : bicgstab<double>(s, b, x, stt);
  return s->fp32 ? fgmres<float>(s, b, x, stt) : fgmres<double>(s, b, x, stt);
}

// b = RHSP + c^-1 D W RF (into BVEC; in_bvec: RHSP is already there),
// projected to mean zero, or with its sum left in bsum for a solver that
// removes the mean on the fly
sim_status schur_rhs(sim_t s, bool in_bvec = false, double *bsum = nullptr) {
  if (!in_bvec) CKH(scale_copy(s->BVEC, s->RHSP, s->N, 1.0, s->st));
  CKH(band_apply(s->ker, true, s->g, s->nt1, s->nt2, s->nactive, s->ACTIVE, s->TLSTART, s->TLIST, s->XS, s->RF,
                 1.0 / s->c, s->BVEC, s->st));
  if (bsum) {
    CKH(dot2(s->BVEC, nullptr, s->N, s->PART, s->st));
    CKH(finalize(s->PART, red_blocks(), 1, bsum, s->st));
    return SIM_OK;
  }
  return project_mean(s, s->BVEC);
}

// Device slots of the isolated solve's deferred means: the sum of b and the
// sum of p' (after the reduction slots of the Krylov solvers)
double *mean_slots(sim_t s) { return s->RED + 3 * (MAX_RESTART + 2); }

// Pressure-force correction on the current RHSP / RF: PP = p', PHIP = Phi'.
// isolated (the Schur solve entry): the pressure right-hand side is already
// in BVEC, and with FGMRES the means of b and p' are not subtracted in passes
// of their own: the solver removes b's on the fly and leaves the sum of p'
// in mean_slots(s)[1] for the entry's output conversion (PP keeps it; a
// constant has no gradient, so Phi' is the same).
sim_status schur_solve_core(sim_t s, sim_solve_stats *stt, bool isolated = false) {
  sim_status rc;
  hipEvent_t e0 = s->ev_solve[0], e1 = s->ev_solve[1];
  CKH(hipEventRecord(e0, s->st));
  const bool defer = isolated && s->cfg.krylov == SIM_KRYLOV_FGMRES;
  double *const bsum = defer ? mean_slots(s) : nullptr, *const xsum = defer ? mean_slots(s) + 1 : nullptr;
  if ((rc = schur_rhs(s, isolated, bsum))) return rc;
  sim_status solve_rc = !defer  ? fgmres_any(s, s->BVEC, s->PP, stt)
                        : s->fp32 ? fgmres<float>(s, s->BVEC, s->PP, stt, bsum, xsum)
                                  : fgmres<double>(s, s->BVEC, s->PP, stt, bsum, xsum);
  if (solve_rc != SIM_OK && solve_rc != SIM_ENOTCONV) return solve_rc;
  // Phi' = c^-1 (B p' - RHS_F) = -c^-1 (W^T G p' + RHS_F)
  CKH(interp_grad<double>(s->ker, s->g, s->nt1, s->nt2, s->nnz, s->NZT, s->TSTART, s->XS, s->PP, -1.0 / s->c, s->RF, -1.0 / s->c, s->PHIP, s->st));
  CKH(hipEventRecord(e1, s->st));
  CKH(hipEventSynchronize(e1));
  float ms = 0;
  CKH(hipEventElapsedTime(&ms, e0, e1));
  if (stt) stt->seconds = ms * 1e-3;
  return solve_rc;
}

// ---------------------------------------------------------------------------
// Momentum solve A u = rhs (faces, split layout): defect correction in FP64,
// each correction by red-black SOR sweeps in precision T.  A has a constant
// interior diagonal a0 + 6 nu/h^2 and red-black ordering makes it consistently
// ordered, so with rho_J = (6 nu/h^2) / (a0 + 6 nu/h^2) the SOR factor
// omega = 2 / (1 + sqrt(1 - rho_J^2)) contracts the error by omega - 1 per
// sweep (boundary rows have no larger Jacobi row ratio: a no-slip ghost adds
// diagonal weight, a free-slip ghost removes an off-diagonal together with
// its share of the diagonal, so rho_J still bounds the Jacobi spectrum).
template <typename T>
sim_status helm_solve(sim_t s, const double *rhs, double *u, sim_solve_stats *stt) {
  hipStream_t st = s->st;
  const sim_config &c = s->cfg;
  const Geo &g = s->g;
  const long long n3 = 3 * s->N;
  const double a0 = 1.5 / c.dt, nuh2 = c.nu / g.h2;
  const double rhoJ = 6.0 * nuh2 / (a0 + 6.0 * nuh2);
  const double omega = 2.0 / (1.0 + sqrt(std::max(0.0, 1.0 - rhoJ * rhoJ)));
  const double rho = omega - 1.0;
  T *R = (T *)s->HR, *E = (T *)s->HE0;
  sim_solve_stats loc{};
  sim_solve_stats &S = stt ? *stt : loc;
  S.iters = 0;
  S.nhist = 0;
  sim_status rc;
  double bn2;
  if ((rc = dev_norm2(s, rhs, n3, &bn2))) return rc;
  double bnorm = sqrt(bn2);
  // sweeps per correction: enough for rho^k to reach the remaining factor
  // to helm_rtol (half of it, for margin), but no more than a safe gain for
  // the correction's precision (1e-5 in float32, two orders above its
  // rounding; 1e-10 in float64, where one correction usually suffices).
  // In float32, 1e-5 against 1e-4 saves a correction per solve at 1e-10:
  // 256^3 steps 11.47 -> 11.08 ms (1e-6: 11.12 ms).
  const double floor_gain = sizeof(T) == 4 ? 1e-5 : 1e-10;
  auto sweeps_for = [&](double rel_now) {
    const double gain = std::min(1.0, std::max(0.5 * c.helm_rtol / std::max(rel_now, 1e-300), floor_gain));
    int k = rho > 1e-12 ? (int)ceil(log(gain) / log(rho)) : 1;
    return std::max(1, std::min(k, 100));
  };
  double rel = 1.0;
  int it = 0;
  int nb = 0;
  for (;; ++it) {
    {
      ProbeScope pr(PR_HELM_RESID, st, 3.0 * s->N * (2 * sizeof(double) + sizeof(T)));  // x, b read, r written
      CKH(helm_resid<T>(g, a0, c.nu, u, rhs, R, s->PART, &nb, st));
    }
    CKH(finalize(s->PART, nb, 1, s->RED, st, s->hpin_dev));
    double r2;
    if ((rc = read_mirror(s, 1, &r2))) return rc;
    if (!isfinite(r2)) return fail(s, SIM_ENONFINITE, "non-finite momentum residual");
    rel = bnorm > 0 ? sqrt(r2) / bnorm : 0.0;
    if (S.nhist < 64) S.hist[S.nhist++] = rel;
    if (rel <= c.helm_rtol || it >= c.helm_maxit) break;
    const int kin = sweeps_for(rel);
    {
      ProbeScope pr(PR_HELM_FIRST, st, 3.0 * s->N * 2 * sizeof(T));  // r read, both colours of e written
      CKH((helm_sor_first<T>(g, a0, c.nu, omega, E, R, st)));
    }
    for (int k = 1; k < kin; ++k) {
      for (int color = 0; color < 2; ++color) {
        // other-colour e, own-colour r and e read, own-colour e written
        ProbeScope pr(PR_HELM_SWEEP, st, 3.0 * s->N * 2 * sizeof(T));
        CKH((helm_sor<T, T>(g, a0, c.nu, omega, E, R, color, st)));
      }
    }
    CKH(add_cast<T>(u, E, n3, st));
  }
  S.iters = it;
  S.rel_res = rel;
  if (rel > c.helm_rtol) return fail(s, SIM_ENOTCONV, "momentum solve iteration limit reached");
  return SIM_OK;
}

sim_status helm_solve_any(sim_t s, const double *rhs, double *u, sim_solve_stats *stt) {
  return s->fp32 ? helm_solve<float>(s, rhs, u, stt) : helm_solve<double>(s, rhs, u, stt);
}

// ---------------------------------------------------------------------------
// One-way (prescribed motion) and two-way (free bodies) time steps.

// Step 2 of both schemes: momentum right-hand side with W Phi^n spread on the
// band, then u* from the extrapolated guess 2 u^n - u^{n-1}.
sim_status predictor(sim_t s, sim_step_stats &S, sim_status &hrc) {
  hipStream_t st = s->st;
  const sim_config &c = s->cfg;
  CKH(gather3(s->K, s->PERM, s->PHIN, s->PHIS, st));
  {
    // u^n, u^{n-1} (three components each) and p^n read; rhs and the guess written
    ProbeScope pr(PR_MOM_RHS, st, 13.0 * s->N * sizeof(double));
    CKH(mom_rhs(s->g, c.dt, s->U, s->UM, s->P, s->RHSU, s->USTAR, st));
  }
  CKH(band_apply(s->ker, false, s->g, s->nt1, s->nt2, s->nactive, s->ACTIVE, s->TLSTART, s->TLIST, s->XS, s->PHIS, 1.0,
                 s->RHSU, st));
  hrc = helm_solve_any(s, s->RHSU, s->USTAR, &S.helm);
  if (hrc != SIM_OK && hrc != SIM_ENOTCONV) return hrc;
  return SIM_OK;
}

// One pressure / force correction on u^(k) = USTAR with the point velocities
// in US: solves eq. Saddle (Sec. 3.1) / eq. pressure_force_iterative_system
// (Sec. 3.2.1), then u += xi tau (-G p' + W Phi'), p += xi p', Phi += xi Phi'.
// Sets S.outer_crit = ||Phi'||_1 / ||Phi^(k+1)||_1 (eq. convergence_criterion)
// when want_crit.
sim_status correction(sim_t s, int k, bool want_crit, sim_step_stats &S, double &divstar, sim_status &src) {
  hipStream_t st = s->st;
  const sim_config &c = s->cfg;
  const long long N = s->N;
  const double tau = 2.0 * c.dt / 3.0;
  sim_status rc;
  CKH(div_apply(s->g, s->USTAR, s->RHSP, -1.0 / tau, st));
  if (k == 0) {
    double d2;
    if ((rc = dev_norm2(s, s->RHSP, N, &d2))) return rc;
    divstar = sqrt(d2) * tau;
  }
  CKH(interp_face(s->ker, s->g, s->nt1, s->nt2, s->nnz, s->NZT, s->TSTART, s->XS, s->USTAR, 1.0 / tau, s->US,
                  -1.0 / tau, s->RF, st));
  src = schur_solve_core(s, &S.schur);
  if (src != SIM_OK && src != SIM_ENOTCONV) return src;
  S.total_schur_iters += S.schur.iters;
  CKH(grad_apply(s->g, s->PP, s->USTAR, -c.xi * tau, s->USTAR, st));
  CKH(band_apply(s->ker, false, s->g, s->nt1, s->nt2, s->nactive, s->ACTIVE, s->TLSTART, s->TLIST, s->XS, s->PHIP,
                 c.xi * tau, s->USTAR, st));
  CKH(axpby(s->P, s->PP, N, c.xi, 1.0, st));
  CKH(scale3(s->K, s->PHIP, c.xi, s->PHIS, 1.0, s->PHIS, st));
  S.outer = k + 1;
  if (want_crit) {
    // ||Phi'||_1 and ||Phi||_1 on the device
    double l1[2] = {0.0, 0.0};
    if (s->K > 0) {
      CKH(abs_sums(s->PHIP, s->PHIS, 3LL * s->K, s->PART, st));
      CKH(finalize(s->PART, red_blocks(), 2, s->RED, st, s->hpin_dev));
      sim_status rc2 = read_mirror(s, 2, l1);
      if (rc2) return rc2;
    }
    const double na = l1[0], nbb = l1[1];
    S.outer_crit = nbb > 0 ? na / nbb : (na > 0 ? INFINITY : 0.0);
  }
  return SIM_OK;
}

// Diagnostics and the rotation of the time levels after the corrections.
sim_status finish_step(sim_t s, double t1, double divstar, sim_step_stats &S) {
  hipStream_t st = s->st;
  const long long N = s->N;
  sim_status rc;
  CKH(scatter3(s->K, s->PERM, s->PHIS, s->PHIN, st));
  CKH(div_apply(s->g, s->USTAR, s->TMPC, 1.0, st));
  if (s->K > 0)
    CKH(interp_face(s->ker, s->g, s->nt1, s->nt2, s->nnz, s->NZT, s->TSTART, s->XS, s->USTAR, 1.0, s->US, -1.0,
                    s->PT3, st));
  // |D u|^2, |slip|^2, |U|^2 in one reduction
  double q3[3];
  CKH(sumsq3(s->TMPC, N, s->K > 0 ? s->PT3 : nullptr, 3LL * s->K, s->K > 0 ? s->US : nullptr, 3LL * s->K, s->PART,
             st));
  CKH(finalize(s->PART, red_blocks(), 3, s->RED, st, s->hpin_dev));
  if ((rc = read_mirror(s, 3, q3))) return rc;
  S.div_rel = divstar > 0 ? sqrt(q3[0]) / divstar : 0.0;
  if (s->K > 0) S.slip_rel = q3[2] > 0 ? sqrt(q3[1] / q3[2]) : 0.0;
  // u^{n-1} <- u^n, u^n <- u^{n+1}
  std::swap(s->UM, s->U);
  std::swap(s->U, s->USTAR);
  s->t = t1;
  ++s->nstep;
  return SIM_OK;
}

struct StepTimer {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipStream_t st;
  explicit StepTimer(hipStream_t s) : st(s) {
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return;
    hipEventRecord(e0, st);
  }
  double seconds() {
    float ms = 0;
    if (e0 && e1 && hipEventRecord(e1, st) == hipSuccess && hipEventSynchronize(e1) == hipSuccess)
      hipEventElapsedTime(&ms, e0, e1);
    return ms * 1e-3;
  }
  ~StepTimer() {
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
  }
};

sim_status step_one_way(sim_t s, sim_step_stats *out) {
  const sim_config &c = s->cfg;
  StepTimer timer(s->st);
  sim_status rc;
  double t1 = s->t + c.dt;
  std::vector<BodyDev> bd = body_states_at(s, t1);
  if ((rc = place_and_bin(s, bd))) return rc;
  sim_step_stats S{};
  sim_status hrc = SIM_OK, src = SIM_OK;
  if ((rc = predictor(s, S, hrc))) return rc;
  double divstar = 0.0;
  for (int k = 0; k < c.outer_iters; ++k) {
    bool want = c.outer_tol > 0 || k + 1 == c.outer_iters;
    if ((rc = correction(s, k, want, S, divstar, src))) return rc;
    if (c.outer_tol > 0 && S.outer_crit < c.outer_tol) break;
  }
  if ((rc = finish_step(s, t1, divstar, S))) return rc;
  S.seconds = timer.seconds();
  s->last = S;
  s->adj_ready = S.outer == 1;
  if (out) *out = S;
  if (hrc == SIM_ENOTCONV) return fail(s, SIM_ENOTCONV, "momentum solve iteration limit reached");
  return src;
}

// Node box of a sphere for the volume integrals: every velocity node within
// a + h sqrt(3)/2 of the centre (the only ones with alpha > 0).
BodySpan body_span(const sim_s *s, const HostBody &hb, const double c[3]) {
  BodySpan sp{};
  sp.k0 = hb.k0;
  sp.kn = hb.kn;
  sp.radius = hb.b.radius;
  const double h = s->g.h;
  for (int a = 0; a < 3; ++a) {
    sp.c[a] = c[a];
    const int n = s->cfg.n[a];
    int lo = (int)floor((c[a] - hb.b.radius) / h) - 2;
    int hi = (int)floor((c[a] + hb.b.radius) / h) + 3;  // exclusive
    int dim = hi - lo;
    if (dim > n) { lo = 0; dim = n; }  // never visit a node twice
    sp.lo[a] = lo;
    sp.dim[a] = dim;
  }
  return sp;
}

// Per-body sums on the device -> host: h3 sum Phi, torque (when phi given)
// and the volume integrals of u at the spans' centres.
sim_status body_sums(sim_t s, const double *phi_nat, const double *u, std::vector<double> &out) {
  hipStream_t st = s->st;
  const int nb = s->nb;
  const double h3 = s->g.h * s->g.h * s->g.h;
  if (phi_nat) CKH(body_force_torque(nb, s->BODIES, s->SPAN, s->OFF, phi_nat, h3, s->BSUM, st));
  CKH(body_volume_integrals(s->g, nb, s->SPAN, u, s->VPART, s->BSUM, st));
  out.assign(12 * (size_t)nb, 0.0);
  CKH(hipMemcpyAsync(out.data(), s->BSUM, sizeof(double) * 12 * nb, hipMemcpyDeviceToHost, st));
  CKH(hipStreamSynchronize(st));
  for (double v : out)
    if (!isfinite(v)) return fail(s, SIM_ENONFINITE, "non-finite body force or volume integral");
  return SIM_OK;
}

sim_status upload_spans(sim_t s, bool predicted) {
  CKH(hipStreamSynchronize(s->st));  // the previous upload has been consumed
  s->hspan.resize(s->nb);
  for (int i = 0; i < s->nb; ++i) {
    const HostBody &hb = s->bodies[i];
    s->hspan[i] = body_span(s, hb, predicted ? hb.xc1 : hb.xc);
  }
  CKH(hipMemcpyAsync(s->SPAN, s->hspan.data(), sizeof(BodySpan) * s->nb, hipMemcpyHostToDevice, s->st));
  return SIM_OK;
}

// R^{n+1} = R^n R_Delta, R_Delta the rotation by the AB2 angle
// dt (3/2 |w^n| - 1/2 |w^{n-1}|) about the body-frame axis of w^n (Sec. 2.2).
void rotation_step(const double R[9], const double w[3], const double wm[3], double dt, double R1[9]) {
  double wn = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
  if (wn == 0.0) {
    memcpy(R1, R, sizeof(double) * 9);
    return;
  }
  double wmn = sqrt(wm[0] * wm[0] + wm[1] * wm[1] + wm[2] * wm[2]);
  double gamma = dt * (1.5 * wn - 0.5 * wmn);
  double e[3] = {w[0] / wn, w[1] / wn, w[2] / wn}, ax[3];
  for (int i = 0; i < 3; ++i) ax[i] = R[i] * e[0] + R[3 + i] * e[1] + R[6 + i] * e[2];  // R^T e
  double Rd[9];
  mat_rodrigues(ax, gamma, Rd);
  mat_mul(R, Rd, R1);
}

// Two-way step (Sec. 3.2.1): Step 1 predicts the body positions and
// orientations; Step 2 is the momentum predictor; Step 3 iterates Newton-Euler
// on the host (from device sums of the forces and of the volume integrals) and
// the pressure-force correction with relaxation xi, up to outer_iters times or
// until ||Phi'||_1 / ||Phi||_1 < outer_tol.
sim_status step_two_way(sim_t s, sim_step_stats *out) {
  hipStream_t st = s->st;
  const sim_config &c = s->cfg;
  StepTimer timer(st);
  sim_status rc;
  const int nb = s->nb;
  const double dt = c.dt, t1 = s->t + dt;
  std::vector<double> sums;
  // volume history at the start: levels n and n-1 both from u^0 at X_c^0
  if (!s->vol_init) {
    if ((rc = upload_spans(s, false))) return rc;
    if ((rc = body_sums(s, nullptr, s->U, sums))) return rc;
    for (int i = 0; i < nb; ++i) {
      HostBody &hb = s->bodies[i];
      for (int a = 0; a < 3; ++a) {
        hb.I_n[a] = hb.I_m[a] = sums[12 * i + 6 + a];
        hb.J_n[a] = hb.J_m[a] = sums[12 * i + 9 + a];
      }
    }
    s->vol_init = true;
  }
  // record for the reverse-mode step: the body state before the step
  const bool rec = c.record_two_way && s->REC_U;
  const long long N = s->N, K3 = 3LL * s->Kmax;
  if (rec) {
    s->rec_pre.assign(18 * (size_t)nb, 0.0);
    s->rec_body.assign(6 * (size_t)nb * c.outer_iters, 0.0);
    for (int i = 0; i < nb; ++i) {
      const HostBody &hb = s->bodies[i];
      double *q = &s->rec_pre[18 * i];
      for (int a = 0; a < 3; ++a) {
        q[a] = hb.xc[a];
        q[3 + a] = hb.xc_m[a];
        q[6 + a] = hb.us[a];
        q[9 + a] = hb.us_m[a];
        q[12 + a] = hb.w[a];
        q[15 + a] = hb.w_m[a];
      }
    }
  }
  // Step 1: X_c^{n+1} = (4 X_c^n - X_c^{n-1}) / 3 + (2 dt / 3) u_s^n, R^{n+1}
  std::vector<BodyDev> bd(nb);
  for (int i = 0; i < nb; ++i) {
    HostBody &hb = s->bodies[i];
    for (int a = 0; a < 3; ++a) hb.xc1[a] = (4.0 * hb.xc[a] - hb.xc_m[a]) / 3.0 + (2.0 * dt / 3.0) * hb.us[a];
    rotation_step(hb.R, hb.w, hb.w_m, dt, hb.R1);
    for (int a = 0; a < 3; ++a) { bd[i].c[a] = hb.xc1[a]; bd[i].v[a] = hb.us[a]; bd[i].w[a] = hb.w[a]; }
    memcpy(bd[i].R, hb.R1, sizeof(double) * 9);
  }
  if ((rc = place_and_bin(s, bd))) return rc;
  if ((rc = upload_spans(s, true))) return rc;
  // Step 2
  sim_step_stats S{};
  sim_status hrc = SIM_OK, src = SIM_OK;
  if ((rc = predictor(s, S, hrc))) return rc;
  // Step 3
  const double tau = 2.0 * dt / 3.0;
  std::vector<double> us_k(3 * (size_t)nb), w_k(3 * (size_t)nb);
  double divstar = 0.0;
  for (int k = 0; k < c.outer_iters; ++k) {
    // forces of Phi^(n,k) (natural order) and volume integrals of u^(k)
    CKH(scatter3(s->K, s->PERM, s->PHIS, s->PT3, st));
    if ((rc = body_sums(s, s->PT3, s->USTAR, sums))) return rc;
    for (int i = 0; i < nb; ++i) {
      const HostBody &hb = s->bodies[i];
      const double a = hb.b.radius, theta = hb.b.density_ratio;
      const double Vp = 4.0 / 3.0 * M_PI * a * a * a, Ip = 0.4 * Vp * a * a;
      const double *F = &sums[12 * i], *T = &sums[12 * i + 3], *Ik = &sums[12 * i + 6], *Jk = &sums[12 * i + 9];
      for (int q = 0; q < 3; ++q) {
        us_k[3 * i + q] = (4.0 * hb.us[q] - hb.us_m[q]) / 3.0 +
                          tau / (theta * Vp) *
                              (-F[q] + (3.0 * Ik[q] - 4.0 * hb.I_n[q] + hb.I_m[q]) / (2.0 * dt) +
                               (theta - 1.0) * Vp * c.g[q]);
        w_k[3 * i + q] = (4.0 * hb.w[q] - hb.w_m[q]) / 3.0 +
                         tau / (theta * Ip) * (-T[q] + (3.0 * Jk[q] - 4.0 * hb.J_n[q] + hb.J_m[q]) / (2.0 * dt));
      }
      for (int q = 0; q < 3; ++q) { bd[i].v[q] = us_k[3 * i + q]; bd[i].w[q] = w_k[3 * i + q]; }
      if (!isfinite(us_k[3 * i] + us_k[3 * i + 1] + us_k[3 * i + 2] + w_k[3 * i] + w_k[3 * i + 1] + w_k[3 * i + 2]))
        return fail(s, SIM_ENONFINITE, "non-finite body velocity");
    }
    // U^(k) = u_s^(k) + omega^(k) x L~ at the predicted points, in tile order
    CKH(hipMemcpyAsync(s->BODIES, bd.data(), sizeof(BodyDev) * nb, hipMemcpyHostToDevice, st));
    CKH(points_place(s->g, s->K, s->BODIES, s->BODYOF, s->OFF, s->XN, s->UN, s->TILE, s->nt0, s->nt1, s->nt2, st));
    CKH(gather3(s->K, s->PERM, s->UN, s->US, st));
    bool want = c.outer_tol > 0 || k + 1 == c.outer_iters;
    if (rec) {
      CKH(hipMemcpyAsync(s->REC_U + k * 3 * N, s->USTAR, sizeof(double) * 3 * N, hipMemcpyDeviceToDevice, st));
      if (s->K > 0)
        CKH(hipMemcpyAsync(s->REC_PHI + k * K3, s->PHIS, sizeof(double) * 3 * s->K, hipMemcpyDeviceToDevice, st));
      for (int i = 0; i < nb; ++i)
        for (int q = 0; q < 3; ++q) {
          s->rec_body[6 * ((size_t)k * nb + i) + q] = us_k[3 * i + q];
          s->rec_body[6 * ((size_t)k * nb + i) + 3 + q] = w_k[3 * i + q];
        }
    }
    if ((rc = correction(s, k, want, S, divstar, src))) return rc;
    if (rec) {
      CKH(hipMemcpyAsync(s->REC_PP + k * N, s->PP, sizeof(double) * N, hipMemcpyDeviceToDevice, st));
      if (s->K > 0) {
        CKH(hipMemcpyAsync(s->REC_PHIP + k * K3, s->PHIP, sizeof(double) * 3 * s->K, hipMemcpyDeviceToDevice, st));
        CKH(hipMemcpyAsync(s->REC_RF + k * K3, s->RF, sizeof(double) * 3 * s->K, hipMemcpyDeviceToDevice, st));
      }
    }
    if (c.outer_tol > 0 && S.outer_crit < c.outer_tol) break;
  }
  // volume integrals of u^{n+1} for the next step's history
  if ((rc = body_sums(s, nullptr, s->USTAR, sums))) return rc;
  for (int i = 0; i < nb; ++i) {
    HostBody &hb = s->bodies[i];
    for (int q = 0; q < 3; ++q) {
      hb.xc_m[q] = hb.xc[q];
      hb.xc[q] = hb.xc1[q];
      hb.us_m[q] = hb.us[q];
      hb.us[q] = us_k[3 * i + q];
      hb.w_m[q] = hb.w[q];
      hb.w[q] = w_k[3 * i + q];
      hb.I_m[q] = hb.I_n[q];
      hb.I_n[q] = sums[12 * i + 6 + q];
      hb.J_m[q] = hb.J_n[q];
      hb.J_n[q] = sums[12 * i + 9 + q];
    }
    memcpy(hb.R, hb.R1, sizeof(double) * 9);
  }
  if ((rc = finish_step(s, t1, divstar, S))) return rc;
  S.seconds = timer.seconds();
  s->last = S;
  // the reverse mode needs the fixed pass count (no early stop on outer_tol)
  s->rec_passes = S.outer;
  s->adj2_ready = rec && c.outer_tol == 0.0 && S.outer == c.outer_iters;
  if (out) *out = S;
  if (hrc == SIM_ENOTCONV) return fail(s, SIM_ENOTCONV, "momentum solve iteration limit reached");
  return src;
}

}  // namespace

// The device address of the static scratch on `device`, which must be the
// current device: taken once per device and kept (each device holds its own
// copy of the array).
constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_noalloc_mu;
void *g_noalloc_ptr[NOALLOC_MAX_DEVICES] = {};

hipError_t noalloc_scratch_setup(int device, void **out) {
  if (device < 0 || device >= NOALLOC_MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  if (!g_noalloc_ptr[device]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_noalloc_ptr[device] = p;
  }
  *out = g_noalloc_ptr[device];
  return hipSuccess;
}

// Frees what sim_create took besides the caller's workspace: the pinned
// reduction mirror, the probe events and the handle itself.
void release_handle(sim_t s) {
  if (s->hpin) hipHostFree(s->hpin);
  probe_free(s->probes);
  for (hipEvent_t e : s->ev_solve)
    if (e) hipEventDestroy(e);
  if (s->ev_iter) hipEventDestroy(s->ev_iter);
  delete s;
}

// sim_solve_schur on whatever solve scratch the handle currently points to
sim_status solve_schur_entry(sim_t s, const double *d_rhs_p, const double *d_rhs_f, double *d_p, double *d_phi,
                             sim_solve_stats *stats) {
  s->adj_ready = false;
  s->adj2_ready = false;
  if (!s->have_bodies) return fail(s, SIM_ESTATE, "no bodies set");
  if (!d_rhs_p || !d_p || (s->K > 0 && (!d_rhs_f || !d_phi))) return fail(s, SIM_EINVAL, "null argument");
  hipStream_t st = s->st;
  CKH(to_split(s->g, 1, d_rhs_p, s->BVEC, st));
  if (s->K > 0) CKH(gather3(s->K, s->PERM, d_rhs_f, s->RF, st));
  sim_status rc = schur_solve_core(s, stats, true);
  if (rc != SIM_OK && rc != SIM_ENOTCONV) return rc;
  const bool deferred = s->cfg.krylov == SIM_KRYLOV_FGMRES;
  CKH(to_natural(s->g, 1, s->PP, d_p, st, deferred ? mean_slots(s) + 1 : nullptr, 1.0 / (double)s->N));
  if (s->K > 0) CKH(scatter3(s->K, s->PERM, s->PHIP, d_phi, st));
  sim_status r2 = sync(s);
  return r2 ? r2 : rc;
}

// ===========================================================================
// C ABI

extern "C" {

sim_status sim_config_check(const sim_config *cfg, int64_t max_points, char *msg, int32_t msg_len) {
  std::vector<int> dims;
  std::string v = validate(cfg, &dims);
  if (v.empty() && (max_points < 0 || max_points > (1LL << 30))) v = "max_points must be 0..2^30";
  if (msg && msg_len > 0) {
    const size_t n = std::min(v.size(), (size_t)msg_len - 1);
    memcpy(msg, v.data(), n);
    msg[n] = '\0';
  }
  return v.empty() ? SIM_OK : SIM_EINVAL;
}

size_t sim_workspace_bytes(const sim_config *cfg, int64_t max_points) {
  std::vector<int> dims;
  if (!validate(cfg, &dims).empty() || max_points < 0 || max_points > (1LL << 30)) return 0;
  return layout(nullptr, cfg, max_points, nullptr, dims);
}

sim_status sim_create(const sim_config *cfg, void *d_workspace, size_t bytes, int64_t max_points, sim_t *out) {
  if (!out) return SIM_EINVAL;
  *out = nullptr;
  std::vector<int> dims;
  std::string v = validate(cfg, &dims);
  if (!v.empty() || max_points < 0 || max_points > (1LL << 30)) return SIM_EINVAL;
  size_t need = layout(nullptr, cfg, max_points, nullptr, dims);
  if (!d_workspace || bytes < need) return SIM_ENOMEM;
  sim_t s = new sim_s();
  s->cfg = *cfg;
  s->st = (hipStream_t)cfg->stream;
  if (hipSetDevice(cfg->device) != hipSuccess) {
    delete s;
    return SIM_EDEVICE;
  }
  char *base = (char *)(((uintptr_t)d_workspace + 255) & ~(uintptr_t)255);
  layout(s, cfg, max_points, base, dims);
  s->g = s->lv[0].g;
  s->N = 2 * s->g.half;
  s->nt0 = cfg->n[0] / 4; s->nt1 = cfg->n[1] / 4; s->nt2 = cfg->n[2] / 4;
  s->ntiles = (long long)s->nt0 * s->nt1 * s->nt2;
  s->Kmax = (int)max_points;
  s->fp32 = cfg->precision == SIM_PREC_FP32MG;
  s->ker = cfg->delta;
  s->c = cfg->lump_c;
  if (hipHostMalloc((void **)&s->hpin, 64 * 1024) != hipSuccess) {
    delete s;
    return SIM_EDEVICE;
  }
  s->probes = probe_new();
  s->dims = dims;
  if (hipEventCreate(&s->ev_solve[0]) != hipSuccess || hipEventCreate(&s->ev_solve[1]) != hipSuccess ||
      hipEventCreateWithFlags(&s->ev_iter, hipEventDisableTiming) != hipSuccess ||
      noalloc_scratch_setup(cfg->device, &s->noalloc_scratch) != hipSuccess) {
    release_handle(s);
    return SIM_EDEVICE;
  }
  if (hipHostGetDevicePointer((void **)&s->hpin_dev, s->hpin, 0) != hipSuccess) {
    release_handle(s);
    return SIM_EDEVICE;
  }
  {
    const Geo &gcoarse = s->lv.back().g;
    const int cn[3] = {gcoarse.n0, gcoarse.n1, gcoarse.n2};
    const int cbc[3] = {cfg->bc[0], cfg->bc[1], cfg->bc[2]};
    std::vector<double> fd((size_t)coarse_fd_size(cn));
    coarse_fd_build(cn, cbc, gcoarse.h, fd.data());
    if (hipMemcpy(s->COARSEFD, fd.data(), sizeof(double) * fd.size(), hipMemcpyHostToDevice) != hipSuccess) {
      release_handle(s);
      return SIM_EDEVICE;
    }
    const size_t nl = s->lv.size();
    if (nl >= 2 && subcycle_fits(s->lv[nl - 2].g, s->lv[nl - 1].g) &&
        (mg_subcycle_tables(s->lv[nl - 2].g, s->lv[nl - 1].g, s->SUBTAB, s->st) != hipSuccess ||
         hipStreamSynchronize(s->st) != hipSuccess)) {
      release_handle(s);
      return SIM_EDEVICE;
    }
    if (s->fdx) {
      const int fn[3] = {cfg->n[0], cfg->n[1], cfg->n[2]};
      std::vector<double> qd((size_t)coarse_fd_size(fn)), blob(fdx_blob_doubles(fn));
      coarse_fd_build(fn, cbc, s->g.h, qd.data());
      fdx_blob_pack(fn, qd.data(), blob.data());
      if (hipMemcpy(s->FDXQ, blob.data(), sizeof(double) * blob.size(), hipMemcpyHostToDevice) != hipSuccess) {
        release_handle(s);
        return SIM_EDEVICE;
      }
    }
    if (s->fastdiag || s->coarse_mfma) {
      const Geo &gq = s->fastdiag ? s->lv[0].g : gcoarse;
      const int fn[3] = {gq.n0, gq.n1, gq.n2};
      std::vector<double> qd((size_t)coarse_fd_size(fn));
      coarse_fd_build(fn, cbc, gq.h, qd.data());
      std::vector<unsigned char> blob(fd_blob_bytes(fn));
      fd_blob_pack(fn, qd.data(), blob.data());
      if (hipMemcpy(s->FDQ, blob.data(), blob.size(), hipMemcpyHostToDevice) != hipSuccess) {
        release_handle(s);
        return SIM_EDEVICE;
      }
    }
  }
  hipStream_t st = s->st;
  bool ok = fill(s->U, 3 * s->N, 0.0, st) == hipSuccess && fill(s->UM, 3 * s->N, 0.0, st) == hipSuccess &&
            fill(s->P, s->N, 0.0, st) == hipSuccess && fill(s->USTAR, 3 * s->N, 0.0, st) == hipSuccess &&
            hipStreamSynchronize(st) == hipSuccess;
  if (!ok) {
    release_handle(s);
    return SIM_EDEVICE;
  }
  *out = s;
  return SIM_OK;
}

sim_status sim_destroy(sim_t s) {
  if (!s) return SIM_EINVAL;
  hipStreamSynchronize(s->st);
  release_handle(s);
  return SIM_OK;
}

const char *sim_last_error(sim_t s) { return s ? s->err.c_str() : "null handle"; }

sim_status sim_set_bodies(sim_t s, int32_t nb, const sim_body *bodies, const double *offsets) {
  if (!s) return SIM_EINVAL;
  if (nb < 0 || nb > MAX_BODIES || (nb > 0 && (!bodies || !offsets))) return fail(s, SIM_EINVAL, "bad body list");
  long long K = 0;
  for (int i = 0; i < nb; ++i) {
    if (bodies[i].n_points < 0 || !(bodies[i].radius >= 0)) return fail(s, SIM_EINVAL, "bad body");
    if (bodies[i].motion != SIM_MOTION_PRESCRIBED && bodies[i].motion != SIM_MOTION_FREE)
      return fail(s, SIM_EINVAL, "bad motion type");
    if (bodies[i].motion == SIM_MOTION_FREE && !(bodies[i].density_ratio > 0 && bodies[i].radius > 0))
      return fail(s, SIM_EINVAL, "free body needs density_ratio > 0 and radius > 0");
    if (bodies[i].motion != bodies[0].motion)
      return fail(s, SIM_EINVAL, "bodies must be all prescribed or all free");
    K += bodies[i].n_points;
  }
  if (K > s->Kmax) return fail(s, SIM_EINVAL, "more points than max_points");
  s->bodies.assign(nb, HostBody());
  std::vector<int> body_of((size_t)std::max<long long>(K, 1));
  long long k0 = 0;
  for (int i = 0; i < nb; ++i) {
    HostBody &hb = s->bodies[i];
    hb.b = bodies[i];
    hb.k0 = (int)k0;
    hb.kn = bodies[i].n_points;
    double r = 0;
    for (int k = 0; k < hb.kn; ++k) {
      const double *o = offsets + 3 * (k0 + k);
      r = std::max(r, sqrt(o[0] * o[0] + o[1] * o[1] + o[2] * o[2]));
      body_of[k0 + k] = i;
    }
    hb.rmax = r;
    double c[3], v[3], R[9];
    prescribed_state(hb.b, s->t, c, v, R);
    if (hb.b.motion == SIM_MOTION_FREE) {
      // steady motion before the first step: X_c^{-1} = X_c^0 - dt u_s^0
      for (int a = 0; a < 3; ++a) {
        hb.xc[a] = bodies[i].center[a];
        hb.xc_m[a] = bodies[i].center[a] - s->cfg.dt * bodies[i].vel[a];
        hb.us[a] = hb.us_m[a] = bodies[i].vel[a];
        hb.w[a] = hb.w_m[a] = bodies[i].omega[a];
        hb.I_n[a] = hb.I_m[a] = hb.J_n[a] = hb.J_m[a] = 0.0;
      }
      for (int q = 0; q < 9; ++q) hb.R[q] = (q % 4 == 0) ? 1.0 : 0.0;
    }
    k0 += hb.kn;
  }
  s->K = (int)K;
  s->nb = nb;
  s->any_free = nb > 0 && bodies[0].motion == SIM_MOTION_FREE;
  s->adj_ready = false;
  s->adj2_ready = false;
  s->vol_init = false;
  hipStream_t st = s->st;
  if (K > 0) {
    CKH(hipMemcpyAsync(s->OFF, offsets, sizeof(double) * 3 * K, hipMemcpyHostToDevice, st));
    CKH(hipMemcpyAsync(s->BODYOF, body_of.data(), sizeof(int) * K, hipMemcpyHostToDevice, st));
    CKH(fill(s->PHIN, 3 * K, 0.0, st));
  }
  std::vector<BodyDev> bd = body_states_at(s, s->t);
  sim_status rc = place_and_bin(s, bd);
  if (rc) return rc;
  s->have_bodies = true;
  return SIM_OK;
}

sim_status sim_set_fields(sim_t s, int32_t level, const double *d_u, const double *d_v, const double *d_w,
                          const double *d_p, const double *d_phi) {
  if (!s || (level != 0 && level != 1)) return fail(s, SIM_EINVAL, "level must be 0 or 1");
  hipStream_t st = s->st;
  double *U = level == 0 ? s->U : s->UM;
  const double *src[3] = {d_u, d_v, d_w};
  for (int d = 0; d < 3; ++d) {
    if (!src[d]) continue;
    // one component at a time: conversion of a single plane
    CKH(to_split(s->g, 1, src[d], U + d * s->N, st));
  }
  CKH(zero_wall_faces(s->g, U, st));
  s->vol_init = false;  // the volume history of free bodies restarts from the new u^n
  s->adj_ready = false;
  s->adj2_ready = false;
  if (level == 0 && d_p) CKH(to_split(s->g, 1, d_p, s->P, st));
  if (level == 0 && d_phi && s->K > 0)
    CKH(hipMemcpyAsync(s->PHIN, d_phi, sizeof(double) * 3 * s->K, hipMemcpyDeviceToDevice, st));
  return sync(s);
}

sim_status sim_get_fields(sim_t s, double *d_u, double *d_v, double *d_w, double *d_p) {
  if (!s) return SIM_EINVAL;
  hipStream_t st = s->st;
  double *dst[3] = {d_u, d_v, d_w};
  for (int d = 0; d < 3; ++d)
    if (dst[d]) CKH(to_natural(s->g, 1, s->U + d * s->N, dst[d], st));
  if (d_p) CKH(to_natural(s->g, 1, s->P, d_p, st));
  return sync(s);
}

sim_status sim_set_time(sim_t s, double t) {
  if (!s) return SIM_EINVAL;
  if (!isfinite(t)) return fail(s, SIM_EINVAL, "time must be finite");
  s->t = t;
  s->adj_ready = false;
  s->adj2_ready = false;
  return SIM_OK;
}

sim_status sim_get_body_state(sim_t s, double *state) {
  if (!s) return SIM_EINVAL;
  if (!s->have_bodies) return fail(s, SIM_ESTATE, "no bodies set");
  if (!state && s->nb > 0) return fail(s, SIM_EINVAL, "null argument");
  std::vector<BodyDev> bd = body_states_at(s, s->t);
  for (int i = 0; i < s->nb; ++i) {
    double *o = state + 18 * i;
    for (int a = 0; a < 3; ++a) {
      o[a] = bd[i].c[a];
      o[3 + a] = bd[i].v[a];
      o[6 + a] = bd[i].w[a];
    }
    memcpy(o + 9, bd[i].R, sizeof(double) * 9);
  }
  return SIM_OK;
}

sim_status sim_get_points(sim_t s, double *d_X, double *d_U) {
  if (!s) return SIM_EINVAL;
  if (!s->have_bodies) return fail(s, SIM_ESTATE, "no bodies set");
  if (s->K > 0) {
    if (d_X) CKH(hipMemcpyAsync(d_X, s->XN, sizeof(double) * 3 * s->K, hipMemcpyDeviceToDevice, s->st));
    if (d_U) CKH(hipMemcpyAsync(d_U, s->UN, sizeof(double) * 3 * s->K, hipMemcpyDeviceToDevice, s->st));
  }
  return sync(s);
}

sim_status sim_get_forces(sim_t s, double *d_f, double *body_ft) {
  if (!s) return SIM_EINVAL;
  if (!s->have_bodies) return fail(s, SIM_ESTATE, "no bodies set");
  hipStream_t st = s->st;
  double h3 = s->g.h * s->g.h * s->g.h;
  if (d_f && s->K > 0) CKH(scale3(s->K, s->PHIN, h3, nullptr, 0.0, d_f, st));
  if (body_ft) {
    std::vector<double> phi(3 * (size_t)s->K), X(3 * (size_t)s->K);
    if (s->K > 0) {
      CKH(hipMemcpyAsync(phi.data(), s->PHIN, sizeof(double) * 3 * s->K, hipMemcpyDeviceToHost, st));
      CKH(hipMemcpyAsync(X.data(), s->XN, sizeof(double) * 3 * s->K, hipMemcpyDeviceToHost, st));
    }
    CKH(hipStreamSynchronize(st));
    std::vector<BodyDev> bd = body_states_at(s, s->t);
    for (int i = 0; i < s->nb; ++i) {
      const HostBody &hb = s->bodies[i];
      double F[3] = {0, 0, 0}, T[3] = {0, 0, 0};
      for (int k = hb.k0; k < hb.k0 + hb.kn; ++k) {
        double l[3] = {X[3 * k] - bd[i].c[0], X[3 * k + 1] - bd[i].c[1], X[3 * k + 2] - bd[i].c[2]};
        const double *f = &phi[3 * k];
        for (int a = 0; a < 3; ++a) F[a] += f[a];
        T[0] += l[1] * f[2] - l[2] * f[1];
        T[1] += l[2] * f[0] - l[0] * f[2];
        T[2] += l[0] * f[1] - l[1] * f[0];
      }
      for (int a = 0; a < 3; ++a) {
        body_ft[6 * i + a] = h3 * F[a];
        body_ft[6 * i + 3 + a] = h3 * T[a];
      }
    }
  }
  return sync(s);
}

sim_status sim_solve_schur(sim_t s, const double *d_rhs_p, const double *d_rhs_f, double *d_p, double *d_phi,
                           sim_solve_stats *stats) {
  if (!s) return SIM_EINVAL;
  ProbeBind probe_bind_(s->probes);
  return solve_schur_entry(s, d_rhs_p, d_rhs_f, d_p, d_phi, stats);
}

sim_status sim_solve_schur_noalloc(sim_t s, const double *d_rhs_p, const double *d_rhs_f, double *d_p,
                                   double *d_phi, sim_solve_stats *stats) {
  if (!s) return SIM_EINVAL;
  ProbeBind probe_bind_(s->probes);
  if (!s->noalloc_scratch) return fail(s, SIM_ESTATE, "static scratch not set up");
  const long long K = s->Kmax > 0 ? s->Kmax : 1;
  Carver sizing(nullptr);
  carve_solve(sizing, &s->cfg, K, 0, s->dims);
  if (sizing.off > NOALLOC_SCRATCH_BYTES) {
    char msg[160];
    snprintf(msg, sizeof msg, "this solve needs %zu bytes of static scratch, more than its %zu", sizing.off,
             (size_t)NOALLOC_SCRATCH_BYTES);
    return fail(s, SIM_EINVAL, msg);
  }
  Carver cv(s->noalloc_scratch);
  const SolveScratch mine = carve_solve(cv, &s->cfg, K, 0, s->dims);
  const SolveScratch own = get_solve_scratch(s);
  put_solve_scratch(s, mine);
  const sim_status rc = solve_schur_entry(s, d_rhs_p, d_rhs_f, d_p, d_phi, stats);
  put_solve_scratch(s, own);
  return rc;
}

sim_status sim_step(sim_t s, int32_t nsteps, sim_step_stats *stats) {
  if (!s) return SIM_EINVAL;
  ProbeBind probe_bind_(s->probes);
  s->adj_ready = false;
  s->adj2_ready = false;
  if (!s->have_bodies) return fail(s, SIM_ESTATE, "no bodies set");
  if (nsteps < 0) return fail(s, SIM_EINVAL, "nsteps < 0");
  sim_status rc = SIM_OK;
  for (int i = 0; i < nsteps; ++i) {
    rc = s->any_free ? step_two_way(s, stats) : step_one_way(s, stats);
    if (rc != SIM_OK && rc != SIM_ENOTCONV) return rc;
  }
  return rc;
}

sim_status sim_step_adjoint(sim_t s, const double *d_gu, const double *d_gv, const double *d_gw, const double *d_gp,
                            const double *d_gphi, double *d_gX, double *gU, double *d_gu_in, double *d_gum_in,
                            double *d_gp_in, double *d_gphi_in) {
  if (!s) return SIM_EINVAL;
  ProbeBind probe_bind_(s->probes);
  if (!s->have_bodies || !s->adj_ready)
    return fail(s, SIM_ESTATE, "no recorded one-way step with one correction to transpose");
  hipStream_t st = s->st;
  const sim_config &c = s->cfg;
  const Geo &g = s->g;
  const long long N = s->N, n3 = 3 * N;
  const int K = s->K, ker = s->ker;
  const double tau = 2.0 * c.dt / 3.0, xi = c.xi, ic = 1.0 / s->c;
  const long long K3 = 3LL * s->Kmax;
  double *A0 = s->ADJ, *A1 = A0 + K3, *A2 = A1 + K3, *A3 = A2 + K3, *A4 = A3 + K3;
  double *UB = s->TMP3, *RB = s->RHSU, *F3 = s->USTAR, *PB = s->RHSP, *BB = s->BVEC;
  sim_status rc;
  auto band = [&](bool div, const double *q, double alpha, double *out) {
    return band_apply(ker, div, g, s->nt1, s->nt2, s->nactive, s->ACTIVE, s->TLSTART, s->TLIST, s->XS, q, alpha, out,
                      st);
  };
  // cotangents of u^{n+1} (masked), p^{n+1}, Phi^{n+1}
  CKH(fill(UB, n3, 0.0, st));
  const double *gin[3] = {d_gu, d_gv, d_gw};
  for (int d = 0; d < 3; ++d)
    if (gin[d]) CKH(to_split(g, 1, gin[d], UB + d * N, st));
  CKH(zero_wall_faces(g, UB, st));
  CKH(fill(PB, N, 0.0, st));
  if (d_gp) CKH(to_split(g, 1, d_gp, PB, st));
  if (K > 0) {
    if (d_gphi) CKH(gather3(K, s->PERM, d_gphi, A0, st));
    else CKH(fill(A0, 3LL * K, 0.0, st));
  }
  // update u+ = u* + xi tau (-G p' + W Phi'), p+ = p + xi p', Phi+ = Phi + xi Phi':
  //   pbar' = xi pbar+ - xi tau G^T ubar = xi pbar+ + xi tau D ubar
  //   Phibar' = xi Phibar+ + xi tau W^T ubar,  Xbar = xi tau d(ubar^T W Phi')
  CKH(div_apply(g, UB, BB, xi * tau, st));
  CKH(axpby(PB, BB, N, 1.0, xi, st));
  CKH(interp_face(ker, g, s->nt1, s->nt2, s->nnz, s->NZT, s->TSTART, s->XS, UB, xi * tau, A0, xi, A1, st));
  CKH(fill(A4, 3LL * K, 0.0, st));
  CKH(interp_dx(ker, g, K, s->XS, UB, s->PHIP, xi * tau, A4, st));
  // force recovery Phi' = c^-1 (-W^T G p' - RHS_F):
  //   pbar' += c^-1 D W Phibar',  RHS_F bar = -c^-1 Phibar'
  CKH(band(true, A1, ic, PB));
  CKH(scale3(K, A1, -ic, nullptr, 0.0, A2, st));
  // Schur solve p' = S~^+ b: bbar = S~^+ P pbar' (S~ symmetric)
  if ((rc = project_mean(s, PB))) return rc;
  sim_solve_stats sst{};
  sim_status src = fgmres_any(s, PB, BB, &sst);
  if (src != SIM_OK && src != SIM_ENOTCONV) return src;
  // q2 = W^T G bbar;  d S~ and d(RHS) terms:
  //   Xbar += d((G bbar)^T W Phi') - c^-1 d((G p')^T W (Phibar' + q2))
  CKH(interp_grad<double>(ker, g, s->nt1, s->nt2, s->nnz, s->NZT, s->TSTART, s->XS, BB, 1.0, nullptr, 0.0, A3, st));
  CKH(grad_apply(g, BB, F3, 1.0, nullptr, st));
  CKH(interp_dx(ker, g, K, s->XS, F3, s->PHIP, 1.0, A4, st));
  CKH(scale3(K, A1, 1.0, A3, 1.0, A1, st));
  CKH(grad_apply(g, s->PP, F3, 1.0, nullptr, st));
  CKH(interp_dx(ker, g, K, s->XS, F3, A1, -ic, A4, st));
  // b = P(RHS_p + c^-1 D W RHS_F): RHS_p bar = bbar, RHS_F bar += -c^-1 W^T G bbar
  CKH(scale3(K, A3, -ic, A2, 1.0, A2, st));
  // RHS_p = -D u*/tau, RHS_F = (W^T u* - U)/tau:
  //   u*bar = ubar + G bbar / tau + W RHS_F bar / tau,  Ubar = -RHS_F bar / tau
  CKH(grad_apply(g, BB, UB, 1.0 / tau, UB, st));
  CKH(band(false, A2, 1.0 / tau, UB));
  CKH(zero_wall_faces(g, UB, st));
  CKH(scale3(K, A2, -1.0 / tau, nullptr, 0.0, A3, st));
  //   Xbar += d(u*^T W RHS_F bar) / tau, u* = u^{n+1} + xi tau (G p' - W Phi')
  CKH(grad_apply(g, s->PP, F3, xi * tau, s->U, st));
  CKH(band(false, s->PHIP, -xi * tau, F3));
  CKH(zero_wall_faces(g, F3, st));
  CKH(interp_dx(ker, g, K, s->XS, F3, A2, 1.0 / tau, A4, st));
  // u* = A^-1 rhs (A symmetric): rhs bar = A^-1 u*bar
  CKH(fill(RB, n3, 0.0, st));
  sim_solve_stats hst{};
  sim_status hrc = helm_solve_any(s, UB, RB, &hst);
  if (hrc != SIM_OK && hrc != SIM_ENOTCONV) return hrc;
  // rhs = (4u^n - u^{n-1})/(2dt) - G p^n + W Phi^n - N(u^n): Xbar += d(rhsbar^T W Phi^n)
  CKH(scale3(K, s->PHIP, -xi, s->PHIS, 1.0, A1, st));  // Phi^n = Phi^{n+1} - xi Phi'
  CKH(interp_dx(ker, g, K, s->XS, RB, A1, 1.0, A4, st));
  // outputs
  if (d_gX && K > 0) CKH(scatter3(K, s->PERM, A4, d_gX, st));
  if (gU && s->nb > 0) {
    CKH(scatter3(K, s->PERM, A3, s->PT3, st));
    CKH(hipStreamSynchronize(st));
    s->hspan.assign(s->nb, BodySpan{});
    for (int i = 0; i < s->nb; ++i) {
      s->hspan[i].k0 = s->bodies[i].k0;
      s->hspan[i].kn = s->bodies[i].kn;
    }
    CKH(hipMemcpyAsync(s->SPAN, s->hspan.data(), sizeof(BodySpan) * s->nb, hipMemcpyHostToDevice, st));
    CKH(body_force_torque(s->nb, s->BODIES, s->SPAN, s->OFF, s->PT3, 1.0, s->BSUM, st));
    std::vector<double> sums(12 * (size_t)s->nb);
    CKH(hipMemcpyAsync(sums.data(), s->BSUM, sizeof(double) * 12 * s->nb, hipMemcpyDeviceToHost, st));
    CKH(hipStreamSynchronize(st));
    for (int i = 0; i < s->nb; ++i)
      for (int q = 0; q < 6; ++q) gU[6 * i + q] = sums[12 * i + q];
  }
  if (d_gphi_in && K > 0) {
    CKH(interp_face(ker, g, s->nt1, s->nt2, s->nnz, s->NZT, s->TSTART, s->XS, RB, 1.0, A0, 1.0, A2, st));
    CKH(scatter3(K, s->PERM, A2, d_gphi_in, st));
  }
  if (d_gp_in) {  // pbar^n = pbar+ - G^T rhsbar = pbar+ + D rhsbar
    CKH(div_apply(g, RB, s->TMPC, 1.0, st));
    CKH(fill(PB, N, 0.0, st));
    if (d_gp) CKH(to_split(g, 1, d_gp, PB, st));
    CKH(axpby(s->TMPC, PB, N, 1.0, 1.0, st));
    CKH(to_natural(g, 1, s->TMPC, d_gp_in, st));
  }
  if (d_gum_in) {
    CKH(scale_copy(F3, RB, n3, -1.0 / (2.0 * c.dt), st));
    for (int d = 0; d < 3; ++d) CKH(to_natural(g, 1, F3 + d * N, d_gum_in + d * N, st));
  }
  if (d_gu_in) {  // ubar^n = M (2/dt rhsbar - J_N(u^n)^T rhsbar); u^n is UM after the step
    CKH(convection_adjoint(g, s->UM, RB, F3, st));
    CKH(axpby(F3, RB, n3, 2.0 / c.dt, -1.0, st));
    CKH(zero_wall_faces(g, F3, st));
    for (int d = 0; d < 3; ++d) CKH(to_natural(g, 1, F3 + d * N, d_gu_in + d * N, st));
  }
  if ((rc = sync(s))) return rc;
  if (src == SIM_ENOTCONV) return fail(s, SIM_ENOTCONV, "adjoint Schur solve iteration limit reached");
  if (hrc == SIM_ENOTCONV) return fail(s, SIM_ENOTCONV, "adjoint momentum solve iteration limit reached");
  return SIM_OK;
}

// Reverse mode of the last two-way step (Sec. 3.2.1 with a fixed number of
// outer passes): the passes in reverse order, each the transposed correction
// (as in sim_step_adjoint, with u^k and U^k of the pass), then U^k = u_s^k +
// w^k x L~, Newton-Euler, the force / torque sums of Phi^(k) and the volume
// integrals of u^k; then the momentum predictor, the points
// X = X_c^{n+1} + L~, L~ = R^{n+1} X~, and Step 1 (X_c^{n+1} by BDF2 and
// R^{n+1} = exp([psi]) R^n with psi = gamma w^n / |w^n|; the cotangent of
// psi is J_l(psi)^T times the rotation cotangent sum L~ x Lbar).
sim_status sim_step_adjoint_two_way(sim_t s, const double *d_gu, const double *d_gv, const double *d_gw,
                                    const double *d_gp, const double *d_gphi, const double *gbody_out,
                                    double *d_gu_in, double *d_gum_in, double *d_gp_in, double *d_gphi_in,
                                    double *gbody_in) {
  if (!s) return SIM_EINVAL;
  ProbeBind probe_bind_(s->probes);
  if (!s->have_bodies || !s->adj2_ready)
    return fail(s, SIM_ESTATE, "no recorded two-way step (record_two_way, outer_tol = 0) to transpose");
  hipStream_t st = s->st;
  const sim_config &c = s->cfg;
  const Geo &g = s->g;
  const long long N = s->N, n3 = 3 * N;
  const int K = s->K, ker = s->ker, nb = s->nb, npass = s->rec_passes;
  const double dt = c.dt, tau = 2.0 * dt / 3.0, xi = c.xi, ic = 1.0 / s->c, h3 = g.h * g.h * g.h;
  const long long K3 = 3LL * s->Kmax;
  double *A0 = s->ADJ, *A1 = A0 + K3, *A2 = A1 + K3, *A3 = A2 + K3, *A4 = A3 + K3;
  double *PBN = s->ADJ2, *LBN = PBN + K3, *UBN = LBN + K3, *XBN = UBN + K3, *PHN = XBN + K3;
  double *COEF = PHN + K3, *VP = COEF + 9 * MAX_BODIES;
  double *UB = s->TMP3, *RB = s->RHSU, *F3 = s->USTAR, *PB = s->RHSP, *PPB = s->PP, *BB = s->BVEC;
  sim_status rc;
  auto band = [&](bool div, const double *q, double alpha, double *out) {
    return band_apply(ker, div, g, s->nt1, s->nt2, s->nactive, s->ACTIVE, s->TLSTART, s->TLIST, s->XS, q, alpha, out,
                      st);
  };
  // per-body sums of a natural-order point vector: (sum v, sum L~ x v)
  std::vector<double> sums(12 * (size_t)nb);
  auto body_sums_of = [&](const double *v) -> sim_status {
    CKH(body_force_torque(nb, s->BODIES, s->SPAN, s->OFF, v, 1.0, s->BSUM, st));
    CKH(hipMemcpyAsync(sums.data(), s->BSUM, sizeof(double) * 12 * nb, hipMemcpyDeviceToHost, st));
    CKH(hipStreamSynchronize(st));
    return SIM_OK;
  };
  // transposed volume integrals of u at X_c^{n+1}: ubar += ..., centre cotangents into xc1b
  std::vector<double> xc1b(3 * (size_t)nb, 0.0), vp(9 * VOL_CHUNKS);
  auto vol_adj = [&](const double *u, int i, const double ib[3], const double jb[3]) -> sim_status {
    CKH(body_volume_adjoint(g, s->hspan[i], ib, jb, u, UB, VP, st));
    CKH(hipMemcpyAsync(vp.data(), VP, sizeof(double) * vp.size(), hipMemcpyDeviceToHost, st));
    CKH(hipStreamSynchronize(st));
    for (int t = 0; t < 3 * VOL_CHUNKS; ++t)
      for (int q = 0; q < 3; ++q) xc1b[3 * i + q] += vp[3 * t + q];
    return SIM_OK;
  };
  if ((rc = upload_spans(s, false))) return rc;  // node boxes at X_c^{n+1}
  // output cotangents
  CKH(fill(UB, n3, 0.0, st));
  const double *gin[3] = {d_gu, d_gv, d_gw};
  for (int d = 0; d < 3; ++d)
    if (gin[d]) CKH(to_split(g, 1, gin[d], UB + d * N, st));
  CKH(zero_wall_faces(g, UB, st));
  CKH(fill(PB, N, 0.0, st));
  if (d_gp) CKH(to_split(g, 1, d_gp, PB, st));
  if (K > 0) {
    if (d_gphi) CKH(scale_copy(PBN, d_gphi, 3LL * K, 1.0, st));
    else CKH(fill(PBN, 3LL * K, 0.0, st));
    CKH(fill(LBN, 3LL * K, 0.0, st));
    CKH(fill(A4, 3LL * K, 0.0, st));
  }
  // per-body output cotangents (xc, us, w, I, J of the step's result) and input accumulators
  std::vector<double> gout(15 * (size_t)nb, 0.0), gin_b(30 * (size_t)nb, 0.0);
  if (gbody_out) std::copy(gbody_out, gbody_out + 15 * nb, gout.begin());
  for (int i = 0; i < nb; ++i)
    for (int q = 0; q < 3; ++q) xc1b[3 * i + q] = gout[15 * i + q];
  for (int i = 0; i < nb; ++i) {
    const double *ib = &gout[15 * i + 9], *jb = &gout[15 * i + 12];
    if (ib[0] != 0.0 || ib[1] != 0.0 || ib[2] != 0.0 || jb[0] != 0.0 || jb[1] != 0.0 || jb[2] != 0.0)
      if ((rc = vol_adj(s->U, i, ib, jb))) return rc;
  }
  CKH(zero_wall_faces(g, UB, st));
  sim_status src = SIM_OK;
  std::vector<double> coef(9 * (size_t)nb);
  for (int k = npass - 1; k >= 0; --k) {
    const double *uk = s->REC_U + k * n3, *ppk = s->REC_PP + k * N;
    const double *phik = s->REC_PHI + k * K3, *phipk = s->REC_PHIP + k * K3, *rfk = s->REC_RF + k * K3;
    if (K > 0) CKH(gather3(K, s->PERM, PBN, A0, st));
    // u^{k+1} = u^k + xi tau (-G p' + W Phi'), p += xi p', Phi += xi Phi'
    CKH(div_apply(g, UB, PPB, xi * tau, st));
    CKH(axpby(PPB, PB, N, xi, 1.0, st));
    CKH(interp_face(ker, g, s->nt1, s->nt2, s->nnz, s->NZT, s->TSTART, s->XS, UB, xi * tau, A0, xi, A1, st));
    CKH(interp_dx(ker, g, K, s->XS, UB, phipk, xi * tau, A4, st));
    // Phi' = c^-1 (-W^T G p' - RHS_F)
    CKH(band(true, A1, ic, PPB));
    CKH(scale3(K, A1, -ic, nullptr, 0.0, A2, st));
    // p' = S~^+ b
    if ((rc = project_mean(s, PPB))) return rc;
    sim_solve_stats sst{};
    sim_status r1 = fgmres_any(s, PPB, BB, &sst);
    if (r1 != SIM_OK && r1 != SIM_ENOTCONV) return r1;
    if (r1 == SIM_ENOTCONV) src = r1;
    CKH(interp_grad<double>(ker, g, s->nt1, s->nt2, s->nnz, s->NZT, s->TSTART, s->XS, BB, 1.0, nullptr, 0.0, A3, st));
    CKH(grad_apply(g, BB, F3, 1.0, nullptr, st));
    CKH(interp_dx(ker, g, K, s->XS, F3, phipk, 1.0, A4, st));
    CKH(scale3(K, A1, 1.0, A3, 1.0, A1, st));
    CKH(grad_apply(g, ppk, F3, 1.0, nullptr, st));
    CKH(interp_dx(ker, g, K, s->XS, F3, A1, -ic, A4, st));
    CKH(scale3(K, A3, -ic, A2, 1.0, A2, st));
    // RHS_p = -D u^k / tau, RHS_F = (W^T u^k - U^k) / tau
    CKH(grad_apply(g, BB, UB, 1.0 / tau, UB, st));
    CKH(band(false, A2, 1.0 / tau, UB));
    CKH(zero_wall_faces(g, UB, st));
    CKH(scale3(K, A2, -1.0 / tau, nullptr, 0.0, A3, st));
    CKH(interp_dx(ker, g, K, s->XS, uk, A2, 1.0 / tau, A4, st));
    // U^k = u_s^k + w^k x L~: per-body sums of Ubar; Newton-Euler transposed on the host
    if (K > 0) CKH(scatter3(K, s->PERM, A3, UBN, st));
    if ((rc = body_sums_of(UBN))) return rc;
    for (int i = 0; i < nb; ++i) {
      const HostBody &hb = s->bodies[i];
      const double a = hb.b.radius, theta = hb.b.density_ratio;
      const double Vp = 4.0 / 3.0 * M_PI * a * a * a, Ip = 0.4 * Vp * a * a;
      const double cu = tau / (theta * Vp), cw = tau / (theta * Ip);
      double usb[3], wb[3], Fb[3], Tb[3], Ikb[3], Jkb[3];
      double *o = &gin_b[30 * i];
      for (int q = 0; q < 3; ++q) {
        usb[q] = sums[12 * i + q] + (k == npass - 1 ? gout[15 * i + 3 + q] : 0.0);
        wb[q] = sums[12 * i + 3 + q] + (k == npass - 1 ? gout[15 * i + 6 + q] : 0.0);
        o[6 + q] += 4.0 / 3.0 * usb[q];     // us
        o[9 + q] -= usb[q] / 3.0;           // us_m
        o[12 + q] += 4.0 / 3.0 * wb[q];     // w
        o[15 + q] -= wb[q] / 3.0;           // w_m
        Fb[q] = -cu * usb[q];
        Tb[q] = -cw * wb[q];
        Ikb[q] = cu * 1.5 / dt * usb[q];
        Jkb[q] = cw * 1.5 / dt * wb[q];
        o[18 + q] -= cu * 2.0 / dt * usb[q];  // I_n
        o[21 + q] += cu * 0.5 / dt * usb[q];  // I_m
        o[24 + q] -= cw * 2.0 / dt * wb[q];   // J_n
        o[27 + q] += cw * 0.5 / dt * wb[q];   // J_m
        coef[9 * i + q] = Fb[q];
        coef[9 * i + 3 + q] = Tb[q];
        coef[9 * i + 6 + q] = s->rec_body[6 * ((size_t)k * nb + i) + 3 + q];
      }
      if ((rc = vol_adj(uk, i, Ikb, Jkb))) return rc;
    }
    CKH(zero_wall_faces(g, UB, st));
    if (K > 0) {
      CKH(hipMemcpyAsync(COEF, coef.data(), sizeof(double) * 9 * nb, hipMemcpyHostToDevice, st));
      CKH(scatter3(K, s->PERM, phik, PHN, st));
      CKH(point_adjoint(K, s->BODYOF, s->OFF, s->BODIES, COEF, h3, PHN, UBN, PBN, LBN, st));
      CKH(hipStreamSynchronize(st));  // coef is reused by the next pass
    }
  }
  // predictor: rhs bar = A^-1 u^0 bar
  CKH(fill(RB, n3, 0.0, st));
  sim_solve_stats hst{};
  sim_status hrc = helm_solve_any(s, UB, RB, &hst);
  if (hrc != SIM_OK && hrc != SIM_ENOTCONV) return hrc;
  CKH(interp_dx(ker, g, K, s->XS, RB, s->REC_PHI, 1.0, A4, st));  // Phi^n = Phi^(0)
  if (d_gphi_in && K > 0) {
    CKH(gather3(K, s->PERM, PBN, A0, st));
    CKH(interp_face(ker, g, s->nt1, s->nt2, s->nnz, s->NZT, s->TSTART, s->XS, RB, 1.0, A0, 1.0, A2, st));
    CKH(scatter3(K, s->PERM, A2, d_gphi_in, st));
  }
  if (d_gp_in) {
    CKH(div_apply(g, RB, s->TMPC, 1.0, st));
    CKH(axpby(s->TMPC, PB, N, 1.0, 1.0, st));
    CKH(to_natural(g, 1, s->TMPC, d_gp_in, st));
  }
  if (d_gum_in) {
    CKH(scale_copy(F3, RB, n3, -1.0 / (2.0 * dt), st));
    for (int d = 0; d < 3; ++d) CKH(to_natural(g, 1, F3 + d * N, d_gum_in + d * N, st));
  }
  if (d_gu_in) {
    CKH(convection_adjoint(g, s->UM, RB, F3, st));
    CKH(axpby(F3, RB, n3, 2.0 / dt, -1.0, st));
    CKH(zero_wall_faces(g, F3, st));
    for (int d = 0; d < 3; ++d) CKH(to_natural(g, 1, F3 + d * N, d_gu_in + d * N, st));
  }
  // points: X = X_c^{n+1} + L~ -> sum Xbar per body; rotation cotangent sum L~ x (Lbar + Xbar)
  if (K > 0) {
    CKH(scatter3(K, s->PERM, A4, XBN, st));
    if ((rc = body_sums_of(XBN))) return rc;
    for (int i = 0; i < nb; ++i)
      for (int q = 0; q < 3; ++q) xc1b[3 * i + q] += sums[12 * i + q];
    CKH(axpby(LBN, XBN, 3LL * K, 1.0, 1.0, st));
    if ((rc = body_sums_of(LBN))) return rc;
  } else {
    std::fill(sums.begin(), sums.end(), 0.0);
  }
  for (int i = 0; i < nb; ++i) {
    const double *pre = &s->rec_pre[18 * i];
    const double *w = pre + 12, *wm = pre + 15;
    double *o = &gin_b[30 * i];
    const double phib[3] = {sums[12 * i + 3], sums[12 * i + 4], sums[12 * i + 5]};
    const double wn = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
    if (wn > 0.0) {
      const double wmn = sqrt(wm[0] * wm[0] + wm[1] * wm[1] + wm[2] * wm[2]);
      const double gam = dt * (1.5 * wn - 0.5 * wmn);
      const double e[3] = {w[0] / wn, w[1] / wn, w[2] / wn};
      const double psi[3] = {gam * e[0], gam * e[1], gam * e[2]};
      // J_l(psi) = I + (1 - cos th)/th^2 [psi] + (th - sin th)/th^3 [psi]^2; psib = J_l^T phib
      const double th = fabs(gam);
      double c1, c2;
      if (th < 1e-8) {
        c1 = 0.5;
        c2 = 1.0 / 6.0;
      } else {
        c1 = (1.0 - cos(th)) / (th * th);
        c2 = (th - sin(th)) / (th * th * th);
      }
      // [psi]^T v = -psi x v, ([psi]^2)^T = [psi]^2: psi x (psi x v)
      const double pxv[3] = {psi[1] * phib[2] - psi[2] * phib[1], psi[2] * phib[0] - psi[0] * phib[2],
                             psi[0] * phib[1] - psi[1] * phib[0]};
      const double ppv[3] = {psi[1] * pxv[2] - psi[2] * pxv[1], psi[2] * pxv[0] - psi[0] * pxv[2],
                             psi[0] * pxv[1] - psi[1] * pxv[0]};
      double psib[3];
      for (int q = 0; q < 3; ++q) psib[q] = phib[q] - c1 * pxv[q] + c2 * ppv[q];
      // d psi / d w = 1.5 dt e e^T + gam (I - e e^T) / |w|;  d psi / d w_m = -0.5 dt e e_m^T
      const double ep = e[0] * psib[0] + e[1] * psib[1] + e[2] * psib[2];
      for (int q = 0; q < 3; ++q) o[12 + q] += 1.5 * dt * e[q] * ep + gam / wn * (psib[q] - e[q] * ep);
      if (wmn > 0.0)
        for (int q = 0; q < 3; ++q) o[15 + q] += -0.5 * dt * (wm[q] / wmn) * ep;
    }
    // X_c^{n+1} = (4 X_c^n - X_c^{n-1}) / 3 + tau u_s^n
    for (int q = 0; q < 3; ++q) {
      o[q] += 4.0 / 3.0 * xc1b[3 * i + q];
      o[3 + q] -= xc1b[3 * i + q] / 3.0;
      o[6 + q] += tau * xc1b[3 * i + q];
    }
  }
  if (gbody_in) std::copy(gin_b.begin(), gin_b.end(), gbody_in);
  if ((rc = sync(s))) return rc;
  if (src == SIM_ENOTCONV) return fail(s, SIM_ENOTCONV, "adjoint Schur solve iteration limit reached");
  if (hrc == SIM_ENOTCONV) return fail(s, SIM_ENOTCONV, "adjoint momentum solve iteration limit reached");
  return SIM_OK;
}

sim_status sim_probe_enable(sim_t s, int32_t probe, int32_t on) {
  if (!s) return SIM_EINVAL;
  if (probe < 0 || probe >= PR_COUNT) return fail(s, SIM_EINVAL, "unknown probe");
  probe_enable(s->probes, probe, on != 0);
  return SIM_OK;
}

sim_status sim_probe_read(sim_t s, int32_t probe, int64_t *launches, double *ms, double *bytes, int32_t reset) {
  if (!s || !launches || !ms) return SIM_EINVAL;
  if (probe < 0 || probe >= PR_COUNT) return fail(s, SIM_EINVAL, "unknown probe");
  long long c = 0;
  double t = 0.0, b = 0.0;
  CKH(probe_read(s->probes, probe, &c, &t, &b, reset != 0));
  *launches = c;
  *ms = t;
  if (bytes) *bytes = b;
  return SIM_OK;
}

// w = S_p z = L z + B^T C^-1 B z with the unlumped C = W^T W (the primal
// Schur complement of Sec. 4.1 before the lumping C ~ c I; B = -W^T G,
// B^T = D W).  C^-1 by conjugate gradients on the Lagrangian vectors in
// float64 to a relative residual of 1e-13, started from the lumped guess
// B z / c; each C product is a spread into a cleared face field followed by
// an interpolation.  An operator-level tool (the spectral checks of Sec. 5),
// not part of the time step.
sim_status exact_schur_matvec(sim_t s, const double *z, double *w, int *cg_iters) {
  hipStream_t st = s->st;
  const Geo &g = s->g;
  const long long N = s->N, n3 = 3LL * s->K;
  sim_status rc;
  CKH(lap_apply<double>(g, z, w, st));
  if (cg_iters) *cg_iters = 0;
  if (s->K == 0) return SIM_OK;
  double *q = s->ADJ, *y = q + n3, *r = y + n3, *pv = r + n3, *ap = pv + n3;
  auto dot = [&](const double *a, const double *b, double *out) -> sim_status {
    CKH(dot2(a, b, n3, s->PART, st));
    CKH(finalize(s->PART, red_blocks(), 1, s->RED, st, s->hpin_dev));
    return read_mirror(s, 1, out);
  };
  auto applyC = [&](const double *v, double *out) -> sim_status {
    CKH(fill(s->TMP3, 3 * N, 0.0, st));
    CKH(band_apply(s->ker, false, g, s->nt1, s->nt2, s->nactive, s->ACTIVE, s->TLSTART, s->TLIST, s->XS, v, 1.0,
                   s->TMP3, st));
    CKH(interp_face(s->ker, g, s->nt1, s->nt2, s->nnz, s->NZT, s->TSTART, s->XS, s->TMP3, 1.0, nullptr, 0.0, out,
                    st));
    return SIM_OK;
  };
  // q = B z
  CKH(interp_grad<double>(s->ker, g, s->nt1, s->nt2, s->nnz, s->NZT, s->TSTART, s->XS, z, -1.0, nullptr, 0.0, q, st));
  CKH(scale3(s->K, q, 1.0 / s->c, nullptr, 0.0, y, st));
  if ((rc = applyC(y, ap))) return rc;
  CKH(scale3(s->K, q, 1.0, ap, -1.0, r, st));
  CKH(scale3(s->K, r, 1.0, nullptr, 0.0, pv, st));
  double q2, rr;
  if ((rc = dot(q, q, &q2)) || (rc = dot(r, r, &rr))) return rc;
  if (!isfinite(q2) || !isfinite(rr)) return fail(s, SIM_ENONFINITE, "non-finite Lagrangian vector");
  int it = 0;
  for (; it < 2000 && rr > 1e-26 * q2; ++it) {
    if ((rc = applyC(pv, ap))) return rc;
    double pap;
    if ((rc = dot(pv, ap, &pap))) return rc;
    if (!(pap > 0)) return fail(s, SIM_ENONFINITE, "W^T W is not positive definite on this point set");
    const double alpha = rr / pap;
    CKH(scale3(s->K, y, 1.0, pv, alpha, y, st));
    CKH(scale3(s->K, r, 1.0, ap, -alpha, r, st));
    double rr2;
    if ((rc = dot(r, r, &rr2))) return rc;
    CKH(scale3(s->K, r, 1.0, pv, rr2 / rr, pv, st));
    rr = rr2;
  }
  if (cg_iters) *cg_iters = it;
  if (rr > 1e-26 * q2) return fail(s, SIM_ENOTCONV, "inner conjugate gradients on W^T W did not converge");
  // w += B^T y = D W y
  CKH(band_apply(s->ker, true, g, s->nt1, s->nt2, s->nactive, s->ACTIVE, s->TLSTART, s->TLIST, s->XS, y, 1.0, w, st));
  return SIM_OK;
}

// ---------------------------------------------------------------------------
// Spectrum of the Laplacian-preconditioned Schur operator L^+ S (the theorem
// of Sec. 5 bounds it by [1, 2] for the primal Schur complement; Sec. 6.2
// measures it for S_p and for the lumped S~).  Lanczos on the pencil (S, L)
// in the L inner product over mean-free pressures; each step applies S once
// and solves L w = S v.  An operator-level tool, not part of the time step.

// x = L^+ b for a mean-free cell field b (split layout) by flexible
// preconditioned conjugate gradients (Polak-Ribiere beta, so that the float32
// V-cycle or the bfloat16 fast diagonalisation may serve as preconditioner)
// to ||b - L x|| <= rtol ||b||; x is returned mean-free.  sc: five cell
// fields of scratch.
sim_status lap_solve(sim_t s, const double *b, double *x, double rtol, int maxit, double *const sc[5], int *iters) {
  hipStream_t st = s->st;
  const Geo &g = s->g;
  const long long N = s->N;
  sim_status rc;
  double *r = sc[0], *zo = sc[1], *zn = sc[2], *p = sc[3], *q = sc[4];
  auto dot = [&](const double *a, const double *c, double *out) -> sim_status {
    CKH(dot2(a, c, N, s->PART, st));
    CKH(finalize(s->PART, red_blocks(), 1, s->RED, st, s->hpin_dev));
    return read_mirror(s, 1, out);
  };
  auto precond = [&](const double *in, double *out) -> sim_status {
    if (s->fastdiag) {
      CKH((fd_precond<double, double>(g, in, out, s->FDW1, s->FDW2, s->FDQ, 1.0f, st)));
    } else if (s->fdx) {
      CKH(fdx_precond(g, in, out, s->FDX1, s->FDX2, s->FDXQ, st));
    } else if (s->fp32) {
      if ((rc = vcycle<float, double>(s, in, (float *)s->Z))) return rc;
      CKH(fill(out, N, 0.0, st));
      CKH(add_cast<float>(out, (const float *)s->Z, N, st));
    } else {
      if ((rc = vcycle<double, double>(s, in, (double *)s->Z))) return rc;
      CKH(scale_copy(out, (const double *)s->Z, N, 1.0, st));
    }
    return project_mean(s, out);
  };
  *iters = 0;
  CKH(fill(x, N, 0.0, st));
  double bb;
  if ((rc = dot(b, b, &bb))) return rc;
  if (!isfinite(bb)) return fail(s, SIM_ENONFINITE, "non-finite right-hand side of the Laplacian solve");
  if (bb == 0.0) return SIM_OK;
  // the residual stays mean-free: its constant part (rounding) is outside the
  // range of L and would stall the stopping test
  CKH(scale_copy(r, b, N, 1.0, st));
  if ((rc = project_mean(s, r))) return rc;
  if ((rc = precond(r, zo))) return rc;
  CKH(scale_copy(p, zo, N, 1.0, st));
  double rz, rr = bb;
  if ((rc = dot(r, zo, &rz))) return rc;
  const double stop = rtol * rtol * bb;
  int it = 0;
  while (it < maxit && rr > stop) {
    CKH(lap_apply<double>(g, p, q, st));
    double pq;
    if ((rc = dot(p, q, &pq))) return rc;
    if (!(pq > 0.0) || !(rz > 0.0)) {
      char msg[160];
      snprintf(msg, sizeof msg, "Laplacian solve broke down (iteration %d: p.Lp = %.3e, r.z = %.3e, |b|^2 = %.3e)",
               it, pq, rz, bb);
      return fail(s, SIM_ENONFINITE, msg);
    }
    const double alpha = rz / pq;
    CKH(axpby(x, p, N, alpha, 1.0, st));   // x += alpha p
    CKH(axpby(r, q, N, -alpha, 1.0, st));  // r -= alpha q
    if ((rc = project_mean(s, r))) return rc;
    ++it;
    if ((rc = dot(r, r, &rr))) return rc;
    if (rr <= stop) break;
    if ((rc = precond(r, zn))) return rc;
    double d2[2];
    CKH(dots2(r, zn, zo, N, s->PART, st));
    CKH(finalize(s->PART, red_blocks(), 2, s->RED, st, s->hpin_dev));
    if ((rc = read_mirror(s, 2, d2))) return rc;
    const double beta = (d2[0] - d2[1]) / rz;
    rz = d2[0];
    CKH(axpby(p, zn, N, 1.0, beta, st));  // p = zn + beta p
    std::swap(zo, zn);
  }
  if ((rc = project_mean(s, x))) return rc;
  *iters = it;
  if (!isfinite(rr)) return fail(s, SIM_ENONFINITE, "non-finite residual in the Laplacian solve");
  if (rr > stop) return fail(s, SIM_ENOTCONV, "Laplacian solve did not reach its tolerance");
  return SIM_OK;
}

// Number of eigenvalues below x of the symmetric tridiagonal matrix with
// diagonal a[0..m) and off-diagonal b[1..m) (Sturm sequence of the LDL^T
// pivots).
int sturm_below(const double *a, const double *b, int m, double x) {
  int cnt = 0;
  double q = a[0] - x;
  if (q < 0.0) ++cnt;
  for (int i = 1; i < m; ++i) {
    const double piv = q != 0.0 ? q : 1e-300;
    q = a[i] - x - b[i] * b[i] / piv;
    if (q < 0.0) ++cnt;
  }
  return cnt;
}

// Eigenvalue number idx (0-based, ascending) of the tridiagonal matrix by
// bisection between its Gershgorin bounds.
double tridiag_eig(const double *a, const double *b, int m, int idx) {
  double lo = a[0], hi = a[0];
  for (int i = 0; i < m; ++i) {
    const double r = (i > 0 ? fabs(b[i]) : 0.0) + (i + 1 < m ? fabs(b[i + 1]) : 0.0);
    lo = std::min(lo, a[i] - r);
    hi = std::max(hi, a[i] + r);
  }
  for (int k = 0; k < 200 && hi - lo > 1e-15 * std::max(fabs(lo), fabs(hi)); ++k) {
    const double mid = 0.5 * (lo + hi);
    if (sturm_below(a, b, m, mid) > idx) hi = mid;
    else lo = mid;
  }
  return 0.5 * (lo + hi);
}

sim_status sim_apply(sim_t s, int32_t op, const double *in, const double *in2, double *out) {
  if (!s) return SIM_EINVAL;
  ProbeBind probe_bind_(s->probes);
  s->adj_ready = false;
  s->adj2_ready = false;
  if (!in || !out) return fail(s, SIM_EINVAL, "null argument");
  hipStream_t st = s->st;
  const Geo &g = s->g;
  const long long N = s->N;
  sim_status rc;
  bool need_points = op == SIM_OP_SCHUR || op == SIM_OP_INTERP || op == SIM_OP_SPREAD || op == SIM_OP_SCHUR_RHS ||
                     op == SIM_OP_SCHUR_EXACT;
  if (need_points && !s->have_bodies) return fail(s, SIM_ESTATE, "no bodies set");
  switch (op) {
    case SIM_OP_LAPLACIAN:
      CKH(to_split(g, 1, in, s->TMPC, st));
      CKH(lap_apply<double>(g, s->TMPC, s->PP, st));
      CKH(to_natural(g, 1, s->PP, out, st));
      break;
    case SIM_OP_SCHUR:
      CKH(to_split(g, 1, in, s->TMPC, st));
      if ((rc = schur_matvec<double>(s, s->TMPC, s->PP))) return rc;
      CKH(to_natural(g, 1, s->PP, out, st));
      break;
    case SIM_OP_PRECOND:
      CKH(to_split(g, 1, in, s->TMPC, st));
      if (s->fastdiag) {
        CKH((fd_precond<double, double>(g, s->TMPC, s->PP, s->FDW1, s->FDW2, s->FDQ, 1.0f, st)));
      } else if (s->fdx) {
        CKH(fdx_precond(g, s->TMPC, s->PP, s->FDX1, s->FDX2, s->FDXQ, st));
      } else if (s->fp32) {
        if ((rc = vcycle<float, double>(s, s->TMPC, (float *)s->Z))) return rc;
        CKH(fill(s->PP, N, 0.0, st));
        CKH(add_cast<float>(s->PP, (const float *)s->Z, N, st));
      } else {
        if ((rc = vcycle<double, double>(s, s->TMPC, (double *)s->Z))) return rc;
        CKH(scale_copy(s->PP, (const double *)s->Z, N, 1.0, st));
      }
      CKH(to_natural(g, 1, s->PP, out, st));
      break;
    case SIM_OP_GRAD:
      CKH(to_split(g, 1, in, s->TMPC, st));
      CKH(grad_apply(g, s->TMPC, s->TMP3, 1.0, nullptr, st));
      CKH(to_natural(g, 3, s->TMP3, out, st));
      break;
    case SIM_OP_DIV:
      CKH(to_split(g, 3, in, s->TMP3, st));
      CKH(zero_wall_faces(g, s->TMP3, st));
      CKH(div_apply(g, s->TMP3, s->PP, 1.0, st));
      CKH(to_natural(g, 1, s->PP, out, st));
      break;
    case SIM_OP_INTERP:
      CKH(to_split(g, 3, in, s->TMP3, st));
      CKH(zero_wall_faces(g, s->TMP3, st));
      CKH(interp_face(s->ker, g, s->nt1, s->nt2, s->nnz, s->NZT, s->TSTART, s->XS, s->TMP3, 1.0, nullptr, 0.0, s->Q, st));
      CKH(scatter3(s->K, s->PERM, s->Q, out, st));
      break;
    case SIM_OP_SPREAD:
      CKH(gather3(s->K, s->PERM, in, s->Q, st));
      CKH(fill(s->TMP3, 3 * N, 0.0, st));
      CKH(band_apply(s->ker, false, g, s->nt1, s->nt2, s->nactive, s->ACTIVE, s->TLSTART, s->TLIST, s->XS, s->Q, 1.0,
                     s->TMP3, st));
      CKH(to_natural(g, 3, s->TMP3, out, st));
      break;
    case SIM_OP_HELMHOLTZ:
      CKH(to_split(g, 3, in, s->TMP3, st));
      CKH(zero_wall_faces(g, s->TMP3, st));
      CKH(helm_apply(g, 1.5 / s->cfg.dt, s->cfg.nu, s->TMP3, s->RHSU, st));
      CKH(to_natural(g, 3, s->RHSU, out, st));
      break;
    case SIM_OP_CONVECTION:
      CKH(to_split(g, 3, in, s->TMP3, st));
      CKH(zero_wall_faces(g, s->TMP3, st));
      CKH(convection(g, s->TMP3, s->RHSU, st));
      CKH(to_natural(g, 3, s->RHSU, out, st));
      break;
    case SIM_OP_HELM_SOLVE: {
      CKH(to_split(g, 3, in, s->RHSU, st));
      CKH(zero_wall_faces(g, s->RHSU, st));
      CKH(fill(s->TMP3, 3 * N, 0.0, st));
      sim_status hr = helm_solve_any(s, s->RHSU, s->TMP3, nullptr);
      if (hr != SIM_OK && hr != SIM_ENOTCONV) return hr;
      CKH(to_natural(g, 3, s->TMP3, out, st));
      break;
    }
    case SIM_OP_SCHUR_EXACT:
      CKH(to_split(g, 1, in, s->TMPC, st));
      if ((rc = exact_schur_matvec(s, s->TMPC, s->PP, nullptr))) return rc;
      CKH(to_natural(g, 1, s->PP, out, st));
      break;
    case SIM_OP_SCHUR_RHS:
      if (s->K > 0 && !in2) return fail(s, SIM_EINVAL, "SCHUR_RHS needs rhs_f");
      CKH(to_split(g, 1, in, s->RHSP, st));
      if (s->K > 0) CKH(gather3(s->K, s->PERM, in2, s->RF, st));
      if ((rc = schur_rhs(s))) return rc;
      CKH(to_natural(g, 1, s->BVEC, out, st));
      break;
    default:
      return fail(s, SIM_EINVAL, "unknown operator");
  }
  return sync(s);
}

sim_status sim_schur_spectrum(sim_t s, int32_t exact, const double *v0, int32_t steps, double lap_rtol,
                              double *alpha, double *beta, int32_t *steps_done, double *lmin, double *lmax) {
  if (!s) return SIM_EINVAL;
  ProbeBind probe_bind_(s->probes);
  s->adj_ready = false;
  s->adj2_ready = false;
  if (!v0) return fail(s, SIM_EINVAL, "null start vector");
  if (steps < 1 || steps > 1024) return fail(s, SIM_EINVAL, "steps must be 1..1024");
  if (!(lap_rtol > 0.0 && lap_rtol < 1.0)) return fail(s, SIM_EINVAL, "lap_rtol must lie in (0, 1)");
  if (!s->have_bodies) return fail(s, SIM_ESTATE, "no bodies set");
  hipStream_t st = s->st;
  const Geo &g = s->g;
  const long long N = s->N;
  sim_status rc;
  // scratch: the momentum work fields and the cell work fields (no state)
  double *vp = s->USTAR, *v = s->USTAR + N, *w = s->USTAR + 2 * N, *sv = s->RHSU, *lw = s->RHSU + N;
  double *const sc[5] = {s->RHSU + 2 * N, s->BVEC, s->RHSP, s->TMPC, s->PP};
  auto dot = [&](const double *a, const double *c, double *out) -> sim_status {
    CKH(dot2(a, c, N, s->PART, st));
    CKH(finalize(s->PART, red_blocks(), 1, s->RED, st, s->hpin_dev));
    return read_mirror(s, 1, out);
  };
  std::vector<double> A(steps, 0.0), Bt(steps + 1, 0.0);
  CKH(to_split(g, 1, v0, v, st));
  if ((rc = project_mean(s, v))) return rc;
  CKH(lap_apply<double>(g, v, lw, st));
  double b0;
  if ((rc = dot(v, lw, &b0))) return rc;
  if (!isfinite(b0)) return fail(s, SIM_ENONFINITE, "non-finite start vector");
  if (!(b0 > 0.0)) return fail(s, SIM_EINVAL, "start vector has no mean-free part");
  CKH(scale_inplace(v, N, 1.0 / sqrt(b0), st));
  CKH(fill(vp, N, 0.0, st));
  Bt[0] = sqrt(b0);
  int m = 0;
  double bj = 0.0;
  for (int j = 0; j < steps; ++j) {
    if (exact) {
      int cg;
      if ((rc = exact_schur_matvec(s, v, sv, &cg))) return rc;
    } else if ((rc = schur_matvec<double>(s, v, sv))) {
      return rc;
    }
    double a;
    if ((rc = dot(v, sv, &a))) return rc;
    int its;
    if ((rc = lap_solve(s, sv, w, lap_rtol, 1000, sc, &its))) return rc;
    // w = L^+ S v - a v - b_j v_prev, kept mean-free: the constant mode has
    // zero L-norm, so rounding in it would grow by 1/beta every step
    CKH(lincomb(w, w, 1.0, v, -a, vp, -bj, nullptr, 0, N, nullptr, st));
    if ((rc = project_mean(s, w))) return rc;
    CKH(lap_apply<double>(g, w, lw, st));
    double bn2;
    if ((rc = dot(w, lw, &bn2))) return rc;
    if (!isfinite(a) || !isfinite(bn2)) return fail(s, SIM_ENONFINITE, "non-finite Lanczos coefficient");
    A[j] = a;
    m = j + 1;
    // an invariant subspace has been found: T holds exact eigenvalues
    if (!(bn2 > 1e-28 * a * a)) break;
    bj = sqrt(bn2);
    Bt[j + 1] = bj;
    double *t = vp;
    vp = v;
    v = w;
    w = t;
    CKH(scale_inplace(v, N, 1.0 / bj, st));
  }
  if (alpha) memcpy(alpha, A.data(), sizeof(double) * m);
  if (beta) memcpy(beta, Bt.data(), sizeof(double) * m);
  if (steps_done) *steps_done = m;
  if (lmin) *lmin = tridiag_eig(A.data(), Bt.data(), m, 0);
  if (lmax) *lmax = tridiag_eig(A.data(), Bt.data(), m, m - 1);
  return sync(s);
}

}  // extern "C"
