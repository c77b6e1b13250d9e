// Host driver of the gamblet library: the C ABI declared in gamblet.h.
//
// gbl_build runs the fine-to-coarse sweep of Algorithm 2 (fine stiffness,
// then for k = q..2 the subband operator, the patch systems, the restriction
// and the Galerkin product, then the coarse factor) as kernel launches
// on the caller's stream.  gbl_solve applies the subband solve of
// Section 4.7 / Theorem 4.15 (restriction, independent subband systems,
// coarse system, reconstruction sum) as an approximate inverse inside
// flexible conjugate gradients on the FP64 fine residual.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <atomic>
#include <chrono>
#include <mutex>
#include <thread>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "../../include/gamblet.h"
#include "gamblet_internal.hpp"
#include "solve_internal.hpp"
#include "autotune.hpp"
#include "exact_host.hpp"

using namespace gbl;

namespace {

thread_local std::string g_last_error = "no error";

// Optional per-kernel timing with HIP events recorded on the launch stream
// around every launch of a kernel class (process-wide, off by default).
struct Profiler {
  unsigned mask = 0;
  std::vector<hipEvent_t> pool;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pending[GBL_PROF_NUM_KERNELS];
  double total_ms[GBL_PROF_NUM_KERNELS] = {};
  long launches[GBL_PROF_NUM_KERNELS] = {};
  hipEvent_t get() {
    if (pool.empty()) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      return e;
    }
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
  }
  void drain() {
    for (int k = 0; k < GBL_PROF_NUM_KERNELS; ++k) {
      for (auto& pr : pending[k]) {
        float ms = 0.f;
        if (hipEventSynchronize(pr.second) == hipSuccess && hipEventElapsedTime(&ms, pr.first, pr.second) == hipSuccess) {
          total_ms[k] += ms;
          launches[k] += 1;
        }
        pool.push_back(pr.first);
        pool.push_back(pr.second);
      }
      pending[k].clear();
    }
  }
};
Profiler g_prof;
std::mutex g_prof_mu;

struct ProfScope {
  int k;
  hipStream_t st;
  hipEvent_t a = nullptr, b = nullptr;
  ProfScope(int kernel, hipStream_t s) : k(kernel), st(s) {
    if (!((g_prof.mask >> k) & 1u)) return;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    a = g_prof.get();
    b = g_prof.get();
    if (a) hipEventRecord(a, st);
  }
  ~ProfScope() {
    if (!a || !b) return;
    hipEventRecord(b, st);
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof.pending[k].emplace_back(a, b);
  }
};

size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }

constexpr int kMaxChunk = 8;   // outer iterations launched between two looks at the estimates

struct Layout {
  int q = 0, n = 0, rho = 0, prec = 0, max_rhs = 1;
  int build64 = 0;           // MIXED_FP64_BUILD: the arena is FP64, the solve reads an FP32 copy of it
  size_t selem = 8;          // bytes of the solve-phase scalar (slot, CG and window vectors)
  size_t hier32_off = 0;     // FP32 copy of the arena (build64 only)
  int mass = 0;              // patch radius of the localized mass inverse at level q (0: nodal basis)
  size_t elem = 8;
  LevelGeom lv[kMaxLevels];
  size_t a_off = 0;          // copy of the coefficient (FP64, n^2)
  size_t hier_off = 0;       // hierarchy arena (T)
  size_t hier_elems = 0;
  size_t acell_off = 0;      // element offset of the coefficient in the hierarchy arena (T)
  size_t L1_off = 0;         // 16 doubles
  size_t status_off = 0;     // 4 ints
  size_t gersh_off = 0;      // per-level bound of lambda_max(M B^(k)) (float bits)
  size_t oscal_off = 0;      // outer scalars
  size_t dpart_off = 0;      // dot partials
  size_t opart_off = 0;      // per-block partials of the outer-iteration kernels (2 x 3 x nblk)
  int onblk = 0;             // blocks of the fine-level slot kernels
  size_t dcnt_off = 0;       // dot ticket
  size_t fine_off[5] = {};   // FP64 slot vectors u, r, z, p, w
  size_t lam_off = 0;        // FP64 nodal adjoint state
  size_t g_off[kMaxLevels] = {};     // T slot vectors per level
  size_t gpad_off = 0, gpad_end = 0;  // the region of all slot vectors and their padding
  size_t cgv_off[kMaxLevels] = {};   // T CG vectors per level (5 x 3 np^2)
  size_t cgscal_off = 0;     // doubles
  size_t cgpart_off[kMaxLevels] = {};
  size_t fcg_off = 0;        // finest-level CG vectors (9 x 3 np^2, T)
  size_t fcgpart_off = 0;    // tile partials (2 per tile)
  size_t fcgscal_off = 0;    // kNumFineScalars doubles
  size_t elog_off = 0;       // per-iteration error estimates of the outer iteration (max_outer + 2 doubles)
  size_t tr_off[kMaxLevels] = {};   // FP64 level vectors of the gamblet transform (nk^2 each)
  size_t sel_off = 0;        // selection state of the compression threshold (4 x 64-bit words + histogram)
  size_t lqtab_off = 0;      // 1-D factors of the localized mass inverse ((n - 1) x (2 kMaxRhoQ + 1) doubles)
  size_t bp_off = 0;         // parent-major copy of one level's B^(k) for the matrix-core patch solves (T)
  // window corrections of the preconditioner (levels 3 <= k < q when window_tol > 0)
  int win_cap[kMaxLevels] = {};      // windows the arrays of level k hold: all (nk/2 - 2)^2
  size_t win_list_off[kMaxLevels] = {}, win_idx_off[kMaxLevels] = {};   // int arrays
  size_t win_inv_off[kMaxLevels] = {}, win_y_off[kMaxLevels] = {};      // T arrays
  size_t wcnt_off = 0;       // kept-window counters (kMaxLevels unsigned)
  // Right-hand sides solved together: the per-solve region [solve_off,
  // solve_off + solve_stride) (outer scalars and vectors, slot vectors, subband
  // iteration vectors, scalars, partial sums, tickets, window apply buffers,
  // error log) is repeated M times, solve_stride bytes apart.
  int M = 1;
  size_t solve_off = 0, solve_stride = 0;
  size_t total = 0;
};

constexpr int kMaxBlock = 64;   // right-hand sides per block solve

int validate_opts(const gbl_opts* o, std::string& msg) {
  if (!o) { msg = "opts is NULL"; return GBL_EINVAL; }
  if (o->rho < 1 || o->rho > kMaxRho) { msg = "rho must be in [1, 5]"; return GBL_EINVAL; }
  if (o->precision != GBL_FP64 && o->precision != GBL_MIXED && o->precision != GBL_MIXED_FP64_BUILD) {
    msg = "unknown precision";
    return GBL_EINVAL;
  }
  if (o->precision == GBL_MIXED_FP64_BUILD && o->level_q_mass > 0) {
    msg = "level_q_mass is not available with MIXED_FP64_BUILD";
    return GBL_EINVAL;
  }
  if (!(o->rtol > 0.0) || !(o->rtol < 1.0)) { msg = "rtol must be in (0, 1)"; return GBL_EINVAL; }
  if (o->max_outer < 1 || o->max_outer > 100000) { msg = "max_outer must be in [1, 100000]"; return GBL_EINVAL; }
  if (o->inner_iters < 1 || o->inner_iters > 100000) { msg = "inner_iters must be in [1, 100000]"; return GBL_EINVAL; }
  if (o->inner_iters_coarse < 0 || o->inner_iters_coarse > 100000) {
    msg = "inner_iters_coarse must be in [0, 100000]";
    return GBL_EINVAL;
  }
  if (o->max_rhs < 1 || o->max_rhs > 4096) { msg = "max_rhs must be in [1, 4096]"; return GBL_EINVAL; }
  if (o->level_q_mass < 0 || o->level_q_mass > kMaxRhoQ) { msg = "level_q_mass must be in [0, 4]"; return GBL_EINVAL; }
  if (o->rho_coarse < 0 || o->rho_coarse > kMaxRhoCoarse) { msg = "rho_coarse must be in [0, 4]"; return GBL_EINVAL; }
  if (o->rho > kMaxRhoCoarse && o->rho_coarse == 0) {
    msg = "rho = 5 (the finest transition) needs rho_coarse in [1, 4] for the levels below";
    return GBL_EINVAL;
  }
  if (o->level_q_mass > 0 && o->inner_kind != GBL_INNER_CHEBYSHEV) {
    msg = "level_q_mass needs Chebyshev inner iterations";
    return GBL_EINVAL;
  }
  if (o->inner_kind != GBL_INNER_CHEBYSHEV && o->inner_kind != GBL_INNER_CG && o->inner_kind != GBL_INNER_CHEB_CG) {
    msg = "unknown inner_kind";
    return GBL_EINVAL;
  }
  if (o->exact != 0 && o->exact != 1) { msg = "exact must be 0 or 1"; return GBL_EINVAL; }
  if (o->geometry != 0 && o->geometry != 1) { msg = "geometry must be 0 or 1"; return GBL_EINVAL; }
  if (o->source != 0 && o->source != 1) { msg = "source must be 0 or 1"; return GBL_EINVAL; }
  if (!o->exact && (o->geometry != 0 || o->source != 0)) {
    msg = "geometry 1 and nodal sources need the exact hierarchy (exact = 1)";
    return GBL_EINVAL;
  }
  if (o->exact && o->precision != GBL_FP64) { msg = "the exact hierarchy is FP64"; return GBL_EINVAL; }
  if (o->w_kind != 0 && o->w_kind != 1) { msg = "w_kind must be 0 or 1"; return GBL_EINVAL; }
  if (o->dim != 2 && o->dim != 3) { msg = "dim must be 2 or 3"; return GBL_EINVAL; }
  if (o->dim == 3 && !o->exact) { msg = "dim 3 needs the exact hierarchy (exact = 1)"; return GBL_EINVAL; }
  if (o->autotune != 0 && o->autotune != 1) { msg = "autotune must be 0 or 1"; return GBL_EINVAL; }
  if (o->tensor != 0 && o->tensor != 1) { msg = "tensor must be 0 or 1"; return GBL_EINVAL; }
  if (o->tensor && !o->exact) { msg = "tensor coefficients need the exact hierarchy (exact = 1)"; return GBL_EINVAL; }
  if (o->w_kind == 1 && !o->exact) {
    msg = "w_kind 1 (Construction 4.11) needs the exact hierarchy: the localized kernels use the orthonormal rows";
    return GBL_EINVAL;
  }
  if (!(o->window_tol >= 0.0) || !(o->window_tol < 1e300)) {
    msg = "window_tol must be finite and >= 0";
    return GBL_EINVAL;
  }
  if (o->window_tol > 0.0 && o->inner_kind == GBL_INNER_CHEBYSHEV) {
    msg = "window_tol needs conjugate gradients on the coarser levels (inner_kind CG or CHEB_CG)";
    return GBL_EINVAL;
  }
  if (o->inner_kind != GBL_INNER_CG) {
    if (o->inner_iters > kMaxCheb || (o->inner_kind == GBL_INNER_CHEBYSHEV && o->inner_iters_coarse > kMaxCheb)) {
      msg = "Chebyshev inner iterations must be at most 32";
      return GBL_EINVAL;
    }
    if (!(o->kappa > 1.0) || !(o->kappa_coarse > 1.0) || !(o->kappa < 1e12) || !(o->kappa_coarse < 1e12)) {
      msg = "kappa and kappa_coarse must be in (1, 1e12)";
      return GBL_EINVAL;
    }
  }
  return GBL_OK;
}

int make_layout(int q, const gbl_opts* o, Layout& L, std::string& msg) {
  if (q < 2 || q > 12) { msg = "q must be in [2, 12]"; return GBL_EINVAL; }
  int st = validate_opts(o, msg);
  if (st) return st;
  L.q = q;
  L.n = 1 << q;
  L.rho = o->rho;
  L.prec = o->precision;
  L.max_rhs = o->max_rhs;
  L.elem = (o->precision == GBL_MIXED) ? 4 : 8;
  L.selem = (o->precision == GBL_FP64) ? 8 : 4;
  L.build64 = (o->precision == GBL_MIXED_FP64_BUILD) ? 1 : 0;
  // stencil widths: A^(q) is the 9-point Q1 stencil; a restriction row of
  // level k-1 spans 2(2 rho_k + 1) level-k slots, so A^(k-1) = R A R^T
  // couples coarse slots up to (4 rho_k + 1 + s_k) / 2 apart.
  for (int k = 1; k <= q; ++k) {
    L.lv[k].k = k;
    L.lv[k].nk = 1 << k;
  }
  L.lv[q].s = std::min(1, L.lv[q].nk - 1);
  if (o->level_q_mass > 0) {
    // A^(q) = Minv^T A Minv couples nodes up to 2 rho_q + 1 steps apart
    const int S = 2 * o->level_q_mass + 1;
    if (L.n - 1 < S) { msg = "level_q_mass needs 2^q - 1 >= 2 level_q_mass + 1"; return GBL_EINVAL; }
    L.lv[q].s = S;
    L.mass = o->level_q_mass;
  }
  for (int k = q; k >= 2; --k) {
    LevelGeom& g = L.lv[k];
    const int nc = g.nk / 2;
    g.rho = std::min((k == q || o->rho_coarse == 0) ? o->rho : o->rho_coarse, nc - 1);
    g.rw = 2 * (2 * g.rho + 1);
    g.t = std::min((g.s + 1) / 2, nc - 1);
    L.lv[k - 1].s = std::min((4 * g.rho + 1 + g.s) / 2, nc - 1);
  }
  size_t e = 0;
  for (int k = 1; k <= q; ++k) {
    LevelGeom& g = L.lv[k];
    const size_t nk2 = (size_t)g.nk * g.nk;
    const size_t S = 2 * g.s + 1;
    g.nA = S * S * nk2;
    g.offA = e;
    e += align_up(g.nA, 64);
    if (k >= 2) {
      const size_t np2 = nk2 / 4;
      const size_t TT = 2 * g.t + 1;
      g.nB = TT * TT * 9 * ((np2 + 63) / 64 * 64);   // block-interleaved, 64 parents per group
      g.offB = e;
      e += align_up(g.nB, 64);
      g.nR = (size_t)g.rw * g.rw * np2;
      g.offR = e;
      e += align_up(g.nR, 64);
      g.nBJ = 9 * np2;
      g.offBJ = e;
      e += align_up(g.nBJ, 64);
    }
  }
  L.acell_off = e;
  e += align_up((size_t)L.n * L.n, 64);
  L.hier_elems = e;
  const size_t n2 = (size_t)L.n * L.n;
  size_t b = 0;
  L.a_off = b; b = align_up(b + n2 * 8);
  L.hier_off = b; b = align_up(b + e * L.elem);
  if (L.build64) { L.hier32_off = b; b = align_up(b + e * 4); }
  L.L1_off = b; b = align_up(b + 16 * 8);
  L.status_off = b; b = align_up(b + 4 * sizeof(int));
  L.gersh_off = b; b = align_up(b + kMaxLevels * sizeof(unsigned));
  // ---- per-solve region (repeated M times)
  L.M = (o->level_q_mass > 0) ? 1 : std::min(o->max_rhs, kMaxBlock);
  L.solve_off = b;
  L.oscal_off = b; b = align_up(b + kNumOuterScalars * 8);
  L.dpart_off = b; b = align_up(b + 3 * kDotBlocks * 8);
  L.dcnt_off = b; b = align_up(b + 4 * sizeof(unsigned));
  L.onblk = (int)((n2 + 255) / 256);
  L.opart_off = b; b = align_up(b + 6 * (size_t)L.onblk * 8);
  for (int i = 0; i < 5; ++i) { L.fine_off[i] = b; b = align_up(b + n2 * 8); }
  L.lam_off = b; b = align_up(b + (size_t)(L.n + 1) * (L.n + 1) * 8);
  // slot vectors with kGPad zero words on each side: the restriction reads up
  // to 2 rho words beyond either end (where R is zero)
  L.gpad_off = b;
  for (int k = 1; k <= q; ++k) {
    L.g_off[k] = b + kGPad * L.selem;
    b = align_up(b + ((size_t)L.lv[k].nk * L.lv[k].nk + 2 * kGPad) * L.selem);
  }
  L.gpad_end = b;
  {
    const size_t np2 = (size_t)L.lv[q].nk * L.lv[q].nk / 4;
    L.fcg_off = b;
    b = align_up(b + 9 * 3 * np2 * L.selem);
    L.fcgpart_off = b;
    b = align_up(b + 2 * std::max<size_t>(1, np2 / 256 + 1) * 8);
  }
  for (int k = 2; k <= q; ++k) {
    const size_t np2 = (size_t)L.lv[k].nk * L.lv[k].nk / 4;
    L.cgv_off[k] = b;
    b = align_up(b + 5 * 3 * np2 * L.selem);
    const size_t nb = std::max((np2 + 255) / 256, (np2 + 63) / 64);
    L.cgpart_off[k] = b;
    b = align_up(b + nb * 8);
  }
  if (o->window_tol > 0.0) {
    for (int k = 3; k < q; ++k) {
      const size_t np = (size_t)L.lv[k].nk / 2;
      L.win_cap[k] = (int)((np - 2) * (np - 2));
      L.win_y_off[k] = b; b = align_up(b + (size_t)L.win_cap[k] * 27 * L.selem);
    }
  }
  L.cgscal_off = b; b = align_up(b + (size_t)kMaxLevels * kNumCGScalars * 8);
  L.fcgscal_off = b; b = align_up(b + kNumFineScalars * 8);
  L.elog_off = b; b = align_up(b + ((size_t)o->max_outer + 2) * 8);
  L.solve_stride = align_up(b - L.solve_off);
  b = L.solve_off + (size_t)L.M * L.solve_stride;
  // ---- shared again
  if (o->window_tol > 0.0) {
    for (int k = 3; k < q; ++k) {
      const size_t np = (size_t)L.lv[k].nk / 2;
      const size_t cap = (size_t)L.win_cap[k];
      L.win_list_off[k] = b; b = align_up(b + cap * sizeof(int));
      L.win_idx_off[k] = b; b = align_up(b + np * np * sizeof(int));
      L.win_inv_off[k] = b; b = align_up(b + cap * 27 * 27 * L.selem);
    }
  }
  // everything from here on is zeroed at the start of a build
  L.wcnt_off = b; b = align_up(b + (size_t)kMaxLevels * sizeof(unsigned));
  for (int k = 1; k <= q; ++k) {
    L.tr_off[k] = b;
    b = align_up(b + (size_t)L.lv[k].nk * L.lv[k].nk * 8);
  }
  L.sel_off = b;
  b = align_up(b + 4 * 8 + (size_t)kSelHistBins * 4);
  L.lqtab_off = b;
  b = align_up(b + (size_t)(L.n - 1) * (2 * kMaxRhoQ + 1) * 8);
  {
    size_t most = 0;
    for (int k = 2; k <= q; ++k) {
      const size_t TT = 2 * L.lv[k].t + 1;
      most = std::max(most, TT * TT * 9 * ((size_t)L.lv[k].nk * L.lv[k].nk / 4));
    }
    L.bp_off = b;
    b = align_up(b + most * L.elem);
  }
  L.total = b;
  return GBL_OK;
}

}  // namespace

struct gbl_ctx {
  Layout L;
  gbl_opts opts;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  std::string err = "no error";
  double* host = nullptr;   // pinned host mirror: outer scalars, then the status word
  CGArgs<float> cgf;     // coarser subband levels (k < q)
  CGArgs<double> cgd;
  FineCG<float> fcgf;    // finest subband level
  FineCG<double> fcgd;
  CGArgs<float> cgqf;    // finest level with a stored B^(q) (level-q gamblets from the mass inverse)
  CGArgs<double> cgqd;
  hipStream_t side = nullptr;           // second stream: coarser subband CG runs beside the finest
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  int device = -1;                      // device whose streams and events these are
  // One outer iteration recorded as a graph (captured on its own stream, so
  // that the caller may pass the null stream) and replayed per iteration.
  hipStream_t cap = nullptr;
  hipGraphExec_t iter_graph = nullptr;
  int iter_graph_m = 0;                 // right-hand sides of the recorded iteration
  bool graph_off = false;               // capture failed once: launch kernel by kernel
  unsigned build_flags = 0;             // GBL_FLAG_* of the build
  float lmax[kMaxLevels] = {};          // bound of lambda_max(M B^(k)) per level
  ChebCoef cheb_fine{};                 // Chebyshev coefficients, finest level
  ChebStep cheb_coarse[kMaxCheb]{};     // Chebyshev coefficients per step, coarser levels
  ChebStep cheb_q[kMaxCheb]{};          // the same for the stored finest level (slot 0)
  bool diverged = false;                // the last solve produced a non-finite estimate or residual
  int nwin[kMaxLevels] = {};            // kept windows of the preconditioner per level
  ExactHier* ex = nullptr;              // the exact (dense) hierarchy when opts.exact
  int tuned[kMaxLevels][2] = {};        // autotuned variants of the level's patch and Galerkin kernels

  // The arena in the scalar T: the build's own (FP64 or FP32), or with
  // MIXED_FP64_BUILD the FP32 copy the solve reads.
  template <typename T>
  T* hier(size_t off) const {
    const size_t base = (sizeof(T) == L.elem) ? L.hier_off : L.hier32_off;
    return reinterpret_cast<T*>(ws + base) + off;
  }
  double* fine(int i) const { return reinterpret_cast<double*>(ws + L.fine_off[i]); }
  int* status() const { return reinterpret_cast<int*>(ws + L.status_off); }
  double* oscal() const { return reinterpret_cast<double*>(ws + L.oscal_off); }
  double* lqtab() const { return reinterpret_cast<double*>(ws + L.lqtab_off); }
  const double* a() const { return reinterpret_cast<const double*>(ws + L.a_off); }
  double* L1() const { return reinterpret_cast<double*>(ws + L.L1_off); }
};

namespace {

int fail(gbl_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg; else g_last_error = msg;
  return code;
}

#define HIPCHK(ctx, call)                                                                   \
  do {                                                                                      \
    hipError_t e_ = (call);                                                                 \
    if (e_ != hipSuccess) return fail((ctx), GBL_EHIP, std::string(#call ": ") + hipGetErrorString(e_)); \
  } while (0)

// The streams, events and pinned host words of a context.  Creating and
// destroying them costs several hundred microseconds of host time, so a
// freed context leaves them, per device, for the next one.
struct CtxResources {
  int device = -1;
  hipStream_t side = nullptr, cap = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  double* host = nullptr;
};
// Pinned host words: outer scalars of every right-hand side of a block, the
// status word, the build's bounds and window counts, then the error
// estimates of a chunk of iterations for every right-hand side.
constexpr size_t kHostStatus = (size_t)kMaxBlock * kNumOuterScalars;
constexpr size_t kHostBits = kHostStatus + 4;
constexpr size_t kHostLog = kHostBits + kMaxLevels;
constexpr size_t kHostWords = kHostLog + (size_t)kMaxBlock * kMaxChunk;
constexpr size_t kMaxPooledResources = 64;
std::mutex g_res_mu;
std::vector<CtxResources> g_res_pool;

void destroy_resources(CtxResources& r) {
  if (r.side) hipStreamDestroy(r.side);
  if (r.cap) hipStreamDestroy(r.cap);
  if (r.ev_fork) hipEventDestroy(r.ev_fork);
  if (r.ev_join) hipEventDestroy(r.ev_join);
  if (r.host) hipHostFree(r.host);
  r = CtxResources{};
}

bool acquire_resources(CtxResources& r) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return false;
  {
    std::lock_guard<std::mutex> lk(g_res_mu);
    for (size_t i = 0; i < g_res_pool.size(); ++i) {
      if (g_res_pool[i].device == dev) {
        r = g_res_pool[i];
        g_res_pool[i] = g_res_pool.back();
        g_res_pool.pop_back();
        return true;
      }
    }
  }
  r.device = dev;
  if (hipHostMalloc(reinterpret_cast<void**>(&r.host), kHostWords * sizeof(double), hipHostMallocDefault) !=
          hipSuccess ||
      hipStreamCreateWithFlags(&r.side, hipStreamNonBlocking) != hipSuccess ||
      hipStreamCreateWithFlags(&r.cap, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&r.ev_fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&r.ev_join, hipEventDisableTiming) != hipSuccess) {
    destroy_resources(r);
    return false;
  }
  return true;
}

void release(gbl_ctx* c) {
  // no work of this context may still run on the second stream
  if (c->side) hipStreamSynchronize(c->side);
  if (c->iter_graph) hipGraphExecDestroy(c->iter_graph);
  CtxResources r;
  r.device = c->device;
  r.side = c->side;
  r.cap = c->cap;
  r.ev_fork = c->ev_fork;
  r.ev_join = c->ev_join;
  r.host = c->host;
  if (r.side && r.cap && r.ev_fork && r.ev_join && r.host) {
    std::lock_guard<std::mutex> lk(g_res_mu);
    if (g_res_pool.size() < kMaxPooledResources) {
      g_res_pool.push_back(r);
      r = CtxResources{};
    }
  }
  destroy_resources(r);
  delete c->ex;
  delete c;
}

template <typename T>
CGArgs<T> make_cg_args(gbl_ctx* c) {
  const Layout& L = c->L;
  CGArgs<T> A{};
  int blk = 0, blks = 0, l = 0;
  for (int k = L.q - 1; k >= 2; --k, ++l) {
    const LevelGeom& g = L.lv[k];
    const size_t np2 = (size_t)g.nk * g.nk / 4;
    CGLev<T>& v = A.lv[l];
    v.B = c->hier<T>(g.offB);
    v.BJ = c->hier<T>(g.offBJ);
    v.g = reinterpret_cast<const T*>(c->ws + L.g_off[k]);
    T* base = reinterpret_cast<T*>(c->ws + L.cgv_off[k]);
    v.x = base;
    v.r = base + 3 * np2;
    v.z = base + 6 * np2;
    v.p = base + 9 * np2;
    v.q = base + 12 * np2;
    v.scal = reinterpret_cast<double*>(c->ws + L.cgscal_off) + l * kNumCGScalars;
    v.part = reinterpret_cast<double*>(c->ws + L.cgpart_off[k]);
    v.np = g.nk / 2;
    v.t = g.t;
    v.fine = (k == L.q) ? 1 : 0;
    v.iters = (k == L.q) ? c->opts.inner_iters : c->opts.inner_iters_coarse;
    v.blk0 = blk;
    v.nblk = (int)((np2 + 255) / 256);
    blk += v.nblk;
    v.blk0s = blks;
    v.nblks = (int)((np2 + 63) / 64);
    blks += v.nblks;
    if (L.win_cap[k] > 0) {
      v.wlist = reinterpret_cast<const int*>(c->ws + L.win_list_off[k]);
      v.widx = reinterpret_cast<const int*>(c->ws + L.win_idx_off[k]);
      v.winv = reinterpret_cast<const T*>(c->ws + L.win_inv_off[k]);
      v.Y = reinterpret_cast<T*>(c->ws + L.win_y_off[k]);
    }
    v.nwin = 0;   // set from the build's counts (set_windows)
    v.win0 = 0;
  }
  A.nlev = l;
  return A;
}

// The kept-window counts of the build into the CG arguments of the coarser levels.
template <typename T>
void set_windows(const gbl_ctx* c, CGArgs<T>& A) {
  int w0 = 0;
  for (int l = 0; l < A.nlev; ++l) {
    const int k = c->L.q - 1 - l;
    A.lv[l].nwin = c->nwin[k];
    A.lv[l].win0 = w0;
    w0 += c->nwin[k];
  }
}

// The finest subband system as a one-level CGArgs over its stored B^(q), for
// hierarchies whose level-q gamblets come from the localized mass inverse
// (their A^(q) is not the nine-point stencil the matrix-free kernels rebuild).
template <typename T>
CGArgs<T> make_cgq_args(gbl_ctx* c) {
  const Layout& L = c->L;
  const int k = L.q;
  const LevelGeom& g = L.lv[k];
  const size_t np2 = (size_t)g.nk * g.nk / 4;
  CGArgs<T> A{};
  CGLev<T>& v = A.lv[0];
  v.B = c->hier<T>(g.offB);
  v.BJ = c->hier<T>(g.offBJ);
  v.g = reinterpret_cast<const T*>(c->ws + L.g_off[k]);
  T* base = reinterpret_cast<T*>(c->ws + L.cgv_off[k]);
  v.x = base;
  v.r = base + 3 * np2;
  v.z = base + 6 * np2;
  v.p = base + 9 * np2;
  v.q = base + 12 * np2;
  // Chebyshev steps use no inner products; the scalar slot is level q - 1's
  v.scal = reinterpret_cast<double*>(c->ws + L.cgscal_off);
  v.part = reinterpret_cast<double*>(c->ws + L.cgpart_off[k]);
  v.np = g.nk / 2;
  v.t = g.t;
  v.fine = 1;
  v.iters = c->opts.inner_iters;
  v.blk0 = 0;
  v.nblk = (int)((np2 + 255) / 256);
  v.blk0s = 0;
  v.nblks = (int)((np2 + 63) / 64);
  A.nlev = 1;
  return A;
}

template <typename T>
FineCG<T> make_fine_cg(gbl_ctx* c) {
  const Layout& L = c->L;
  const LevelGeom& g = L.lv[L.q];
  const size_t np2 = (size_t)g.nk * g.nk / 4;
  FineCG<T> F{};
  F.g = reinterpret_cast<const T*>(c->ws + L.g_off[L.q]);
  F.acell = c->hier<T>(L.acell_off);
  F.BJ = c->hier<T>(g.offBJ);
  T* base = reinterpret_cast<T*>(c->ws + L.fcg_off);
  F.x = base;
  F.u = base + 3 * np2;
  F.p = base + 6 * np2;
  F.r[0] = base + 9 * np2;
  F.r[1] = base + 12 * np2;
  F.w[0] = base + 15 * np2;
  F.w[1] = base + 18 * np2;
  F.s[0] = base + 21 * np2;
  F.s[1] = base + 24 * np2;
  F.scal = reinterpret_cast<double*>(c->ws + L.fcgscal_off);
  F.part = reinterpret_cast<double*>(c->ws + L.fcgpart_off);
  F.np = g.nk / 2;
  const int tp = std::min(16, F.np);
  F.nblk = (F.np / tp) * (F.np / tp);
  return F;
}

// Chebyshev coefficients (recurrence documented with ChebCoef) for the
// interval [G / kappa, G].  A small margin on G covers the FP32 rounding of
// the bound itself.
void cheb_coefs(double G, double kappa, int K, float& c0, float* ca, float* cb) {
  const double lmax = (G > 0.0 && std::isfinite(G)) ? 1.001 * G : 1.0;
  const double lmin = lmax / kappa;
  const double theta = 0.5 * (lmax + lmin), delta = 0.5 * (lmax - lmin), sigma = theta / delta;
  double rho_prev = 1.0 / sigma;
  c0 = (float)(1.0 / theta);
  ca[0] = cb[0] = 0.0f;
  for (int k = 1; k < K && k < kMaxCheb; ++k) {
    const double rho = 1.0 / (2.0 * sigma - rho_prev);
    ca[k] = (float)(rho * rho_prev);
    cb[k] = (float)(2.0 * rho / delta);
    rho_prev = rho;
  }
}

void make_cheb_tables(gbl_ctx* c) {
  const Layout& L = c->L;
  ChebCoef& f = c->cheb_fine;
  cheb_coefs(c->lmax[L.q], c->opts.kappa, c->opts.inner_iters, f.c0, f.ca, f.cb);
  for (int step = 0; step < kMaxCheb; ++step) {
    c->cheb_q[step].c0[0] = f.c0;
    c->cheb_q[step].ca[0] = f.ca[step];
    c->cheb_q[step].cb[0] = f.cb[step];
  }
  // coarser levels: slot l of the CG arguments is level q - 1 - l
  for (int l = 0; l + 2 <= L.q - 1 && l < kMaxLevels; ++l) {
    const int k = L.q - 1 - l;
    ChebCoef t{};
    cheb_coefs(c->lmax[k], c->opts.kappa_coarse, c->opts.inner_iters_coarse, t.c0, t.ca, t.cb);
    for (int step = 0; step < kMaxCheb; ++step) {
      c->cheb_coarse[step].c0[l] = t.c0;
      c->cheb_coarse[step].ca[l] = t.ca[step];
      c->cheb_coarse[step].cb[l] = t.cb[step];
    }
  }
}

// The variant of a build step to launch: kVariantDefault without autotuning;
// with it, the recorded choice for this device, precision and level shape,
// or (first time) the faster of the applicable candidates, each launched once
// to warm up and twice under events on the build stream.  Every candidate
// rewrites the same outputs from the same inputs, and the chosen one runs
// again afterwards, so the build's result is the chosen kernel's; the status
// word is restored around the trials.
template <typename T, typename Launch, typename Ok>
int tuned_variant(gbl_ctx* c, const std::string& key, Ok ok, Launch launch, hipStream_t st) {
  if (!c->opts.autotune) return kVariantDefault;
  const std::string path = c->opts.autotune_path ? c->opts.autotune_path : "";
  const std::string full = tune_device_name() + (sizeof(T) == 8 ? ":f64:" : ":f32:") + key;
  const int known = tune_lookup(path, full);
  if (known >= 0 && ok(known)) return known;
  double us[2] = {-1.0, -1.0};
  int best = -1;
  int saved = 0;
  if (hipMemcpyAsync(&saved, c->status(), sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return kVariantDefault;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) hipEventDestroy(e0);
    return kVariantDefault;
  }
  for (int v = 0; v < 2; ++v) {
    if (!ok(v)) continue;
    launch(v);
    hipEventRecord(e0, st);
    launch(v);
    launch(v);
    hipEventRecord(e1, st);
    float ms = 0.f;
    if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) continue;
    us[v] = 500.0 * ms;   // per launch
    if (best < 0 || us[v] < us[best]) best = v;
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  (void)hipGetLastError();
  if (hipMemcpyAsync(c->status(), &saved, sizeof(int), hipMemcpyHostToDevice, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return kVariantDefault;
  if (best < 0) return kVariantDefault;
  tune_store(path, full, best, us, 2);
  return best;
}

template <typename T>
int build_impl(gbl_ctx* c, hipStream_t st) {
  const Layout& L = c->L;
  const int q = L.q;
  {
    ProfScope ps(GBL_PROF_ASSEMBLE, st);
    if (L.mass > 0) {
      // level-q gamblets from the localized mass inverse (Algorithm 2;
      // Definition 5.2): A^(q) = Minv^T A Minv on the empty-slot grid
      launch_mass_inverse_table(L.n, L.mass, c->lqtab(), st);
      launch_zero<T>(L.lv[q].nA, c->hier<T>(L.lv[q].offA), st);
      launch_level_q_operator_arena<T>(L.n, L.mass, c->a(), c->lqtab(), c->hier<T>(L.lv[q].offA), c->status(), st);
    } else {
      launch_assemble_fine<T>(c->a(), c->hier<T>(L.lv[q].offA), L.n, c->status(), st);
    }
    launch_convert<T, double>((size_t)L.n * L.n, c->a(), c->hier<T>(L.acell_off), st);
  }
  for (int k = q; k >= 2; --k) {
    const LevelGeom& g = L.lv[k];
    const bool fine = (k == q);
    {
      ProfScope ps(GBL_PROF_SUBBAND_OPERATOR, st);
      launch_subband_operator<T>(g, c->hier<T>(g.offA), c->hier<T>(g.offB), c->hier<T>(g.offBJ), fine, st);
      // scratch: the level's subband solve vectors, unused while building
      T* scratch = reinterpret_cast<T*>(c->ws + (k == q ? L.fcg_off : L.cgv_off[k]));
      launch_gershgorin<T>(g, c->hier<T>(g.offB), scratch, reinterpret_cast<unsigned*>(c->ws + L.gersh_off) + k, st);
      if (L.win_cap[k] > 0 && sizeof(T) == L.selem)
        launch_win_build<T>(g, c->hier<T>(g.offB), c->opts.window_tol, L.win_cap[k],
                            reinterpret_cast<int*>(c->ws + L.win_list_off[k]),
                            reinterpret_cast<int*>(c->ws + L.win_idx_off[k]),
                            reinterpret_cast<T*>(c->ws + L.win_inv_off[k]),
                            reinterpret_cast<unsigned*>(c->ws + L.wcnt_off) + k, c->status(), st);
    }
    {
      const int cls = patch_class(g, fine);
      auto patch = [&](int v) {
        launch_patch_solve<T>(g, c->hier<T>(g.offA), c->hier<T>(g.offB), c->hier<T>(g.offR),
                              reinterpret_cast<T*>(c->ws + L.bp_off), fine, c->status(), st, v);
      };
      char key[160];
      std::snprintf(key, sizeof key, "%s:nk%d:rho%d:s%d:t%d:fine%d:mass%d", cls == kKernelBand ? "band" : "patch",
                    g.nk, g.rho, g.s, g.t, fine ? 1 : 0, L.mass);
      const int pv = tuned_variant<T>(c, key, [&](int v) { return patch_variant_ok<T>(g, fine, v); }, patch, st);
      if (c->opts.autotune) c->tuned[k][0] = pv;
      ProfScope ps(cls == kKernelBand ? GBL_PROF_PATCH_BAND : GBL_PROF_PATCH_SOLVE, st);
      patch(pv);
    }
    {
      const LevelGeom& gc = L.lv[k - 1];
      auto galerkin = [&](int v) {
        launch_galerkin<T>(g, gc, c->hier<T>(g.offA), c->hier<T>(g.offR), c->hier<T>(gc.offA), st, v);
      };
      char key[160];
      std::snprintf(key, sizeof key, "galerkin:nk%d:rho%d:s%d:sc%d", g.nk, g.rho, g.s, gc.s);
      const int gv =
          tuned_variant<T>(c, key, [&](int v) { return galerkin_variant_ok<T>(g, gc, v); }, galerkin, st);
      if (c->opts.autotune) c->tuned[k][1] = gv;
      ProfScope ps(GBL_PROF_GALERKIN, st);
      galerkin(gv);
    }
  }
  launch_coarse_factor<T>(c->hier<T>(L.lv[1].offA), L.lv[1].s, c->L1(), c->status(), st);
  HIPCHK(c, hipGetLastError());
  return GBL_OK;
}

// z = S r: the subband solve of the localized hierarchy applied to the fine
// residual r (FP64 slot vectors); inner arithmetic in T.  The finest subband
// system runs on the caller's stream while the coarser ones run beside it on
// a second stream (the subband systems are independent, Section 4.7).
template <typename T>
const FineCG<T>& fcg_of(const gbl_ctx* c);
template <typename T>
const CGArgs<T>& cgq_of(const gbl_ctx* c);

// r_converted: g^(q) already holds T(r).  When dots is set, the finest
// prolongation also forms (z, z), (u, u), (z, w) into dots[0..3).
template <typename T>
void precondition(gbl_ctx* c, const CGArgs<T>& cg, const double* r, double* z, hipStream_t st,
                  bool r_converted = false, const double* uo = nullptr, const double* wo = nullptr,
                  double* dots = nullptr, Zb zb = Zb()) {
  const Layout& L = c->L;
  const int q = L.q;
  const size_t n2 = (size_t)L.n * L.n;
  T* g[kMaxLevels];
  for (int k = 1; k <= q; ++k) g[k] = reinterpret_cast<T*>(c->ws + L.g_off[k]);
  const FineCG<T>& F = fcg_of<T>(c);
  // levels 2..kc (at most 16 x 16 slots, never the finest) run in one workgroup
  const int kc = std::min(q - 1, 4);
  ChainArgs<T> chain{};
  chain.n = std::max(0, kc - 1);
  chain.g1 = g[1];
  for (int k = 2; k <= kc; ++k) {
    ChainLevel<T>& cl = chain.lv[k - 2];
    cl.R = c->hier<T>(L.lv[k].offR);
    cl.gf = g[k];
    cl.gc = g[k - 1];
    cl.w = cg.lv[q - 1 - k].x;
    cl.nk = L.lv[k].nk;
    cl.rho = L.lv[k].rho;
    cl.fine = 0;
  }
  if (L.mass > 0)
    launch_mass_load_slots<T>(L.n, L.mass, c->lqtab(), r, g[q], st);   // g^(q) = Minv^T r
  else if (!r_converted)
    launch_convert<T, double>(n2, r, g[q], st, zb);
  // The subband systems are independent (Section 4.7), so they run beside each
  // other: the finest one on the caller's stream (it needs only g^(q)), and
  // the restriction chain, the coarser systems and the prolongation down to
  // level q - 1 on the second stream.
  hipStream_t cs = c->side ? c->side : st;
  const bool cheb = c->opts.inner_kind != GBL_INNER_CG;                // finest level
  const bool cheb_coarse = c->opts.inner_kind == GBL_INNER_CHEBYSHEV;  // coarser levels
  const bool coarse = cg.nlev > 0 && c->opts.inner_iters_coarse > 0;
  bool windows = false;
  for (int l = 0; l < cg.nlev; ++l) windows = windows || cg.lv[l].nwin > 0;
  if (c->side) {
    hipEventRecord(c->ev_fork, st);
    hipStreamWaitEvent(cs, c->ev_fork, 0);
  }
  const int K = c->opts.inner_iters_coarse;
  for (int k = q; k > kc; --k) {
    ProfScope ps(GBL_PROF_RESTRICT, cs);
    launch_restrict<T>(L.lv[k], c->hier<T>(L.lv[k].offR), g[k], g[k - 1], cs, zb);
  }
  {
    ProfScope ps(GBL_PROF_RESTRICT, cs);
    launch_restrict_chain<T>(chain, cs, zb);
  }
  if (coarse) {
    if (cheb_coarse) {
      {
        ProfScope ps(GBL_PROF_CG_INIT, cs);
        launch_cheb_init<T>(cg, c->cheb_coarse[0], 0, cg.nlev, cs, zb);
      }
      for (int j = 1; j < K; ++j) {
        ProfScope ps(GBL_PROF_CG_SPMV, cs);
        launch_cheb_step<T>(cg, c->cheb_coarse[j], j, 0, cg.nlev, cs, zb);
      }
    } else {
      const CGLev<T>& last = cg.lv[cg.nlev - 1];
      {
        ProfScope ps(GBL_PROF_CG_INIT, cs);
        launch_cg_init<T>(cg, last.blk0 + last.nblk, cs, zb);
        if (windows) launch_win_correct<T>(cg, 0, true, cs, zb);
      }
      for (int it = 0; it < K; ++it) {
        {
          ProfScope ps(GBL_PROF_CG_SPMV, cs);
          launch_cg_spmv<T>(cg, last.blk0s + last.nblks, it, cs, zb);
        }
        ProfScope ps(GBL_PROF_CG_UPDATE, cs);
        launch_cg_update<T>(cg, last.blk0 + last.nblk, it, cs, zb);
        if (windows && it + 1 < K) launch_win_correct<T>(cg, it, false, cs, zb);
      }
    }
  } else {
    for (int l = 0; l < cg.nlev; ++l) launch_zero<T>(3 * (size_t)cg.lv[l].np * cg.lv[l].np, cg.lv[l].x, cs, zb);
  }
  {
    ProfScope ps(GBL_PROF_PROLONG, cs);
    launch_prolong_chain<T>(chain, c->L1(), cs, zb);
  }
  for (int k = kc + 1; k < q; ++k) {
    ProfScope ps(GBL_PROF_PROLONG, cs);
    launch_prolong<T>(L.lv[k], c->hier<T>(L.lv[k].offR), g[k - 1], cg.lv[q - 1 - k].x, g[k], false, cs, zb);
  }
  // finest level (enqueued after the coarser chain, the longer of the two
  // branches, so that a replayed graph starts that chain first): Chebyshev
  // steps fused four per launch, or one CG iteration per launch (whose last
  // step x += alpha p is applied inside the prolongation)
  if (cheb && L.mass > 0) {
    // stored B^(q): the generic Chebyshev kernels on a one-level argument set
    const CGArgs<T>& Q = cgq_of<T>(c);
    {
      ProfScope ps(GBL_PROF_FINE_CG, st);
      launch_cheb_init<T>(Q, c->cheb_q[0], 0, 1, st);
    }
    for (int j = 1; j < c->opts.inner_iters; ++j) {
      ProfScope ps(GBL_PROF_FINE_CG, st);
      launch_cheb_step<T>(Q, c->cheb_q[j], j, 0, 1, st);
    }
  } else if (cheb) {
    const int K = c->opts.inner_iters;
    int fuse = 4;   // steps per launch (GBL_CHEB_FUSE = 1..4; the halo is 4 parents)
    if (const char* e = getenv("GBL_CHEB_FUSE")) {
      const int v = atoi(e);
      if (v >= 1 && v <= 4) fuse = v;
    }
    int k0 = 0, rd = 0;
    do {
      const int ns = std::min(fuse, K - 1 - k0);
      ProfScope ps(GBL_PROF_FINE_CG, st);
      launch_fine_cheb<T>(F, c->cheb_fine, K, k0, ns, rd, st, zb);
      k0 += ns;
      rd ^= 1;
    } while (k0 < K - 1);
  } else {
    for (int it = 0; it < c->opts.inner_iters; ++it) {
      ProfScope ps(GBL_PROF_FINE_CG, st);
      launch_fine_cg<T>(F, it, st, zb);
    }
  }
  if (c->side) {
    hipEventRecord(c->ev_join, cs);
    hipStreamWaitEvent(st, c->ev_join, 0);
  }
  ProfScope ps(GBL_PROF_PROLONG, st);
  double* part = reinterpret_cast<double*>(c->ws + L.dpart_off);
  unsigned* cnt = reinterpret_cast<unsigned*>(c->ws + L.dcnt_off);
  // the partial sums (z, z), (u, u), (z, w) go to the second half of the outer partials
  double* opart = reinterpret_cast<double*>(c->ws + L.opart_off) + 3 * (size_t)L.onblk;
  if (L.mass > 0) {
    // v^(q) in the level-q slots, then the nodal vector z = Minv v^(q)
    launch_prolong<T>(L.lv[q], c->hier<T>(L.lv[q].offR), g[q - 1], cgq_of<T>(c).lv[0].x, g[q], true, st);
    launch_mass_nodal_dots<T>(L.n, L.mass, c->lqtab(), g[q], z, dots ? uo : z, dots ? wo : z, opart, st);
  } else {
    launch_prolong_fine_dots<T>(L.lv[q], c->hier<T>(L.lv[q].offR), g[q - 1], F, z, dots ? uo : z, dots ? wo : z,
                                opart, cheb ? 1 : 0, st, zb);
  }
  (void)part;
  (void)cnt;
}

// One outer iteration of flexible CG on the FP64 fine system, with the subband
// solve as preconditioner: w = A p, u += alpha p, r -= alpha w, z = S r, and
// the new direction p = z + beta p, whose kernel also logs the iteration's
// error estimate on the device.
template <typename T>
void outer_iteration(gbl_ctx* c, const CGArgs<T>& cg, hipStream_t st, Zb zb) {
  const Layout& L = c->L;
  const int n = L.n;
  const int len = n * n;
  double* u = c->fine(0);
  double* r = c->fine(1);
  double* z = c->fine(2);
  double* p = c->fine(3);
  double* w = c->fine(4);
  double* sc = c->oscal();
  double* partA = reinterpret_cast<double*>(c->ws + L.opart_off);
  double* partB = partA + 3 * (size_t)L.onblk;
  double* elog = reinterpret_cast<double*>(c->ws + L.elog_off);
  T* gq = reinterpret_cast<T*>(c->ws + L.g_off[L.q]);
  {
    ProfScope ps(GBL_PROF_FINE_APPLY, st);
    launch_apply_fine_dots(c->a(), n, p, r, w, partA, st, zb);
  }
  launch_outer_update_convert<T>(len, partA, L.onblk, sc, u, r, p, w, gq, st, zb);
  precondition<T>(c, cg, r, z, st, true, u, w, sc, zb);
  launch_outer_direction(len, sc, partB, L.onblk, z, p, elog, 0, st, zb);
}

// Kernel classes launched inside the outer iteration: while any of them is
// being timed, iterations are launched kernel by kernel.
constexpr unsigned kIterationClasses =
    (1u << GBL_PROF_RESTRICT) | (1u << GBL_PROF_CG_INIT) | (1u << GBL_PROF_CG_SPMV) | (1u << GBL_PROF_CG_UPDATE) |
    (1u << GBL_PROF_PROLONG) | (1u << GBL_PROF_FINE_APPLY) | (1u << GBL_PROF_FINE_CG);

// Enqueue m outer iterations on st: replays of the recorded iteration graph
// (recorded on first use), or kernel-by-kernel launches.
bool iteration_graph_enabled() {
  const char* e = getenv("GBL_ITER_GRAPH");
  return !(e && e[0] == '0');
}

template <typename T>
int run_iterations(gbl_ctx* c, const CGArgs<T>& cg, int m, hipStream_t st, Zb zb) {
  if (!(g_prof.mask & kIterationClasses) && !c->graph_off && iteration_graph_enabled()) {
    if (c->iter_graph && c->iter_graph_m != zb.m) {
      hipGraphExecDestroy(c->iter_graph);   // recorded for another number of right-hand sides
      c->iter_graph = nullptr;
    }
    if (!c->iter_graph) {
      hipGraph_t g = nullptr;
      bool ok = hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal) == hipSuccess;
      if (ok) {
        outer_iteration<T>(c, cg, c->cap, zb);
        ok = hipStreamEndCapture(c->cap, &g) == hipSuccess && g != nullptr;
      }
      if (ok) ok = hipGraphInstantiate(&c->iter_graph, g, nullptr, nullptr, 0) == hipSuccess;
      c->iter_graph_m = zb.m;
      if (g) hipGraphDestroy(g);
      if (!ok) {
        c->iter_graph = nullptr;
        c->graph_off = true;
        (void)hipGetLastError();
      }
    }
    if (c->iter_graph) {
      for (int j = 0; j < m; ++j) HIPCHK(c, hipGraphLaunch(c->iter_graph, st));
      return GBL_OK;
    }
  }
  for (int j = 0; j < m; ++j) outer_iteration<T>(c, cg, st, zb);
  return GBL_OK;
}

// Ratio of the error left in the iterate to its current estimate.  When the
// estimates contract by c per iteration the remaining error is about
// estimate / (1 - c).  c is the larger of two geometric means, over the last
// kRateWindow iterations and over the whole run: CG's contraction is uneven
// from one iteration to the next and speeds up late in a run, and with a weak
// preconditioner the estimates under-read the error by more than the recent
// contraction alone suggests (measured: a factor 11 at rho = 1 on the
// 512 x 512 benchmark problem, where the last 16 iterations gave 10).  The
// ratio is never taken below 3, the margin for estimates read through loose
// inner solves.  A slowly contracting iteration (a small patch radius, a high
// contrast) thus has to go further below rtol before it stops.
constexpr int kRateWindow = 16;
double tail_factor(const std::vector<double>& h) {
  const size_t k = h.size();
  if (k <= 4) return 3.0;
  const size_t w = std::min(k - 1, (size_t)kRateWindow);
  const double a = h[k - 1], b = h[k - 1 - w], b0 = h[0];
  if (!(a > 0.0) || !(b > 0.0) || !(b0 > 0.0)) return 3.0;
  const double c_recent = std::pow(a / b, 1.0 / (double)w);
  const double c_run = std::pow(a / b0, 1.0 / (double)(k - 1));
  const double c = std::min(std::max(c_recent, c_run), 0.995);
  return std::max(3.0, 1.0 / (1.0 - c));
}

// Iterations to launch before the next look at the error estimates: the
// estimates so far are extrapolated geometrically to the iteration that
// reaches rtol / tail_factor, so that few iterations run past it.
int next_chunk(const std::vector<double>& h, double rtol) {
  const size_t k = h.size();
  if (k < 3) return 2;
  const double tol = rtol / tail_factor(h);
  const double a = h[k - 1], b = h[k - 3];
  const double cur = std::max(h[k - 1], h[k - 2]);
  if (!(a > 0.0) || !(b > 0.0) || !(a < b) || !(cur > tol)) return 1;
  const double rate = std::sqrt(a / b);
  const double rem = std::log(tol / cur) / std::log(rate);
  return (int)std::min((double)kMaxChunk, std::max(1.0, std::floor(rem)));
}

// Flexible CG on the FP64 fine system with the subband solve as
// preconditioner, for zb.m right-hand sides at once (each with its own
// scalars in its copy of the per-solve region).  mode 0: source given per
// cell; mode 1: nodal right-hand side.  src and u_nodal hold the right-hand
// sides src_stride and u_stride doubles apart.  The block stops when every
// right-hand side has met the stopping rule (or produced a non-finite
// estimate); right-hand sides that finished earlier keep iterating, which only
// lowers their error.
template <typename T>
int fcg_solve(gbl_ctx* c, const CGArgs<T>& cg, int mode, const double* src, size_t src_stride, double* u_nodal,
              size_t u_stride, gbl_solve_info* info, hipStream_t st, Zb zb) {
  const Layout& L = c->L;
  const int n = L.n;
  const int len = n * n;
  const int m = zb.m;
  double* u = c->fine(0);
  double* r = c->fine(1);
  double* z = c->fine(2);
  double* p = c->fine(3);
  double* w = c->fine(4);
  double* sc = c->oscal();
  double* part = reinterpret_cast<double*>(c->ws + L.dpart_off);
  unsigned* cnt = reinterpret_cast<unsigned*>(c->ws + L.dcnt_off);
  double* partB = reinterpret_cast<double*>(c->ws + L.opart_off) + 3 * (size_t)L.onblk;
  const double* elog = reinterpret_cast<const double*>(c->ws + L.elog_off);
  launch_residual(c->a(), n, mode, src, u_nodal, nullptr, r, st, zb, src_stride, u_stride);
  launch_fill((size_t)len, 0.0, u, st, zb);
  launch_fill(1, 0.0, sc + kSIter, st, zb);
  launch_dots(len, 1, r, r, nullptr, nullptr, nullptr, nullptr, part, cnt, sc + kSBB, st, zb);
  precondition<T>(c, cg, r, z, st, false, u, w, sc, zb);
  launch_outer_direction(len, sc, partB, L.onblk, z, p, nullptr, 1, st, zb);
  // Error estimate of iteration i (logged by the direction kernel): z = S r
  // approximates the error and alpha p is the last correction; either alone
  // can under-read the error when the inner solves are loose, so the larger
  // of the two over the last two iterations, times tail_factor, is tested
  // against rtol.  Iterations that run past the first passing one only lower
  // the A-norm error further.
  const double rtol = c->opts.rtol;
  double* hl = c->host + kHostLog;   // host copy of a chunk of estimates, kMaxChunk per right-hand side
  std::vector<std::vector<double>> hist(m);
  std::vector<int> done_rhs(m, 0), status(m, GBL_ENOCONV);
  std::vector<double> est(m, 1.0), prev(m, INFINITY);
  int done = 0;
  // GBL_PROGRESS=1: a line on stderr about every 15 s of a long solve
  const char* pe = getenv("GBL_PROGRESS");
  const bool progress = pe && pe[0] == '1';
  auto t_last = std::chrono::steady_clock::now();
  while (done < c->opts.max_outer) {
    int chunk = kMaxChunk;
    for (int j = 0; j < m; ++j)
      if (!done_rhs[j]) chunk = std::min(chunk, next_chunk(hist[j], rtol));
    chunk = std::min(chunk, c->opts.max_outer - done);
    const int rs = run_iterations<T>(c, cg, chunk, st, zb);
    if (rs) return rs;
    HIPCHK(c, hipMemcpy2DAsync(hl, kMaxChunk * sizeof(double), elog + done, L.solve_stride,
                               (size_t)chunk * sizeof(double), m, hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipStreamSynchronize(st));
    done += chunk;
    int open = 0;
    for (int j = 0; j < m; ++j) {
      for (int i = 0; i < chunk && !done_rhs[j]; ++i) {
        const double cur = hl[j * kMaxChunk + i];
        hist[j].push_back(cur);
        if (!std::isfinite(cur)) {
          est[j] = cur;
          status[j] = GBL_ENOCONV;
          done_rhs[j] = 1;
        } else {
          est[j] = std::max(cur, prev[j]);
          prev[j] = cur;
          if (est[j] * tail_factor(hist[j]) <= rtol) {
            status[j] = GBL_OK;
            done_rhs[j] = 1;
          }
        }
      }
      open += done_rhs[j] ? 0 : 1;
    }
    if (!open) break;
    if (progress) {
      const auto now = std::chrono::steady_clock::now();
      if (std::chrono::duration<double>(now - t_last).count() >= 15.0) {
        double worst_est = 0.0;
        for (int j = 0; j < m; ++j)
          if (!done_rhs[j]) worst_est = std::max(worst_est, est[j]);
        std::fprintf(stderr, "gbl: %d right-hand side(s), outer iteration %d, %d open, largest estimate %.3e\n", m,
                     done, open, worst_est);
        std::fflush(stderr);
        t_last = now;
      }
    }
  }
  const int it = done;
  launch_slots_to_nodal(n, u, u_nodal, st, zb, u_stride);
  // final residual of the returned iterate
  launch_residual(c->a(), n, mode, src, u_nodal, u, r, st, zb, src_stride, u_stride);
  launch_dots(len, 1, r, r, nullptr, nullptr, nullptr, nullptr, part, cnt, sc + kSRR, st, zb);
  HIPCHK(c, hipMemcpy2DAsync(c->host, kNumOuterScalars * sizeof(double), sc, L.solve_stride,
                             kNumOuterScalars * sizeof(double), m, hipMemcpyDeviceToHost, st));
  HIPCHK(c, hipStreamSynchronize(st));
  HIPCHK(c, hipGetLastError());
  int worst = GBL_OK;
  for (int j = 0; j < m; ++j) {
    const double* hs = c->host + (size_t)j * kNumOuterScalars;
    const double bb = hs[kSBB], rr = hs[kSRR];
    const double rel_res = bb > 0.0 ? std::sqrt(rr / bb) : std::sqrt(rr);
    if (info) {
      // maxima over right-hand sides that keep a NaN visible
      auto worse = [](double a, double b) { return (std::isnan(a) || std::isnan(b)) ? NAN : std::max(a, b); };
      info->outer_iters = std::max(info->outer_iters, it);
      info->rel_update = worse(info->rel_update, est[j]);
      info->rel_residual = worse(info->rel_residual, rel_res);
    }
    if (!std::isfinite(est[j]) || !std::isfinite(rel_res)) c->diverged = true;
    if (status[j] != GBL_OK) worst = status[j];
  }
  return worst;
}

template <typename T>
const CGArgs<T>& cg_of(const gbl_ctx* c);
template <>
const CGArgs<float>& cg_of<float>(const gbl_ctx* c) { return c->cgf; }
template <>
const CGArgs<double>& cg_of<double>(const gbl_ctx* c) { return c->cgd; }
template <typename T>
const FineCG<T>& fcg_of(const gbl_ctx* c);
template <>
const FineCG<float>& fcg_of<float>(const gbl_ctx* c) { return c->fcgf; }
template <>
const FineCG<double>& fcg_of<double>(const gbl_ctx* c) { return c->fcgd; }
template <>
const CGArgs<float>& cgq_of<float>(const gbl_ctx* c) { return c->cgqf; }
template <>
const CGArgs<double>& cgq_of<double>(const gbl_ctx* c) { return c->cgqd; }

template <typename T>
// Right-hand sides in blocks of up to M solved together (M copies of the
// per-solve region).
int solve_many(gbl_ctx* c, int nrhs, int mode, const double* src, size_t src_stride, double* u,
               gbl_solve_info* info, hipStream_t st) {
  int worst = GBL_OK;
  const size_t us = (size_t)(c->L.n + 1) * (c->L.n + 1);
  for (int r0 = 0; r0 < nrhs; r0 += c->L.M) {
    Zb zb;
    zb.m = std::min(c->L.M, nrhs - r0);
    zb.zs = c->L.solve_stride;
    const int s = fcg_solve<T>(c, cg_of<T>(c), mode, src + r0 * src_stride, src_stride, u + r0 * us, us, info, st,
                               zb);
    if (s == GBL_EHIP) return s;
    if (s != GBL_OK) worst = s;
  }
  return worst;
}

}  // namespace

// Geometry, hierarchy operators and FP64 level vectors of the gamblet transform
template <typename T>
TransformArgs transform_args(const gbl_ctx* c) {
  const Layout& L = c->L;
  TransformArgs a;
  a.q = L.q;
  a.n = L.n;
  for (int k = 1; k <= L.q; ++k) {
    a.lv[k] = L.lv[k];
    a.U[k] = reinterpret_cast<double*>(c->ws + L.tr_off[k]);
    if (k >= 2) {
      a.R[k] = c->hier<T>(L.lv[k].offR);
      a.B[k] = c->hier<T>(L.lv[k].offB);
    }
  }
  a.A1 = c->hier<T>(L.lv[1].offA);
  return a;
}

extern "C" {

int gbl_version(void) { return GBL_VERSION; }

int gbl_default_opts(gbl_opts* o) {
  if (!o) return fail(nullptr, GBL_EINVAL, "opts is NULL");
  o->rho = 3;
  o->precision = GBL_MIXED;
  o->rtol = 1e-8;
  o->max_outer = 100;
  o->inner_iters = 16;
  o->max_rhs = 1;
  o->inner_iters_coarse = 2;
  o->inner_kind = GBL_INNER_CHEBYSHEV;
  o->kappa = 200.0;
  o->kappa_coarse = 10.0;
  o->level_q_mass = 0;
  o->rho_coarse = 0;
  o->window_tol = 0.0;
  o->exact = 0;
  o->geometry = 0;
  o->source = 0;
  o->w_kind = 0;
  o->dim = 2;
  o->autotune = 0;
  o->autotune_path = nullptr;
  o->tensor = 0;
  return GBL_OK;
}

int gbl_workspace_bytes(int q, const gbl_opts* opts, size_t* bytes) {
  if (!bytes) return fail(nullptr, GBL_EINVAL, "bytes is NULL");
  std::string msg;
  if (opts && opts->exact) {
    int st = validate_opts(opts, msg);
    ExactHier E;
    if (!st) st = exact_layout(E, q, opts->dim, opts->geometry, opts->w_kind, opts->tensor, opts->max_rhs, msg);
    if (st) return fail(nullptr, st, msg);
    *bytes = E.total;
    return GBL_OK;
  }
  Layout L;
  const int st = make_layout(q, opts, L, msg);
  if (st) return fail(nullptr, st, msg);
  *bytes = L.total;
  return GBL_OK;
}

int gbl_build(gbl_ctx** out, int q, const double* a_dev, const gbl_opts* opts, void* ws_dev, size_t ws_bytes,
              void* stream) {
  if (!out) return fail(nullptr, GBL_EINVAL, "out is NULL");
  *out = nullptr;
  if (!a_dev) return fail(nullptr, GBL_EINVAL, "a_dev is NULL");
  if (!ws_dev) return fail(nullptr, GBL_EINVAL, "ws_dev is NULL");
  std::string msg;
  if (opts && opts->exact) {
    int st = validate_opts(opts, msg);
    ExactHier E;
    if (!st) st = exact_layout(E, q, opts->dim, opts->geometry, opts->w_kind, opts->tensor, opts->max_rhs, msg);
    if (st) return fail(nullptr, st, msg);
    if (ws_bytes < E.total)
      return fail(nullptr, GBL_ENOMEM, "workspace too small: need " + std::to_string(E.total) + " bytes");
    gbl_ctx* c = new (std::nothrow) gbl_ctx();
    if (c) c->ex = new (std::nothrow) ExactHier(E);
    if (!c || !c->ex) {
      delete c;
      return fail(nullptr, GBL_ENOMEM, "host allocation failed");
    }
    c->opts = *opts;
    c->L.q = q;
    c->L.n = E.nc;
    c->L.prec = GBL_FP64;
    c->L.elem = c->L.selem = 8;
    c->ws = static_cast<char*>(ws_dev);
    c->ws_bytes = ws_bytes;
    c->ex->ws = c->ws;
    st = exact_build(*c->ex, a_dev, static_cast<hipStream_t>(stream), msg);
    if (st) {
      g_last_error = msg;
      release(c);
      return st;
    }
    *out = c;
    return GBL_OK;
  }
  Layout L;
  int st = make_layout(q, opts, L, msg);
  if (st) return fail(nullptr, st, msg);
  if (ws_bytes < L.total)
    return fail(nullptr, GBL_ENOMEM, "workspace too small: need " + std::to_string(L.total) + " bytes");
  gbl_ctx* c = new (std::nothrow) gbl_ctx();
  if (!c) return fail(nullptr, GBL_ENOMEM, "host allocation failed");
  c->L = L;
  c->opts = *opts;
  c->ws = static_cast<char*>(ws_dev);
  c->ws_bytes = ws_bytes;
  hipStream_t s = static_cast<hipStream_t>(stream);
  {
    CtxResources r;
    if (!acquire_resources(r)) {
      delete c;
      return fail(nullptr, GBL_EHIP, "stream, event or pinned host allocation failed");
    }
    c->device = r.device;
    c->side = r.side;
    c->cap = r.cap;
    c->ev_fork = r.ev_fork;
    c->ev_join = r.ev_join;
    c->host = r.host;
  }
  auto bail = [&](int code) {
    g_last_error = c->err;
    release(c);
    return code;
  };
  const size_t n2 = (size_t)L.n * L.n;
  if (hipMemcpyAsync(c->ws + L.a_off, a_dev, n2 * sizeof(double), hipMemcpyDeviceToDevice, s) != hipSuccess) {
    c->err = "copy of the coefficient failed";
    return bail(GBL_EHIP);
  }
  // zero the status word, reduction tickets and the coarse factor
  {
    // coarse factor, status, bounds and every copy of the per-solve region
    launch_fill((L.solve_off + (size_t)L.M * L.solve_stride - L.L1_off) / 8, 0.0,
                reinterpret_cast<double*>(c->ws + L.L1_off), s);
    launch_fill((L.total - L.wcnt_off) / 8, 0.0, reinterpret_cast<double*>(c->ws + L.wcnt_off), s);
  }
  c->cgf = make_cg_args<float>(c);
  c->cgd = make_cg_args<double>(c);
  c->cgqf = make_cgq_args<float>(c);
  c->cgqd = make_cgq_args<double>(c);
  c->fcgf = make_fine_cg<float>(c);
  c->fcgd = make_fine_cg<double>(c);
  st = (L.elem == 8) ? build_impl<double>(c, s) : build_impl<float>(c, s);
  if (st) return bail(st);
  if (L.build64) {
    // the solve reads an FP32 copy of the FP64 hierarchy; its window
    // corrections are formed from that copy (the operator the solve applies)
    launch_convert<float, double>(L.hier_elems, c->hier<double>(0), c->hier<float>(0), s);
    for (int k = 3; k < L.q; ++k) {
      if (L.win_cap[k] <= 0) continue;
      const LevelGeom& g = L.lv[k];
      launch_win_build<float>(g, c->hier<float>(g.offB), opts->window_tol, L.win_cap[k],
                              reinterpret_cast<int*>(c->ws + L.win_list_off[k]),
                              reinterpret_cast<int*>(c->ws + L.win_idx_off[k]),
                              reinterpret_cast<float*>(c->ws + L.win_inv_off[k]),
                              reinterpret_cast<unsigned*>(c->ws + L.wcnt_off) + k, c->status(), s);
    }
    if (hipGetLastError() != hipSuccess) {
      c->err = "launch failed";
      return bail(GBL_EHIP);
    }
  }
  unsigned* hbits = reinterpret_cast<unsigned*>(c->host + kHostBits);
  unsigned* wbits = hbits + kMaxLevels;
  static_assert(2 * kMaxLevels * sizeof(unsigned) <= (kHostLog - kHostBits) * sizeof(double),
                "pinned host words hold the bounds and the window counts");
  if (hipMemcpyAsync(c->host + kHostStatus, c->status(), sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipMemcpyAsync(hbits, c->ws + L.gersh_off, kMaxLevels * sizeof(unsigned), hipMemcpyDeviceToHost, s) !=
          hipSuccess ||
      hipMemcpyAsync(wbits, c->ws + L.wcnt_off, kMaxLevels * sizeof(unsigned), hipMemcpyDeviceToHost, s) !=
          hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess) {
    c->err = "status read failed";
    return bail(GBL_EHIP);
  }
  for (int k = 0; k < kMaxLevels; ++k) std::memcpy(&c->lmax[k], &hbits[k], sizeof(float));
  make_cheb_tables(c);
  int bits = 0;
  std::memcpy(&bits, c->host + kHostStatus, sizeof(int));
  if (bits & kBadCoefficient) {
    c->err = "coefficient must be positive and finite in every cell";
    return bail(GBL_EINVAL);
  }
  if (bits & kRegularizedPivot) c->build_flags |= GBL_FLAG_PIVOTS_REGULARIZED;
  if (bits & kWindowOverflow) {
    c->err = "more kept windows than the workspace holds";
    return bail(GBL_ENOMEM);
  }
  for (int k = 0; k < kMaxLevels; ++k) c->nwin[k] = (int)std::min<unsigned>(wbits[k], (unsigned)L.win_cap[k]);
  set_windows(c, c->cgf);
  set_windows(c, c->cgd);
  if (bits & kBadPivot) {
    c->err = "non-positive pivot in a patch or coarse matrix";
    return bail(GBL_ENOTSPD);
  }
  *out = c;
  return GBL_OK;
}

int gbl_solve(gbl_ctx* c, int nrhs, const double* g_dev, double* u_dev, gbl_solve_info* info, void* stream) {
  if (!c) return fail(nullptr, GBL_EINVAL, "ctx is NULL");
  if (!g_dev || !u_dev) return fail(c, GBL_EINVAL, "g_dev and u_dev must not be NULL");
  if (nrhs < 1) return fail(c, GBL_EINVAL, "nrhs must be at least 1");
  if (info) std::memset(info, 0, sizeof(*info));
  c->diverged = false;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (c->ex) {
    std::string msg;
    const int st = exact_solve(*c->ex, nrhs, c->opts.source, g_dev, u_dev, 2, s, msg);
    if (info) info->status = st;
    return st ? fail(c, st, msg) : GBL_OK;
  }
  const size_t n2 = (size_t)c->L.n * c->L.n;
  const int st = (c->L.selem == 8) ? solve_many<double>(c, nrhs, 0, g_dev, n2, u_dev, info, s)
                                         : solve_many<float>(c, nrhs, 0, g_dev, n2, u_dev, info, s);
  if (info) info->status = st;
  if (st == GBL_ENOCONV)
    return fail(c, st, c->diverged ? "solve diverged (non-finite error estimate or residual)"
                                   : "solve did not reach rtol within max_outer iterations");
  return st;
}

int gbl_adjoint(gbl_ctx* c, int nrhs, const double* u_dev, const double* dJdu_dev, double* dJdloga_dev,
                double* dJdg_dev, double* lambda_dev, gbl_solve_info* info, void* stream) {
  if (!c) return fail(nullptr, GBL_EINVAL, "ctx is NULL");
  if (!u_dev || !dJdu_dev || !dJdloga_dev) return fail(c, GBL_EINVAL, "u, dJdu and dJdloga must not be NULL");
  if (c->ex) return fail(c, GBL_EINVAL, "the exact hierarchy has no adjoint call");
  if (nrhs < 1) return fail(c, GBL_EINVAL, "nrhs must be at least 1");
  if (info) std::memset(info, 0, sizeof(*info));
  c->diverged = false;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int n = c->L.n;
  const size_t n2 = (size_t)n * n, us = (size_t)(n + 1) * (n + 1);
  int worst = GBL_OK;
  for (int r0 = 0; r0 < nrhs; r0 += c->L.M) {
    Zb zb;
    zb.m = std::min(c->L.M, nrhs - r0);
    zb.zs = c->L.solve_stride;
    // the adjoint states: the caller's array, or the per-solve copies of the workspace
    double* lam = lambda_dev ? lambda_dev + r0 * us : reinterpret_cast<double*>(c->ws + c->L.lam_off);
    const size_t ls = lambda_dev ? us : c->L.solve_stride / sizeof(double);
    for (int j = 0; j < zb.m; ++j) launch_fill(us, 0.0, lam + j * ls, s);
    const int st = (c->L.selem == 8)
                       ? fcg_solve<double>(c, c->cgd, 1, dJdu_dev + r0 * us, us, lam, ls, info, s, zb)
                       : fcg_solve<float>(c, c->cgf, 1, dJdu_dev + r0 * us, us, lam, ls, info, s, zb);
    if (st == GBL_EHIP) return st;
    if (st != GBL_OK) worst = st;
    ProfScope ps(GBL_PROF_GRADIENT, s);
    for (int j = 0; j < zb.m; ++j) {
      const int r = r0 + j;
      launch_cell_gradient(c->a(), n, u_dev + r * us, lam + j * ls, dJdloga_dev + r * n2,
                           dJdg_dev ? dJdg_dev + r * n2 : nullptr, s);
    }
  }
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipStreamSynchronize(s));
  if (info) info->status = worst;
  if (worst == GBL_ENOCONV)
    return fail(c, worst, c->diverged ? "adjoint solve diverged (non-finite error estimate or residual)"
                                      : "adjoint solve did not reach rtol within max_outer iterations");
  return worst;
}

// ---------------------------------------------------------------------------
// Batches of independent problems.  A problem of depth 6..8 leaves most of the
// GPU idle (its kernels are latency-bound), so the problems of a batch run
// concurrently: a pool of host threads, each with its own HIP stream, takes
// problems largest first (work ~ 4^q x right-hand sides).  The pool's streams
// start after the work already enqueued on the caller's stream and the caller's
// stream waits for all of them before the call returns.
// ---------------------------------------------------------------------------
}  // extern "C"

namespace {

int batch_workers(int nprob) {
  int w = 8;
  if (const char* e = getenv("GBL_BATCH_WORKERS")) {
    const int v = atoi(e);
    if (v >= 1 && v <= 64) w = v;
  }
  return std::max(1, std::min(w, nprob));
}

// Runs job(i, stream) for every problem i on the pool; returns the first
// non-OK status in problem order (status[i] holds each one) and the message
// of that failure in msg.
template <typename Job>
int run_batch(int nprob, const std::vector<double>& work, int* status, hipStream_t caller, Job job,
              std::string& msg) {
  std::vector<int> order(nprob);
  for (int i = 0; i < nprob; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return work[x] > work[y]; });
  const int nw = batch_workers(nprob);
  hipEvent_t start = nullptr;
  if (hipEventCreateWithFlags(&start, hipEventDisableTiming) != hipSuccess || hipEventRecord(start, caller) != hipSuccess) {
    msg = "event creation failed";
    return GBL_EHIP;
  }
  std::vector<hipStream_t> streams(nw, nullptr);
  std::vector<hipEvent_t> done(nw, nullptr);
  int setup = GBL_OK;
  for (int w = 0; w < nw; ++w) {
    if (hipStreamCreateWithFlags(&streams[w], hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&done[w], hipEventDisableTiming) != hipSuccess ||
        hipStreamWaitEvent(streams[w], start, 0) != hipSuccess) {
      setup = GBL_EHIP;
    }
  }
  std::vector<std::string> msgs(nprob);
  if (setup == GBL_OK) {
    int dev = 0;
    hipGetDevice(&dev);
    std::atomic<int> next{0};
    std::vector<std::thread> pool;
    for (int w = 0; w < nw; ++w) {
      pool.emplace_back([&, w]() {
        hipSetDevice(dev);
        for (;;) {
          const int k = next.fetch_add(1);
          if (k >= nprob) break;
          const int i = order[k];
          status[i] = job(i, streams[w], msgs[i]);
        }
        hipEventRecord(done[w], streams[w]);
      });
    }
    for (auto& t : pool) t.join();
    for (int w = 0; w < nw; ++w) hipStreamWaitEvent(caller, done[w], 0);
  }
  for (int w = 0; w < nw; ++w) {
    if (streams[w]) {
      hipStreamSynchronize(streams[w]);
      hipStreamDestroy(streams[w]);
    }
    if (done[w]) hipEventDestroy(done[w]);
  }
  hipEventDestroy(start);
  if (setup != GBL_OK) {
    msg = "stream creation for the batch failed";
    return setup;
  }
  for (int i = 0; i < nprob; ++i) {
    if (status[i] != GBL_OK) {
      msg = "problem " + std::to_string(i) + ": " + msgs[i];
      return status[i];
    }
  }
  return GBL_OK;
}

}  // namespace

extern "C" {

int gbl_build_batched(int nprob, const int* q, const double* const* a_dev, const gbl_opts* opts,
                      void* const* ws_dev, const size_t* ws_bytes, gbl_ctx** ctx_out, int* status, void* stream) {
  if (nprob < 1 || !q || !a_dev || !opts || !ws_dev || !ws_bytes || !ctx_out || !status)
    return fail(nullptr, GBL_EINVAL, "batched build: null argument or nprob < 1");
  if (opts->exact) return fail(nullptr, GBL_EINVAL, "batched build: the exact hierarchy is built one problem at a time");
  std::vector<double> work(nprob);
  for (int i = 0; i < nprob; ++i) {
    ctx_out[i] = nullptr;
    status[i] = GBL_EINVAL;
    work[i] = (q[i] >= 2 && q[i] <= 12) ? std::ldexp(1.0, 2 * q[i]) : 0.0;
  }
  std::string msg;
  const int st = run_batch(nprob, work, status, static_cast<hipStream_t>(stream),
                           [&](int i, hipStream_t s, std::string& m) {
                             const int r = gbl_build(&ctx_out[i], q[i], a_dev[i], opts, ws_dev[i], ws_bytes[i], s);
                             if (r != GBL_OK) m = gbl_last_error(nullptr);
                             return r;
                           },
                           msg);
  if (st != GBL_OK) return fail(nullptr, st, "batched build: " + msg);
  return GBL_OK;
}

int gbl_solve_batched(int nprob, gbl_ctx* const* ctx, const int* nrhs, const double* const* g_dev,
                      double* const* u_dev, gbl_solve_info* info, int* status, void* stream) {
  if (nprob < 1 || !ctx || !nrhs || !g_dev || !u_dev || !status)
    return fail(nullptr, GBL_EINVAL, "batched solve: null argument or nprob < 1");
  std::vector<double> work(nprob);
  for (int i = 0; i < nprob; ++i) {
    status[i] = GBL_EINVAL;
    work[i] = ctx[i] ? std::ldexp(1.0, 2 * ctx[i]->L.q) * std::max(1, nrhs[i]) : 0.0;
  }
  std::string msg;
  const int st = run_batch(nprob, work, status, static_cast<hipStream_t>(stream),
                           [&](int i, hipStream_t s, std::string& m) {
                             const int r = gbl_solve(ctx[i], nrhs[i], g_dev[i], u_dev[i], info ? &info[i] : nullptr, s);
                             if (r != GBL_OK) m = gbl_last_error(ctx[i]);
                             return r;
                           },
                           msg);
  if (st != GBL_OK) return fail(nullptr, st, "batched solve: " + msg);
  return GBL_OK;
}

int gbl_build_flags(const gbl_ctx* c, unsigned* flags) {
  if (!c || !flags) return fail(nullptr, GBL_EINVAL, "ctx or flags is NULL");
  *flags = c->build_flags;
  return GBL_OK;
}

int gbl_level_layout(const gbl_ctx* c, int k, gbl_level_desc* d) {
  if (!c || !d) return fail(nullptr, GBL_EINVAL, "ctx and desc must not be NULL");
  if (k < 1 || k > c->L.q) return fail(const_cast<gbl_ctx*>(c), GBL_EINVAL, "level out of range");
  if (c->ex) {
    const ExactHier& E = *c->ex;
    std::memset(d, 0, sizeof(*d));
    d->k = k;
    d->dense = 1;
    d->n = (int)E.N[k];
    d->nsub = k >= 2 ? E.rp * E.np2[k] : 0;
    d->nk = k == c->L.q ? E.m : (1 << k);
    d->elem_bytes = 8;
    d->A = E.A(k);
    d->B = k >= 2 ? E.B(k) : nullptr;
    d->R = k >= 2 ? E.R(k) : nullptr;
    d->patch_kernel = kVariantDefault;
    d->galerkin_kernel = kVariantDefault;
    return GBL_OK;
  }
  const LevelGeom& g = c->L.lv[k];
  d->k = k;
  d->nk = g.nk;
  d->s = g.s;
  d->t = k >= 2 ? g.t : 0;
  d->rw = k >= 2 ? g.rw : 0;
  d->rho = k >= 2 ? g.rho : 0;
  d->elem_bytes = (int)c->L.elem;
  const char* base = c->ws + c->L.hier_off;
  d->A = base + g.offA * c->L.elem;
  d->B = k >= 2 ? base + g.offB * c->L.elem : nullptr;
  d->R = k >= 2 ? base + g.offR * c->L.elem : nullptr;
  d->nwin = (k >= 2 && k < c->L.q) ? c->nwin[k] : 0;
  d->wlist = d->nwin > 0 ? reinterpret_cast<const int*>(c->ws + c->L.win_list_off[k]) : nullptr;
  d->winv = d->nwin > 0 ? c->ws + c->L.win_inv_off[k] : nullptr;
  d->dense = 0;
  d->n = 0;
  d->nsub = 0;
  d->patch_kernel = (c->opts.autotune && k >= 2) ? c->tuned[k][0] : kVariantDefault;
  d->galerkin_kernel = (c->opts.autotune && k >= 2) ? c->tuned[k][1] : kVariantDefault;
  return GBL_OK;
}

int gbl_profile_enable(unsigned mask) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof.mask = mask;
  return GBL_OK;
}

int gbl_profile_reset(void) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof.drain();
  for (int k = 0; k < GBL_PROF_NUM_KERNELS; ++k) {
    g_prof.total_ms[k] = 0.0;
    g_prof.launches[k] = 0;
  }
  return GBL_OK;
}

int gbl_profile_read(int kernel, double* total_ms, long* launches) {
  if (kernel < 0 || kernel >= GBL_PROF_NUM_KERNELS || !total_ms || !launches)
    return fail(nullptr, GBL_EINVAL, "bad profile query");
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof.drain();
  *total_ms = g_prof.total_ms[kernel];
  *launches = g_prof.launches[kernel];
  return GBL_OK;
}

int gbl_transform_size(const gbl_ctx* c, size_t* count) {
  if (!c || !count) return fail(nullptr, GBL_EINVAL, "ctx or count is NULL");
  *count = c->ex ? (size_t)c->ex->ncoef : (size_t)1 << (2 * c->L.q);
  return GBL_OK;
}

int gbl_transform(gbl_ctx* c, const double* u_dev, double* coef_dev, void* stream) {
  if (!c) return fail(nullptr, GBL_EINVAL, "ctx is NULL");
  if (!u_dev || !coef_dev) return fail(c, GBL_EINVAL, "u and coef must not be NULL");
  if (c->L.mass > 0) return fail(c, GBL_EINVAL, "the transform needs the nodal-basis level-q gamblets");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (c->ex) return exact_transform(*c->ex, u_dev, coef_dev, s) ? fail(c, GBL_EHIP, "launch failed") : GBL_OK;
  if (c->L.elem == 8) launch_transform<double>(transform_args<double>(c), u_dev, coef_dev, s);
  else launch_transform<float>(transform_args<float>(c), u_dev, coef_dev, s);
  HIPCHK(c, hipGetLastError());
  return GBL_OK;
}

int gbl_inverse_transform(gbl_ctx* c, const double* coef_dev, double* u_dev, void* stream) {
  if (!c) return fail(nullptr, GBL_EINVAL, "ctx is NULL");
  if (!u_dev || !coef_dev) return fail(c, GBL_EINVAL, "u and coef must not be NULL");
  if (c->L.mass > 0) return fail(c, GBL_EINVAL, "the transform needs the nodal-basis level-q gamblets");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (c->ex)
    return exact_inverse_transform(*c->ex, coef_dev, u_dev, s) ? fail(c, GBL_EHIP, "launch failed") : GBL_OK;
  if (c->L.elem == 8) launch_inverse_transform<double>(transform_args<double>(c), coef_dev, u_dev, s);
  else launch_inverse_transform<float>(transform_args<float>(c), coef_dev, u_dev, s);
  HIPCHK(c, hipGetLastError());
  return GBL_OK;
}

int gbl_compress(gbl_ctx* c, double* coef_dev, long keep, double* threshold, void* stream) {
  if (!c) return fail(nullptr, GBL_EINVAL, "ctx is NULL");
  if (!coef_dev) return fail(c, GBL_EINVAL, "coef must not be NULL");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const long n = c->ex ? c->ex->ncoef : (long)1 << (2 * c->L.q);
  double* thr = c->ex ? c->ex->at(c->ex->offThr) : c->oscal() + kSSpare;   // device scalar
  if (keep <= 0) {
    launch_fill((size_t)n, 0.0, coef_dev, s);
    if (threshold) *threshold = HUGE_VAL;
  } else if (keep >= n) {
    if (threshold) *threshold = 0.0;
  } else {
    auto* sel = reinterpret_cast<unsigned long long*>(c->ws + (c->ex ? c->ex->offSel : c->L.sel_off));
    launch_select_threshold(coef_dev, n, keep, sel, reinterpret_cast<unsigned*>(sel + 4), thr, s);
    launch_zero_below(thr, n, coef_dev, s);
    if (threshold) {
      HIPCHK(c, hipMemcpyAsync(threshold, thr, sizeof(double), hipMemcpyDeviceToHost, s));
      HIPCHK(c, hipStreamSynchronize(s));
    }
  }
  HIPCHK(c, hipGetLastError());
  return GBL_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Compression without allocation: the selection of gbl_compress with its
// state words, histogram and threshold in a fixed array of this library's
// device memory instead of a hierarchy workspace.  Host code never passes
// `scratch` itself to a kernel: the array's device address on the current
// device comes from hipGetSymbolAddress, taken once per device on the first
// call there.
// ---------------------------------------------------------------------------
namespace {

constexpr size_t kNaStateOff = 0;      // 4 words of 64 bits
constexpr size_t kNaThrOff = 64;       // the threshold (one double)
constexpr size_t kNaHistOff = 256;     // kSelHistBins counters of 32 bits
constexpr size_t kNaScratchBytes = kNaHistOff + (size_t)kSelHistBins * sizeof(unsigned);
constexpr long kNaMaxCount = 4294967295L;   // the histogram counters are 32-bit
constexpr int kNaMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kNaScratchBytes];

std::mutex g_na_mu;
unsigned char* g_na_ptr[kNaMaxDevices] = {};

int noalloc_scratch(unsigned char** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(nullptr, GBL_EHIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
  if (dev < 0 || dev >= kNaMaxDevices) return fail(nullptr, GBL_EINVAL, "device ordinal beyond 63");
  std::lock_guard<std::mutex> lk(g_na_mu);
  if (!g_na_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(nullptr, GBL_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_na_ptr[dev] = static_cast<unsigned char*>(p);
  }
  *out = g_na_ptr[dev];
  return GBL_OK;
}

}  // namespace

extern "C" {

int gbl_compress_noalloc(double* coef_dev, long count, long keep, double* threshold, void* stream) {
  if (!coef_dev) return fail(nullptr, GBL_EINVAL, "coef must not be NULL");
  if (count < 1 || count > kNaMaxCount)
    return fail(nullptr, GBL_EINVAL, "count must be in [1, 4294967295] (32-bit histogram counters)");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (keep <= 0) {
    launch_fill((size_t)count, 0.0, coef_dev, s);
    if (threshold) *threshold = HUGE_VAL;
  } else if (keep >= count) {
    if (threshold) *threshold = 0.0;
  } else {
    unsigned char* base = nullptr;
    const int st = noalloc_scratch(&base);
    if (st) return st;
    auto* state = reinterpret_cast<unsigned long long*>(base + kNaStateOff);
    auto* hist = reinterpret_cast<unsigned*>(base + kNaHistOff);
    double* thr = reinterpret_cast<double*>(base + kNaThrOff);
    launch_select_threshold(coef_dev, count, keep, state, hist, thr, s);
    launch_zero_below(thr, count, coef_dev, s);
    if (threshold) {
      hipError_t e = hipMemcpyAsync(threshold, thr, sizeof(double), hipMemcpyDeviceToHost, s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
      if (e != hipSuccess) return fail(nullptr, GBL_EHIP, std::string("threshold read: ") + hipGetErrorString(e));
    }
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(nullptr, GBL_EHIP, std::string("launch: ") + hipGetErrorString(e));
  return GBL_OK;
}

int gbl_energy_norm(gbl_ctx* c, const double* u_dev, double* norm, void* stream) {
  if (!c || !norm) return fail(c, GBL_EINVAL, "ctx and norm must not be NULL");
  if (!u_dev) return fail(c, GBL_EINVAL, "u must not be NULL");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (c->ex) return exact_energy_norm(*c->ex, u_dev, norm, s) ? fail(c, GBL_EHIP, "energy norm failed") : GBL_OK;
  const Layout& L = c->L;
  const int n = L.n;
  double* sl = c->fine(0);
  double* w = c->fine(1);
  double* out = c->oscal() + kSSpare + 1;
  launch_nodal_to_slots(n, u_dev, sl, s);
  launch_apply_fine(c->a(), n, sl, w, s);
  launch_dots(n * n, 1, sl, w, nullptr, nullptr, nullptr, nullptr, reinterpret_cast<double*>(c->ws + L.dpart_off),
              reinterpret_cast<unsigned*>(c->ws + L.dcnt_off), out, s);
  HIPCHK(c, hipMemcpyAsync(c->host, out, sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
  HIPCHK(c, hipGetLastError());
  *norm = std::sqrt(std::max(c->host[0], 0.0));
  return GBL_OK;
}

// Level-q gamblets from the localized mass inverse (Algorithm 2; Definition
// 5.2).  These calls need no hierarchy: they take q, the patch radius and
// device pointers, and launch on stream.
static int check_level_q(int q, int rho_q) {
  if (q < 2 || q > 12) return fail(nullptr, GBL_EINVAL, "q must be in [2, 12]");
  if (rho_q < 1 || rho_q > kMaxRhoQ) return fail(nullptr, GBL_EINVAL, "rho_q must be in [1, 4]");
  return GBL_OK;
}

static int launched() {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(nullptr, GBL_EHIP, std::string("kernel launch: ") + hipGetErrorString(e));
  return GBL_OK;
}

int gbl_mass_inverse(int q, int rho_q, double* table_dev, void* stream) {
  if (int st = check_level_q(q, rho_q)) return st;
  if (!table_dev) return fail(nullptr, GBL_EINVAL, "table must not be NULL");
  launch_mass_inverse_table(1 << q, rho_q, table_dev, static_cast<hipStream_t>(stream));
  return launched();
}

int gbl_level_q_gamblets(int q, int rho_q, const double* table_dev, double* psi_dev, void* stream) {
  if (int st = check_level_q(q, rho_q)) return st;
  if (!table_dev || !psi_dev) return fail(nullptr, GBL_EINVAL, "table and psi must not be NULL");
  launch_level_q_weights(1 << q, rho_q, table_dev, psi_dev, static_cast<hipStream_t>(stream));
  return launched();
}

int gbl_level_q_load(int q, int rho_q, const double* table_dev, const double* b_dev, double* gq_dev, void* stream) {
  if (int st = check_level_q(q, rho_q)) return st;
  if (!table_dev || !b_dev || !gq_dev) return fail(nullptr, GBL_EINVAL, "table, b and gq must not be NULL");
  if (b_dev == gq_dev) return fail(nullptr, GBL_EINVAL, "b and gq must not overlap");
  launch_level_q_load(1 << q, rho_q, table_dev, b_dev, gq_dev, static_cast<hipStream_t>(stream));
  return launched();
}

int gbl_level_q_operator(int q, int rho_q, const double* a_dev, const double* table_dev, double* aq_dev,
                         void* stream) {
  if (int st = check_level_q(q, rho_q)) return st;
  if (!a_dev || !table_dev || !aq_dev) return fail(nullptr, GBL_EINVAL, "a, table and aq must not be NULL");
  launch_level_q_operator(1 << q, rho_q, a_dev, table_dev, aq_dev, static_cast<hipStream_t>(stream));
  return launched();
}

int gbl_level_q_to_nodal(int q, int rho_q, const double* table_dev, const double* U_dev, double* u_dev,
                         void* stream) {
  if (int st = check_level_q(q, rho_q)) return st;
  if (!table_dev || !U_dev || !u_dev) return fail(nullptr, GBL_EINVAL, "table, U and u must not be NULL");
  if (U_dev == u_dev) return fail(nullptr, GBL_EINVAL, "U and u must not overlap");
  launch_level_q_to_nodal(1 << q, rho_q, table_dev, U_dev, u_dev, static_cast<hipStream_t>(stream));
  return launched();
}

int gbl_destroy(gbl_ctx* c) {
  if (!c) return GBL_OK;
  release(c);
  return GBL_OK;
}

const char* gbl_last_error(const gbl_ctx* c) {
  if (c) return c->err.c_str();
  return g_last_error.c_str();
}

}  // extern "C"
