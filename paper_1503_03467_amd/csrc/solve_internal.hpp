// Solve-phase structures shared by the host driver and kernels_solve.hip.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>

#include "gamblet_internal.hpp"

namespace gbl {

// Outer (FP64) scalar slots.
constexpr int kSPW = 0;   // (p, A p)
constexpr int kSPR = 1;   // (p, r)
constexpr int kSPP = 2;   // (p, p)
constexpr int kSZZ = 3;   // (z, z)
constexpr int kSUU = 4;   // (u, u)
constexpr int kSZW = 5;   // (z, A p)
constexpr int kSRR = 6;   // (r, r)
constexpr int kSBB = 7;   // (b, b)
constexpr int kSIter = 8;    // outer iterations whose error estimate has been logged
constexpr int kSSpare = 9;   // unused slots
constexpr int kNumOuterScalars = 12;
constexpr int kDotBlocks = 1024;
constexpr int kUpdateBlocks = 256;   // blocks of the kernels that re-add block partials

// Per-level CG scalar slots.
constexpr int kCRZ = 0;
constexpr int kCPQ = 1;
constexpr int kCALPHA = 2;
constexpr int kCBETA = 3;
constexpr int kCRZD = 4;   // (r, D^-1 r) of a level with window corrections, before their part
constexpr int kNumCGScalars = 5;
// steps of k_cg_scalars (which partial sums it adds and which scalars it sets)
constexpr int kCGPhaseInit = 0;
constexpr int kCGPhaseSpmv = 1;
constexpr int kCGPhaseUpdate = 2;
constexpr int kCGPhaseWinInit = 3;
constexpr int kCGPhaseWin = 4;

template <typename T>
struct CGLev {
  const T* B;      // B^(k), offset-major
  const T* BJ;     // inverse 3x3 diagonal blocks
  const T* g;      // level-k right-hand side g^(k) (slots)
  T* x;            // w^(k)
  T* r;
  T* z;
  T* p;
  T* q;            // B p
  double* scal;    // kNumCGScalars
  double* part;    // one partial sum per block (added by k_cg_scalars)
  int np;          // parents per dimension (n_{k-1})
  int t;           // parent-stencil half-width
  int fine;        // k == q
  int iters;       // CG iteration budget of this level
  int blk0;        // first block of this level in the update/init grid (256 parents per block)
  int nblk;        // update/init blocks of this level
  int blk0s;       // first block of this level in the operator grid (64 parents per block)
  int nblks;       // operator blocks of this level
  // window corrections of the preconditioner (levels k < q; nwin = 0: none)
  const T* winv;   // [nwin][27][27] B_w^-1
  T* Y;            // [nwin][27] B_w^-1 r_w of the current iteration
  const int* wlist;   // window origins x0 * np + y0
  const int* widx;    // [np^2] slot of the window with that origin, or -1
  int nwin;
  int win0;        // first window of this level in the window grid
};

template <typename T>
struct CGArgs {
  CGLev<T> lv[kMaxLevels];
  int nlev;
};

// Several right-hand sides solved together.  Right-hand side z of a launch
// (blockIdx.z, z < m) works on the copy of the per-solve region of the
// workspace (vectors, scalars, partial sums, tickets) that sits zs bytes
// after the previous one; the hierarchy (operators, factors, windows) is
// shared.  Pointers that are null stay null.
struct Zb {
  int m = 1;
  size_t zs = 0;
};
template <typename P>
__device__ __forceinline__ P* zsh(P* p, size_t off) {
  return p ? reinterpret_cast<P*>(reinterpret_cast<char*>(p) + off) : p;
}
template <typename P>
__device__ __forceinline__ const P* zsh(const P* p, size_t off) {
  return p ? reinterpret_cast<const P*>(reinterpret_cast<const char*>(p) + off) : p;
}
template <typename T>
__device__ __forceinline__ CGLev<T> zlev(CGLev<T> L, size_t off) {
  L.g = zsh(L.g, off);
  L.x = zsh(L.x, off);
  L.r = zsh(L.r, off);
  L.z = zsh(L.z, off);
  L.p = zsh(L.p, off);
  L.q = zsh(L.q, off);
  L.scal = zsh(L.scal, off);
  L.part = zsh(L.part, off);
  L.Y = zsh(L.Y, off);
  return L;
}

// After the CG start (init) or CG iteration it: z += sum_w P_w^T B_w^-1 P_w r
// on the levels with kept windows, and their (r, z) / beta update.
template <typename T>
void launch_win_correct(const CGArgs<T>& a, int it, bool init, hipStream_t st, Zb zb = Zb());

// Finest subband level, conjugate gradients in the Chronopoulos-Gear form
// (one reduction and one launch per iteration).  r, w (= B u) and s (= B p)
// are double buffered because tiles read their neighbours' old values.
constexpr int kFGamma = 0;   // (r_i, u_i)
constexpr int kFAlpha = 1;
constexpr int kFBeta = 2;
constexpr int kNumFineScalars = 4;

template <typename T>
struct FineCG {
  const T* g;        // level-q right-hand side (slots)
  const T* acell;    // cell coefficient
  const T* BJ;       // inverse 3x3 parent blocks
  T* x;
  T* u;
  T* p;
  T* r[2];
  T* w[2];
  T* s[2];
  double* scal;
  double* part;
  int np;
  int nblk;          // tiles
};
template <typename T>
__device__ __forceinline__ FineCG<T> zfine(FineCG<T> F, size_t off) {
  F.g = zsh(F.g, off);
  F.x = zsh(F.x, off);
  F.u = zsh(F.u, off);
  F.p = zsh(F.p, off);
  for (int i = 0; i < 2; ++i) {
    F.r[i] = zsh(F.r[i], off);
    F.w[i] = zsh(F.w[i], off);
    F.s[i] = zsh(F.s[i], off);
  }
  F.scal = zsh(F.scal, off);
  F.part = zsh(F.part, off);
  return F;
}

// Chebyshev iteration for the subband systems (an alternative to CG with no
// inner products: the preconditioner it defines is a fixed polynomial in
// M B, so the outer iteration sees one linear operator).  With
// [lmin, lmax] = [G / kappa, G], G an upper bound of lambda_max(M B),
//   theta = (lmax + lmin) / 2, delta = (lmax - lmin) / 2, sigma = theta / delta,
//   d_0 = M r_0 / theta,  r_k = r_{k-1} - B d_{k-1},
//   rho_0 = 1 / sigma, rho_k = 1 / (2 sigma - rho_{k-1}),
//   d_k = rho_k rho_{k-1} d_{k-1} + (2 rho_k / delta) M r_k,
//   x = d_0 + ... + d_{K-1}.
constexpr int kMaxCheb = 32;   // largest K
struct ChebCoef {
  float c0;              // 1 / theta
  float ca[kMaxCheb];    // rho_k rho_{k-1}
  float cb[kMaxCheb];    // 2 rho_k / delta
};
// One step of the coarser levels: coefficients of step k for every level.
struct ChebStep {
  float ca[kMaxLevels];
  float cb[kMaxLevels];
  float c0[kMaxLevels];
};

template <typename T>
void launch_fine_cheb(const FineCG<T>& f, const ChebCoef& c, int K, int k0, int nsteps, int rd, hipStream_t st,
                      Zb zb = Zb());
// levels l0 .. l1-1 of the coarser subband systems (CGArgs order)
template <typename T>
void launch_cheb_init(const CGArgs<T>& a, const ChebStep& s, int l0, int l1, hipStream_t st, Zb zb = Zb());
template <typename T>
void launch_cheb_step(const CGArgs<T>& a, const ChebStep& s, int k, int l0, int l1, hipStream_t st, Zb zb = Zb());

template <typename T>
void launch_fine_cg(const FineCG<T>& f, int it, hipStream_t st, Zb zb = Zb());
// Level-q gamblets from the localized mass inverse: g^(q) = Minv^T r, and
// z = Minv v^(q) with the partial sums of launch_prolong_fine_dots.
template <typename T>
void launch_mass_load_slots(int n, int rho, const double* Y, const double* r, T* g, hipStream_t st);
template <typename T>
void launch_mass_nodal_dots(int n, int rho, const double* Y, const T* v, double* z, const double* uo,
                            const double* wo, double* part, hipStream_t st);
template <typename T>
void launch_prolong_fine_dots(const LevelGeom& L, const T* R, const T* vc, const FineCG<T>& F, double* z,
                              const double* uo, const double* wo, double* part, int cheb, hipStream_t st,
                              Zb zb = Zb());
template <typename T>
void launch_outer_update_convert(int len, const double* part, int nblk, double* sc, double* u, double* r,
                                 const double* p, const double* w, T* g, hipStream_t st, Zb zb = Zb());
void launch_apply_fine_dots(const double* a, int n, const double* p, const double* r, double* w, double* part,
                            hipStream_t st, Zb zb = Zb());

// Small levels handled inside one workgroup (restriction and prolongation
// chains).  Entry j is level k = kmin + j: R = R^(k-1,k), gf = level-k
// vector, gc = level-(k-1) vector, w = subband solution of level k.
template <typename T>
struct ChainLevel {
  const T* R;
  T* gf;
  T* gc;
  const T* w;
  int nk;
  int rho;
  int fine;
};

template <typename T>
struct ChainArgs {
  ChainLevel<T> lv[kMaxLevels];
  int n;   // levels 2 .. 2+n-1, ordered by increasing level for prolongation
  T* g1;   // level-1 vector (coarse solve in place)
};
template <typename T>
__device__ __forceinline__ ChainLevel<T> zchain(ChainLevel<T> L, size_t off) {
  L.gf = zsh(L.gf, off);
  L.gc = zsh(L.gc, off);
  L.w = zsh(L.w, off);
  return L;
}

template <typename T>
void launch_restrict_chain(const ChainArgs<T>& c, hipStream_t st, Zb zb = Zb());
template <typename T>
void launch_prolong_chain(const ChainArgs<T>& c, const double* L1, hipStream_t st, Zb zb = Zb());

template <typename T>
void launch_cg_scalars(const CGArgs<T>& a, int it, int phase, hipStream_t st, Zb zb = Zb());
template <typename T>
void launch_cg_init(const CGArgs<T>& a, int nblocks, hipStream_t st, Zb zb = Zb());
template <typename T>
void launch_cg_spmv(const CGArgs<T>& a, int nblocks, int it, hipStream_t st, Zb zb = Zb());
template <typename T>
void launch_cg_update(const CGArgs<T>& a, int nblocks, int it, hipStream_t st, Zb zb = Zb());
template <typename T>
void launch_zero(size_t len, T* x, hipStream_t st, Zb zb = Zb());
template <typename TD, typename TS>
void launch_convert(size_t len, const TS* s, TD* d, hipStream_t st, Zb zb = Zb());

template <typename T>
void launch_restrict(const LevelGeom& L, const T* R, const T* gf, T* gc, hipStream_t st, Zb zb = Zb());
template <typename T>
void launch_prolong(const LevelGeom& L, const T* R, const T* vc, const T* w, T* vf, bool fine,
                    hipStream_t st, Zb zb = Zb());

// src_stride / u_stride: doubles between the right-hand sides of the
// caller's source and nodal arrays
void launch_residual(const double* a, int n, int mode, const double* src, const double* u_nodal,
                     const double* u_slot, double* r, hipStream_t st, Zb zb = Zb(), size_t src_stride = 0,
                     size_t u_stride = 0);
void launch_apply_fine(const double* a, int n, const double* p, double* w, hipStream_t st);
void launch_dots(int len, int nv, const double* x0, const double* y0, const double* x1, const double* y1,
                 const double* x2, const double* y2, double* part, unsigned* cnt, double* out,
                 hipStream_t st, Zb zb = Zb());
void launch_outer_direction(int len, double* sc, const double* partz, int nblkz, const double* z, double* p,
                            double* elog, int first, hipStream_t st, Zb zb = Zb());
void launch_slots_to_nodal(int n, const double* s, double* u, hipStream_t st, Zb zb = Zb(), size_t u_stride = 0);
void launch_fill(size_t len, double v, double* x, hipStream_t st, Zb zb = Zb());
void launch_cell_gradient(const double* a, int n, const double* u, const double* lam, double* dloga,
                          double* dg, hipStream_t st);

}  // namespace gbl
