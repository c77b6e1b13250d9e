// Internal declarations shared by the host driver and the kernel files.
//
// Geometry used by every kernel ("slot" layout).  The fine mesh has n = 2^q
// cells per dimension.  Level k (1 <= k <= q) is a square grid of nk = 2^k
// slots, index x*nk + y.  For k < q a slot is a dyadic cell of side 2^-k;
// for k = q slot (x, y) is the mesh node (x, y) and slots with x = 0 or
// y = 0 carry no unknown (they are boundary nodes).  The parent of slot
// (x, y) of level k is slot (x/2, y/2) of level k-1, its child position is
// t = 2 (x mod 2) + (y mod 2) (nested aggregation, Construction 4.2, with the
// nodal measurements at level q allowed in the discussion of Algorithm 1).
//
// Subband unknowns of level k (Lemma 4.9) are stored three per parent,
// index 3 * parent + t, t = 0..2; for parents of level q-1 that have fewer
// than four children the missing rows are padded with identity rows (zero
// right-hand side), which leaves every result unchanged.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

#include "../../include/gamblet.h"

namespace gbl {

constexpr int kMaxLevels = 13;     // q <= 12
constexpr int kMaxRho = 5;         // the finest transition; below it at most kMaxRhoCoarse
constexpr int kMaxRhoCoarse = 4;
constexpr int kMaxRhoQ = 4;   // patch radius of the localized mass inverse
// zero words before and after every level slot vector g^(k)
constexpr int kGPad = 16;
static_assert(kGPad >= 2 * kMaxRho, "the restriction reads 2 rho words beyond the slot vector");

// Device status bits (or-ed into the workspace status word).
constexpr int kBadCoefficient = 1;
constexpr int kBadPivot = 2;
constexpr int kBadInput = 4;
constexpr int kRegularizedPivot = 8;   // FP32 patch or coarse pivots raised to the floor (not an error)
constexpr int kWindowOverflow = 16;    // more kept windows than their arrays hold

struct LevelGeom {
  int k = 0;       // level
  int nk = 0;      // side (slots)
  int s = 0;       // A^(k) stencil half-width
  int t = 0;       // B^(k) parent-stencil half-width (k >= 2)
  int rho = 0;     // effective patch radius for the patches of level k-1 (k >= 2)
  int rw = 0;      // R^(k-1,k) block width 2(2 rho + 1) (k >= 2)
  size_t offA = 0, offB = 0, offR = 0, offBJ = 0;   // element offsets into the hierarchy arena
  size_t nA = 0, nB = 0, nR = 0, nBJ = 0;            // element counts
  int nparent() const { return (nk / 2) * (nk / 2); }
  int nsub() const { return 3 * nparent(); }
};

// Launchers (defined in kernels_*.hip), templated on the hierarchy scalar T.
template <typename T>
void launch_assemble_fine(const double* a, T* A, int n, int* status, hipStream_t st);
template <typename T>
void launch_subband_operator(const LevelGeom& L, const T* A, T* B, T* BJ, bool fine, hipStream_t st);
// Bound of lambda_max(M B^(k)) (block Gershgorin); scratch holds 6 np^2 T values.
template <typename T>
void launch_gershgorin(const LevelGeom& L, const T* B, T* scratch, unsigned* out, hipStream_t st);
// Bp: scratch of TT^2 * 9 * (nk/2)^2 T values for a parent-major copy of B^(k)
// (read by the matrix-core kernel's patch gather).
// variant (a build-kernel choice, kVariantDefault: the built-in rule): for
// the dense patch solves 0 = register-tiled, 1 = matrix cores; for the band
// patch solves of level q 0 = LDS band, 1 = register band (two patches per
// wavefront); for the Galerkin product 0 = one workgroup per coarse row,
// 1 = strips of coarse rows.
constexpr int kVariantDefault = -1;
enum BuildKernelClass { kKernelPatch = 0, kKernelBand = 1, kKernelGalerkin = 2 };
// candidates of a class at this level (0 when the class does not run here)
int patch_class(const LevelGeom& L, bool fine);   // kKernelPatch or kKernelBand
template <typename T>
bool patch_variant_ok(const LevelGeom& L, bool fine, int variant);
template <typename T>
bool galerkin_variant_ok(const LevelGeom& L, const LevelGeom& C, int variant);
template <typename T>
void launch_patch_solve(const LevelGeom& L, const T* A, const T* B, T* R, T* Bp, bool fine, int* status,
                        hipStream_t st, int variant = kVariantDefault);
template <typename T>
void launch_galerkin(const LevelGeom& L, const LevelGeom& C, const T* A, const T* R, T* Ac,
                     hipStream_t st, int variant = kVariantDefault);
// Window corrections of the subband preconditioner (kernels_window.hip):
// for every 3 x 3 group of parents of level k < q, B_w^-1 is kept when
// tr(D_w B_w^-1) > tol (D_w the 3 x 3 parent blocks of B_w).  cap windows fit
// in wlist / winv; widx has one slot index (or -1) per parent position.
template <typename T>
void launch_win_build(const LevelGeom& g, const T* B, double tol, int cap, int* wlist, int* widx, T* winv,
                      unsigned* count, int* status, hipStream_t st);
template <typename T>
void launch_coarse_factor(const T* A1, int s1, double* L1, int* status, hipStream_t st);

// Solve-phase launchers (declared with their batching argument in solve_internal.hpp).
template <typename T>
void launch_coarse_solve(const double* L1, const T* g1, T* v1, hipStream_t st);

// Gamblet transform of a level-q vector and its inverse (kernels_transform.hip).
// Level k's normalized coefficients sit at offset 4^(k-1) of the coefficient
// vector (level 1: 4 values by slot; level k >= 2: 3 (nk/2)^2 values, entry
// t (nk/2)^2 + parent, zero on padding rows); 4^q values in all.
struct TransformArgs {
  int q = 0;
  int n = 0;                        // cells per dimension (2^q)
  LevelGeom lv[kMaxLevels];
  const void* A1 = nullptr;         // A^(1) stencil (hierarchy scalar)
  const void* R[kMaxLevels] = {};   // R^(k-1,k), k >= 2
  const void* B[kMaxLevels] = {};   // B^(k), k >= 2
  double* U[kMaxLevels] = {};       // FP64 level vectors, nk^2 slots each
};
template <typename T>
void launch_transform(const TransformArgs& a, const double* u_nodal, double* coef, hipStream_t st);
template <typename T>
void launch_inverse_transform(const TransformArgs& a, const double* coef, double* u_nodal, hipStream_t st);
// threshold = the keep-th largest |c| (keep >= 1), written to *thr on the device
// Selection state for launch_select_threshold: 4 words of 64 bits, then
// kSelHistBins counters of 32 bits (caller-provided device memory).
constexpr int kSelHistBins = 2048;
void launch_select_threshold(const double* c, long n, long keep, unsigned long long* state, unsigned* hist,
                             double* thr, hipStream_t st);
void launch_zero_below(const double* thr, long n, double* c, hipStream_t st);
void launch_nodal_to_slots(int n, const double* u_nodal, double* s, hipStream_t st);

// Level-q gamblets from the localized mass inverse (kernels_level_q.hip).
// n = 2^q cells per side; vectors over the (n-1)^2 interior nodes; Y is the
// [(n-1)][2 rho + 1] table of one-dimensional factors.
void launch_mass_inverse_table(int n, int rho, double* Y, hipStream_t st);
void launch_level_q_weights(int n, int rho, const double* Y, double* W, hipStream_t st);
void launch_level_q_load(int n, int rho, const double* Y, const double* b, double* gq, hipStream_t st);
void launch_level_q_to_nodal(int n, int rho, const double* Y, const double* U, double* u, hipStream_t st);
void launch_level_q_operator(int n, int rho, const double* a, const double* Y, double* AQ, hipStream_t st);
// the same operator into the hierarchy's level-q stencil (offset-major, half
// width 2 rho + 1, slots shifted by one), after a check of the coefficient
template <typename T>
void launch_level_q_operator_arena(int n, int rho, const double* a, const double* Y, T* A, int* status,
                                   hipStream_t st);

}  // namespace gbl
