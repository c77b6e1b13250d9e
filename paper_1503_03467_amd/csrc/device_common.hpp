// Device helpers shared by the kernel files: the subband matrices W^(k) of
// Construction 4.13 (rows of the normalised Helmert matrices of Lemma 4.12)
// and the averaging weights pibar (Section 4.7), per parent type.
#pragma once

#include <hip/hip_runtime.h>

namespace gbl {

// Parent types.  Away from the two low edges of level q-1 every parent has
// four children.  At level q-1 a parent with px = 0 keeps only its children
// with dx = 1 (child positions 2, 3), one with py = 0 only those with dy = 1
// (positions 1, 3), and the corner parent only position 3.
//   0: full, 1: px == 0, 2: py == 0, 3: corner.
__device__ __forceinline__ int parent_type(bool fine, int px, int py) {
  if (!fine) return 0;
  return (px == 0 ? 1 : 0) | (py == 0 ? 2 : 0);
}

// W rows (3 per parent, over the four child positions) and pibar weights.
// Helmert rows for m = 4: (1,-1,0,0)/sqrt2, (1,1,-2,0)/sqrt6, (1,1,1,-3)/sqrt12;
// for m = 2 over the two present children: (1,-1)/sqrt2.  Rows of parents with
// fewer children are zero (padding rows).
__device__ __forceinline__ double wcoef(int type, int t, int d) {
  constexpr double r2 = 0.70710678118654752440;
  constexpr double r6 = 0.40824829046386301637;
  constexpr double r12 = 0.28867513459481288225;
  if (type == 0) {
    if (t == 0) return d == 0 ? r2 : (d == 1 ? -r2 : 0.0);
    if (t == 1) return d < 2 ? r6 : (d == 2 ? -2.0 * r6 : 0.0);
    return d < 3 ? r12 : -3.0 * r12;
  }
  if (t != 0 || type == 3) return 0.0;
  if (type == 1) return d == 2 ? r2 : (d == 3 ? -r2 : 0.0);
  return d == 1 ? r2 : (d == 3 ? -r2 : 0.0);   // type 2
}

__device__ __forceinline__ double pibar(int type, int d) {
  if (type == 0) return 0.25;
  if (type == 3) return d == 3 ? 1.0 : 0.0;
  if (type == 1) return d >= 2 ? 0.5 : 0.0;
  return (d == 1 || d == 3) ? 0.5 : 0.0;   // type 2
}

// True for padding subband rows (parents with fewer than four children).
__device__ __forceinline__ bool is_pad_row(int type, int t) {
  if (type == 0) return false;
  if (type == 3) return true;
  return t != 0;
}

// Map a linear workgroup id so that consecutive logical ids run on the same
// XCD (workgroups are dispatched round-robin over the 8 XCDs, each with its
// own L2): neighbouring patches then share cached operator rows.
__device__ __forceinline__ int xcd_remap(int bid, int nblocks) {
  const int nx = 8;
  const int full = (nblocks / nx) * nx;
  if (bid >= full) return bid;
  const int per = full / nx;
  return (bid % nx) * per + bid / nx;
}

// Block-interleaved index of the subband operator B^(k): the (2t+1)^2 x 9
// entries of every group of 64 consecutive parents are contiguous, lanes
// (parents) fastest: B[p / 64][o][e][p % 64], o = ox (2t+1) + oy, e = 3i + j.
__device__ __forceinline__ size_t b_index(int o, int e, int p, int TT) {
  return ((size_t)(p >> 6) * (size_t)(TT * TT * 9) + (size_t)(o * 9 + e)) * 64 + (p & 63);
}

// Pivot of a patch factorisation whose matrix is scaled to a unit diagonal.
// In FP64 a pivot that is not positive is an error (bad is set).  In FP32 a
// pivot below kPivotFloor is the rounding of a Schur complement that lies
// under single-precision resolution (a patch straddling a coefficient jump of
// many orders of magnitude): it is raised to the floor and reg is set.  The
// patch solve is then perturbed, but every D gives a full-rank
// R = pibar + D W, so the hierarchy stays symmetric positive definite and the
// FP64 outer iteration absorbs the perturbation.
constexpr float kPivotFloor = 1e-6f;
template <typename T>
__device__ __forceinline__ T patch_pivot(T pv, int& bad, int& reg) {
  if (sizeof(T) == 4) {
    if (!(pv > T(kPivotFloor))) {
      reg = 1;
      return T(kPivotFloor);
    }
    return pv;
  }
  if (!(pv > T(0))) {
    bad = 1;
    return T(1);
  }
  return pv;
}

template <typename T>
__device__ __forceinline__ T my_sqrt(T x);
template <>
__device__ __forceinline__ double my_sqrt<double>(double x) { return sqrt(x); }
template <>
__device__ __forceinline__ float my_sqrt<float>(float x) { return sqrtf(x); }

}  // namespace gbl
