// Device reductions shared by the solve-phase kernel files.
#pragma once

#include <hip/hip_runtime.h>

namespace gbl {

// ---------------------------------------------------------------------------
// Reductions: block sum, then the last block to finish (atomic ticket) adds
// the per-block partials in a fixed order -- deterministic, no waiting.
// ---------------------------------------------------------------------------
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* sh) {
  // sh: NV * 8 doubles (one per wave of a 256-thread block... up to 16 waves)
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double x = v[k];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
    if (lane == 0) sh[k * 16 + wid] = x;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      double x = 0.0;
      for (int w = 0; w < nw; ++w) x += sh[k * 16 + w];
      v[k] = x;
    }
  }
  __syncthreads();
}

// Publish this block's partial sums; the last block to arrive (atomic
// ticket) then reduces all partials with every one of its threads, in a
// fixed order, and thread 0 receives the totals in out[] with *is_last set.
// Must be called by all threads of the block (it contains barriers).
template <int NV>
__device__ __forceinline__ void finish_reduction(const double (&v)[NV], double* part, int nblk, int blk,
                                                 unsigned* cnt, double* out, bool* is_last, double* sh) {
  __shared__ int last_flag;
  *is_last = false;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) part[k * nblk + blk] = v[k];
    __threadfence();
    const unsigned ticket = atomicAdd(cnt, 1u);
    last_flag = (ticket == (unsigned)(nblk - 1)) ? 1 : 0;
  }
  __syncthreads();
  if (last_flag) {
    __threadfence();
    const volatile double* vp = part;
    double acc[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      double x = 0.0;
      for (int b = threadIdx.x; b < nblk; b += blockDim.x) x += vp[k * nblk + b];
      acc[k] = x;
    }
    block_sum<NV>(acc, sh);
    if (threadIdx.x == 0) {
#pragma unroll
      for (int k = 0; k < NV; ++k) out[k] = acc[k];
      *cnt = 0u;
      *is_last = true;
    }
  }
}

// The same for the right-hand sides of a block solve at once: value k of this
// block goes to the partial array of right-hand side k (part0 + k * stride
// bytes), one atomic ticket on cnt elects the last block, and that block
// reduces every right-hand side's partials exactly as finish_reduction does
// for one (same loops, same order), so each total is bit-identical to the
// single-right-hand-side reduction.  Only the first nv values are used.
template <int NV>
__device__ __forceinline__ void finish_reduction_rhs(const double (&v)[NV], int nv, double* part0, size_t stride,
                                                     int nblk, int blk, unsigned* cnt, double (&out)[NV],
                                                     bool* is_last, double* sh) {
  __shared__ int last_flag;
  *is_last = false;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k)
      if (k < nv) reinterpret_cast<double*>(reinterpret_cast<char*>(part0) + k * stride)[blk] = v[k];
    __threadfence();
    const unsigned ticket = atomicAdd(cnt, 1u);
    last_flag = (ticket == (unsigned)(nblk - 1)) ? 1 : 0;
  }
  __syncthreads();
  if (last_flag) {
    __threadfence();
    double acc[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      double x = 0.0;
      if (k < nv) {
        const volatile double* vp =
            reinterpret_cast<const volatile double*>(reinterpret_cast<const char*>(part0) + k * stride);
        for (int b = threadIdx.x; b < nblk; b += blockDim.x) x += vp[b];
      }
      acc[k] = x;
    }
    block_sum<NV>(acc, sh);
    if (threadIdx.x == 0) {
#pragma unroll
      for (int k = 0; k < NV; ++k) out[k] = acc[k];
      *cnt = 0u;
      *is_last = true;
    }
  }
}

}  // namespace gbl
