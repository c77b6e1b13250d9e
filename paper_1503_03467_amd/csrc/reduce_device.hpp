// Device reductions shared by the solve-phase kernel files.
#pragma once

#include <hip/hip_runtime.h>

namespace gbl {

// ---------------------------------------------------------------------------
// Reductions: block sum, then the per-block partials are added in a fixed
// order -- deterministic, no waiting.  Either the last block to finish adds
// them (atomic ticket; each block then pays an agent-scope release fence,
// which writes back its XCD's L2, so this is kept for small grids), or the
// kernel only stores its partials and a one-workgroup step adds them.
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

// Partial sums only (no ticket): thread 0 stores this block's sums (after
// block_sum); a later kernel adds them in block order.
template <int NV>
__device__ __forceinline__ void write_partials(const double (&v)[NV], double* part, int nblk, int blk) {
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) part[k * nblk + blk] = v[k];
  }
}

// Total of nblk per-block partial sums by one workgroup, in the order the
// last block of finish_reduction uses (thread b adds partials b, b +
// blockDim.x, ... in turn, then the block sum), so for the same block size a
// reduction split into a partial-writing kernel and this step gives the same
// bits as the ticketed one.  Thread 0 receives the totals.  Sum k of block b sits at
// part[k * nblk + b].  Must be called by all threads of the block.
template <int NV>
__device__ __forceinline__ void total_partials(const double* __restrict__ part, int nblk, double (&out)[NV],
                                               double* sh) {
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double x = 0.0;
    for (int b = threadIdx.x; b < nblk; b += blockDim.x) x += part[k * nblk + b];
    out[k] = x;
  }
  block_sum<NV>(out, sh);
}

}  // namespace gbl
