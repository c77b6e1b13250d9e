// Gamblet transform of a given level-q vector, its inverse, and the
// selection used to compress it: the representation of u in the basis
// psi^(1)_i / ||psi^(1)_i||_a, chi^(k)_j / ||chi^(k)_j||_a (discussion of
// Example 5.1, Figures 10-11).
//
// Measurements of level k-1 are sums of level-k measurements over the
// children (R^(k-1,k) pi^(k-1,k)T = I for every R = pibar + D W), so the
// level-(k-1) coefficients of u are U^(k-1) = pi U^(k), and the detail
// U^(k) - R^T U^(k-1) lies in the range of W^T: w^(k) = W (U^(k) - R^T U^(k-1))
// (the rows of W are orthonormal, Construction 4.13).  The inverse is the
// reconstruction of Theorem 4.15.  ||chi^(k)_j||_a^2 = B^(k)_jj and
// ||psi^(1)_i||_a^2 = A^(1)_ii scale the coefficients.  All arithmetic is
// FP64; the hierarchy operators are read in their stored precision.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "device_common.hpp"
#include "gamblet_internal.hpp"

namespace gbl {

// sum_i R_{i,(fx,fy)} v_i over the level-(k-1) rows whose restriction block
// covers level-k slot (fx, fy); rows outside the level are weighted by zero
template <typename T, int RHO>
__device__ __forceinline__ double rt_apply_r(const T* __restrict__ R, const double* __restrict__ vc, int nk, int fx,
                                             int fy) {
  const int nc = nk / 2;
  const size_t nc2 = (size_t)nc * nc;
  const int px = fx >> 1, py = fy >> 1;
  constexpr int rw = 2 * (2 * RHO + 1);
  double acc = 0.0;
#pragma unroll
  for (int dx = -RHO; dx <= RHO; ++dx) {
    const int ix = px + dx;
    const bool okx = ix >= 0 && ix < nc;
    const int ixc = min(max(ix, 0), nc - 1);
    const int bx = fx - 2 * (ixc - RHO);
#pragma unroll
    for (int dy = -RHO; dy <= RHO; ++dy) {
      const int iy = py + dy;
      const bool ok = okx && iy >= 0 && iy < nc;
      const int iyc = min(max(iy, 0), nc - 1);
      const int by = fy - 2 * (iyc - RHO);
      const int bxc = min(max(bx, 0), rw - 1), byc = min(max(by, 0), rw - 1);
      const int i = ixc * nc + iyc;
      acc += (double)R[(size_t)(bxc * rw + byc) * nc2 + i] * (vc[i] * (ok ? 1.0 : 0.0));
    }
  }
  return acc;
}

template <typename T>
__device__ __forceinline__ double rt_apply(const T* __restrict__ R, const double* __restrict__ vc, int nk, int rho,
                                           int fx, int fy) {
  switch (rho) {
    case 1: return rt_apply_r<T, 1>(R, vc, nk, fx, fy);
    case 2: return rt_apply_r<T, 2>(R, vc, nk, fx, fy);
    case 3: return rt_apply_r<T, 3>(R, vc, nk, fx, fy);
    case 4: return rt_apply_r<T, 4>(R, vc, nk, fx, fy);
    default: return rt_apply_r<T, 5>(R, vc, nk, fx, fy);
  }
}

// level-q slots from nodal values: slot (x, y) is node (x, y); the slots of
// row or column 0 are boundary nodes, not unknowns, and hold zero
__global__ void k_nodal_to_slots(int n, const double* __restrict__ u, double* __restrict__ s) {
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= n * n) return;
  const int x = id / n, y = id % n;
  s[id] = (x == 0 || y == 0) ? 0.0 : u[x * (n + 1) + y];
}

// interior nodes from level-q slots; boundary nodes are set to zero
__global__ void k_slots_to_nodal_all(int n, const double* __restrict__ s, double* __restrict__ u) {
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  const int m = n + 1;
  if (id >= m * m) return;
  const int x = id / m, y = id % m;
  u[id] = (x == 0 || y == 0 || x == n || y == n) ? 0.0 : s[x * n + y];
}

// U^(k-1) = pi U^(k): each parent sums its four child slots
__global__ void k_child_sum(int nc, const double* __restrict__ f, double* __restrict__ c) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nc * nc) return;
  const int px = p / nc, py = p % nc, nk = 2 * nc;
  const double* r0 = f + (size_t)(2 * px) * nk + 2 * py;
  c[p] = (r0[0] + r0[1]) + (r0[nk] + r0[nk + 1]);
}

// detail of every level-k slot, in place: f = U^(k) - R^T U^(k-1) (U^(k) is
// no longer needed once the child sums are formed)
template <typename T>
__global__ void k_detail_slots(const T* __restrict__ R, const double* __restrict__ c, double* __restrict__ f, int nk,
                               int rho) {
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= nk * nk) return;
  const int fx = id / nk, fy = id % nk;
  f[id] -= rt_apply<T>(R, c, nk, rho, fx, fy);
}

// level-k normalized coefficients of one parent: w = W (detail of its four
// children), times sqrt(B^(k)_jj); padding rows are zero
template <typename T>
__global__ void k_detail(const T* __restrict__ B, const double* __restrict__ f, double* __restrict__ out, int nk,
                         int t, int fine) {
  const int np = nk / 2;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= np * np) return;
  const int px = p / np, py = p % np;
  const int tp = parent_type(fine != 0, px, py);
  double r[4];
#pragma unroll
  for (int d = 0; d < 4; ++d) r[d] = f[(size_t)(2 * px + (d >> 1)) * nk + 2 * py + (d & 1)];
  const int TT = 2 * t + 1;
  const size_t np2 = (size_t)np * np;
#pragma unroll
  for (int tt = 0; tt < 3; ++tt) {
    double w = 0.0;
#pragma unroll
    for (int d = 0; d < 4; ++d) w += wcoef(tp, tt, d) * r[d];
    const double bd = is_pad_row(tp, tt) ? 0.0 : (double)B[b_index(t * TT + t, 4 * tt, p, TT)];
    out[tt * np2 + p] = bd > 0.0 ? w * sqrt(bd) : 0.0;
  }
}

// level 1: c = U sqrt(A^(1)_ii) (forward) or U = c / sqrt(A^(1)_ii) (inverse)
template <typename T>
__global__ void k_level1(const T* __restrict__ A1, int s1, const double* __restrict__ in, double* __restrict__ out,
                         int inverse) {
  const int i = threadIdx.x;
  if (i >= 4) return;
  const int S1 = 2 * s1 + 1;
  const double d = (double)A1[(size_t)(s1 * S1 + s1) * 4 + i];
  const double sc = d > 0.0 ? sqrt(d) : 0.0;
  out[i] = inverse ? (sc > 0.0 ? in[i] / sc : 0.0) : in[i] * sc;
}

// v^(k) = R^(k,k-1) v^(k-1) + W^(k)T w^(k), w from the normalized coefficients
template <typename T>
__global__ void k_recon(const T* __restrict__ R, const T* __restrict__ B, const double* __restrict__ vc,
                        const double* __restrict__ cf, double* __restrict__ vf, int nk, int rho, int t, int fine) {
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= nk * nk) return;
  const int fx = id / nk, fy = id % nk;
  const int np = nk / 2;
  double acc = rt_apply<T>(R, vc, nk, rho, fx, fy);
  const int px = fx >> 1, py = fy >> 1;
  const int d = 2 * (fx & 1) + (fy & 1);
  const int tp = parent_type(fine != 0, px, py);
  const int p = px * np + py;
  const int TT = 2 * t + 1;
  const size_t np2 = (size_t)np * np;
#pragma unroll
  for (int tt = 0; tt < 3; ++tt) {
    if (is_pad_row(tp, tt)) continue;
    const double bd = (double)B[b_index(t * TT + t, 4 * tt, p, TT)];
    if (bd > 0.0) acc += wcoef(tp, tt, d) * (cf[tt * np2 + p] / sqrt(bd));
  }
  vf[id] = acc;
}

// The keep-th largest |c| (1 <= keep <= n): the largest tau with
// count(|c| >= tau) >= keep.  Non-negative doubles order like their bit
// patterns, so tau is found digit by digit on the 63-bit pattern of |c|, from
// the top (radix selection): for each digit a histogram of the entries that
// agree with the digits fixed so far, built by many workgroups (LDS counts,
// then one global atomic per non-empty bin), then one workgroup walks the bins
// from the top and fixes the digit at which the running count reaches the
// rank still needed.  NaN entries are never counted; if fewer than keep
// entries are numbers, tau = 0 (every number is kept).
//
// Selection state: st[0] digits fixed so far, st[1] rank still needed within
// them, st[2] set when no bin reaches that rank; then hist[kSelBins].
constexpr int kSelBins = kSelHistBins;
constexpr unsigned long long kAbsMask = 0x7FFFFFFFFFFFFFFFull;
constexpr unsigned long long kInfBits = 0x7FF0000000000000ull;

__global__ void k_sel_init(unsigned long long* __restrict__ st, unsigned* __restrict__ hist, long keep) {
  for (int b = threadIdx.x; b < kSelBins; b += blockDim.x) hist[b] = 0u;
  if (threadIdx.x == 0) {
    st[0] = 0ull;
    st[1] = (unsigned long long)keep;
    st[2] = 0ull;
  }
}

__global__ __launch_bounds__(256) void k_sel_hist(const double* __restrict__ c, long n, int shift, int width,
                                                  const unsigned long long* __restrict__ st,
                                                  unsigned* __restrict__ hist) {
  __shared__ unsigned h[kSelBins];
  const int nb = 1 << width;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) h[b] = 0u;
  __syncthreads();
  const int top = shift + width;   // <= 63
  const unsigned long long want = st[0] >> top;
  const unsigned mask = (unsigned)nb - 1u;
  const long stride = (long)gridDim.x * blockDim.x;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const unsigned long long key = (unsigned long long)__double_as_longlong(c[i]) & kAbsMask;
    if (key <= kInfBits && (key >> top) == want) atomicAdd(&h[(unsigned)(key >> shift) & mask], 1u);
  }
  __syncthreads();
  for (int b = threadIdx.x; b < nb; b += blockDim.x)
    if (h[b]) atomicAdd(&hist[b], h[b]);
}

// 256 threads; thread t holds bins nb-1-per*t ... (descending), so the
// exclusive scan of the per-thread sums gives every bin's count of entries in
// higher bins.  The histogram is cleared for the next digit.
__global__ __launch_bounds__(256) void k_sel_pick(unsigned long long* __restrict__ st, unsigned* __restrict__ hist,
                                                  int shift, int width, int last, double* __restrict__ thr) {
  __shared__ unsigned long long wsum[4];
  __shared__ unsigned long long pick[2];   // bin found, rank still needed within it
  __shared__ int found;
  const int nb = 1 << width;
  const int per = nb / 256;   // 8 or 4
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  if (tid == 0) found = 0;
  unsigned cnt[8];
  unsigned long long mine = 0;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    cnt[j] = j < per ? hist[nb - 1 - (tid * per + j)] : 0u;
    mine += cnt[j];
  }
  // inclusive scan over the wavefront, then over the four wavefronts
  unsigned long long incl = mine;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const unsigned long long v = __shfl_up(incl, off, 64);
    if (lane >= off) incl += v;
  }
  if (lane == 63) wsum[wv] = incl;
  __syncthreads();
  unsigned long long before = incl - mine;
  for (int w = 0; w < wv; ++w) before += wsum[w];
  const unsigned long long need = st[1];
  if (st[2] == 0ull && before < need && before + mine >= need) {
    unsigned long long run = before;
    for (int j = 0; j < per; ++j) {
      if (run + cnt[j] >= need) {
        pick[0] = (unsigned long long)(nb - 1 - (tid * per + j));
        pick[1] = need - run;
        found = 1;
        break;
      }
      run += cnt[j];
    }
  }
#pragma unroll
  for (int j = 0; j < 8; ++j)
    if (j < per) hist[nb - 1 - (tid * per + j)] = 0u;
  __syncthreads();
  if (tid == 0) {
    // no bin reaches the rank: fewer numbers than keep (first digit only)
    unsigned long long failed = st[2];
    unsigned long long prefix = st[0];
    if (!failed && found) {
      prefix |= pick[0] << shift;
      st[0] = prefix;
      st[1] = pick[1];
    } else {
      failed = 1ull;
      st[2] = 1ull;
    }
    if (last) *thr = failed ? 0.0 : __longlong_as_double((long long)prefix);
  }
}

__global__ void k_zero_below(const double* __restrict__ thr, long n, double* __restrict__ c) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double t = *thr;
  if (!(fabs(c[i]) >= t)) c[i] = 0.0;
}

template <typename T>
void launch_transform(const TransformArgs& a, const double* u_nodal, double* coef, hipStream_t st) {
  const int q = a.q;
  const int nq = a.n;
  hipLaunchKernelGGL(k_nodal_to_slots, dim3((nq * nq + 255) / 256), dim3(256), 0, st, nq, u_nodal, a.U[q]);
  for (int k = q; k >= 2; --k) {
    const LevelGeom& g = a.lv[k];
    const int nc = g.nk / 2;
    hipLaunchKernelGGL(k_child_sum, dim3((nc * nc + 255) / 256), dim3(256), 0, st, nc, a.U[k], a.U[k - 1]);
    double* out = coef + (size_t)nc * nc;   // level k starts at 4^(k-1) = (nk/2)^2
    hipLaunchKernelGGL((k_detail_slots<T>), dim3((g.nk * g.nk + 255) / 256), dim3(256), 0, st,
                       static_cast<const T*>(a.R[k]), a.U[k - 1], a.U[k], g.nk, g.rho);
    hipLaunchKernelGGL((k_detail<T>), dim3((nc * nc + 255) / 256), dim3(256), 0, st, static_cast<const T*>(a.B[k]),
                       a.U[k], out, g.nk, g.t, k == q ? 1 : 0);
  }
  hipLaunchKernelGGL((k_level1<T>), dim3(1), dim3(64), 0, st, static_cast<const T*>(a.A1), a.lv[1].s, a.U[1], coef, 0);
}

template <typename T>
void launch_inverse_transform(const TransformArgs& a, const double* coef, double* u_nodal, hipStream_t st) {
  const int q = a.q;
  hipLaunchKernelGGL((k_level1<T>), dim3(1), dim3(64), 0, st, static_cast<const T*>(a.A1), a.lv[1].s, coef, a.U[1], 1);
  for (int k = 2; k <= q; ++k) {
    const LevelGeom& g = a.lv[k];
    const int nc = g.nk / 2;
    const double* cf = coef + (size_t)nc * nc;
    hipLaunchKernelGGL((k_recon<T>), dim3((g.nk * g.nk + 255) / 256), dim3(256), 0, st, static_cast<const T*>(a.R[k]),
                       static_cast<const T*>(a.B[k]), a.U[k - 1], cf, a.U[k], g.nk, g.rho, g.t, k == q ? 1 : 0);
  }
  const int m = a.n + 1;
  hipLaunchKernelGGL(k_slots_to_nodal_all, dim3((m * m + 255) / 256), dim3(256), 0, st, a.n, a.U[q], u_nodal);
}

void launch_select_threshold(const double* c, long n, long keep, unsigned long long* state, unsigned* hist,
                             double* thr, hipStream_t st) {
  // digits of the 63-bit pattern, top first: 11 (exponent), 11, 11, 10, 10, 10
  static const int kShift[6] = {52, 41, 30, 20, 10, 0};
  static const int kWidth[6] = {11, 11, 11, 10, 10, 10};
  const long per_block = 256L * 4;
  const unsigned grid = (unsigned)std::max(1L, std::min(1024L, (n + per_block - 1) / per_block));
  hipLaunchKernelGGL(k_sel_init, dim3(1), dim3(256), 0, st, state, hist, keep);
  for (int d = 0; d < 6; ++d) {
    hipLaunchKernelGGL(k_sel_hist, dim3(grid), dim3(256), 0, st, c, n, kShift[d], kWidth[d], state, hist);
    hipLaunchKernelGGL(k_sel_pick, dim3(1), dim3(256), 0, st, state, hist, kShift[d], kWidth[d], d == 5 ? 1 : 0, thr);
  }
}

void launch_zero_below(const double* thr, long n, double* c, hipStream_t st) {
  hipLaunchKernelGGL(k_zero_below, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, thr, n, c);
}

void launch_nodal_to_slots(int n, const double* u_nodal, double* s, hipStream_t st) {
  hipLaunchKernelGGL(k_nodal_to_slots, dim3((n * n + 255) / 256), dim3(256), 0, st, n, u_nodal, s);
}

template void launch_transform<float>(const TransformArgs&, const double*, double*, hipStream_t);
template void launch_transform<double>(const TransformArgs&, const double*, double*, hipStream_t);
template void launch_inverse_transform<float>(const TransformArgs&, const double*, double*, hipStream_t);
template void launch_inverse_transform<double>(const TransformArgs&, const double*, double*, hipStream_t);

}  // namespace gbl
