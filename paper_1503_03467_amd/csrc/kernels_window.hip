// Window corrections of the subband preconditioner (levels k < q).
//
// The subband systems B^(k) w = W g^(k) (Section 4.7) are solved inexactly
// with block-Jacobi preconditioning (the 3 x 3 block of every parent).  The
// bound on the condition number of B^(k) grows with the contrast of the
// coefficient (Section 4.8), and with inclusions of very high coefficient
// that contrast shows up as a few localized modes: an inclusion that spans
// several parents of level k-1 but contains none of them can move almost
// rigidly at the cost of the surrounding low coefficient, while every parent
// block on its own sees the high coefficient.  Such a mode has a tiny
// Rayleigh quotient relative to the block-Jacobi preconditioner.
//
// A window is a 3 x 3 group of parents (27 subband unknowns).  At build time
// every window's principal submatrix B_w is factorized in FP64 and the
// indicator tr(D_w B_w^-1) is formed, D_w the block diagonal of B_w: it lies
// between 1/lambda_min and 27/lambda_min of the pencil (B_w, D_w), so it is
// large exactly when the window holds such a mode.  Windows whose indicator
// exceeds a threshold keep B_w^-1; the preconditioner becomes the additive
// Schwarz operator M^-1 = D^-1 + sum_w P_w^T B_w^-1 P_w, still symmetric
// positive definite, used inside conjugate gradients.
//
// Layout (per level, in the workspace): wlist[cap] window origins
// (x0 * np + y0), widx[np^2] slot of the window with that origin or -1,
// winv[cap][27][27] (column j of B_w^-1 at [j][0..26], i fastest) and the
// apply buffer Y[cap][27].  Local unknown i of a window is
// (3 dx + dy) * 3 + t for parent (x0 + dx, y0 + dy) and subband index t.
#include <hip/hip_runtime.h>

#include "device_common.hpp"
#include "gamblet_internal.hpp"
#include "solve_internal.hpp"
#include "reduce_device.hpp"

namespace gbl {

constexpr int kWinN = 27;
constexpr int kWinLd = 28;   // LDS row stride of the window matrix (doubles)

// One wavefront per window origin, four windows per 256-thread workgroup.
template <typename T>
__global__ __launch_bounds__(256) void k_win_build(const T* __restrict__ B, int np, int t, double tol, int cap,
                                                   int* __restrict__ wlist, int* __restrict__ widx,
                                                   T* __restrict__ winv, unsigned* __restrict__ count,
                                                   int* __restrict__ status) {
  __shared__ double sm[4][kWinN * kWinLd];
  __shared__ int bad[4];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int nw = np - 2;   // origins per dimension
  const int w = blockIdx.x * 4 + wv;
  const bool live = w < nw * nw;
  const int x0 = live ? w / nw : 0, y0 = live ? w % nw : 0;
  const int TT = 2 * t + 1;
  double* M = sm[wv];
  if (lane == 0) bad[wv] = 0;
  // gather B_w (entries coupling parents more than t apart are zero)
  for (int e = lane; e < kWinN * kWinN; e += 64) {
    const int i = e / kWinN, j = e % kWinN;
    const int pi = i / 3, ti = i % 3, pj = j / 3, tj = j % 3;
    const int ox = pj / 3 - pi / 3, oy = pj % 3 - pi % 3;
    double v = 0.0;
    if (live && ox >= -t && ox <= t && oy >= -t && oy <= t) {
      const int p = (x0 + pi / 3) * np + (y0 + pi % 3);
      v = (double)B[b_index((ox + t) * TT + (oy + t), 3 * ti + tj, p, TT)];
    }
    M[i * kWinLd + j] = v;
  }
  __syncthreads();
  // block-diagonal entries of column j (lane j), kept for the indicator
  double dcol[3] = {0.0, 0.0, 0.0};
  if (lane < kWinN) {
    const int b0 = (lane / 3) * 3;
#pragma unroll
    for (int a = 0; a < 3; ++a) dcol[a] = M[(b0 + a) * kWinLd + lane];
  }
  __syncthreads();
  // Cholesky, lower triangle in place
  for (int c = 0; c < kWinN; ++c) {
    const double d = M[c * kWinLd + c];
    __syncthreads();
    if (!(d > 0.0)) {
      if (lane == 0) bad[wv] = 1;
    }
    const double s = (d > 0.0) ? sqrt(d) : 1.0;
    if (lane >= c && lane < kWinN) M[lane * kWinLd + c] = (lane == c) ? s : M[lane * kWinLd + c] / s;
    __syncthreads();
    const int m = kWinN - 1 - c;
    for (int e = lane; e < m * m; e += 64) {
      const int i = c + 1 + e / m, j = c + 1 + e % m;
      if (j <= i) M[i * kWinLd + j] -= M[i * kWinLd + c] * M[j * kWinLd + c];
    }
    __syncthreads();
  }
  // column j of B_w^-1 by a forward and a backward substitution (lane j)
  double x[kWinN];
#pragma unroll
  for (int i = 0; i < kWinN; ++i) x[i] = (i == lane) ? 1.0 : 0.0;
#pragma unroll
  for (int i = 0; i < kWinN; ++i) {
    double v = x[i];
#pragma unroll
    for (int k = 0; k < i; ++k) v -= M[i * kWinLd + k] * x[k];
    x[i] = v / M[i * kWinLd + i];
  }
#pragma unroll
  for (int i = kWinN - 1; i >= 0; --i) {
    double v = x[i];
#pragma unroll
    for (int k = i + 1; k < kWinN; ++k) v -= M[k * kWinLd + i] * x[k];
    x[i] = v / M[i * kWinLd + i];
  }
  // indicator tr(D_w B_w^-1) = sum_j sum_{i in block(j)} D_ij (B_w^-1)_ij
  double tr = 0.0;
  if (lane < kWinN) {
    const int b0 = (lane / 3) * 3;
#pragma unroll
    for (int i = 0; i < kWinN; ++i)
      if (i >= b0 && i < b0 + 3) tr += dcol[i - b0] * x[i];
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) tr += __shfl_xor(tr, off, 64);
  const bool flag = live && !bad[wv] && tr > tol;
  int slot = -1;
  if (flag && lane == 0) slot = (int)atomicAdd(count, 1u);
  slot = __shfl(slot, 0, 64);
  if (flag && slot >= cap) {
    if (lane == 0) atomicOr(status, kWindowOverflow);
    slot = -1;
  }
  if (live && lane == 0) widx[x0 * np + y0] = slot;
  if (slot >= 0) {
    if (lane == 0) wlist[slot] = x0 * np + y0;
    if (lane < kWinN) {
      T* out = winv + (size_t)slot * kWinN * kWinN + (size_t)lane * kWinN;
#pragma unroll
      for (int i = 0; i < kWinN; ++i) out[i] = (T)x[i];
    }
  }
}

template <typename T>
void launch_win_build(const LevelGeom& g, const T* B, double tol, int cap, int* wlist, int* widx, T* winv,
                      unsigned* count, int* status, hipStream_t st) {
  const int np = g.nk / 2;
  if (np < 3) return;
  const int nwin = (np - 2) * (np - 2);
  hipLaunchKernelGGL(k_win_build<T>, dim3((nwin + 3) / 4), dim3(256), 0, st, B, np, g.t, tol, cap, wlist, widx,
                     winv, count, status);
}

// Y_w = B_w^-1 r_w for every kept window of the windowed levels (one
// wavefront per window; the level of a block from its window range).
template <typename T>
__global__ __launch_bounds__(256) void k_win_apply(CGArgs<T> args, int it, size_t zs) {
  __shared__ T rs[4][32];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int gw = blockIdx.x * 4 + wv;
  int l = 0;
  while (l + 1 < args.nlev && gw >= args.lv[l + 1].win0) ++l;
  const CGLev<T> L = zlev(args.lv[l], blockIdx.z * zs);
  const int w = gw - L.win0;
  const bool live = (it < L.iters - 1) && w >= 0 && w < L.nwin;
  const int np = L.np;
  const size_t np2 = (size_t)np * np;
  int o = 0;
  if (live) o = L.wlist[w];
  const int x0 = o / np, y0 = o - (o / np) * np;
  if (live && lane < kWinN) {
    const int pl = lane / 3, tl = lane % 3;
    rs[wv][lane] = L.r[tl * np2 + (size_t)(x0 + pl / 3) * np + (y0 + pl % 3)];
  }
  __syncthreads();
  if (live && lane < kWinN) {
    const T* col = L.winv + (size_t)w * kWinN * kWinN + lane;
    T acc = T(0);
#pragma unroll
    for (int j = 0; j < kWinN; ++j) acc += col[(size_t)j * kWinN] * rs[wv][j];
    L.Y[(size_t)w * kWinN + lane] = acc;
  }
}

// z += sum over the kept windows containing the parent of their Y entries
// (a fixed order: origins by dx, then dy), and the per-block partials of
// (r, sum); the scalar step then forms (r, z) = (r, D^-1 r) (left in kCRZD
// by the CG kernel) + (r, sum).
template <typename T>
__global__ __launch_bounds__(256) void k_win_gather(CGLev<T> L0, int it, int init, size_t zs) {
  __shared__ double sh[16];
  const CGLev<T> L = zlev(L0, blockIdx.z * zs);
  if (!init && it >= L.iters - 1) return;
  const int blk = blockIdx.x;
  const int p = blk * 256 + threadIdx.x;
  const int np = L.np;
  const size_t np2 = (size_t)np * np;
  double v[1] = {0.0};
  if (p < np * np) {
    const int px = p / np, py = p - (p / np) * np;
    T dz[3] = {T(0), T(0), T(0)};
#pragma unroll
    for (int dx = 0; dx < 3; ++dx) {
#pragma unroll
      for (int dy = 0; dy < 3; ++dy) {
        const int x0 = px - dx, y0 = py - dy;
        if (x0 < 0 || y0 < 0 || x0 > np - 3 || y0 > np - 3) continue;
        const int s = L.widx[x0 * np + y0];
        if (s < 0) continue;
        const T* y = L.Y + (size_t)s * kWinN + (3 * dx + dy) * 3;
        dz[0] += y[0];
        dz[1] += y[1];
        dz[2] += y[2];
      }
    }
#pragma unroll
    for (int t = 0; t < 3; ++t) {
      L.z[t * np2 + p] += dz[t];
      v[0] += (double)(L.r[t * np2 + p] * dz[t]);
    }
  }
  block_sum<1>(v, sh);
  write_partials<1>(v, L.part, L.nblk, blk);
}

template <typename T>
void launch_win_correct(const CGArgs<T>& a, int it, bool init, hipStream_t st, Zb zb) {
  const CGLev<T>& last = a.lv[a.nlev - 1];
  const int total = last.win0 + last.nwin;
  if (total <= 0) return;
  hipLaunchKernelGGL(k_win_apply<T>, dim3((total + 3) / 4, 1, zb.m), dim3(256), 0, st, a, init ? -1 : it, zb.zs);
  for (int l = 0; l < a.nlev; ++l) {
    if (a.lv[l].nwin <= 0) continue;
    hipLaunchKernelGGL(k_win_gather<T>, dim3(a.lv[l].nblk, 1, zb.m), dim3(256), 0, st, a.lv[l], it, init ? 1 : 0,
                       zb.zs);
  }
  launch_cg_scalars<T>(a, it, init ? kCGPhaseWinInit : kCGPhaseWin, st, zb);
}

template void launch_win_build<float>(const LevelGeom&, const float*, double, int, int*, int*, float*, unsigned*,
                                      int*, hipStream_t);
template void launch_win_build<double>(const LevelGeom&, const double*, double, int, int*, int*, double*,
                                       unsigned*, int*, hipStream_t);
template void launch_win_correct<float>(const CGArgs<float>&, int, bool, hipStream_t, Zb);
template void launch_win_correct<double>(const CGArgs<double>&, int, bool, hipStream_t, Zb);

}  // namespace gbl
