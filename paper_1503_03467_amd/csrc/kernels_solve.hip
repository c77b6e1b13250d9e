// Solve-phase kernels for gfx950: fine residual (FP64, matrix-free from the
// cell coefficient), restriction g^(k-1) = R g^(k), the subband systems
// B^(k) w^(k) = W^(k) g^(k) for all levels at once (block-Jacobi
// preconditioned CG, one launch per CG phase covering every level), the
// coarse solve, prolongation and the reconstruction sum, outer flexible-CG
// vector operations, and the adjoint gradient.
#include <hip/hip_runtime.h>

#include "device_common.hpp"
#include "gamblet_internal.hpp"
#include "solve_internal.hpp"
#include "reduce_device.hpp"

namespace gbl {

// Every block adds the nblk partials of sum k (fixed order per thread, then
// a fixed-order block reduction); the total is broadcast through LDS.
__device__ __forceinline__ double sum_partials(const double* __restrict__ part, int nblk, int k, double* sh) {
  __shared__ double bcast;
  double acc[1] = {0.0};
  for (int b = threadIdx.x; b < nblk; b += blockDim.x) acc[0] += part[k * nblk + b];
  block_sum<1>(acc, sh);
  if (threadIdx.x == 0) bcast = acc[0];
  __syncthreads();
  const double r = bcast;
  __syncthreads();
  return r;
}

// ---------------------------------------------------------------------------
// Fine operator, matrix-free from the cell coefficient (FP64).  For node
// (x, y) the cells around it are (x-1,y-1), (x,y-1), (x-1,y), (x,y).
// ---------------------------------------------------------------------------
template <typename F>
__device__ __forceinline__ double apply_fine(const double* __restrict__ a, int n, int x, int y, F U) {
  const double a00 = a[(x - 1) * n + (y - 1)];
  const double a10 = a[x * n + (y - 1)];
  const double a01 = a[(x - 1) * n + y];
  const double a11 = a[x * n + y];
  double s = (2.0 / 3.0) * (a00 + a10 + a01 + a11) * U(x, y);
  s -= (a10 + a11) * (1.0 / 6.0) * U(x + 1, y);
  s -= (a00 + a01) * (1.0 / 6.0) * U(x - 1, y);
  s -= (a01 + a11) * (1.0 / 6.0) * U(x, y + 1);
  s -= (a00 + a10) * (1.0 / 6.0) * U(x, y - 1);
  s -= a11 * (1.0 / 3.0) * U(x + 1, y + 1);
  s -= a00 * (1.0 / 3.0) * U(x - 1, y - 1);
  s -= a10 * (1.0 / 3.0) * U(x + 1, y - 1);
  s -= a01 * (1.0 / 3.0) * U(x - 1, y + 1);
  return s;
}

// r = b - A u over interior node slots.  b comes from the cell source
// (mode 0: b_i = (h^2/4) sum of g over the four cells at node i) or from a
// nodal array (mode 1).  u is nodal with boundary values; its interior
// values are read from u_slot when given (else taken as zero).
__global__ void k_residual(const double* __restrict__ a, int n, int mode, const double* __restrict__ src,
                           const double* __restrict__ u_nodal, const double* __restrict__ u_slot,
                           double* __restrict__ r, size_t zs, size_t src_stride, size_t u_stride) {
  const size_t zo = blockIdx.z * zs;
  src += blockIdx.z * src_stride;
  u_nodal += blockIdx.z * u_stride;
  u_slot = zsh(u_slot, zo);
  r = zsh(r, zo);
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= n * n) return;
  const int x = id / n, y = id % n;
  if (x == 0 || y == 0) {
    r[id] = 0.0;
    return;
  }
  const int s1 = n + 1;
  double b;
  if (mode == 0) {
    const double h = 1.0 / n;
    b = 0.25 * h * h *
        (src[(x - 1) * n + (y - 1)] + src[x * n + (y - 1)] + src[(x - 1) * n + y] + src[x * n + y]);
  } else {
    b = src[x * s1 + y];
  }
  auto U = [&](int i, int j) -> double {
    if (i == 0 || j == 0 || i == n || j == n) return u_nodal[i * s1 + j];
    return u_slot ? u_slot[i * n + j] : 0.0;
  };
  r[id] = b - apply_fine(a, n, x, y, U);
}

// w = A p for an interior slot vector p (zero Dirichlet data).
__global__ void k_apply_fine(const double* __restrict__ a, int n, const double* __restrict__ p,
                             double* __restrict__ w) {
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= n * n) return;
  const int x = id / n, y = id % n;
  if (x == 0 || y == 0) {
    w[id] = 0.0;
    return;
  }
  auto U = [&](int i, int j) -> double {
    if (i == 0 || j == 0 || i == n || j == n) return 0.0;
    return p[i * n + j];
  };
  w[id] = apply_fine(a, n, x, y, U);
}

// Up to three dot products of FP64 slot vectors at once -> out[0..nv).
__global__ __launch_bounds__(256) void k_dots(int len, int nv, const double* __restrict__ x0,
                                              const double* __restrict__ y0, const double* __restrict__ x1,
                                              const double* __restrict__ y1, const double* __restrict__ x2,
                                              const double* __restrict__ y2, double* part, unsigned* cnt,
                                              double* out, size_t zs) {
  __shared__ double sh[3 * 16];
  const size_t zo = blockIdx.z * zs;
  x0 = zsh(x0, zo);
  y0 = zsh(y0, zo);
  x1 = zsh(x1, zo);
  y1 = zsh(y1, zo);
  x2 = zsh(x2, zo);
  y2 = zsh(y2, zo);
  part = zsh(part, zo);
  cnt = zsh(cnt, zo);
  out = zsh(out, zo);
  double v[3] = {0.0, 0.0, 0.0};
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < len; i += gridDim.x * blockDim.x) {
    v[0] += x0[i] * y0[i];
    if (nv > 1) v[1] += x1[i] * y1[i];
    if (nv > 2) v[2] += x2[i] * y2[i];
  }
  block_sum<3>(v, sh);
  bool last;
  double res[3];
  finish_reduction<3>(v, part, gridDim.x, blockIdx.x, cnt, res, &last, sh);
  if (last) {
    for (int k = 0; k < nv; ++k) out[k] = res[k];
  }
}

// Outer flexible CG steps (scalars live on the device).
//   beta = -(z, w) / (p, w);  p = z + beta p   (A-orthogonalise against the last direction)
// (z, w) is re-added from the partials of the finest prolongation kernel.
// When elog is set, block 0 also forms the error estimate of the iteration
// that has just finished, max(||z|| / ||u||, |alpha| ||p|| / ||u||) with
// z = S r the preconditioned residual and alpha p the last correction, and
// appends it to elog at the position counted by sc[kSIter] (a NaN in either
// term is kept).
__global__ __launch_bounds__(256) void k_outer_direction(int len, double* __restrict__ sc,
                                                         const double* __restrict__ partz, int nblkz,
                                                         const double* __restrict__ z, double* __restrict__ p,
                                                         double* __restrict__ elog, int first, size_t zs) {
  __shared__ double sh[16];
  const size_t zo = blockIdx.z * zs;
  sc = zsh(sc, zo);
  partz = zsh(partz, zo);
  z = zsh(z, zo);
  p = zsh(p, zo);
  elog = zsh(elog, zo);
  double beta = 0.0;
  if (!first) {
    const double zw = sum_partials(partz, nblkz, 2, sh);
    const double pw = sc[kSPW];
    beta = (pw > 0.0) ? -zw / pw : 0.0;
    if (blockIdx.x == 0 && elog != nullptr) {
      const double zz = sum_partials(partz, nblkz, 0, sh);
      const double uu = sum_partials(partz, nblkz, 1, sh);
      if (threadIdx.x == 0) {
        const double pr = sc[kSPR], pp = sc[kSPP];
        const double alpha = (pw > 0.0) ? pr / pw : 0.0;
        double cur;
        if (uu > 0.0) {
          const double e1 = sqrt(zz / uu), e2 = fabs(alpha) * sqrt(pp / uu);
          cur = (e1 > e2 || e1 != e1) ? e1 : e2;
        } else {
          cur = (zz > 0.0 || pp > 0.0) ? 1.0 : 0.0;
        }
        const int i = (int)sc[kSIter];
        elog[i] = cur;
        sc[kSIter] = (double)(i + 1);
      }
    }
  }
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < len; i += gridDim.x * blockDim.x)
    p[i] = first ? z[i] : z[i] + beta * p[i];
}

// w = A p fused with the per-block partial sums of (p, w), (p, r), (p, p).
__global__ __launch_bounds__(256) void k_apply_fine_dots(const double* __restrict__ a, int n,
                                                         const double* __restrict__ p, const double* __restrict__ r,
                                                         double* __restrict__ w, double* part, size_t zs) {
  __shared__ double sh[3 * 16];
  const size_t zo = blockIdx.z * zs;
  p = zsh(p, zo);
  r = zsh(r, zo);
  w = zsh(w, zo);
  part = zsh(part, zo);
  double v[3] = {0.0, 0.0, 0.0};
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id < n * n) {
    const int x = id / n, y = id % n;
    double wv = 0.0;
    if (x != 0 && y != 0) {
      auto U = [&](int i, int j) -> double {
        if (i == 0 || j == 0 || i == n || j == n) return 0.0;
        return p[i * n + j];
      };
      wv = apply_fine(a, n, x, y, U);
    }
    w[id] = wv;
    const double pv = p[id];
    v[0] = pv * wv;
    v[1] = pv * r[id];
    v[2] = pv * pv;
  }
  block_sum<3>(v, sh);
  write_partials<3>(v, part, gridDim.x, blockIdx.x);
}

// alpha = (p, r) / (p, w) from the partials of the operator kernel;
// u += alpha p; r -= alpha w; g = T(r) (input of the subband solve).  Block 0
// also stores (p, w), (p, r), (p, p) for the host and the next kernels.
template <typename T>
__global__ __launch_bounds__(256) void k_outer_update_convert(int len, const double* __restrict__ part, int nblk,
                                                              double* __restrict__ sc, double* __restrict__ u,
                                                              double* __restrict__ r, const double* __restrict__ p,
                                                              const double* __restrict__ w, T* __restrict__ g,
                                                              size_t zs) {
  __shared__ double sh[16];
  const size_t zo = blockIdx.z * zs;
  part = zsh(part, zo);
  sc = zsh(sc, zo);
  u = zsh(u, zo);
  r = zsh(r, zo);
  p = zsh(p, zo);
  w = zsh(w, zo);
  g = zsh(g, zo);
  const double pw = sum_partials(part, nblk, 0, sh);
  const double pr = sum_partials(part, nblk, 1, sh);
  if (blockIdx.x == 0) {
    const double pp = sum_partials(part, nblk, 2, sh);
    if (threadIdx.x == 0) {
      sc[kSPW] = pw;
      sc[kSPR] = pr;
      sc[kSPP] = pp;
    }
  }
  const double alpha = (pw > 0.0) ? pr / pw : 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < len; i += gridDim.x * blockDim.x) {
    u[i] += alpha * p[i];
    const double rn = r[i] - alpha * w[i];
    r[i] = rn;
    g[i] = T(rn);
  }
}

// slot vector -> nodal interior (boundary entries untouched)
__global__ void k_slots_to_nodal(int n, const double* __restrict__ s, double* __restrict__ u, size_t zs,
                                 size_t u_stride) {
  s = zsh(s, blockIdx.z * zs);
  u += blockIdx.z * u_stride;
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= n * n) return;
  const int x = id / n, y = id % n;
  if (x == 0 || y == 0) return;
  u[x * (n + 1) + y] = s[id];
}

__global__ void k_fill(size_t len, double v, double* __restrict__ x, size_t zs) {
  x = zsh(x, blockIdx.z * zs);
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < len) x[i] = v;
}

template <typename T>
__global__ void k_fill_t(size_t len, T* __restrict__ x, size_t zs) {
  x = zsh(x, blockIdx.z * zs);
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < len) x[i] = T(0);
}

template <typename TD, typename TS>
__global__ void k_convert(size_t len, const TS* __restrict__ s, TD* __restrict__ d, size_t zs) {
  s = zsh(s, blockIdx.z * zs);
  d = zsh(d, blockIdx.z * zs);
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < len) d[i] = TD(s[i]);
}

// Right-hand sides per chunk of the kernels that read a shared operator once
// for several right-hand sides (registers bound the count).
template <typename T>
constexpr int kChunkRhs = sizeof(T) == 4 ? 8 : 4;

// Copy r of a per-solve vector (each copy zs bytes after the previous one).
template <typename P>
__device__ __forceinline__ P* rhs_ptr(P* p, int r, size_t zs) {
  return reinterpret_cast<P*>(reinterpret_cast<char*>(p) + (size_t)r * zs);
}
template <typename P>
__device__ __forceinline__ const P* rhs_ptr(const P* p, int r, size_t zs) {
  return reinterpret_cast<const P*>(reinterpret_cast<const char*>(p) + (size_t)r * zs);
}

// ---------------------------------------------------------------------------
// Restriction g^(k-1)_i = sum_c R_{i,c} g^(k)_c (eq. g^(k) = R g^(k+1),
// Section 4.7; the right-hand side step of Algorithm 2).  One thread per coarse slot; R is
// entry-major (R[e][cell]) so consecutive threads read consecutive words.
// ---------------------------------------------------------------------------
template <typename T, int RHO>
__device__ __forceinline__ T restrict_row(const T* __restrict__ R, const T* __restrict__ gf, int nk, int i, int bx) {
  // Row bx of coarse slot i's restriction block (uniform over the wavefront in
  // k_restrict, so the R addresses are scalar there).
  // The patch solves store explicit zeros in R at support positions outside
  // the level, so those terms need no mask: the row index is clamped into the
  // level and y positions outside it read a neighbouring row of g^(k) or the
  // zero padding around the vector (at most 2 RHO words past either end),
  // each multiplied by a zero of R.  The loads of a row then share one
  // address, with immediate offsets, and are all in flight together.
  constexpr int rw = 2 * (2 * RHO + 1);
  const int nc = nk / 2;
  const int nc2 = nc * nc;
  const int cx = i / nc, cy = i - (i / nc) * nc;
  const int fx = min(max(2 * (cx - RHO) + bx, 0), nk - 1);
  const T* gr = gf + fx * nk + 2 * (cy - RHO);
  const T* Rr = R + (size_t)(bx * rw) * nc2;
  T acc = T(0);
#pragma unroll
  for (int by = 0; by < rw; ++by) acc += Rr[by * nc2 + i] * gr[by];
  return acc;
}

template <typename T, int RHO>
__global__ __launch_bounds__(128) void k_restrict(const T* __restrict__ R, const T* __restrict__ gf,
                                                  T* __restrict__ gc, int nk, size_t zs) {
  gf = zsh(gf, blockIdx.z * zs);
  gc = zsh(gc, blockIdx.z * zs);
  // 64 consecutive coarse slots per workgroup, one per lane, so every load of
  // R reads 64 consecutive words.  The restriction block has 2 (2 RHO + 1)
  // rows: wavefront w sums rows w (2 RHO + 1) ... w (2 RHO + 1) + 2 RHO (a
  // compile-time count, so all its loads are issued together) and the two
  // partial sums are added in LDS.
  constexpr int half = 2 * RHO + 1;
  __shared__ T red[64];
  const int nc = nk / 2;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int i = min((int)blockIdx.x * 64 + lane, nc * nc - 1);
  T acc = T(0);
  const int w0 = __builtin_amdgcn_readfirstlane(w * half);
#pragma unroll
  for (int j = 0; j < half; ++j) acc += restrict_row<T, RHO>(R, gf, nk, i, w0 + j);
  if (w == 1) red[lane] = acc;
  __syncthreads();
  if (w == 0 && (int)blockIdx.x * 64 + lane < nc * nc) gc[i] = acc + red[lane];
}

// One launch per level for every right-hand side of a block (grid z): a
// variant that applied each R word to a chunk of 8 right-hand sides was 2.5x
// slower at 2048 x 2048 cells (the gathers of g, reused by about 80 coarse
// slots each, then come from 8 vectors at once and miss the L2).
template <typename T>
void launch_restrict(const LevelGeom& L, const T* R, const T* gf, T* gc, hipStream_t st, Zb zb) {
  const int nc = L.nk / 2;
  const dim3 grid((nc * nc + 63) / 64, 1, zb.m), block(128);
  switch (L.rho) {
    case 1: hipLaunchKernelGGL((k_restrict<T, 1>), grid, block, 0, st, R, gf, gc, L.nk, zb.zs); break;
    case 2: hipLaunchKernelGGL((k_restrict<T, 2>), grid, block, 0, st, R, gf, gc, L.nk, zb.zs); break;
    case 3: hipLaunchKernelGGL((k_restrict<T, 3>), grid, block, 0, st, R, gf, gc, L.nk, zb.zs); break;
    case 4: hipLaunchKernelGGL((k_restrict<T, 4>), grid, block, 0, st, R, gf, gc, L.nk, zb.zs); break;
    default: hipLaunchKernelGGL((k_restrict<T, 5>), grid, block, 0, st, R, gf, gc, L.nk, zb.zs); break;
  }
}

// ---------------------------------------------------------------------------
// Prolongation and subband sum: v^(k) = R^(k,k-1) v^(k-1) + W^(k)T w^(k)
// (Theorem 4.15; the subband gamblets are never formed, discussion of
// Algorithm 1 in Section 5.2).  One thread per level-k slot, gathering the
// restriction rows of the (2 rho + 1)^2 coarse slots whose patch covers it.
// ---------------------------------------------------------------------------
// (R^T v)_c for level-k slot c = (fx, fy): the (2 rho + 1)^2 coarse rows whose
// restriction block covers c.  RHO is a compile-time radius so the gather
// is unrolled; rows outside the level are clamped and masked out.
template <typename T, int RHO>
__device__ __forceinline__ T prolong_at_r(const T* __restrict__ R, const T* __restrict__ vc, int nk, int fx, int fy) {
  const int nc = nk / 2;
  const size_t nc2 = (size_t)nc * nc;
  const int px = fx >> 1, py = fy >> 1;
  constexpr int rw = 2 * (2 * RHO + 1);
  T acc = T(0);
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
      // rows outside the level are clamped to real rows and weighted by zero:
      // a product with a 0/1 factor (not a select) keeps every load
      // unconditional, so they can all be in flight together
      acc += R[(size_t)(bxc * rw + byc) * nc2 + i] * (vc[i] * T(ok ? 1 : 0));
    }
  }
  return acc;
}

// The coarse values a workgroup of 256 consecutive level-k slots in one row
// (fine row fx, columns fy0 .. fy0 + 255; nk a multiple of 256) gathers in
// the chunked prolongation: coarse rows px - RHO .. px + RHO and columns py0 -
// RHO .. py0 + 127 + RHO of every right-hand side's coarse vector, clamped
// into the level as prolong_at_r clamps them (the zero weight of the terms
// outside the level is applied at the gather), copied once into LDS: the
// gather otherwise fetched each of them through L2 for every one of the
// (2 RHO + 1)^2 terms.  Must be called by all threads of the workgroup.
template <typename T, int RHO, int MC>
__device__ __forceinline__ void stage_coarse_rows(const T* __restrict__ vc0, size_t zs, int nr, int nc, int px,
                                                  int py0, T* zl) {
  constexpr int RW = 2 * RHO + 1, CW = 128 + 2 * RHO;
  for (int e = threadIdx.x; e < MC * RW * CW; e += blockDim.x) {
    const int r = e / (RW * CW);
    const int rem = e - r * (RW * CW);
    const int dx = rem / CW, col = rem - (rem / CW) * CW;
    if (r < nr) {
      const int ixc = min(max(px - RHO + dx, 0), nc - 1);
      const int iyc = min(max(py0 - RHO + col, 0), nc - 1);
      zl[e] = rhs_ptr(vc0, r, zs)[ixc * nc + iyc];
    }
  }
  __syncthreads();
}

// (R^T v)_c for a chunk of right-hand sides, with the coarse values from
// stage_coarse_rows: each R word is loaded once and applied to the nr coarse
// vectors, each sum in the terms and order of prolong_at_r.
template <typename T, int RHO, int MC>
__device__ __forceinline__ void prolong_at_mr_staged(const T* __restrict__ R, const T* __restrict__ zl, int nr, int nk,
                                                     int fx, int fy, int py0, T (&acc)[MC]) {
  const int nc = nk / 2;
  const size_t nc2 = (size_t)nc * nc;
  const int px = fx >> 1, py = fy >> 1;
  constexpr int rw = 2 * (2 * RHO + 1);
  constexpr int RW = 2 * RHO + 1, CW = 128 + 2 * RHO;
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
      const T rv = R[(size_t)(bxc * rw + byc) * nc2 + i];
      const T okv = T(ok ? 1 : 0);
      const int col = py - py0 + dy + RHO;
#pragma unroll
      for (int r = 0; r < MC; ++r)
        if (r < nr) acc[r] += rv * (zl[(r * RW + dx + RHO) * CW + col] * okv);
    }
  }
}

template <typename T>
__device__ __forceinline__ T prolong_at(const T* __restrict__ R, const T* __restrict__ vc, int nk, int rho,
                                        int fx, int fy) {
  switch (rho) {
    case 1: return prolong_at_r<T, 1>(R, vc, nk, fx, fy);
    case 2: return prolong_at_r<T, 2>(R, vc, nk, fx, fy);
    case 3: return prolong_at_r<T, 3>(R, vc, nk, fx, fy);
    case 4: return prolong_at_r<T, 4>(R, vc, nk, fx, fy);
    default: return prolong_at_r<T, 5>(R, vc, nk, fx, fy);
  }
}

// w^(k) for the subband sum: the CG iterate, or for the finest level the
// iterate plus its pending last step x + alpha (u + beta p) when scal is set.
template <typename T>
__global__ void k_prolong(const T* __restrict__ R, const T* __restrict__ vc, const T* __restrict__ w,
                          T* __restrict__ vf, int nk, int rho, int fine, const T* __restrict__ u,
                          const T* __restrict__ pdir, const double* __restrict__ scal, double* __restrict__ zout,
                          size_t zs) {
  const size_t zo = blockIdx.z * zs;
  vc = zsh(vc, zo);
  w = zsh(w, zo);
  vf = zsh(vf, zo);
  u = zsh(u, zo);
  pdir = zsh(pdir, zo);
  scal = zsh(scal, zo);
  zout = zsh(zout, zo);
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= nk * nk) return;
  const int nc = nk / 2;
  const size_t nc2 = (size_t)nc * nc;
  const int fx = id / nk, fy = id % nk;
  T acc = prolong_at<T>(R, vc, nk, rho, fx, fy);
  const int px = fx >> 1, py = fy >> 1;
  const int d = 2 * (fx & 1) + (fy & 1);
  const int tp = parent_type(fine != 0, px, py);
  const int p = px * nc + py;
  T alpha = T(0), beta = T(0);
  if (scal) {
    alpha = T(scal[kFAlpha]);
    beta = T(scal[kFBeta]);
  }
#pragma unroll
  for (int t = 0; t < 3; ++t) {
    T wt = w[t * nc2 + p];
    if (scal) wt += alpha * (u[t * nc2 + p] + beta * pdir[t * nc2 + p]);
    acc += T(wcoef(tp, t, d)) * wt;
  }
  if (zout) zout[id] = (double)acc;
  else vf[id] = acc;
}

// v^(k) = R^T v^(k-1) + W^T w^(k) of a coarser level for a chunk of
// right-hand sides (R read once per chunk; per right-hand side the sums of
// k_prolong in the same order).
template <typename T, int RHO, int MC>
__global__ __launch_bounds__(256) void k_prolong_mr(const T* __restrict__ R, const T* __restrict__ vc0,
                                                    const T* __restrict__ w0, T* __restrict__ vf0, int nk, int m,
                                                    size_t zs) {
  __shared__ T zl[MC * (2 * RHO + 1) * (128 + 2 * RHO)];
  const int r0 = (int)blockIdx.z * MC;
  const int nr = min(MC, m - r0);
  vc0 = rhs_ptr(vc0, r0, zs);
  w0 = rhs_ptr(w0, r0, zs);
  vf0 = rhs_ptr(vf0, r0, zs);
  const int nc = nk / 2;
  const int first = (int)blockIdx.x * (int)blockDim.x;
  const int py0 = (first % nk) >> 1;
  stage_coarse_rows<T, RHO, MC>(vc0, zs, nr, nc, (first / nk) >> 1, py0, zl);
  const int id = first + (int)threadIdx.x;
  if (id >= nk * nk) return;
  const size_t nc2 = (size_t)nc * nc;
  const int fx = id / nk, fy = id % nk;
  T acc[MC];
#pragma unroll
  for (int r = 0; r < MC; ++r) acc[r] = T(0);
  prolong_at_mr_staged<T, RHO, MC>(R, zl, nr, nk, fx, fy, py0, acc);
  const int px = fx >> 1, py = fy >> 1;
  const int d = 2 * (fx & 1) + (fy & 1);
  const int tp = parent_type(false, px, py);
  const int p = px * nc + py;
#pragma unroll
  for (int r = 0; r < MC; ++r) {
    if (r < nr) {
      const T* w = rhs_ptr(w0, r, zs);
      T a = acc[r];
#pragma unroll
      for (int t = 0; t < 3; ++t) {
        const T wt = w[t * nc2 + p];
        a += T(wcoef(tp, t, d)) * wt;
      }
      rhs_ptr(vf0, r, zs)[id] = a;
    }
  }
}

template <typename T, int RHO>
void launch_prolong_mr(const LevelGeom& L, const T* R, const T* vc, const T* w, T* vf, hipStream_t st, Zb zb) {
  constexpr int MC = kChunkRhs<T>;
  const int tot = L.nk * L.nk;
  hipLaunchKernelGGL((k_prolong_mr<T, RHO, MC>), dim3((tot + 255) / 256, 1, (zb.m + MC - 1) / MC), dim3(256), 0, st,
                     R, vc, w, vf, L.nk, zb.m, zb.zs);
}

// Levels from this many points up take the chunked prolongation in a block
// solve: there R^(k) is large and its reads dominate; on smaller levels the
// kernels are latency-bound and a thread per right-hand side is faster (at
// 64 x 64 to 256 x 256 cells the chunked kernels made a block solve 1.6x
// slower).
constexpr size_t kChunkedProlongPoints = size_t(1) << 18;

template <typename T>
void launch_prolong(const LevelGeom& L, const T* R, const T* vc, const T* w, T* vf, bool fine,
                    hipStream_t st, Zb zb) {
  if (zb.m > 1 && !fine && (size_t)L.nk * L.nk >= kChunkedProlongPoints && L.nk % 256 == 0) {
    switch (L.rho) {
      case 1: launch_prolong_mr<T, 1>(L, R, vc, w, vf, st, zb); break;
      case 2: launch_prolong_mr<T, 2>(L, R, vc, w, vf, st, zb); break;
      case 3: launch_prolong_mr<T, 3>(L, R, vc, w, vf, st, zb); break;
      case 4: launch_prolong_mr<T, 4>(L, R, vc, w, vf, st, zb); break;
      default: launch_prolong_mr<T, 5>(L, R, vc, w, vf, st, zb); break;
    }
    return;
  }
  const int tot = L.nk * L.nk;
  hipLaunchKernelGGL(k_prolong<T>, dim3((tot + 255) / 256, 1, zb.m), dim3(256), 0, st, R, vc, w, vf, L.nk, L.rho,
                     fine ? 1 : 0, (const T*)nullptr, (const T*)nullptr, (const double*)nullptr, (double*)nullptr,
                     zb.zs);
}

// Finest level: z = R^T v^(q-1) + W^T (x + alpha (u + beta p)) in FP64,
// fused with the sums (z, z), (u_out, u_out), (z, w_out) of the outer iteration.
template <typename T>
__global__ __launch_bounds__(256) void k_prolong_fine_dots(const T* __restrict__ R, const T* __restrict__ vc,
                                                           FineCG<T> F0, int nk, int rho, double* __restrict__ z,
                                                           const double* __restrict__ uo,
                                                           const double* __restrict__ wo, double* part, int cheb,
                                                           size_t zs) {
  __shared__ double sh[3 * 16];
  const size_t zo = blockIdx.z * zs;
  const FineCG<T> F = zfine(F0, zo);
  vc = zsh(vc, zo);
  z = zsh(z, zo);
  uo = zsh(uo, zo);
  wo = zsh(wo, zo);
  part = zsh(part, zo);
  const int nc = nk / 2;
  const size_t nc2 = (size_t)nc * nc;
  const T alpha = cheb ? T(0) : T(F.scal[kFAlpha]), beta = cheb ? T(0) : T(F.scal[kFBeta]);
  double v[3] = {0.0, 0.0, 0.0};
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id < nk * nk) {
    const int fx = id / nk, fy = id % nk;
    T acc = prolong_at<T>(R, vc, nk, rho, fx, fy);
    const int px = fx >> 1, py = fy >> 1;
    const int d = 2 * (fx & 1) + (fy & 1);
    const int tp = parent_type(true, px, py);
    const int pp = px * nc + py;
#pragma unroll
    for (int t = 0; t < 3; ++t) {
      const T wt = cheb ? F.x[t * nc2 + pp] : F.x[t * nc2 + pp] + alpha * (F.u[t * nc2 + pp] + beta * F.p[t * nc2 + pp]);
      acc += T(wcoef(tp, t, d)) * wt;
    }
    const double zv = (double)acc;
    z[id] = zv;
    const double uv = uo[id];
    v[0] = zv * zv;
    v[1] = uv * uv;
    v[2] = zv * wo[id];
  }
  block_sum<3>(v, sh);
  write_partials<3>(v, part, gridDim.x, blockIdx.x);
}

// The same for a chunk of right-hand sides (R read once per chunk); per
// right-hand side the sums, block sums and partials of k_prolong_fine_dots.
template <typename T, int RHO, int MC>
__global__ __launch_bounds__(256) void k_prolong_fine_dots_mr(const T* __restrict__ R, const T* __restrict__ vc0,
                                                              FineCG<T> F0, int nk, double* z0, const double* uo0,
                                                              const double* wo0, double* part0, int cheb, int m,
                                                              size_t zs) {
  __shared__ double sh[3 * MC * 16];
  __shared__ T zl[MC * (2 * RHO + 1) * (128 + 2 * RHO)];
  const int r0 = (int)blockIdx.z * MC;
  const int nr = min(MC, m - r0);
  vc0 = rhs_ptr(vc0, r0, zs);
  z0 = rhs_ptr(z0, r0, zs);
  uo0 = rhs_ptr(uo0, r0, zs);
  wo0 = rhs_ptr(wo0, r0, zs);
  part0 = rhs_ptr(part0, r0, zs);
  const int nc = nk / 2;
  const size_t nc2 = (size_t)nc * nc;
  const int first = (int)blockIdx.x * (int)blockDim.x;
  const int py0 = (first % nk) >> 1;
  stage_coarse_rows<T, RHO, MC>(vc0, zs, nr, nc, (first / nk) >> 1, py0, zl);
  double v[3 * MC];
#pragma unroll
  for (int k = 0; k < 3 * MC; ++k) v[k] = 0.0;
  const int id = first + (int)threadIdx.x;
  if (id < nk * nk) {
    const int fx = id / nk, fy = id % nk;
    T acc[MC];
#pragma unroll
    for (int r = 0; r < MC; ++r) acc[r] = T(0);
    prolong_at_mr_staged<T, RHO, MC>(R, zl, nr, nk, fx, fy, py0, acc);
    const int px = fx >> 1, py = fy >> 1;
    const int d = 2 * (fx & 1) + (fy & 1);
    const int tp = parent_type(true, px, py);
    const int pp = px * nc + py;
#pragma unroll
    for (int r = 0; r < MC; ++r) {
      if (r < nr) {
        const FineCG<T> F = zfine(F0, (size_t)(r0 + r) * zs);
        const T alpha = cheb ? T(0) : T(F.scal[kFAlpha]), beta = cheb ? T(0) : T(F.scal[kFBeta]);
        T a = acc[r];
#pragma unroll
        for (int t = 0; t < 3; ++t) {
          const T wt =
              cheb ? F.x[t * nc2 + pp] : F.x[t * nc2 + pp] + alpha * (F.u[t * nc2 + pp] + beta * F.p[t * nc2 + pp]);
          a += T(wcoef(tp, t, d)) * wt;
        }
        const double zv = (double)a;
        rhs_ptr(z0, r, zs)[id] = zv;
        const double uv = rhs_ptr(uo0, r, zs)[id];
        v[3 * r] = zv * zv;
        v[3 * r + 1] = uv * uv;
        v[3 * r + 2] = zv * rhs_ptr(wo0, r, zs)[id];
      }
    }
  }
  block_sum<3 * MC>(v, sh);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int r = 0; r < MC; ++r) {
      if (r < nr) {
        double* part = rhs_ptr(part0, r, zs);
#pragma unroll
        for (int k = 0; k < 3; ++k) part[k * gridDim.x + blockIdx.x] = v[3 * r + k];
      }
    }
  }
}

template <typename T, int RHO>
void launch_prolong_fine_dots_mr(const LevelGeom& L, const T* R, const T* vc, const FineCG<T>& F, double* z,
                                 const double* uo, const double* wo, double* part, int cheb, hipStream_t st, Zb zb) {
  constexpr int MC = kChunkRhs<T>;
  const int tot = L.nk * L.nk;
  hipLaunchKernelGGL((k_prolong_fine_dots_mr<T, RHO, MC>), dim3((tot + 255) / 256, 1, (zb.m + MC - 1) / MC),
                     dim3(256), 0, st, R, vc, F, L.nk, z, uo, wo, part, cheb, zb.m, zb.zs);
}

template <typename T>
void launch_prolong_fine_dots(const LevelGeom& L, const T* R, const T* vc, const FineCG<T>& F, double* z,
                              const double* uo, const double* wo, double* part, int cheb, hipStream_t st, Zb zb) {
  if (zb.m > 1 && (size_t)L.nk * L.nk >= kChunkedProlongPoints && L.nk % 256 == 0) {
    switch (L.rho) {
      case 1: launch_prolong_fine_dots_mr<T, 1>(L, R, vc, F, z, uo, wo, part, cheb, st, zb); break;
      case 2: launch_prolong_fine_dots_mr<T, 2>(L, R, vc, F, z, uo, wo, part, cheb, st, zb); break;
      case 3: launch_prolong_fine_dots_mr<T, 3>(L, R, vc, F, z, uo, wo, part, cheb, st, zb); break;
      case 4: launch_prolong_fine_dots_mr<T, 4>(L, R, vc, F, z, uo, wo, part, cheb, st, zb); break;
      default: launch_prolong_fine_dots_mr<T, 5>(L, R, vc, F, z, uo, wo, part, cheb, st, zb); break;
    }
    return;
  }
  const int tot = L.nk * L.nk;
  hipLaunchKernelGGL(k_prolong_fine_dots<T>, dim3((tot + 255) / 256, 1, zb.m), dim3(256), 0, st, R, vc, F, L.nk,
                     L.rho, z, uo, wo, part, cheb, zb.zs);
}

template <typename T>
void launch_outer_update_convert(int len, const double* part, int nblk, double* sc, double* u, double* r,
                                 const double* p, const double* w, T* g, hipStream_t st, Zb zb) {
  int nb = (len + 255) / 256;
  if (nb > kUpdateBlocks) nb = kUpdateBlocks;
  hipLaunchKernelGGL(k_outer_update_convert<T>, dim3(nb, 1, zb.m), dim3(256), 0, st, len, part, nblk, sc, u, r, p, w,
                     g, zb.zs);
}

void launch_apply_fine_dots(const double* a, int n, const double* p, const double* r, double* w, double* part,
                            hipStream_t st, Zb zb) {
  hipLaunchKernelGGL(k_apply_fine_dots, dim3((n * n + 255) / 256, 1, zb.m), dim3(256), 0, st, a, n, p, r, w, part,
                     zb.zs);
}

// Small levels in one workgroup.  Restriction g^(k-1) = R g^(k) for k = khi..2;
// then the coarse solve and the prolongations v^(k) for k = 2..khi, with a
// workgroup barrier between levels.
template <typename T>
__global__ __launch_bounds__(1024) void k_restrict_chain(ChainArgs<T> c, size_t zs) {
  __shared__ T red[256 * 18];   // (cell, row) partial sums of the largest chain level (16 x 16 cells, rw <= 18)
  const size_t zo = blockIdx.z * zs;
  for (int j = c.n - 1; j >= 0; --j) {
    const ChainLevel<T> L = zchain(c.lv[j], zo);
    const int nc = L.nk / 2;
    const int rw = 2 * (2 * L.rho + 1);
    // work item (cell i, row bx): partial sum over the row, then rows are added
    for (int e = threadIdx.x; e < nc * nc * rw; e += blockDim.x) {
      const int i = e / rw, bx = e - (e / rw) * rw;
      T acc;
      switch (L.rho) {
        case 1: acc = restrict_row<T, 1>(L.R, L.gf, L.nk, i, bx); break;
        case 2: acc = restrict_row<T, 2>(L.R, L.gf, L.nk, i, bx); break;
        case 3: acc = restrict_row<T, 3>(L.R, L.gf, L.nk, i, bx); break;
        default: acc = restrict_row<T, 4>(L.R, L.gf, L.nk, i, bx); break;
      }
      red[e] = acc;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nc * nc; i += blockDim.x) {
      T acc = T(0);
      for (int bx = 0; bx < rw; ++bx) acc += red[i * rw + bx];
      L.gc[i] = acc;
    }
    __syncthreads();
  }
}

// One level of the prolongation chain, v^(k) = R^(k,k-1) v^(k-1) + W^(k)T w^(k),
// by the whole workgroup.  The level's vectors come in as restrict-qualified
// arguments (not through the chain structure) so that the gathers of a slot
// can all be in flight together.
template <typename T, int RHO>
__device__ __forceinline__ void prolong_level(const T* __restrict__ R, const T* __restrict__ vc,
                                              const T* __restrict__ w, T* __restrict__ vf, int nk, int fine) {
  const int nc = nk / 2;
  const int nc2 = nc * nc;
  for (int id = threadIdx.x; id < nk * nk; id += blockDim.x) {
    const int fx = id / nk, fy = id % nk;
    T acc = prolong_at_r<T, RHO>(R, vc, nk, fx, fy);
    const int px = fx >> 1, py = fy >> 1;
    const int d = 2 * (fx & 1) + (fy & 1);
    const int tp = parent_type(fine != 0, px, py);
    const int p = px * nc + py;
#pragma unroll
    for (int t = 0; t < 3; ++t) acc += T(wcoef(tp, t, d)) * w[t * nc2 + p];
    vf[id] = acc;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_prolong_chain(ChainArgs<T> c, const double* __restrict__ L1, size_t zs) {
  const size_t zo = blockIdx.z * zs;
  T* g1 = zsh(c.g1, zo);
  if (threadIdx.x == 0) {
    // coarsest system with the FP64 Cholesky factor of A^(1)
    double y[4];
    for (int i = 0; i < 4; ++i) {
      double v = (double)g1[i];
      for (int k = 0; k < i; ++k) v -= L1[i * 4 + k] * y[k];
      y[i] = v / L1[i * 4 + i];
    }
    for (int i = 3; i >= 0; --i) {
      double v = y[i];
      for (int k = i + 1; k < 4; ++k) v -= L1[k * 4 + i] * y[k];
      y[i] = v / L1[i * 4 + i];
    }
    for (int i = 0; i < 4; ++i) g1[i] = T(y[i]);
  }
  __syncthreads();
  for (int j = 0; j < c.n; ++j) {
    const ChainLevel<T> L = zchain(c.lv[j], zo);
    switch (L.rho) {
      case 1: prolong_level<T, 1>(L.R, L.gc, L.w, L.gf, L.nk, L.fine); break;
      case 2: prolong_level<T, 2>(L.R, L.gc, L.w, L.gf, L.nk, L.fine); break;
      case 3: prolong_level<T, 3>(L.R, L.gc, L.w, L.gf, L.nk, L.fine); break;
      default: prolong_level<T, 4>(L.R, L.gc, L.w, L.gf, L.nk, L.fine); break;
    }
    __syncthreads();
  }
}

template <typename T>
void launch_restrict_chain(const ChainArgs<T>& c, hipStream_t st, Zb zb) {
  if (c.n == 0) return;
  hipLaunchKernelGGL(k_restrict_chain<T>, dim3(1, 1, zb.m), dim3(1024), 0, st, c, zb.zs);
}
template <typename T>
void launch_prolong_chain(const ChainArgs<T>& c, const double* L1, hipStream_t st, Zb zb) {
  hipLaunchKernelGGL(k_prolong_chain<T>, dim3(1, 1, zb.m), dim3(256), 0, st, c, L1, zb.zs);
}

// Coarsest system A^(1) U^(1) = g^(1) (last solve of Algorithm 2) with the FP64
// Cholesky factor computed at build time.
template <typename T>
__global__ void k_coarse_solve(const double* __restrict__ L1, const T* __restrict__ g1, T* __restrict__ v1) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double y[4];
  for (int i = 0; i < 4; ++i) {
    double v = (double)g1[i];
    for (int k = 0; k < i; ++k) v -= L1[i * 4 + k] * y[k];
    y[i] = v / L1[i * 4 + i];
  }
  for (int i = 3; i >= 0; --i) {
    double v = y[i];
    for (int k = i + 1; k < 4; ++k) v -= L1[k * 4 + i] * y[k];
    y[i] = v / L1[i * 4 + i];
  }
  for (int i = 0; i < 4; ++i) v1[i] = T(y[i]);
}

template <typename T>
void launch_coarse_solve(const double* L1, const T* g1, T* v1, hipStream_t st) {
  hipLaunchKernelGGL(k_coarse_solve<T>, dim3(1), dim3(64), 0, st, L1, g1, v1);
}

// ---------------------------------------------------------------------------
// Subband systems B^(k) w^(k) = W^(k) g^(k) (eq. for w^(k), Section 4.7;
// subband solve of Algorithm 2), all levels in one grid.  Conjugate gradients
// (Section 4.9) with a block-Jacobi preconditioner (inverse 3x3 parent
// blocks).  Subband vectors are stored t-major: v[t * np^2 + parent].
// The direction update is folded into the operator application using
// B p_new = B z + beta B p_old, so each iteration takes two launches.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ int find_level(const CGArgs<T>& A, int b) {
  int l = 0;
  while (l + 1 < A.nlev && b >= A.lv[l + 1].blk0) ++l;
  return l;
}

template <typename T>
__device__ __forceinline__ int find_level_s(const CGArgs<T>& A, int b) {
  int l = 0;
  while (l + 1 < A.nlev && b >= A.lv[l + 1].blk0s) ++l;
  return l;
}

// Operator kernels of a block of m right-hand sides run as one 1-D grid in
// which the m workgroups of one stencil group (64 parents) sit on the same
// XCD and are dispatched next to each other (workgroups go round-robin over
// the 8 XCDs by linear id): id = (g / 8) 8m + r 8 + g % 8 for group g and
// right-hand side r.  The group's block of B^(k) is then fetched from HBM
// once and read from that XCD's L2 by the other m - 1.  Returns false for
// the padding ids past the last group.
__device__ __forceinline__ bool xcd_group_rhs(int id, int m, int ngroups, int& grp, int& rhs) {
  const int per = 8 * m;
  const int hi = id / per, rem = id - hi * per;
  rhs = rem >> 3;
  grp = hi * 8 + (rem & 7);
  return grp < ngroups;
}
inline unsigned xcd_group_grid(int ngroups, int m) { return (unsigned)(((ngroups + 7) / 8) * 8 * m); }

template <typename T>
__global__ __launch_bounds__(256) void k_cg_init(CGArgs<T> args, size_t zs) {
  __shared__ double sh[16];
  const int l = find_level(args, blockIdx.x);
  const CGLev<T> L = zlev(args.lv[l], blockIdx.z * zs);
  const int blk = blockIdx.x - L.blk0;
  const int p = blk * 256 + threadIdx.x;
  const int np = L.np;
  const size_t np2 = (size_t)np * np;
  const int nk = 2 * np;
  double v[1] = {0.0};
  if (p < np * np) {
    const int px = p / np, py = p % np;
    const int tp = parent_type(L.fine != 0, px, py);
    T gch[4];
#pragma unroll
    for (int d = 0; d < 4; ++d) gch[d] = L.g[(2 * px + (d >> 1)) * nk + 2 * py + (d & 1)];
    T r[3];
#pragma unroll
    for (int t = 0; t < 3; ++t) {
      T acc = T(0);
#pragma unroll
      for (int d = 0; d < 4; ++d) acc += T(wcoef(tp, t, d)) * gch[d];
      r[t] = acc;
    }
    T z[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      T acc = T(0);
#pragma unroll
      for (int j = 0; j < 3; ++j) acc += L.BJ[(i * 3 + j) * np2 + p] * r[j];
      z[i] = acc;
    }
#pragma unroll
    for (int t = 0; t < 3; ++t) {
      L.x[t * np2 + p] = T(0);
      L.r[t * np2 + p] = r[t];
      L.z[t * np2 + p] = z[t];
      L.p[t * np2 + p] = T(0);
      L.q[t * np2 + p] = T(0);
      v[0] += (double)(r[t] * z[t]);
    }
  }
  block_sum<1>(v, sh);
  write_partials<1>(v, L.part, L.nblk, blk);
}

// Coarser levels, stored block stencil.  A workgroup covers 64 consecutive
// parents (the lanes of every wavefront) and has one wavefront per neighbour
// row ox of the parent stencil, so each load instruction of a wavefront
// reads 64 consecutive words; the rows are summed in LDS.
// q = B z + beta q, p = z + beta p and the partial sums of (p, q); the last
// block of each level forms alpha = (r, z) / (p, q).
// Neighbour rows ox = wv, wv + nw, ... of one parent for a compile-time
// stencil width TT (the oy loop is unrolled so that a row's loads are all
// in flight together).
template <typename T, int TT>
__device__ __forceinline__ void coarse_rows(const CGLev<T>& L, const T* __restrict__ zs, int p, int wv, int nw,
                                            T& acc0, T& acc1, T& acc2) {
  constexpr int t = TT / 2;
  const int np = L.np;
  const size_t np2 = (size_t)np * np;
  const int px = p / np, py = p - (p / np) * np;
  for (int ox = wv; ox < TT; ox += nw) {
    const int qx = px + ox - t;
    if (qx < 0 || qx >= np) continue;
    const T* Bo = L.B + b_index(ox * TT, 0, p, TT);
    const int qb = qx * np + py - t;
    // B is stored as zero for neighbours outside the level, so the z index is
    // only clamped and every load of the row is unconditional
#pragma unroll
    for (int oy = 0; oy < TT; ++oy) {
      const int qy = min(max(py + oy - t, 0), np - 1);
      const int qn = qb + t + (qy - py);
      const T z0 = zs[qn], z1 = zs[np2 + qn], z2 = zs[2 * np2 + qn];
      const T* Bb = Bo + oy * 9 * 64;
      acc0 += Bb[0] * z0 + Bb[64] * z1 + Bb[128] * z2;
      acc1 += Bb[192] * z0 + Bb[256] * z1 + Bb[320] * z2;
      acc2 += Bb[384] * z0 + Bb[448] * z1 + Bb[512] * z2;
    }
  }
}

template <typename T>
__device__ __forceinline__ void coarse_apply(const CGLev<T>& L, const T* zs, int TT, int p, int wv, int nw, T& acc0,
                                             T& acc1, T& acc2) {
  switch (TT) {
    case 1: coarse_rows<T, 1>(L, zs, p, wv, nw, acc0, acc1, acc2); break;
    case 3: coarse_rows<T, 3>(L, zs, p, wv, nw, acc0, acc1, acc2); break;
    case 5: coarse_rows<T, 5>(L, zs, p, wv, nw, acc0, acc1, acc2); break;
    case 7: coarse_rows<T, 7>(L, zs, p, wv, nw, acc0, acc1, acc2); break;
    case 9: coarse_rows<T, 9>(L, zs, p, wv, nw, acc0, acc1, acc2); break;
    case 11: coarse_rows<T, 11>(L, zs, p, wv, nw, acc0, acc1, acc2); break;
    case 13: coarse_rows<T, 13>(L, zs, p, wv, nw, acc0, acc1, acc2); break;
    case 15: coarse_rows<T, 15>(L, zs, p, wv, nw, acc0, acc1, acc2); break;
    default: coarse_rows<T, 17>(L, zs, p, wv, nw, acc0, acc1, acc2); break;
  }
}

template <typename T>
__global__ __launch_bounds__(1024) void k_cg_spmv(CGArgs<T> args, int it, int blk_begin, int ngroups, int m,
                                                 size_t zs) {
  __shared__ double sh[16];
  __shared__ T red[3 * 16 * 64];
  int grp, rhs;
  if (!xcd_group_rhs((int)blockIdx.x, m, ngroups, grp, rhs)) return;
  const int gb = blk_begin + grp;
  const int l = find_level_s(args, gb);
  const CGLev<T> L = zlev(args.lv[l], rhs * zs);
  if (it >= L.iters) return;
  const int blk = gb - L.blk0s;
  const int np = L.np;
  const size_t np2 = (size_t)np * np;
  const int TT = 2 * L.t + 1;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
  const int p = blk * 64 + lane;
  T acc0 = T(0), acc1 = T(0), acc2 = T(0);
  if (p < np * np) {
    coarse_apply<T>(L, L.z, TT, p, wv, nw, acc0, acc1, acc2);
  }
  red[(0 * 16 + wv) * 64 + lane] = acc0;
  red[(1 * 16 + wv) * 64 + lane] = acc1;
  red[(2 * 16 + wv) * 64 + lane] = acc2;
  __syncthreads();
  double v[1] = {0.0};
  if (threadIdx.x < 64 && p < np * np) {
    const T beta = T(L.scal[kCBETA]);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      T sum = T(0);
      for (int w = 0; w < nw; ++w) sum += red[(i * 16 + w) * 64 + lane];
      const T qv = sum + beta * L.q[i * np2 + p];
      const T pv = L.z[i * np2 + p] + beta * L.p[i * np2 + p];
      L.q[i * np2 + p] = qv;
      L.p[i * np2 + p] = pv;
      v[0] += (double)(pv * qv);
    }
  }
  block_sum<1>(v, sh);
  write_partials<1>(v, L.part, L.nblks, blk);
}

template <typename T>
__global__ __launch_bounds__(256) void k_cg_update(CGArgs<T> args, int it, size_t zs) {
  __shared__ double sh[16];
  const int l = find_level(args, blockIdx.x);
  const CGLev<T> L = zlev(args.lv[l], blockIdx.z * zs);
  if (it >= L.iters) return;
  const int blk = blockIdx.x - L.blk0;
  const int p = blk * 256 + threadIdx.x;
  const int np = L.np;
  const size_t np2 = (size_t)np * np;
  double v[1] = {0.0};
  if (p < np * np) {
    const T alpha = T(L.scal[kCALPHA]);
    T r[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      L.x[i * np2 + p] += alpha * L.p[i * np2 + p];
      r[i] = L.r[i * np2 + p] - alpha * L.q[i * np2 + p];
      L.r[i * np2 + p] = r[i];
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      T acc = T(0);
#pragma unroll
      for (int j = 0; j < 3; ++j) acc += L.BJ[(i * 3 + j) * np2 + p] * r[j];
      L.z[i * np2 + p] = acc;
      v[0] += (double)(acc * r[i]);
    }
  }
  block_sum<1>(v, sh);
  write_partials<1>(v, L.part, L.nblk, blk);
}

// The scalar steps of the subband CG, one workgroup per (level, right-hand
// side): the per-block partials that the init, operator, update or window
// kernel stored are added in a fixed order (no tickets: a release fence per
// block of those grids costs more than the streaming work itself) and
//   init:    (r, z) -> rz, beta = alpha = 0
//   spmv:    (p, q) -> pq, alpha = rz / pq
//   update:  (r, z) -> beta = rz_new / rz, rz = rz_new
// On a level with window corrections the (r, D^-1 r) part goes to kCRZD and
// the window step completes it:
//   window:  rz_new = kCRZD + (r, sum of window terms), then as update (or
//            as init for the first one).
template <typename T>
__global__ __launch_bounds__(256) void k_cg_scalars(CGArgs<T> args, int it, int phase, size_t zs) {
  __shared__ double sh[16];
  const CGLev<T> L = zlev(args.lv[blockIdx.x], blockIdx.z * zs);
  int nblk = L.nblk;
  switch (phase) {
    case kCGPhaseInit: break;
    case kCGPhaseSpmv:
      if (it >= L.iters) return;
      nblk = L.nblks;
      break;
    case kCGPhaseUpdate:
      if (it >= L.iters) return;
      break;
    case kCGPhaseWinInit:
      if (L.nwin <= 0) return;
      break;
    default:   // kCGPhaseWin
      if (L.nwin <= 0 || it >= L.iters - 1) return;
      break;
  }
  double res[1];
  total_partials<1>(L.part, nblk, res, sh);
  if (threadIdx.x != 0) return;
  const double s = res[0];
  double* sc = L.scal;
  switch (phase) {
    case kCGPhaseInit:
      if (L.nwin > 0) {
        sc[kCRZD] = s;
      } else {
        sc[kCRZ] = s;
        sc[kCBETA] = 0.0;
        sc[kCALPHA] = 0.0;
      }
      break;
    case kCGPhaseSpmv:
      sc[kCPQ] = s;
      sc[kCALPHA] = (s > 0.0) ? sc[kCRZ] / s : 0.0;
      break;
    case kCGPhaseUpdate:
      if (L.nwin > 0 && it < L.iters - 1) {
        sc[kCRZD] = s;
      } else {
        const double rz = sc[kCRZ];
        sc[kCBETA] = (rz > 0.0) ? s / rz : 0.0;
        sc[kCRZ] = s;
      }
      break;
    case kCGPhaseWinInit:
      sc[kCRZ] = sc[kCRZD] + s;
      sc[kCBETA] = 0.0;
      sc[kCALPHA] = 0.0;
      break;
    default: {
      const double rz = sc[kCRZD] + s, old = sc[kCRZ];
      sc[kCBETA] = (old > 0.0) ? rz / old : 0.0;
      sc[kCRZ] = rz;
      break;
    }
  }
}

// ---------------------------------------------------------------------------
// The same operator steps for a block of right-hand sides with B^(k) read
// once per chunk of up to MC of them: every B word a lane loads is applied to
// the chunk's MC vectors (each in its own per-solve copy, zs bytes apart)
// before the next load.  Per right-hand side the sums run in the order of the
// single-vector kernels, so results are the same bit for bit.
// ---------------------------------------------------------------------------
template <typename T, int TT, int MC>
__device__ __forceinline__ void coarse_rows_mr(const CGLev<T>& L, const T* __restrict__ zs0, size_t zs, int nr,
                                               int p, int wv, int nw, T (&acc)[MC][3]) {
  constexpr int t = TT / 2;
  const int np = L.np;
  const size_t np2 = (size_t)np * np;
  const int px = p / np, py = p - (p / np) * np;
  for (int ox = wv; ox < TT; ox += nw) {
    const int qx = px + ox - t;
    if (qx < 0 || qx >= np) continue;
    const T* Bo = L.B + b_index(ox * TT, 0, p, TT);
    const int qb = qx * np + py - t;
#pragma unroll
    for (int oy = 0; oy < TT; ++oy) {
      const int qy = min(max(py + oy - t, 0), np - 1);
      const int qn = qb + t + (qy - py);
      const T* Bb = Bo + oy * 9 * 64;
      const T b0 = Bb[0], b1 = Bb[64], b2 = Bb[128], b3 = Bb[192], b4 = Bb[256], b5 = Bb[320];
      const T b6 = Bb[384], b7 = Bb[448], b8 = Bb[512];
#pragma unroll
      for (int r = 0; r < MC; ++r) {
        if (r < nr) {
          const T* zr = reinterpret_cast<const T*>(reinterpret_cast<const char*>(zs0) + (size_t)r * zs);
          const T z0 = zr[qn], z1 = zr[np2 + qn], z2 = zr[2 * np2 + qn];
          acc[r][0] += b0 * z0 + b1 * z1 + b2 * z2;
          acc[r][1] += b3 * z0 + b4 * z1 + b5 * z2;
          acc[r][2] += b6 * z0 + b7 * z1 + b8 * z2;
        }
      }
    }
  }
}

// The same rows for a workgroup whose 64 parents lie in one grid row (np >=
// 64), with the coarse vectors staged in LDS: for each of its offset rows a
// wavefront first copies the segment of grid row qx it needs (columns py0 - t
// .. py0 + 63 + t clamped into the level as in coarse_rows_mr, three
// components of every right-hand side of the chunk) into its own slice zl,
// then runs the row from there.  The gathers otherwise re-read every z word
// through L2 once per stencil offset oy (the kernel was bound by the L2
// request rate); the products and their order are those of coarse_rows_mr.
template <typename T, int TT, int MC>
__device__ __forceinline__ void coarse_rows_mr_staged(const CGLev<T>& L, const T* __restrict__ zs0, size_t zs, int nr,
                                                      int p, int wv, int nw, T (&acc)[MC][3], T* zl) {
  constexpr int t = TT / 2;
  constexpr int ZW = 64 + 2 * t;
  const int np = L.np;
  const size_t np2 = (size_t)np * np;
  const int lane = threadIdx.x & 63;
  const int px = p / np, py = p - (p / np) * np;
  const int py0 = py - lane;
  T* zw = zl + (size_t)wv * MC * 3 * ZW;
  const int rounds = (TT + nw - 1) / nw;
  for (int k = 0; k < rounds; ++k) {
    const int ox = wv + k * nw;
    const int qx = px + ox - t;
    const bool row = ox < TT && qx >= 0 && qx < np;
    if (row) {
      for (int idx = lane; idx < ZW; idx += 64) {
        const size_t q = (size_t)qx * np + min(max(py0 - t + idx, 0), np - 1);
#pragma unroll
        for (int r = 0; r < MC; ++r) {
          if (r < nr) {
            const T* zr = rhs_ptr(zs0, r, zs);
            zw[(r * 3 + 0) * ZW + idx] = zr[q];
            zw[(r * 3 + 1) * ZW + idx] = zr[np2 + q];
            zw[(r * 3 + 2) * ZW + idx] = zr[2 * np2 + q];
          }
        }
      }
    }
    __syncthreads();
    if (row) {
      const T* Bo = L.B + b_index(ox * TT, 0, p, TT);
#pragma unroll
      for (int oy = 0; oy < TT; ++oy) {
        const T* Bb = Bo + oy * 9 * 64;
        const T b0 = Bb[0], b1 = Bb[64], b2 = Bb[128], b3 = Bb[192], b4 = Bb[256], b5 = Bb[320];
        const T b6 = Bb[384], b7 = Bb[448], b8 = Bb[512];
#pragma unroll
        for (int r = 0; r < MC; ++r) {
          if (r < nr) {
            const T z0 = zw[(r * 3 + 0) * ZW + lane + oy], z1 = zw[(r * 3 + 1) * ZW + lane + oy];
            const T z2 = zw[(r * 3 + 2) * ZW + lane + oy];
            acc[r][0] += b0 * z0 + b1 * z1 + b2 * z2;
            acc[r][1] += b3 * z0 + b4 * z1 + b5 * z2;
            acc[r][2] += b6 * z0 + b7 * z1 + b8 * z2;
          }
        }
      }
    }
    __syncthreads();
  }
}

template <typename T, int MC>
__device__ __forceinline__ void coarse_apply_mr_staged(const CGLev<T>& L, const T* zs0, size_t zs, int nr, int TT,
                                                       int p, int wv, int nw, T (&acc)[MC][3], T* zl) {
  switch (TT) {
    case 1: coarse_rows_mr_staged<T, 1, MC>(L, zs0, zs, nr, p, wv, nw, acc, zl); break;
    case 3: coarse_rows_mr_staged<T, 3, MC>(L, zs0, zs, nr, p, wv, nw, acc, zl); break;
    case 5: coarse_rows_mr_staged<T, 5, MC>(L, zs0, zs, nr, p, wv, nw, acc, zl); break;
    case 7: coarse_rows_mr_staged<T, 7, MC>(L, zs0, zs, nr, p, wv, nw, acc, zl); break;
    case 9: coarse_rows_mr_staged<T, 9, MC>(L, zs0, zs, nr, p, wv, nw, acc, zl); break;
    case 11: coarse_rows_mr_staged<T, 11, MC>(L, zs0, zs, nr, p, wv, nw, acc, zl); break;
    case 13: coarse_rows_mr_staged<T, 13, MC>(L, zs0, zs, nr, p, wv, nw, acc, zl); break;
    case 15: coarse_rows_mr_staged<T, 15, MC>(L, zs0, zs, nr, p, wv, nw, acc, zl); break;
    default: coarse_rows_mr_staged<T, 17, MC>(L, zs0, zs, nr, p, wv, nw, acc, zl); break;
  }
}

template <typename T, int MC>
__device__ __forceinline__ void coarse_apply_mr(const CGLev<T>& L, const T* zs0, size_t zs, int nr, int TT, int p,
                                                int wv, int nw, T (&acc)[MC][3]) {
  switch (TT) {
    case 1: coarse_rows_mr<T, 1, MC>(L, zs0, zs, nr, p, wv, nw, acc); break;
    case 3: coarse_rows_mr<T, 3, MC>(L, zs0, zs, nr, p, wv, nw, acc); break;
    case 5: coarse_rows_mr<T, 5, MC>(L, zs0, zs, nr, p, wv, nw, acc); break;
    case 7: coarse_rows_mr<T, 7, MC>(L, zs0, zs, nr, p, wv, nw, acc); break;
    case 9: coarse_rows_mr<T, 9, MC>(L, zs0, zs, nr, p, wv, nw, acc); break;
    case 11: coarse_rows_mr<T, 11, MC>(L, zs0, zs, nr, p, wv, nw, acc); break;
    case 13: coarse_rows_mr<T, 13, MC>(L, zs0, zs, nr, p, wv, nw, acc); break;
    case 15: coarse_rows_mr<T, 15, MC>(L, zs0, zs, nr, p, wv, nw, acc); break;
    default: coarse_rows_mr<T, 17, MC>(L, zs0, zs, nr, p, wv, nw, acc); break;
  }
}

// Right-hand sides per chunk of the shared-B kernels (LDS holds 3 x waves x
// 64 partial sums per right-hand side).

template <typename T, int MC>
__global__ __launch_bounds__(1024) void k_cg_spmv_mr(CGArgs<T> args, int it, int blk_begin, int ngroups, int nchunks,
                                                   int m, size_t zs) {
  __shared__ double sh[16 * MC];
  extern __shared__ unsigned char red_raw[];
  T* red = reinterpret_cast<T*>(red_raw);   // [MC][3][nw][64]
  int grp, chunk;
  if (!xcd_group_rhs((int)blockIdx.x, nchunks, ngroups, grp, chunk)) return;
  const int r0 = chunk * MC;
  const int nr = min(MC, m - r0);
  const int gb = blk_begin + grp;
  const int l = find_level_s(args, gb);
  const CGLev<T> L0 = zlev(args.lv[l], r0 * zs);
  if (it >= L0.iters) return;
  const int blk = gb - L0.blk0s;
  const int np = L0.np;
  const size_t np2 = (size_t)np * np;
  const int TT = 2 * L0.t + 1;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
  const int p = blk * 64 + lane;
  T acc[MC][3];
#pragma unroll
  for (int r = 0; r < MC; ++r) acc[r][0] = acc[r][1] = acc[r][2] = T(0);
  if (np >= 64) {
    // the staging buffer shares the dynamic LDS with the wavefront sums below;
    // the staged rows end with a barrier
    coarse_apply_mr_staged<T, MC>(L0, L0.z, zs, nr, TT, p, wv, nw, acc, red);
  } else if (p < np * np) {
    coarse_apply_mr<T, MC>(L0, L0.z, zs, nr, TT, p, wv, nw, acc);
  }
#pragma unroll
  for (int r = 0; r < MC; ++r)
#pragma unroll
    for (int i = 0; i < 3; ++i) red[((r * 3 + i) * nw + wv) * 64 + lane] = acc[r][i];
  __syncthreads();
  // (p, q) of every right-hand side of the chunk, block sums for all of them
  // in one pass, each stored as that right-hand side's partial
  double v[MC];
#pragma unroll
  for (int r = 0; r < MC; ++r) v[r] = 0.0;
  for (int r = 0; r < nr; ++r) {
    const CGLev<T> L = zlev(args.lv[l], (r0 + r) * zs);
    if (threadIdx.x < 64 && p < np * np) {
      const T beta = T(L.scal[kCBETA]);
      double vr = 0.0;
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        T sum = T(0);
        for (int w = 0; w < nw; ++w) sum += red[((r * 3 + i) * nw + w) * 64 + lane];
        const T qv = sum + beta * L.q[i * np2 + p];
        const T pv = L.z[i * np2 + p] + beta * L.p[i * np2 + p];
        L.q[i * np2 + p] = qv;
        L.p[i * np2 + p] = pv;
        vr += (double)(pv * qv);
      }
#pragma unroll
      for (int k = 0; k < MC; ++k)
        if (k == r) v[k] = vr;
    }
  }
  block_sum<MC>(v, sh);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < MC; ++k)
      if (k < nr) zsh(L0.part, (size_t)k * zs)[blk] = v[k];
  }
}

template <typename T, int MC>
__global__ __launch_bounds__(1024) void k_cheb_step_mr(CGArgs<T> args, ChebStep cs, int k, int blk_begin, int ngroups,
                                                     int nchunks, int m, size_t zs) {
  extern __shared__ unsigned char red_raw[];
  T* red = reinterpret_cast<T*>(red_raw);   // [MC][3][nw][64]
  int grp, chunk;
  if (!xcd_group_rhs((int)blockIdx.x, nchunks, ngroups, grp, chunk)) return;
  const int r0 = chunk * MC;
  const int nr = min(MC, m - r0);
  const int gb = blk_begin + grp;
  const int l = find_level_s(args, gb);
  const CGLev<T> L0 = zlev(args.lv[l], r0 * zs);
  if (k >= L0.iters) return;
  const int blk = gb - L0.blk0s;
  const int np = L0.np;
  const size_t np2 = (size_t)np * np;
  const int TT = 2 * L0.t + 1;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
  const int p = blk * 64 + lane;
  T acc[MC][3];
#pragma unroll
  for (int r = 0; r < MC; ++r) acc[r][0] = acc[r][1] = acc[r][2] = T(0);
  if (p < np * np) coarse_apply_mr<T, MC>(L0, (k & 1) ? L0.z : L0.p, zs, nr, TT, p, wv, nw, acc);
#pragma unroll
  for (int r = 0; r < MC; ++r)
#pragma unroll
    for (int i = 0; i < 3; ++i) red[((r * 3 + i) * nw + wv) * 64 + lane] = acc[r][i];
  __syncthreads();
  if (threadIdx.x < 64 && p < np * np) {
    const T ca = T(cs.ca[l]), cb = T(cs.cb[l]);
    for (int r = 0; r < nr; ++r) {
      const CGLev<T> L = zlev(args.lv[l], (r0 + r) * zs);
      const T* dold = (k & 1) ? L.z : L.p;
      T* dnew = (k & 1) ? L.p : L.z;
      T rr[3];
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        T sum = T(0);
        for (int w = 0; w < nw; ++w) sum += red[((r * 3 + i) * nw + w) * 64 + lane];
        rr[i] = L.r[i * np2 + p] - sum;
        L.r[i * np2 + p] = rr[i];
      }
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        T acc1 = T(0);
#pragma unroll
        for (int j = 0; j < 3; ++j) acc1 += L.BJ[(i * 3 + j) * np2 + p] * rr[j];
        const T dn = ca * dold[i * np2 + p] + cb * acc1;
        dnew[i * np2 + p] = dn;
        L.x[i * np2 + p] += dn;
      }
    }
  }
}

template <typename T>
void launch_cg_scalars(const CGArgs<T>& a, int it, int phase, hipStream_t st, Zb zb) {
  hipLaunchKernelGGL(k_cg_scalars<T>, dim3(a.nlev, 1, zb.m), dim3(256), 0, st, a, it, phase, zb.zs);
}
template <typename T>
void launch_cg_init(const CGArgs<T>& a, int nblocks, hipStream_t st, Zb zb) {
  hipLaunchKernelGGL(k_cg_init<T>, dim3(nblocks, 1, zb.m), dim3(256), 0, st, a, zb.zs);
  launch_cg_scalars<T>(a, 0, kCGPhaseInit, st, zb);
}
// The largest coarse level (first in the list) gets its own launch with
// one wavefront per stencil row; the smaller levels share a second launch.
template <typename T>
void launch_cg_spmv(const CGArgs<T>& a, int nblocks, int it, hipStream_t st, Zb zb) {
  const int n0 = a.lv[0].nblks < nblocks ? a.lv[0].nblks : nblocks;
  const int t0 = 2 * a.lv[0].t + 1;
  int tmax = 1;
  for (int l = 1; l < a.nlev; ++l) tmax = tmax > 2 * a.lv[l].t + 1 ? tmax : 2 * a.lv[l].t + 1;
  const int w0 = t0 < 16 ? t0 : 16, w1 = tmax < 16 ? tmax : 16;
  if (zb.m == 1) {
    hipLaunchKernelGGL(k_cg_spmv<T>, dim3(xcd_group_grid(n0, 1)), dim3(64 * w0), 0, st, a, it, 0, n0, 1, zb.zs);
    if (nblocks > n0)
      hipLaunchKernelGGL(k_cg_spmv<T>, dim3(xcd_group_grid(nblocks - n0, 1)), dim3(64 * w1), 0, st, a, it, n0,
                         nblocks - n0, 1, zb.zs);
    launch_cg_scalars<T>(a, it, kCGPhaseSpmv, st, zb);
    return;
  }
  constexpr int MC = kChunkRhs<T>;
  const int nch = (zb.m + MC - 1) / MC;
  // dynamic LDS: the wavefront sums [MC][3][w][64], or the staged z rows
  // [w][MC][3][64 + 2t] of the widest stencil in the launch (the larger)
  const size_t lds0 = (size_t)MC * 3 * w0 * (64 + 2 * a.lv[0].t) * sizeof(T);
  const size_t lds1 = (size_t)MC * 3 * w1 * (64 + 2 * ((tmax - 1) / 2)) * sizeof(T);
  hipLaunchKernelGGL((k_cg_spmv_mr<T, MC>), dim3(xcd_group_grid(n0, nch)), dim3(64 * w0), lds0, st, a, it, 0, n0,
                     nch, zb.m, zb.zs);
  if (nblocks > n0)
    hipLaunchKernelGGL((k_cg_spmv_mr<T, MC>), dim3(xcd_group_grid(nblocks - n0, nch)), dim3(64 * w1), lds1, st, a,
                       it, n0, nblocks - n0, nch, zb.m, zb.zs);
  launch_cg_scalars<T>(a, it, kCGPhaseSpmv, st, zb);
}
template <typename T>
void launch_cg_update(const CGArgs<T>& a, int nblocks, int it, hipStream_t st, Zb zb) {
  hipLaunchKernelGGL(k_cg_update<T>, dim3(nblocks, 1, zb.m), dim3(256), 0, st, a, it, zb.zs);
  launch_cg_scalars<T>(a, it, kCGPhaseUpdate, st, zb);
}

// ---------------------------------------------------------------------------
// Chebyshev iteration on the coarser subband levels (all levels in one grid;
// coefficients of the step per level in ChebStep).  d_k alternates between
// the z (k even) and p (k odd) vectors; x accumulates d_0 + ... + d_k.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_cheb_init(CGArgs<T> args, ChebStep cs, int blk_begin, size_t zs) {
  const int gb = blk_begin + (int)blockIdx.x;
  const int l = find_level(args, gb);
  const CGLev<T> L = zlev(args.lv[l], blockIdx.z * zs);
  const int p = (gb - L.blk0) * 256 + threadIdx.x;
  const int np = L.np;
  const size_t np2 = (size_t)np * np;
  const int nk = 2 * np;
  if (p >= np * np) return;
  const int px = p / np, py = p % np;
  const int tp = parent_type(L.fine != 0, px, py);
  T gch[4];
#pragma unroll
  for (int d = 0; d < 4; ++d) gch[d] = L.g[(2 * px + (d >> 1)) * nk + 2 * py + (d & 1)];
  T r[3];
#pragma unroll
  for (int t = 0; t < 3; ++t) {
    T acc = T(0);
#pragma unroll
    for (int d = 0; d < 4; ++d) acc += T(wcoef(tp, t, d)) * gch[d];
    r[t] = acc;
  }
  const T c0 = T(cs.c0[l]);
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    T acc = T(0);
#pragma unroll
    for (int j = 0; j < 3; ++j) acc += L.BJ[(i * 3 + j) * np2 + p] * r[j];
    const T d0 = c0 * acc;
    L.r[i * np2 + p] = r[i];
    L.z[i * np2 + p] = d0;
    L.x[i * np2 + p] = d0;
  }
}

// Step k >= 1: r -= B d_{k-1};  d_k = ca d_{k-1} + cb M r;  x += d_k.  The
// operator part is that of k_cg_spmv (64 parents per workgroup, one
// wavefront per stencil row).
template <typename T>
__global__ __launch_bounds__(1024) void k_cheb_step(CGArgs<T> args, ChebStep cs, int k, int blk_begin, int ngroups,
                                                   int m, size_t zs) {
  __shared__ T red[3 * 16 * 64];
  int grp, rhs;
  if (!xcd_group_rhs((int)blockIdx.x, m, ngroups, grp, rhs)) return;
  const int gb = blk_begin + grp;
  const int l = find_level_s(args, gb);
  const CGLev<T> L = zlev(args.lv[l], rhs * zs);
  if (k >= L.iters) return;
  const int blk = gb - L.blk0s;
  const int np = L.np;
  const size_t np2 = (size_t)np * np;
  const int TT = 2 * L.t + 1;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
  const int p = blk * 64 + lane;
  const T* dold = (k & 1) ? L.z : L.p;
  T* dnew = (k & 1) ? L.p : L.z;
  T acc0 = T(0), acc1 = T(0), acc2 = T(0);
  if (p < np * np) coarse_apply<T>(L, dold, TT, p, wv, nw, acc0, acc1, acc2);
  red[(0 * 16 + wv) * 64 + lane] = acc0;
  red[(1 * 16 + wv) * 64 + lane] = acc1;
  red[(2 * 16 + wv) * 64 + lane] = acc2;
  __syncthreads();
  if (threadIdx.x < 64 && p < np * np) {
    const T ca = T(cs.ca[l]), cb = T(cs.cb[l]);
    T r[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      T sum = T(0);
      for (int w = 0; w < nw; ++w) sum += red[(i * 16 + w) * 64 + lane];
      r[i] = L.r[i * np2 + p] - sum;
      L.r[i * np2 + p] = r[i];
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      T acc = T(0);
#pragma unroll
      for (int j = 0; j < 3; ++j) acc += L.BJ[(i * 3 + j) * np2 + p] * r[j];
      const T dn = ca * dold[i * np2 + p] + cb * acc;
      dnew[i * np2 + p] = dn;
      L.x[i * np2 + p] += dn;
    }
  }
}

template <typename T>
void launch_cheb_init(const CGArgs<T>& a, const ChebStep& s, int l0, int l1, hipStream_t st, Zb zb) {
  const int b0 = a.lv[l0].blk0, b1 = a.lv[l1 - 1].blk0 + a.lv[l1 - 1].nblk;
  hipLaunchKernelGGL(k_cheb_init<T>, dim3(b1 - b0, 1, zb.m), dim3(256), 0, st, a, s, b0, zb.zs);
}
// One launch for the levels l0 .. l1-1: one wavefront per stencil row of the
// largest of them (its blocks dominate); wider stencils loop over their rows.
template <typename T>
void launch_cheb_step(const CGArgs<T>& a, const ChebStep& s, int k, int l0, int l1, hipStream_t st, Zb zb) {
  const int b0 = a.lv[l0].blk0s, b1 = a.lv[l1 - 1].blk0s + a.lv[l1 - 1].nblks;
  const int t0 = 2 * a.lv[l0].t + 1;
  const int w0 = t0 < 16 ? t0 : 16;
  if (zb.m == 1) {
    hipLaunchKernelGGL(k_cheb_step<T>, dim3(xcd_group_grid(b1 - b0, 1)), dim3(64 * w0), 0, st, a, s, k, b0, b1 - b0,
                       1, zb.zs);
    return;
  }
  constexpr int MC = kChunkRhs<T>;
  const int nch = (zb.m + MC - 1) / MC;
  hipLaunchKernelGGL((k_cheb_step_mr<T, MC>), dim3(xcd_group_grid(b1 - b0, nch)), dim3(64 * w0),
                     (size_t)MC * 3 * w0 * 64 * sizeof(T), st, a, s, k, b0, b1 - b0, nch, zb.m, zb.zs);
}

// ---------------------------------------------------------------------------
// Chebyshev iteration on the finest subband level, several steps per launch.
// A workgroup owns a tile of 8 x 8 parents and works on the tile plus a halo
// of H parents (one thread per parent of the 16 x 16 region).  Each step needs
// d on a one-parent halo of the region where r and d are formed, so after s
// steps the values are exact on the region shrunk by s parents; with s <= H
// the tile itself stays exact and only it is stored.  The operator B^(q) is
// applied matrix-free: nodal W^T d in LDS (with a zero border), the Q1
// stencil from the cell coefficients held in registers, then W.  The launch
// with k0 = 0 starts from r_0 = W g, d_0 = M r_0 / theta, x = d_0.  r and d are
// double buffered (buffer rd is read, rd ^ 1 written) because tiles read
// their neighbours' values.
// ---------------------------------------------------------------------------
template <typename T, int H>
__global__ __launch_bounds__(256) void k_fine_cheb(FineCG<T> F0, ChebCoef cf, int k0, int nsteps, int rd, size_t zs) {
  const FineCG<T> F = zfine(F0, blockIdx.z * zs);
  constexpr int TPM = 8;
  constexpr int VWM = 2 * (TPM + 2 * H) + 2;
  __shared__ T vl[VWM * VWM];
  const int np = F.np;
  const int nk = 2 * np;
  const size_t np2 = (size_t)np * np;
  const int TP = np < TPM ? np : TPM;
  const int ntx = np / TP;
  const int RW = TP + 2 * H;
  const int VW = 2 * RW + 2;
  const int blk = xcd_remap((int)blockIdx.x, (int)gridDim.x);
  const int tx = blk / ntx, ty = blk - (blk / ntx) * ntx;
  const int tid = threadIdx.x;
  const bool act = tid < RW * RW;
  const int rx = act ? tid / RW : 0, ry = act ? tid - (tid / RW) * RW : 0;
  const int px = tx * TP - H + rx, py = ty * TP - H + ry;
  const bool in = act && px >= 0 && py >= 0 && px < np && py < np;
  const bool interior = act && rx >= H && rx < H + TP && ry >= H && ry < H + TP;
  const int q = in ? px * np + py : 0;
  const int tp = in ? parent_type(true, px, py) : 3;
  // buffers picked by selects, not by an index into F's arrays (an index
  // that is not a compile-time constant moves F to scratch memory)
  const T* const r_in = rd ? F.r[1] : F.r[0];
  const T* const d_in = rd ? F.w[1] : F.w[0];
  T* const r_out = rd ? F.r[0] : F.r[1];
  T* const d_out = rd ? F.w[0] : F.w[1];
  for (int e = tid; e < VW * VW; e += blockDim.x) vl[e] = T(0);

  T bj[9], ac[3][3], r[3], d[3], x[3];
#pragma unroll
  for (int e = 0; e < 9; ++e) bj[e] = in ? F.BJ[e * np2 + q] : T(0);
#pragma unroll
  for (int i = 0; i < 3; ++i) {
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const int cx = 2 * px - 1 + i, cy = 2 * py - 1 + j;
      ac[i][j] = (in && cx >= 0 && cy >= 0 && cx < nk && cy < nk) ? F.acell[(size_t)cx * nk + cy] : T(0);
    }
  }
  if (k0 == 0) {
    T gc[4];
#pragma unroll
    for (int dd = 0; dd < 4; ++dd) gc[dd] = in ? F.g[(2 * px + (dd >> 1)) * nk + 2 * py + (dd & 1)] : T(0);
#pragma unroll
    for (int t = 0; t < 3; ++t)
      r[t] = T(wcoef(tp, t, 0)) * gc[0] + T(wcoef(tp, t, 1)) * gc[1] + T(wcoef(tp, t, 2)) * gc[2] +
             T(wcoef(tp, t, 3)) * gc[3];
    const T c0 = T(cf.c0);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      d[i] = c0 * (bj[3 * i] * r[0] + bj[3 * i + 1] * r[1] + bj[3 * i + 2] * r[2]);
      x[i] = d[i];
    }
  } else {
#pragma unroll
    for (int t = 0; t < 3; ++t) {
      r[t] = in ? r_in[t * np2 + q] : T(0);
      d[t] = in ? d_in[t * np2 + q] : T(0);
      x[t] = interior ? F.x[t * np2 + q] : T(0);
    }
  }
  __syncthreads();
  for (int s2 = 0; s2 < nsteps; ++s2) {
    const int k = k0 + 1 + s2;
    if (act) {
#pragma unroll
      for (int dd = 0; dd < 4; ++dd) {
        const T v = T(wcoef(tp, 0, dd)) * d[0] + T(wcoef(tp, 1, dd)) * d[1] + T(wcoef(tp, 2, dd)) * d[2];
        vl[(2 * rx + (dd >> 1) + 1) * VW + 2 * ry + (dd & 1) + 1] = v;
      }
    }
    __syncthreads();
    if (in) {
      T Av[4];
#pragma unroll
      for (int dd = 0; dd < 4; ++dd) {
        const int dx = dd >> 1, dy = dd & 1;
        if (2 * px + dx == 0 || 2 * py + dy == 0) {
          Av[dd] = T(0);
          continue;
        }
        const T a00 = ac[dx][dy], a10 = ac[dx + 1][dy], a01 = ac[dx][dy + 1], a11 = ac[dx + 1][dy + 1];
        const T* vp = vl + (2 * rx + dx + 1) * VW + 2 * ry + dy + 1;
        T acc = T(2.0 / 3.0) * (a00 + a10 + a01 + a11) * vp[0];
        acc -= (a10 + a11) * T(1.0 / 6.0) * vp[VW];
        acc -= (a00 + a01) * T(1.0 / 6.0) * vp[-VW];
        acc -= (a01 + a11) * T(1.0 / 6.0) * vp[1];
        acc -= (a00 + a10) * T(1.0 / 6.0) * vp[-1];
        acc -= a11 * T(1.0 / 3.0) * vp[VW + 1];
        acc -= a00 * T(1.0 / 3.0) * vp[-VW - 1];
        acc -= a10 * T(1.0 / 3.0) * vp[VW - 1];
        acc -= a01 * T(1.0 / 3.0) * vp[-VW + 1];
        Av[dd] = acc;
      }
#pragma unroll
      for (int t = 0; t < 3; ++t) {
        const T bd = is_pad_row(tp, t) ? d[t]
                                        : T(wcoef(tp, t, 0)) * Av[0] + T(wcoef(tp, t, 1)) * Av[1] +
                                              T(wcoef(tp, t, 2)) * Av[2] + T(wcoef(tp, t, 3)) * Av[3];
        r[t] -= bd;
      }
      const T ca = T(cf.ca[k]), cb = T(cf.cb[k]);
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        d[i] = ca * d[i] + cb * (bj[3 * i] * r[0] + bj[3 * i + 1] * r[1] + bj[3 * i + 2] * r[2]);
        x[i] += d[i];
      }
    }
    __syncthreads();
  }
  if (interior) {
#pragma unroll
    for (int t = 0; t < 3; ++t) {
      r_out[t * np2 + q] = r[t];
      d_out[t * np2 + q] = d[t];
      F.x[t * np2 + q] = x[t];
    }
  }
}

template <typename T>
void launch_fine_cheb(const FineCG<T>& f, const ChebCoef& c, int K, int k0, int nsteps, int rd, hipStream_t st,
                      Zb zb) {
  (void)K;
  const int TP = f.np < 8 ? f.np : 8;
  const int nb = (f.np / TP) * (f.np / TP);
  hipLaunchKernelGGL((k_fine_cheb<T, 4>), dim3(nb, 1, zb.m), dim3(256), 0, st, f, c, k0, nsteps, rd, zb.zs);
}

// ---------------------------------------------------------------------------
// Finest subband system B^(q) w = W g^(q), preconditioned CG in the
// Chronopoulos-Gear arrangement: iteration i forms, per parent,
//   p_{i-1} = u_{i-1} + b p_{i-2},  s_{i-1} = w_{i-1} + b s_{i-2},
//   x_i = x_{i-1} + a p_{i-1},      r_i = r_{i-1} - a s_{i-1},
//   u_i = M r_i,  w_i = B u_i,  and the sums (r_i, u_i), (w_i, u_i),
// from which the last block forms the next a, b.  B u needs u on a
// one-parent halo of the tile; the halo values are recomputed from the old
// r, w, s (double buffered), so a single launch covers one iteration.
// it == 0 starts from x = 0, r = W g.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_fine_cg(FineCG<T> F0, int it, size_t zs) {
  const FineCG<T> F = zfine(F0, blockIdx.z * zs);
  __shared__ double sh[32];
  __shared__ T lds[3 * 18 * 18 + 36 * 36 + 33 * 33 + 3 * 16 * 16];
  const int np = F.np;
  const int nk = 2 * np;
  const size_t np2 = (size_t)np * np;
  const int TP = np < 16 ? np : 16;
  const int ntx = np / TP;
  const int blk = xcd_remap((int)blockIdx.x, (int)gridDim.x);
  const int tx = blk / ntx, ty = blk - (blk / ntx) * ntx;
  const int px0 = tx * TP, py0 = ty * TP;
  const int HW = TP + 2;
  const int VW = 2 * TP + 4;
  const int AW = 2 * TP + 1;
  T* ul = lds;                 // u at tile + halo parents, [t][hx][hy]
  T* vl = ul + 3 * HW * HW;    // nodal W^T u
  T* al = vl + VW * VW;        // cell coefficients
  T* rl = al + AW * AW;        // r_i of the tile's own parents, [t][lx][ly]
  const int tid = threadIdx.x;
  // cell coefficients do not depend on the iteration: stage them first
  for (int e = tid; e < AW * AW; e += blockDim.x) {
    const int cxl = e / AW, cyl = e - (e / AW) * AW;
    const int cx = 2 * px0 - 1 + cxl, cy = 2 * py0 - 1 + cyl;
    al[e] = (cx >= 0 && cy >= 0 && cx < nk && cy < nk) ? F.acell[(size_t)cx * nk + cy] : T(0);
  }
  const int rd = (it + 1) & 1, wr = it & 1;   // buffers read / written by this iteration
  // picked by selects (a run-time index into F's arrays would move F to scratch memory)
  const T* const w_rd = rd ? F.w[1] : F.w[0];
  const T* const s_rd = rd ? F.s[1] : F.s[0];
  const T* const r_rd = rd ? F.r[1] : F.r[0];
  T* const r_wr = wr ? F.r[1] : F.r[0];
  T* const s_wr = wr ? F.s[1] : F.s[0];
  T* const w_wr = wr ? F.w[1] : F.w[0];
  const T alpha = it ? T(F.scal[kFAlpha]) : T(0);
  const T beta = it ? T(F.scal[kFBeta]) : T(0);

  for (int e = tid; e < HW * HW; e += blockDim.x) {
    const int hx = e / HW, hy = e - (e / HW) * HW;
    const int px = px0 - 1 + hx, py = py0 - 1 + hy;
    T u3[3] = {T(0), T(0), T(0)};
    if (px >= 0 && py >= 0 && px < np && py < np) {
      const int q = px * np + py;
      const int tp = parent_type(true, px, py);
      T r3[3], s3[3];
      if (it == 0) {
        T gc[4];
#pragma unroll
        for (int d = 0; d < 4; ++d) gc[d] = F.g[(2 * px + (d >> 1)) * nk + 2 * py + (d & 1)];
#pragma unroll
        for (int t = 0; t < 3; ++t) {
          r3[t] = T(wcoef(tp, t, 0)) * gc[0] + T(wcoef(tp, t, 1)) * gc[1] + T(wcoef(tp, t, 2)) * gc[2] +
                  T(wcoef(tp, t, 3)) * gc[3];
          s3[t] = T(0);
        }
      } else {
#pragma unroll
        for (int t = 0; t < 3; ++t) {
          s3[t] = w_rd[t * np2 + q] + beta * s_rd[t * np2 + q];
          r3[t] = r_rd[t * np2 + q] - alpha * s3[t];
        }
      }
#pragma unroll
      for (int i = 0; i < 3; ++i)
        u3[i] = F.BJ[(i * 3 + 0) * np2 + q] * r3[0] + F.BJ[(i * 3 + 1) * np2 + q] * r3[1] +
                F.BJ[(i * 3 + 2) * np2 + q] * r3[2];
      if (hx >= 1 && hx <= TP && hy >= 1 && hy <= TP) {
#pragma unroll
        for (int t = 0; t < 3; ++t) {
          const size_t o = t * np2 + q;
          if (it == 0) {
            F.x[o] = T(0);
            F.p[o] = T(0);
          } else {
            const T pn = F.u[o] + beta * F.p[o];
            F.p[o] = pn;
            F.x[o] += alpha * pn;
          }
          F.u[o] = u3[t];
          r_wr[o] = r3[t];
          s_wr[o] = s3[t];
          rl[(t * TP + hx - 1) * TP + hy - 1] = r3[t];
        }
      }
    }
#pragma unroll
    for (int t = 0; t < 3; ++t) ul[(t * HW + hx) * HW + hy] = u3[t];
  }
  __syncthreads();
  for (int e = tid; e < HW * HW; e += blockDim.x) {
    const int hx = e / HW, hy = e - (e / HW) * HW;
    const int px = px0 - 1 + hx, py = py0 - 1 + hy;
    const bool in = px >= 0 && py >= 0 && px < np && py < np;
    const int tp = in ? parent_type(true, px, py) : 3;
    const T u0 = ul[(0 * HW + hx) * HW + hy], u1 = ul[(1 * HW + hx) * HW + hy], u2 = ul[(2 * HW + hx) * HW + hy];
#pragma unroll
    for (int d = 0; d < 4; ++d) {
      T v = T(0);
      if (in) v = T(wcoef(tp, 0, d)) * u0 + T(wcoef(tp, 1, d)) * u1 + T(wcoef(tp, 2, d)) * u2;
      vl[(2 * hx + (d >> 1)) * VW + 2 * hy + (d & 1)] = v;
    }
  }
  __syncthreads();
  double v[2] = {0.0, 0.0};
  if (tid < TP * TP) {
    const int lx = tid / TP, ly = tid - (tid / TP) * TP;
    const int px = px0 + lx, py = py0 + ly;
    const int tp = parent_type(true, px, py);
    T Av[4];
#pragma unroll
    for (int d = 0; d < 4; ++d) {
      const int x = 2 * px + (d >> 1), yy = 2 * py + (d & 1);
      if (x == 0 || yy == 0) {
        Av[d] = T(0);
        continue;
      }
      const int vx = x - 2 * (px0 - 1), vy = yy - 2 * (py0 - 1);
      const int ax = x - (2 * px0 - 1), ay = yy - (2 * py0 - 1);
      const T a00 = al[(ax - 1) * AW + (ay - 1)], a10 = al[ax * AW + (ay - 1)];
      const T a01 = al[(ax - 1) * AW + ay], a11 = al[ax * AW + ay];
      const T* vp = vl + vx * VW + vy;
      T acc = T(2.0 / 3.0) * (a00 + a10 + a01 + a11) * vp[0];
      acc -= (a10 + a11) * T(1.0 / 6.0) * vp[VW];
      acc -= (a00 + a01) * T(1.0 / 6.0) * vp[-VW];
      acc -= (a01 + a11) * T(1.0 / 6.0) * vp[1];
      acc -= (a00 + a10) * T(1.0 / 6.0) * vp[-1];
      acc -= a11 * T(1.0 / 3.0) * vp[VW + 1];
      acc -= a00 * T(1.0 / 3.0) * vp[-VW - 1];
      acc -= a10 * T(1.0 / 3.0) * vp[VW - 1];
      acc -= a01 * T(1.0 / 3.0) * vp[-VW + 1];
      Av[d] = acc;
    }
    const int q = px * np + py;
#pragma unroll
    for (int t = 0; t < 3; ++t) {
      const T ut = ul[(t * HW + lx + 1) * HW + ly + 1];
      T wt;
      if (is_pad_row(tp, t)) {
        wt = ut;
      } else {
        wt = T(wcoef(tp, t, 0)) * Av[0] + T(wcoef(tp, t, 1)) * Av[1] + T(wcoef(tp, t, 2)) * Av[2] +
             T(wcoef(tp, t, 3)) * Av[3];
      }
      w_wr[t * np2 + q] = wt;
      v[0] += (double)(rl[(t * TP + lx) * TP + ly] * ut);
      v[1] += (double)(wt * ut);
    }
  }
  block_sum<2>(v, sh);
  write_partials<2>(v, F.part, F.nblk, blk);
}

// Scalars of the finest-level CG step from the tile partials of (r, u) and
// (w, u), added in a fixed order by one workgroup per right-hand side.
template <typename T>
__global__ __launch_bounds__(256) void k_fine_cg_scalars(FineCG<T> F0, int it, size_t zs) {
  __shared__ double sh[2 * 16];
  const FineCG<T> F = zfine(F0, blockIdx.z * zs);
  double res[2];
  total_partials<2>(F.part, F.nblk, res, sh);
  if (threadIdx.x != 0) return;
  const double gam = res[0], del = res[1];
  double b = 0.0, eta = del;
  if (it > 0) {
    const double gprev = F.scal[kFGamma], aprev = F.scal[kFAlpha];
    b = (gprev > 0.0) ? gam / gprev : 0.0;
    eta = (aprev != 0.0) ? del - b * gam / aprev : del;
  }
  F.scal[kFGamma] = gam;
  F.scal[kFBeta] = b;
  F.scal[kFAlpha] = (eta > 0.0) ? gam / eta : 0.0;
}

// Last update x += a p after the final iteration (no operator application).
template <typename T>
__global__ void k_fine_cg_finish(FineCG<T> F0, int it, size_t zs) {
  const FineCG<T> F = zfine(F0, blockIdx.z * zs);
  const size_t np2 = (size_t)F.np * F.np;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 3 * np2) return;
  const T alpha = T(F.scal[kFAlpha]), beta = T(F.scal[kFBeta]);
  const T pn = F.u[i] + beta * F.p[i];
  F.x[i] += alpha * pn;
}

template <typename T>
void launch_fine_cg(const FineCG<T>& f, int it, hipStream_t st, Zb zb) {
  if (it >= 0) {
    hipLaunchKernelGGL(k_fine_cg<T>, dim3(f.nblk, 1, zb.m), dim3(256), 0, st, f, it, zb.zs);
    hipLaunchKernelGGL(k_fine_cg_scalars<T>, dim3(1, 1, zb.m), dim3(256), 0, st, f, it, zb.zs);
  } else {
    const size_t n = 3 * (size_t)f.np * f.np;
    hipLaunchKernelGGL(k_fine_cg_finish<T>, dim3((unsigned)((n + 255) / 256), 1, zb.m), dim3(256), 0, st, f, it,
                       zb.zs);
  }
}

// ---------------------------------------------------------------------------
// Adjoint gradient per cell (not in the paper): dJ/dlog a_e = -a_e lam_e^T K u_e
// and dJ/dg_e = (h^2/4) sum of lam at the cell's corners, with the unit
// bilinear element stiffness K (local order (0,0),(1,0),(0,1),(1,1)).
// ---------------------------------------------------------------------------
__global__ void k_cell_gradient(const double* __restrict__ a, int n, const double* __restrict__ u,
                                const double* __restrict__ lam, double* __restrict__ dloga,
                                double* __restrict__ dg) {
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= n * n) return;
  const int ex = id / n, ey = id % n;
  const int s1 = n + 1;
  const int nd[4] = {ex * s1 + ey, (ex + 1) * s1 + ey, ex * s1 + ey + 1, (ex + 1) * s1 + ey + 1};
  double ue[4], le[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    ue[i] = u[nd[i]];
    le[i] = lam[nd[i]];
  }
  const double K[4][4] = {{4.0, -1.0, -1.0, -2.0}, {-1.0, 4.0, -2.0, -1.0}, {-1.0, -2.0, 4.0, -1.0},
                          {-2.0, -1.0, -1.0, 4.0}};
  double e = 0.0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    double ku = 0.0;
#pragma unroll
    for (int j = 0; j < 4; ++j) ku += K[i][j] * ue[j];
    e += le[i] * ku;
  }
  dloga[id] = -a[id] * e * (1.0 / 6.0);
  if (dg) {
    const double h = 1.0 / n;
    dg[id] = 0.25 * h * h * (le[0] + le[1] + le[2] + le[3]);
  }
}

// ---------------------------------------------------------------------------
// Host launch helpers for the non-templated kernels.
// ---------------------------------------------------------------------------
void launch_residual(const double* a, int n, int mode, const double* src, const double* u_nodal,
                     const double* u_slot, double* r, hipStream_t st, Zb zb, size_t src_stride, size_t u_stride) {
  hipLaunchKernelGGL(k_residual, dim3((n * n + 255) / 256, 1, zb.m), dim3(256), 0, st, a, n, mode, src, u_nodal,
                     u_slot, r, zb.zs, src_stride, u_stride);
}
void launch_apply_fine(const double* a, int n, const double* p, double* w, hipStream_t st) {
  hipLaunchKernelGGL(k_apply_fine, dim3((n * n + 255) / 256), dim3(256), 0, st, a, n, p, w);
}
void launch_dots(int len, int nv, const double* x0, const double* y0, const double* x1, const double* y1,
                 const double* x2, const double* y2, double* part, unsigned* cnt, double* out,
                 hipStream_t st, Zb zb) {
  int nb = (len + 255) / 256;
  if (nb > kDotBlocks) nb = kDotBlocks;
  hipLaunchKernelGGL(k_dots, dim3(nb, 1, zb.m), dim3(256), 0, st, len, nv, x0, y0, x1, y1, x2, y2, part, cnt, out,
                     zb.zs);
}
void launch_outer_direction(int len, double* sc, const double* partz, int nblkz, const double* z, double* p,
                            double* elog, int first, hipStream_t st, Zb zb) {
  int nb = (len + 255) / 256;
  if (nb > kUpdateBlocks) nb = kUpdateBlocks;
  hipLaunchKernelGGL(k_outer_direction, dim3(nb, 1, zb.m), dim3(256), 0, st, len, sc, partz, nblkz, z, p, elog, first,
                     zb.zs);
}
void launch_slots_to_nodal(int n, const double* s, double* u, hipStream_t st, Zb zb, size_t u_stride) {
  hipLaunchKernelGGL(k_slots_to_nodal, dim3((n * n + 255) / 256, 1, zb.m), dim3(256), 0, st, n, s, u, zb.zs,
                     u_stride);
}
void launch_fill(size_t len, double v, double* x, hipStream_t st, Zb zb) {
  if (len == 0) return;
  hipLaunchKernelGGL(k_fill, dim3((unsigned)((len + 255) / 256), 1, zb.m), dim3(256), 0, st, len, v, x, zb.zs);
}
template <typename T>
void launch_zero(size_t len, T* x, hipStream_t st, Zb zb) {
  if (len == 0) return;
  hipLaunchKernelGGL(k_fill_t<T>, dim3((unsigned)((len + 255) / 256), 1, zb.m), dim3(256), 0, st, len, x, zb.zs);
}
template <typename TD, typename TS>
void launch_convert(size_t len, const TS* s, TD* d, hipStream_t st, Zb zb) {
  if (len == 0) return;
  hipLaunchKernelGGL((k_convert<TD, TS>), dim3((unsigned)((len + 255) / 256), 1, zb.m), dim3(256), 0, st, len, s, d,
                     zb.zs);
}
void launch_cell_gradient(const double* a, int n, const double* u, const double* lam, double* dloga,
                          double* dg, hipStream_t st) {
  hipLaunchKernelGGL(k_cell_gradient, dim3((n * n + 255) / 256), dim3(256), 0, st, a, n, u, lam, dloga, dg);
}

// ---------------------------------------------------------------------------
// Level-q gamblets from the localized mass inverse (Algorithm 2; Definition
// 5.2): the finest subband right-hand side is g^(q) = Minv^T r and the finest
// prolongation v^(q) stands for the nodal vector z = Minv v^(q).  Slot (x, y),
// x, y >= 1, holds interior node (x - 1, y - 1); Y is the table of 1-D
// factors ([n - 1][2 rho + 1]) and a node's weight at offset (dx, dy) is
// Y[ix][dx] Y[iy][dy].
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_mass_load_slots(int n, int rho, const double* __restrict__ Y, const double* __restrict__ r,
                                  T* __restrict__ g) {
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= n * n) return;
  const int x = id / n, y = id % n;
  if (x == 0 || y == 0) {
    g[id] = T(0);
    return;
  }
  const int m = n - 1, w = 2 * rho + 1;
  const int ix = x - 1, iy = y - 1;
  double acc = 0.0;
  for (int dx = -rho; dx <= rho; ++dx) {
    const int lx = ix + dx;
    if (lx < 0 || lx >= m) continue;
    double row = 0.0;
    for (int dy = -rho; dy <= rho; ++dy) {
      const int ly = iy + dy;
      if (ly < 0 || ly >= m) continue;
      row += Y[(size_t)iy * w + dy + rho] * r[(size_t)(lx + 1) * n + ly + 1];
    }
    acc += Y[(size_t)ix * w + dx + rho] * row;
  }
  g[id] = T(acc);
}

// z = Minv v (FP64 slots, zero on the empty slots) and the partial sums
// (z, z), (u, u), (z, w) of k_prolong_fine_dots, in its layout.
template <typename T>
__global__ __launch_bounds__(256) void k_mass_nodal_dots(int n, int rho, const double* __restrict__ Y,
                                                         const T* __restrict__ v, double* __restrict__ z,
                                                         const double* __restrict__ uo,
                                                         const double* __restrict__ wo, double* part) {
  __shared__ double sh[3 * 16];
  double acc3[3] = {0.0, 0.0, 0.0};
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id < n * n) {
    const int x = id / n, y = id % n;
    double zv = 0.0;
    if (x > 0 && y > 0) {
      const int m = n - 1, w = 2 * rho + 1;
      const int lx = x - 1, ly = y - 1;
      for (int dx = -rho; dx <= rho; ++dx) {
        const int ix = lx - dx;
        if (ix < 0 || ix >= m) continue;
        double row = 0.0;
        for (int dy = -rho; dy <= rho; ++dy) {
          const int iy = ly - dy;
          if (iy < 0 || iy >= m) continue;
          row += Y[(size_t)iy * w + dy + rho] * (double)v[(size_t)(ix + 1) * n + iy + 1];
        }
        zv += Y[(size_t)ix * w + dx + rho] * row;
      }
    }
    z[id] = zv;
    const double uv = uo[id];
    acc3[0] = zv * zv;
    acc3[1] = uv * uv;
    acc3[2] = zv * wo[id];
  }
  block_sum<3>(acc3, sh);
  write_partials<3>(acc3, part, gridDim.x, blockIdx.x);
}

template <typename T>
void launch_mass_load_slots(int n, int rho, const double* Y, const double* r, T* g, hipStream_t st) {
  hipLaunchKernelGGL(k_mass_load_slots<T>, dim3((n * n + 255) / 256), dim3(256), 0, st, n, rho, Y, r, g);
}

template <typename T>
void launch_mass_nodal_dots(int n, int rho, const double* Y, const T* v, double* z, const double* uo,
                            const double* wo, double* part, hipStream_t st) {
  hipLaunchKernelGGL(k_mass_nodal_dots<T>, dim3((n * n + 255) / 256), dim3(256), 0, st, n, rho, Y, v, z, uo, wo,
                     part);
}

#define GBL_INST(T)                                                                                      \
  template void launch_mass_load_slots<T>(int, int, const double*, const double*, T*, hipStream_t);     \
  template void launch_mass_nodal_dots<T>(int, int, const double*, const T*, double*, const double*,    \
                                          const double*, double*, hipStream_t);                         \
  template void launch_restrict<T>(const LevelGeom&, const T*, const T*, T*, hipStream_t, Zb);          \
  template void launch_prolong<T>(const LevelGeom&, const T*, const T*, const T*, T*, bool, hipStream_t, Zb); \
  template void launch_coarse_solve<T>(const double*, const T*, T*, hipStream_t);                       \
  template void launch_cg_init<T>(const CGArgs<T>&, int, hipStream_t, Zb);                              \
  template void launch_cg_scalars<T>(const CGArgs<T>&, int, int, hipStream_t, Zb);                      \
  template void launch_cg_spmv<T>(const CGArgs<T>&, int, int, hipStream_t, Zb);                         \
  template void launch_cg_update<T>(const CGArgs<T>&, int, int, hipStream_t, Zb);                       \
  template void launch_zero<T>(size_t, T*, hipStream_t, Zb);                                            \
  template void launch_fine_cg<T>(const FineCG<T>&, int, hipStream_t, Zb);                             \
  template void launch_fine_cheb<T>(const FineCG<T>&, const ChebCoef&, int, int, int, int, hipStream_t, Zb); \
  template void launch_cheb_init<T>(const CGArgs<T>&, const ChebStep&, int, int, hipStream_t, Zb);      \
  template void launch_cheb_step<T>(const CGArgs<T>&, const ChebStep&, int, int, int, hipStream_t, Zb); \
  template void launch_prolong_fine_dots<T>(const LevelGeom&, const T*, const T*, const FineCG<T>&,      \
                                            double*, const double*, const double*, double*, int,         \
                                            hipStream_t, Zb);                                           \
  template void launch_outer_update_convert<T>(int, const double*, int, double*, double*, double*,      \
                                               const double*, const double*, T*, hipStream_t, Zb);      \
  template void launch_restrict_chain<T>(const ChainArgs<T>&, hipStream_t, Zb);                         \
  template void launch_prolong_chain<T>(const ChainArgs<T>&, const double*, hipStream_t, Zb);
GBL_INST(float)
GBL_INST(double)
#undef GBL_INST
template void launch_convert<float, double>(size_t, const double*, float*, hipStream_t, Zb);
template void launch_convert<double, float>(size_t, const float*, double*, hipStream_t, Zb);
template void launch_convert<double, double>(size_t, const double*, double*, hipStream_t, Zb);

}  // namespace gbl
