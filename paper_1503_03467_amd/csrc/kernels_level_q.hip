// Level-q gamblets from the localized inverse of the mass matrix (Algorithm
// 2, the mass-inverse and level-q lines; Definition 5.2): for every interior
// node i, y^(i) solves M^(i,rho) y = e_i on the patch of nodes within rho node
// steps of i (a box, clipped to the interior), psi^(q)_i = sum_j y^(i)_j phi_j,
// g^(q)_i = sum_j y^(i)_j b_j and A^(q) = Minv^T A Minv.
//
// On a uniform grid the Q1 mass matrix is (h T) (x) (h T), T = tridiag(1, 4,
// 1) / 6, and a box patch is a product of two intervals, so the patch matrix
// is a Kronecker product and y^(i) = y_x (x) y_y, each factor the solution of
// a tridiagonal system of at most 2 rho + 1 unknowns.  The factors depend on
// one coordinate only: the table Y[x][d] (x an interior coordinate, d in
// [-rho, rho]) holds them, and every kernel below reads weights as
// Y[ix][dx] Y[iy][dy].  This replaces the paper's per-node iterative patch
// solves by 2 (2^q - 1) tridiagonal solves.
//
// The level-q operator row i is A^(q)_ij = sum_m c_m Minv_mj with c = A Minv e_i
// (support: the patch grown by one node).  The weights of column j factor,
// so the sum over m = (mx, my) runs as two one-dimensional contractions:
// t[dx][my] = sum_mx c[mx][my] Y[ix+dx][mx-ix-dx], then
// A^(q)_{i, i+(dx,dy)} = sum_my t[dx][my] Y[iy+dy][my-iy-dy].
#include <hip/hip_runtime.h>

#include "gamblet_internal.hpp"

namespace gbl {

// Y[x][d + rho] = (6/h) (tridiag(1, 4, 1) restricted to [lo, hi))^-1 e_x at
// x + d, zero outside [lo, hi); lo = max(0, x - rho), hi = min(m, x + rho + 1).
__global__ void k_mass_inverse_table(int m, int rho, double inv_h, double* __restrict__ Y) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= m) return;
  constexpr int kMax = 2 * kMaxRhoQ + 1;
  const int lo = max(0, x - rho), hi = min(m, x + rho + 1), L = hi - lo;
  double cp[kMax], dp[kMax], y[kMax];
  // forward sweep of the Thomas algorithm (diagonally dominant: no pivoting)
  double denom = 4.0;
  cp[0] = 1.0 / denom;
  dp[0] = (lo == x) ? 1.0 / denom : 0.0;
  for (int r = 1; r < L; ++r) {
    denom = 4.0 - cp[r - 1];
    cp[r] = 1.0 / denom;
    const double e = (lo + r == x) ? 1.0 : 0.0;
    dp[r] = (e - dp[r - 1]) / denom;
  }
  y[L - 1] = dp[L - 1];
  for (int r = L - 2; r >= 0; --r) y[r] = dp[r] - cp[r] * y[r + 1];
  const int w = 2 * rho + 1;
  for (int d = -rho; d <= rho; ++d) {
    const int p = x + d;
    Y[(size_t)x * w + d + rho] = (p >= lo && p < hi) ? 6.0 * inv_h * y[p - lo] : 0.0;
  }
}

// psi^(q)_i in the phi basis: W[i][(dx + rho)(2 rho + 1) + dy + rho]
__global__ void k_level_q_weights(int m, int rho, const double* __restrict__ Y, double* __restrict__ W) {
  const int w = 2 * rho + 1;
  const size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t total = (size_t)m * m * w * w;
  if (id >= total) return;
  const size_t i = id / (w * w);
  const int e = (int)(id % (w * w));
  const int ix = (int)(i / m), iy = (int)(i % m);
  W[id] = Y[(size_t)ix * w + e / w] * Y[(size_t)iy * w + e % w];
}

// g^(q)_i = sum_{l in patch(i)} Y[ix][lx-ix] Y[iy][ly-iy] b_l
__global__ void k_level_q_load(int m, int rho, const double* __restrict__ Y, const double* __restrict__ b,
                               double* __restrict__ gq) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m * m) return;
  const int w = 2 * rho + 1;
  const int ix = i / m, iy = i % m;
  double acc = 0.0;
  for (int dx = -rho; dx <= rho; ++dx) {
    const int lx = ix + dx;
    if (lx < 0 || lx >= m) continue;
    double row = 0.0;
    for (int dy = -rho; dy <= rho; ++dy) {
      const int ly = iy + dy;
      if (ly < 0 || ly >= m) continue;
      row += Y[(size_t)iy * w + dy + rho] * b[(size_t)lx * m + ly];
    }
    acc += Y[(size_t)ix * w + dx + rho] * row;
  }
  gq[i] = acc;
}

// u_l = sum_{i : l in patch(i)} Y[ix][lx-ix] Y[iy][ly-iy] U_i
__global__ void k_level_q_to_nodal(int m, int rho, const double* __restrict__ Y, const double* __restrict__ U,
                                   double* __restrict__ u) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= m * m) return;
  const int w = 2 * rho + 1;
  const int lx = l / m, ly = l % m;
  double acc = 0.0;
  for (int dx = -rho; dx <= rho; ++dx) {
    const int ix = lx - dx;
    if (ix < 0 || ix >= m) continue;
    double row = 0.0;
    for (int dy = -rho; dy <= rho; ++dy) {
      const int iy = ly - dy;
      if (iy < 0 || iy >= m) continue;
      row += Y[(size_t)iy * w + dy + rho] * U[(size_t)ix * m + iy];
    }
    acc += Y[(size_t)ix * w + dx + rho] * row;
  }
  u[l] = acc;
}

// A_{l, l+s} of the Q1 stiffness matrix, s in {-1, 0, 1}^2, from the cell
// coefficient and the unit element matrix (diagonal 4/6, edge neighbour
// -1/6 per shared cell, diagonal neighbour -2/6).  The cells are a block held
// in LDS: sa[u * CA + v] is the cell (x0 + u, y0 + v), and (LX, LY) are the
// node coordinates of l relative to (x0, y0) (node (X, Y) is the corner
// shared by cells X-1 .. X and Y-1 .. Y).
template <int CA>
__device__ __forceinline__ double stiffness_lds(const double* __restrict__ sa, int LX, int LY, int sx, int sy) {
  if (sx == 0 && sy == 0)
    return (4.0 / 6.0) * (sa[(LX - 1) * CA + LY - 1] + sa[LX * CA + LY - 1] + sa[(LX - 1) * CA + LY] + sa[LX * CA + LY]);
  const int cx = sx < 0 ? LX - 1 : LX;
  const int cy = sy < 0 ? LY - 1 : LY;
  if (sy == 0) return (-1.0 / 6.0) * (sa[cx * CA + LY - 1] + sa[cx * CA + LY]);
  if (sx == 0) return (-1.0 / 6.0) * (sa[(LX - 1) * CA + cy] + sa[LX * CA + cy]);
  return (-2.0 / 6.0) * sa[cx * CA + cy];
}

// One wavefront per interior node i, four nodes per workgroup.  Output row i
// of A^(q): AQ[i][(dx + S)(2S + 1) + dy + S], S = 2 RHO + 1, zero where
// i + (dx, dy) is not an interior node.  The cells under the grown patch
// (2 RHO + 4 per side) are staged in LDS first.
// With ARENA set the row goes to the hierarchy's offset-major level-q
// operator instead: AQ[(dx + S)(2S + 1) + dy + S][slot], slot = (ix + 1) n +
// iy + 1, in the hierarchy's precision T (the empty slots x = 0 or y = 0 are
// left to the caller).
template <int RHO, typename T = double, bool ARENA = false>
__global__ __launch_bounds__(256) void k_level_q_operator(int n, const double* __restrict__ a,
                                                          const double* __restrict__ Y, T* __restrict__ AQ) {
  constexpr int P = 2 * RHO + 1;      // patch width
  constexpr int CW = 2 * RHO + 3;     // width of the support of c = A Minv e_i
  constexpr int S = 2 * RHO + 1;      // half width of the level-q stencil
  constexpr int AW = 2 * S + 1;
  __shared__ double sy[4][2][AW][P];  // 1-D factors at ix + dx and iy + dy, dx, dy in [-S, S]
  __shared__ double sc[4][CW][CW];
  __shared__ double st[4][AW][CW];
  constexpr int CA = 2 * RHO + 4;     // cells under the grown patch, per side
  __shared__ double sa[4][CA * CA];
  const int m = n - 1;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const long i = (long)blockIdx.x * 4 + wv;
  const bool valid = i < (long)m * m;
  const int ix = valid ? (int)(i / m) : 0, iy = valid ? (int)(i % m) : 0;
  // node (ix + ox, iy + oy), interior coordinates, has node coordinates
  // (ix + ox + 1, ...) and touches cells ix + ox .. ix + ox + 1: the block
  // starts at cell x0 = ix - RHO - 1
  const int x0 = ix - RHO - 1, y0 = iy - RHO - 1;
  for (int e = lane; e < CA * CA; e += 64) {
    const int cx = x0 + e / CA, cy = y0 + e % CA;
    sa[wv][e] = (cx >= 0 && cx < n && cy >= 0 && cy < n) ? a[(size_t)cx * n + cy] : 0.0;
  }
  // 1. factors of the patches of the nodes in the stencil's reach
  for (int e = lane; e < 2 * AW * P; e += 64) {
    const int dim = e / (AW * P), k = (e / P) % AW, d = e % P;
    const int p = (dim == 0 ? ix : iy) + k - S;
    sy[wv][dim][k][d] = (p >= 0 && p < m) ? Y[(size_t)p * P + d] : 0.0;
  }
  __syncthreads();
  // 2. c = A Minv e_i on the grown patch: c[ox][oy] at node i + o
  for (int e = lane; e < CW * CW; e += 64) {
    const int ox = e / CW - (RHO + 1), oy = e % CW - (RHO + 1);
    const int lx = ix + ox, ly = iy + oy;
    double acc = 0.0;
    if (valid && lx >= 0 && lx < m && ly >= 0 && ly < m) {
#pragma unroll
      for (int sx = -1; sx <= 1; ++sx) {
        const int wx = ox + sx;   // offset of the neighbour from i
        if (wx < -RHO || wx > RHO) continue;
        const double fx = sy[wv][0][S][wx + RHO];
#pragma unroll
        for (int sy_ = -1; sy_ <= 1; ++sy_) {
          const int wy = oy + sy_;
          if (wy < -RHO || wy > RHO) continue;
          const double f = fx * sy[wv][1][S][wy + RHO];
          if (f != 0.0) acc += stiffness_lds<CA>(sa[wv], ox + RHO + 2, oy + RHO + 2, sx, sy_) * f;
        }
      }
    }
    sc[wv][ox + RHO + 1][oy + RHO + 1] = acc;
  }
  __syncthreads();
  // 3. t[dx][my] = sum_mx c[mx][my] Y[ix + dx][mx - dx], offsets from i
  for (int e = lane; e < AW * CW; e += 64) {
    const int kx = e / CW, cy = e % CW;
    const int dx = kx - S;
    double acc = 0.0;
#pragma unroll
    for (int cx = 0; cx < CW; ++cx) {
      const int d = (cx - (RHO + 1)) - dx;   // node i + mx relative to node i + dx
      if (d >= -RHO && d <= RHO) acc += sc[wv][cx][cy] * sy[wv][0][kx][d + RHO];
    }
    st[wv][kx][cy] = acc;
  }
  __syncthreads();
  // 4. A^(q)_{i, i + (dx, dy)} = sum_my t[dx][my] Y[iy + dy][my - dy]
  if (valid) {
    for (int e = lane; e < AW * AW; e += 64) {
      const int kx = e / AW, ky = e % AW;
      const int dy = ky - S;
      double acc = 0.0;
#pragma unroll
      for (int cy = 0; cy < CW; ++cy) {
        const int d = (cy - (RHO + 1)) - dy;
        if (d >= -RHO && d <= RHO) acc += st[wv][kx][cy] * sy[wv][1][ky][d + RHO];
      }
      if (ARENA)
        AQ[(size_t)e * n * n + (size_t)(ix + 1) * n + iy + 1] = T(acc);
      else
        AQ[(size_t)i * AW * AW + e] = T(acc);
    }
  }
}

void launch_mass_inverse_table(int n, int rho, double* Y, hipStream_t st) {
  const int m = n - 1;
  hipLaunchKernelGGL(k_mass_inverse_table, dim3((m + 63) / 64), dim3(64), 0, st, m, rho, (double)n, Y);
}

void launch_level_q_weights(int n, int rho, const double* Y, double* W, hipStream_t st) {
  const int m = n - 1, w = 2 * rho + 1;
  const size_t total = (size_t)m * m * w * w;
  hipLaunchKernelGGL(k_level_q_weights, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, m, rho, Y, W);
}

void launch_level_q_load(int n, int rho, const double* Y, const double* b, double* gq, hipStream_t st) {
  const int m = n - 1;
  hipLaunchKernelGGL(k_level_q_load, dim3((m * m + 255) / 256), dim3(256), 0, st, m, rho, Y, b, gq);
}

void launch_level_q_to_nodal(int n, int rho, const double* Y, const double* U, double* u, hipStream_t st) {
  const int m = n - 1;
  hipLaunchKernelGGL(k_level_q_to_nodal, dim3((m * m + 255) / 256), dim3(256), 0, st, m, rho, Y, U, u);
}

void launch_level_q_operator(int n, int rho, const double* a, const double* Y, double* AQ, hipStream_t st) {
  const long m2 = (long)(n - 1) * (n - 1);
  const dim3 grid((unsigned)((m2 + 3) / 4)), block(256);
  switch (rho) {
    case 1: hipLaunchKernelGGL(k_level_q_operator<1>, grid, block, 0, st, n, a, Y, AQ); break;
    case 2: hipLaunchKernelGGL(k_level_q_operator<2>, grid, block, 0, st, n, a, Y, AQ); break;
    case 3: hipLaunchKernelGGL(k_level_q_operator<3>, grid, block, 0, st, n, a, Y, AQ); break;
    default: hipLaunchKernelGGL(k_level_q_operator<4>, grid, block, 0, st, n, a, Y, AQ); break;
  }
}

// Positive, finite cell coefficients (the nodal-basis build checks them in
// its assembly kernel).
__global__ void k_check_cells(const double* __restrict__ a, int n, int* __restrict__ status) {
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= n * n) return;
  const double v = a[id];
  if (!(v > 0.0) || !(v < INFINITY)) atomicOr(status, kBadCoefficient);
}

template <typename T>
void launch_level_q_operator_arena(int n, int rho, const double* a, const double* Y, T* A, int* status,
                                   hipStream_t st) {
  const long m2 = (long)(n - 1) * (n - 1);
  const dim3 grid((unsigned)((m2 + 3) / 4)), block(256);
  hipLaunchKernelGGL(k_check_cells, dim3((n * n + 255) / 256), dim3(256), 0, st, a, n, status);
  switch (rho) {
    case 1: hipLaunchKernelGGL((k_level_q_operator<1, T, true>), grid, block, 0, st, n, a, Y, A); break;
    case 2: hipLaunchKernelGGL((k_level_q_operator<2, T, true>), grid, block, 0, st, n, a, Y, A); break;
    case 3: hipLaunchKernelGGL((k_level_q_operator<3, T, true>), grid, block, 0, st, n, a, Y, A); break;
    default: hipLaunchKernelGGL((k_level_q_operator<4, T, true>), grid, block, 0, st, n, a, Y, A); break;
  }
}
template void launch_level_q_operator_arena<float>(int, int, const double*, const double*, float*, int*,
                                                   hipStream_t);
template void launch_level_q_operator_arena<double>(int, int, const double*, const double*, double*, int*,
                                                    hipStream_t);

}  // namespace gbl
