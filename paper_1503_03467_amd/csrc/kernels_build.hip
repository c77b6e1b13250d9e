// Build-phase kernels of the localized gamblet hierarchy (Algorithm 2,
// fine-to-coarse sweep) for gfx950.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdlib>

#include "device_common.hpp"
#include "gamblet_internal.hpp"

namespace gbl {

// ---------------------------------------------------------------------------
// Fine stiffness A^(q) = A (first step of Algorithm 2; level-q gamblets are the
// nodal basis functions).  Bilinear element on a square cell with
// coefficient a_e: diagonal 2/3 a_e, edge neighbours -1/6 a_e, opposite
// corner -1/3 a_e.  One thread per node slot; the nine couplings are
// written offset-major, A[ox*3+oy][x*n+y].  Couplings to boundary nodes and
// the rows of boundary slots are zero.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_assemble_fine(const double* __restrict__ a, T* __restrict__ A, int n,
                                int* __restrict__ status) {
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= n * n) return;
  const int x = id / n, y = id % n;
  const size_t nn = (size_t)n * n;
  if (x == 0 || y == 0) {
    for (int e = 0; e < 9; ++e) A[e * nn + id] = T(0);
    return;
  }
  // cells around node (x, y): (x-1,y-1), (x,y-1), (x-1,y), (x,y)
  const double a00 = a[(x - 1) * n + (y - 1)];
  const double a10 = a[x * n + (y - 1)];
  const double a01 = a[(x - 1) * n + y];
  const double a11 = a[x * n + y];
  if (!(a00 > 0.0 && a10 > 0.0 && a01 > 0.0 && a11 > 0.0) ||
      !(a00 < INFINITY && a10 < INFINITY && a01 < INFINITY && a11 < INFINITY)) {
    atomicOr(status, kBadCoefficient);
  }
  double v[3][3];
  v[1][1] = (2.0 / 3.0) * (a00 + a10 + a01 + a11);
  v[2][1] = -(a10 + a11) / 6.0;
  v[0][1] = -(a00 + a01) / 6.0;
  v[1][2] = -(a01 + a11) / 6.0;
  v[1][0] = -(a00 + a10) / 6.0;
  v[2][2] = -a11 / 3.0;
  v[0][0] = -a00 / 3.0;
  v[2][0] = -a10 / 3.0;
  v[0][2] = -a01 / 3.0;
  for (int ox = 0; ox < 3; ++ox) {
    for (int oy = 0; oy < 3; ++oy) {
      const int xx = x + ox - 1, yy = y + oy - 1;
      const bool inner = xx >= 1 && xx <= n - 1 && yy >= 1 && yy <= n - 1;
      A[(ox * 3 + oy) * nn + id] = inner ? T(v[ox][oy]) : T(0);
    }
  }
}

template <typename T>
void launch_assemble_fine(const double* a, T* A, int n, int* status, hipStream_t st) {
  const int tot = n * n;
  hipLaunchKernelGGL(k_assemble_fine<T>, dim3((tot + 255) / 256), dim3(256), 0, st, a, A, n, status);
}

// ---------------------------------------------------------------------------
// Subband operator B^(k) = W^(k) A^(k) W^(k)T (eq. defining B, Section 4.7;
// Algorithm 2) in parent-block stencil form (entry (o, 3i + j) of
// parent p couples subband row (p, i) to (p + o - t, j); block-interleaved
// layout, see b_index), plus the inverse of every 3x3 diagonal block
// (block-Jacobi preconditioner of the subband CG).  One thread per
// (parent, neighbour parent) pair; the 64 lanes of a wavefront take 64
// consecutive parents and one neighbour offset, so each store of B (and each
// read of a stencil plane of A) covers consecutive words.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T a_entry(const T* __restrict__ A, int nk, int s, int cx, int cy, int dx,
                                     int dy) {
  // A^(k)_{(cx,cy),(dx,dy)}; zero outside the grid or the stencil
  if (cx < 0 || cy < 0 || cx >= nk || cy >= nk) return T(0);
  if (dx < 0 || dy < 0 || dx >= nk || dy >= nk) return T(0);
  const int ox = dx - cx + s, oy = dy - cy + s;
  const int S = 2 * s + 1;
  if (ox < 0 || oy < 0 || ox >= S || oy >= S) return T(0);
  return A[(size_t)(ox * S + oy) * nk * nk + cx * nk + cy];
}

template <typename T>
__global__ void k_subband_operator(const T* __restrict__ A, T* __restrict__ B, T* __restrict__ BJ,
                                   int nk, int s, int t, int fine) {
  const int np = nk / 2;
  const int TT = 2 * t + 1;
  const long id = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long g = id >> 6;   // (group of 64 parents, offset)
  const int o = (int)(g % (TT * TT));
  const int p = (int)((g / (TT * TT)) * 64 + (id & 63));
  if (p >= np * np) return;
  const int px = p / np, py = p % np;
  const int ox = o / TT, oy = o % TT;
  const int qx = px + ox - t, qy = py + oy - t;
  const size_t np2 = (size_t)np * np;
  T* out = B + b_index(o, 0, p, TT);   // entry e at out[64 e]
  if (qx < 0 || qy < 0 || qx >= np || qy >= np) {
    for (int e = 0; e < 9; ++e) out[64 * e] = T(0);
    return;
  }
  const int tp = parent_type(fine != 0, px, py);
  const int tq = parent_type(fine != 0, qx, qy);
  // M[d][d'] = A_{child d of p, child d' of q}
  double M[4][4];
  for (int d = 0; d < 4; ++d) {
    for (int e = 0; e < 4; ++e) {
      M[d][e] = (double)a_entry(A, nk, s, 2 * px + (d >> 1), 2 * py + (d & 1), 2 * qx + (e >> 1),
                                2 * qy + (e & 1));
    }
  }
  double Bl[3][3];
  for (int i = 0; i < 3; ++i) {
    double tmp[4];
    for (int e = 0; e < 4; ++e) {
      double acc = 0.0;
      for (int d = 0; d < 4; ++d) acc += wcoef(tp, i, d) * M[d][e];
      tmp[e] = acc;
    }
    for (int j = 0; j < 3; ++j) {
      double acc = 0.0;
      for (int e = 0; e < 4; ++e) acc += tmp[e] * wcoef(tq, j, e);
      Bl[i][j] = acc;
    }
  }
  const bool center = (ox == t && oy == t);
  if (center) {
    for (int i = 0; i < 3; ++i) {
      if (is_pad_row(tp, i)) {
        for (int j = 0; j < 3; ++j) Bl[i][j] = Bl[j][i] = 0.0;
        Bl[i][i] = 1.0;
      }
    }
  }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) out[64 * (i * 3 + j)] = T(Bl[i][j]);
  if (center) {
    // inverse of the symmetric 3x3 diagonal block by cofactors
    const double a0 = Bl[0][0], a1 = Bl[0][1], a2 = Bl[0][2];
    const double b1 = Bl[1][1], b2 = Bl[1][2], c2 = Bl[2][2];
    const double C00 = b1 * c2 - b2 * b2, C01 = -(a1 * c2 - a2 * b2), C02 = a1 * b2 - a2 * b1;
    const double C11 = a0 * c2 - a2 * a2, C12 = -(a0 * b2 - a1 * a2), C22 = a0 * b1 - a1 * a1;
    const double det = a0 * C00 + a1 * C01 + a2 * C02;
    const double id = det != 0.0 ? 1.0 / det : 0.0;
    T* bj = BJ + p;   // BJ[e * np2 + p]
    bj[0 * np2] = T(C00 * id); bj[1 * np2] = T(C01 * id); bj[2 * np2] = T(C02 * id);
    bj[3 * np2] = T(C01 * id); bj[4 * np2] = T(C11 * id); bj[5 * np2] = T(C12 * id);
    bj[6 * np2] = T(C02 * id); bj[7 * np2] = T(C12 * id); bj[8 * np2] = T(C22 * id);
  }
}

template <typename T>
void launch_subband_operator(const LevelGeom& L, const T* A, T* B, T* BJ, bool fine, hipStream_t st) {
  const int np = L.nk / 2;
  const int TT = 2 * L.t + 1;
  const long tot = (long)((np * np + 63) / 64) * 64 * TT * TT;   // whole groups of 64 parents
  hipLaunchKernelGGL(k_subband_operator<T>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, A, B,
                     BJ, L.nk, L.s, L.t, fine ? 1 : 0);
}

// ---------------------------------------------------------------------------
// Patch solves and restriction (Definition 5.3; Algorithm 2).
//
// One workgroup of 256 threads (a 16 x 16 thread grid) per coarse cell i of
// level k-1.  The patch is the box of coarse cells within rho of i, clipped
// to the domain; its unknowns are the subband indices of those parents
// (3 per parent).  The patch matrix B^(i,rho), symmetrically scaled by the
// inverse square roots of its diagonal, is held in registers in a
// block-cyclic layout: thread (tr, tc) owns entries (tr + 16 a, tc + 16 b),
// a >= b.  The right-hand side -(W A pibar^T)_{i^chi, i} is appended as an
// extra last row, so the right-looking Cholesky factorisation also performs
// the forward substitution.  Column j is broadcast through LDS (double
// buffered, one barrier per column); a back substitution follows.  The
// patch solution y gives the restriction row
// R_i = pibar_i + sum_{j in i^chi} y_j W_j.
// ---------------------------------------------------------------------------
template <typename T, int MB>
__global__ __launch_bounds__(256) void k_patch_solve(const T* __restrict__ A, const T* __restrict__ B,
                                                     T* __restrict__ R, int nk, int s, int t, int rho,
                                                     int fine, int* __restrict__ status) {
  constexpr int P = 16 * MB;
  constexpr int NE = MB * (MB + 1) / 2;
  const int nc = nk / 2;
  const int ci = xcd_remap((int)blockIdx.x, (int)gridDim.x);
  const int cx = ci / nc, cy = ci % nc;
  const int x0 = max(0, cx - rho), x1 = min(nc - 1, cx + rho);
  const int y0 = max(0, cy - rho), y1 = min(nc - 1, cy + rho);
  const int wy = y1 - y0 + 1;
  const int npar = (x1 - x0 + 1) * wy;
  const int p = 3 * npar;   // unknowns; row p carries the right-hand side
  const int tid = threadIdx.x;
  const int tr = tid >> 4, tc = tid & 15;
  const int TT = 2 * t + 1;
  const int S = 2 * s + 1;
  const int ti = parent_type(fine != 0, cx, cy);
  const size_t nc2 = (size_t)nc * nc;

  __shared__ T colbuf[2][P];
  __shared__ T pivv[P];
  __shared__ T ldiag[P];
  __shared__ T zb[P];
  __shared__ T sc[P];
  __shared__ int flag;
  if (tid == 0) flag = 0;

  // scaling and right-hand side
  for (int r = tid; r < P; r += 256) {
    T scale = T(1), rhs = T(0);
    if (r < p) {
      const int lp = r / 3, tt = r - 3 * lp;
      const int px = x0 + lp / wy, py = y0 + lp % wy;
      const T d = B[b_index(t * TT + t, tt * 4, px * nc + py, TT)];
      if (d > T(0)) {
        scale = T(1) / my_sqrt<T>(d);
      } else {
        atomicOr(status, kBadPivot);
      }
      const int tp = parent_type(fine != 0, px, py);
      // b_(p,tt) = - sum_d W_tt(p)[d] sum_e pibar_i[e] A_{2p+d, 2i+e}
      if (abs(px - cx) <= t && abs(py - cy) <= t && !is_pad_row(tp, tt)) {
        double acc = 0.0;
        for (int d = 0; d < 4; ++d) {
          const double wd = wcoef(tp, tt, d);
          if (wd == 0.0) continue;
          const int fx = 2 * px + (d >> 1), fy = 2 * py + (d & 1);
          double inner = 0.0;
          for (int e = 0; e < 4; ++e) {
            const double pe = pibar(ti, e);
            if (pe == 0.0) continue;
            const int gx = 2 * cx + (e >> 1), gy = 2 * cy + (e & 1);
            const int ox = gx - fx + s, oy = gy - fy + s;
            if (ox < 0 || oy < 0 || ox >= S || oy >= S) continue;
            inner += pe * (double)A[(size_t)(ox * S + oy) * nk * nk + fx * nk + fy];
          }
          acc += wd * inner;
        }
        rhs = T(-acc);
      }
    }
    sc[r] = scale;
    zb[r] = rhs * scale;
  }
  __syncthreads();

  // load the scaled patch matrix (lower triangle) and the right-hand-side row
  T a[NE];
#pragma unroll
  for (int ai = 0; ai < MB; ++ai) {
#pragma unroll
    for (int bi = 0; bi <= ai; ++bi) {
      const int r = tr + 16 * ai, c = tc + 16 * bi;
      T v;
      if (r < p && c < p) {
        if (r >= c) {
          const int lr = r / 3, trr = r - 3 * lr;
          const int lc = c / 3, tcc = c - 3 * lc;
          const int rx = x0 + lr / wy, ry = y0 + lr % wy;
          const int qx = x0 + lc / wy, qy = y0 + lc % wy;
          const int ox = qx - rx + t, oy = qy - ry + t;
          T bv = T(0);
          if (ox >= 0 && oy >= 0 && ox < TT && oy < TT)
            bv = B[b_index(ox * TT + oy, trr * 3 + tcc, rx * nc + ry, TT)];
          v = bv * sc[r] * sc[c];
        } else {
          v = T(0);
        }
      } else if (r == p && c < p) {
        v = zb[c];
      } else {
        v = (r == c) ? T(1) : T(0);
      }
      a[ai * (ai + 1) / 2 + bi] = v;
    }
  }

  // first column broadcast
  if (tc == 0) {
#pragma unroll
    for (int ai = 0; ai < MB; ++ai) {
      const int r = tr + 16 * ai;
      const T v = a[ai * (ai + 1) / 2];
      colbuf[0][r] = (r > 0 && r <= p) ? v : T(0);
      if (r == 0) pivv[0] = v;
    }
  }
  __syncthreads();

  for (int j = 0; j < p; ++j) {
    const T* cur = colbuf[j & 1];
    T* nxt = colbuf[(j + 1) & 1];
    int pbad = 0, preg = 0;
    const T pv = patch_pivot<T>(pivv[j], pbad, preg);
    if (tid == 0 && (pbad | preg)) flag |= pbad | (preg << 1);
    const T sq = my_sqrt<T>(pv);
    const T inv = T(1) / pv;
    const T rs = T(1) / sq;
    T cr[MB], cc[MB];
#pragma unroll
    for (int m = 0; m < MB; ++m) {
      cr[m] = cur[tr + 16 * m];
      cc[m] = cur[tc + 16 * m] * inv;
    }
    // scale the owned part of column j into L
    const int bj = j >> 4;
    if (tc == (j & 15)) {
#pragma unroll
      for (int bi = 0; bi < MB; ++bi) {
        if (bi == bj) {
#pragma unroll
          for (int ai = bi; ai < MB; ++ai) {
            const int r = tr + 16 * ai;
            T& e = a[ai * (ai + 1) / 2 + bi];
            if (r > j) e = e * rs;
            else if (r == j) { e = sq; ldiag[j] = sq; }
          }
        }
      }
    }
    // trailing update a_rc -= c_r c_c / pivot (entries of retired columns see c = 0)
#pragma unroll
    for (int bi = 0; bi < MB; ++bi) {
      if (16 * bi + 15 > j) {
#pragma unroll
        for (int ai = bi; ai < MB; ++ai) a[ai * (ai + 1) / 2 + bi] -= cr[ai] * cc[bi];
      }
    }
    // publish column j+1
    const int jn = j + 1;
    if (jn < p && tc == (jn & 15)) {
      const int bn = jn >> 4;
#pragma unroll
      for (int bi = 0; bi < MB; ++bi) {
        if (bi == bn) {
#pragma unroll
          for (int ai = bi; ai < MB; ++ai) {
            const int r = tr + 16 * ai;
            const T v = a[ai * (ai + 1) / 2 + bi];
            nxt[r] = (r > jn && r <= p) ? v : T(0);
            if (r == jn) pivv[jn] = v;
          }
        }
      }
    }
    __syncthreads();
  }

  // forward-substitution result z = L^{-1} b sits in row p
  if (tr == (p & 15)) {
    const int ap = p >> 4;
#pragma unroll
    for (int ai = 0; ai < MB; ++ai) {
      if (ai == ap) {
#pragma unroll
        for (int bi = 0; bi <= ai; ++bi) {
          const int c = tc + 16 * bi;
          if (c < p) zb[c] = a[ai * (ai + 1) / 2 + bi];
        }
      }
    }
  }
  __syncthreads();
  // back substitution L^T x = z, row j of L owned by threads with tr = j mod 16
  for (int j = p - 1; j >= 0; --j) {
    if (tr == (j & 15)) {
      const int aj = j >> 4;
      const T xj = zb[j] / ldiag[j];
#pragma unroll
      for (int ai = 0; ai < MB; ++ai) {
        if (ai == aj) {
#pragma unroll
          for (int bi = 0; bi <= ai; ++bi) {
            const int c = tc + 16 * bi;
            if (c < j) zb[c] -= a[ai * (ai + 1) / 2 + bi] * xj;
          }
        }
      }
      if (tc == (j & 15)) pivv[j] = xj;   // x_j (pivot values are no longer needed)
    }
    __syncthreads();
  }
  // unscale: y_r = sc_r x_r
  for (int r = tid; r < p; r += 256) zb[r] = pivv[r] * sc[r];
  if (tid == 0 && (flag & 1)) atomicOr(status, kBadPivot);
  if (tid == 0 && (flag & 2)) atomicOr(status, kRegularizedPivot);
  __syncthreads();

  // R_i[bx][by] over level-k slots c = 2(cx - rho) + bx
  const int rw = 2 * (2 * rho + 1);
  const int ox0 = 2 * (cx - rho), oy0 = 2 * (cy - rho);
  T* Ri = R + ci;   // R[e * nc2 + ci]
  for (int e = tid; e < rw * rw; e += 256) {
    const int bx = e / rw, by = e % rw;
    const int fx = ox0 + bx, fy = oy0 + by;
    double v = 0.0;
    if (fx >= 0 && fy >= 0 && fx < nk && fy < nk) {
      const int px = fx >> 1, py = fy >> 1;
      const int d = 2 * (fx & 1) + (fy & 1);
      const int tp = parent_type(fine != 0, px, py);
      if (px == cx && py == cy) v = pibar(tp, d);
      const int lp = (px - x0) * wy + (py - y0);
      for (int tt = 0; tt < 3; ++tt) v += (double)zb[3 * lp + tt] * wcoef(tp, tt, d);
    }
    Ri[(size_t)e * nc2] = T(v);
  }
}

template <typename T>
void launch_patch_solve_band(const LevelGeom& L, const T* A, const T* B, T* R, int* status, hipStream_t st,
                             int variant);
template <typename T, int NT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_patch_chol_mfma(const T* __restrict__ A, const T* __restrict__ B,
                                                         const T* __restrict__ Bp, T* __restrict__ R, int nk,
                                                         int s, int t, int rho, int fine,
                                                         int* __restrict__ status);

// B^(k) with the (2t+1)^2 x 9 entries of each parent contiguous, Bp[p][o][e]
// (the operators keep 64 parents fastest; a patch gathers one parent's
// entries at a time).  Tiles of 64 parents x 32 entries through LDS, so that
// both the reads and the writes are coalesced.
template <typename T>
__global__ __launch_bounds__(256) void k_b_parent_major(const T* __restrict__ B, T* __restrict__ Bp, int np2,
                                                        int per) {
  __shared__ T tile[32][65];
  const int grp = blockIdx.x;
  const int oe0 = blockIdx.y * 32;
  for (int e = threadIdx.x; e < 32 * 64; e += 256) {
    const int r = e >> 6, pl = e & 63;
    const int oe = oe0 + r;
    tile[r][pl] = (oe < per) ? B[((size_t)grp * per + oe) * 64 + pl] : T(0);
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 32 * 64; e += 256) {
    const int pl = e >> 5, r = e & 31;
    const int p = grp * 64 + pl, oe = oe0 + r;
    if (p < np2 && oe < per) Bp[(size_t)p * per + oe] = tile[r][pl];
  }
}

// Dense patch kernel choice: the matrix-core kernel for FP32 patches, the
// register-tiled kernel for FP64 ones (whose accumulator tiles would leave one
// workgroup per compute unit).  GBL_PATCH_MFMA=1 or 0 forces one kernel for
// both; the parity tests run both.
// Dense patch solves on the matrix cores by default, in FP32 and in FP64
// (timed faster than the register-tiled kernel on every level but the
// smallest, where both take a few microseconds); GBL_PATCH_MFMA=0 selects
// the register-tiled kernel.
template <typename T>
static bool patch_mfma_enabled() {
  const char* e = getenv("GBL_PATCH_MFMA");
  return !(e && e[0] == '0');
}

int patch_class(const LevelGeom& L, bool fine) {
  return (fine && L.t == 1 && L.nk / 2 > 2 * L.rho + 1) ? kKernelBand : kKernelPatch;
}

template <typename T>
bool patch_variant_ok(const LevelGeom& L, bool fine, int variant) {
  const int nc = L.nk / 2;
  if (patch_class(L, fine) == kKernelBand) return variant == 0 || (variant == 1 && L.rho <= 3);
  const int wmax = (2 * L.rho + 1) < nc ? (2 * L.rho + 1) : nc;
  return variant == 0 || (variant == 1 && 3 * wmax * wmax + 1 <= 160);
}

template <typename T>
void launch_patch_solve(const LevelGeom& L, const T* A, const T* B, T* R, T* Bp, bool fine, int* status,
                        hipStream_t st, int variant) {
  const int nc = L.nk / 2;
  if (patch_class(L, fine) == kKernelBand) {
    launch_patch_solve_band<T>(L, A, B, R, status, st, variant);
    return;
  }
  const int wmax = (2 * L.rho + 1) < nc ? (2 * L.rho + 1) : nc;
  const int need = 3 * wmax * wmax + 1;
  const dim3 grid(nc * nc), block(256);
  const int f = fine ? 1 : 0;
  const bool mfma = variant == kVariantDefault ? patch_mfma_enabled<T>() : variant == 1;
  if (mfma && need <= 160) {
    const int np2 = nc * nc, TT = 2 * L.t + 1, per = TT * TT * 9;
    hipLaunchKernelGGL(k_b_parent_major<T>, dim3((np2 + 63) / 64, (per + 31) / 32), dim3(256), 0, st, B, Bp, np2, per);
    hipLaunchKernelGGL((k_patch_chol_mfma<T, 10>), grid, block, 0, st, A, B, Bp, R, L.nk, L.s, L.t, L.rho, f,
                       status);
    return;
  }
  if (need <= 32) {
    hipLaunchKernelGGL((k_patch_solve<T, 2>), grid, block, 0, st, A, B, R, L.nk, L.s, L.t, L.rho, f, status);
  } else if (need <= 80) {
    hipLaunchKernelGGL((k_patch_solve<T, 5>), grid, block, 0, st, A, B, R, L.nk, L.s, L.t, L.rho, f, status);
  } else if (need <= 160) {
    hipLaunchKernelGGL((k_patch_solve<T, 10>), grid, block, 0, st, A, B, R, L.nk, L.s, L.t, L.rho, f, status);
  } else {
    hipLaunchKernelGGL((k_patch_solve<T, 16>), grid, block, 0, st, A, B, R, L.nk, L.s, L.t, L.rho, f, status);
  }
}

// ---------------------------------------------------------------------------
// Patch solves on matrix cores (levels k < q): blocked right-looking Cholesky
// with 16 x 16 tiles.  The scaled patch matrix, with the right-hand side as
// row p, is held as MFMA accumulator tiles (I, J), J <= I, dealt round-robin
// to the four wavefronts (tile number I (I + 1) / 2 + J = 4 m + wave).  For
// each panel P:
//   1. the panel tiles (I, P) go to LDS;
//   2. lanes 0..15 of wavefront 0 hold the rows of the diagonal tile in
//      registers and factor it, L_PP, exchanging column values with lane
//      reads (no LDS round trips);
//   3. one thread per panel row solves l L_PP^T = a (rows of L_IP, I > P),
//      and sixteen more threads solve it for the unit rows, giving the rows
//      of L_PP^{-T} used by the back substitution;
//   4. A_IJ -= L_IP L_JP^T for P < J <= I on the matrix cores.
// Row p of the factor is z = L^{-1} b; a blocked back substitution with the
// stored L_PP^{-T} gives x = L^{-T} z.  Scaling, right-hand side and the
// restriction row are those of the register-tiled kernel.
// ---------------------------------------------------------------------------
typedef float gbl_v4f __attribute__((ext_vector_type(4)));
typedef double gbl_v4d __attribute__((ext_vector_type(4)));

template <typename T>
struct Mfma;
template <>
struct Mfma<float> {
  typedef gbl_v4f acc_t;
  static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // accumulator element r of lane l is tile row row(l, r), column l % 16
  static __device__ __forceinline__ int row(int l, int r) { return 4 * (l >> 4) + r; }
  static __device__ __forceinline__ float lane_value(float v, int lane) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
  }
};
template <>
struct Mfma<double> {
  typedef gbl_v4d acc_t;
  static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int l, int r) { return (l >> 4) + 4 * r; }
  static __device__ __forceinline__ double lane_value(double v, int lane) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
  }
};

// 1 / sqrt(pivot) of a Cholesky step: the hardware reciprocal square root
// in FP32 (about one unit of roundoff, well inside the accuracy the conditioning
// of the FP32 patch systems allows), correctly rounded operations in FP64
template <typename T>
__device__ __forceinline__ T pivot_rsqrt(T x);
template <>
__device__ __forceinline__ float pivot_rsqrt<float>(float x) { return __builtin_amdgcn_rsqf(x); }
template <>
__device__ __forceinline__ double pivot_rsqrt<double>(double x) { return 1.0 / my_sqrt<double>(x); }

template <typename T, int NT>
struct CholLds {
  T panel[NT][16][17];   // column-P tiles; rows of L_IP after the solve
  T lpp[16][16];         // factored diagonal tile
  T dinv[16];
  T linvt[NT][16][16];   // rows of L_PP^{-T}
  T sc[16 * NT];
  T rhs[16 * NT];        // scaled right-hand side, later z, then x
  T part[NT][16];
  int rowinfo[16 * NT];  // patch row r: parent (x, y) and subband index, packed (x << 20 | y << 8 | t)
  int bad;
};

// tile (I, J) of tile number tix = I (I + 1) / 2 + J; slots past the last tile get I = NT
__host__ __device__ constexpr int tile_row(int tix, int ntile, int nt) {
  int i = 0;
  while ((i + 1) * (i + 2) / 2 <= tix) ++i;
  return tix < ntile ? i : nt;
}
__host__ __device__ constexpr int tile_col(int tix) {
  int i = 0;
  while ((i + 1) * (i + 2) / 2 <= tix) ++i;
  return tix - i * (i + 1) / 2;
}

// Body of the kernel for wavefront W: its slots m hold the tiles numbered
// 4 m + W, so every tile coordinate is a compile-time constant.
template <typename T, int NT, int W>
__device__ __forceinline__ void patch_chol_mfma_body(CholLds<T, NT>& sm, const T* __restrict__ A,
                                                     const T* __restrict__ B, const T* __restrict__ Bp,
                                                     T* __restrict__ R, int nk, int s, int t, int rho, int fine,
                                                     int* __restrict__ status) {
  typedef typename Mfma<T>::acc_t acc_t;
  constexpr int NTILE = NT * (NT + 1) / 2;
  constexpr int SLOTS = (NTILE + 3) / 4;
  constexpr int P16 = 16 * NT;

  const int nc = nk / 2;
  const int ci = xcd_remap((int)blockIdx.x, (int)gridDim.x);
  const int cx = ci / nc, cy = ci % nc;
  const int x0 = max(0, cx - rho), x1 = min(nc - 1, cx + rho);
  const int y0 = max(0, cy - rho), y1 = min(nc - 1, cy + rho);
  const int wy = y1 - y0 + 1;
  const int npar = (x1 - x0 + 1) * wy;
  const int p = 3 * npar;
  const int nta = (p + 1 + 15) / 16;    // tiles holding rows 0..p
  const int tid = threadIdx.x;
  const int l = tid & 63, lc = l & 15;
  const int TT = 2 * t + 1;
  const int S = 2 * s + 1;
  const int ti = parent_type(fine != 0, cx, cy);
  if (tid == 0) sm.bad = 0;

  // patch rows: parent and subband index (integer work only)
  for (int r = tid; r < p; r += 256) {
    const int lp = r / 3, tt = r - 3 * lp;
    sm.rowinfo[r] = ((x0 + lp / wy) << 20) | ((y0 + lp % wy) << 8) | tt;
  }
  __syncthreads();

  // this wavefront's tiles, gathered from B^(k) unscaled, issued together
  // with the loads of the scaling and right-hand side below (one round of
  // global-memory latency instead of two); the scaling is applied after the
  // barrier, in the same order of products
  acc_t acc[SLOTS];
#pragma unroll
  for (int m = 0; m < SLOTS; ++m) {
    const int I = tile_row(4 * m + W, NTILE, NT), J = tile_col(4 * m + W);
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[m][r] = T(0);
    if (I < nta) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = 16 * I + Mfma<T>::row(l, r), j = 16 * J + lc;
        T v;
        if (i < p && j < p) {
          if (i >= j) {
            const int ri = sm.rowinfo[i], rj = sm.rowinfo[j];
            const int rx = ri >> 20, ry = (ri >> 8) & 0xfff, trr = ri & 0xff;
            const int qx = rj >> 20, qy = (rj >> 8) & 0xfff, tcc = rj & 0xff;
            const int ox = qx - rx + t, oy = qy - ry + t;
            T bv = T(0);
            if (ox >= 0 && oy >= 0 && ox < TT && oy < TT)
              bv = Bp[(size_t)(rx * nc + ry) * (TT * TT * 9) + (ox * TT + oy) * 9 + trr * 3 + tcc];
            v = bv;
          } else {
            v = T(0);
          }
        } else if (i == p && j < p) {
          v = T(0);   // right-hand side, filled in after the barrier
        } else {
          v = (i == j) ? T(1) : T(0);
        }
        acc[m][r] = v;
      }
    }
  }

  // scaling and right-hand side
  for (int r = tid; r < P16; r += 256) {
    T scale = T(1), rv = T(0);
    if (r < p) {
      const int lp = r / 3, tt = r - 3 * lp;
      const int px = x0 + lp / wy, py = y0 + lp % wy;
      const T d = B[b_index(t * TT + t, tt * 4, px * nc + py, TT)];
      if (d > T(0)) scale = T(1) / my_sqrt<T>(d);
      else atomicOr(status, kBadPivot);
      const int tp = parent_type(fine != 0, px, py);
      if (abs(px - cx) <= t && abs(py - cy) <= t && !is_pad_row(tp, tt)) {
        double rsum = 0.0;
        for (int dd = 0; dd < 4; ++dd) {
          const double wd = wcoef(tp, tt, dd);
          if (wd == 0.0) continue;
          const int fx = 2 * px + (dd >> 1), fy = 2 * py + (dd & 1);
          double inner = 0.0;
          for (int e = 0; e < 4; ++e) {
            const double pe = pibar(ti, e);
            if (pe == 0.0) continue;
            const int gx = 2 * cx + (e >> 1), gy = 2 * cy + (e & 1);
            const int ox = gx - fx + s, oy = gy - fy + s;
            if (ox < 0 || oy < 0 || ox >= S || oy >= S) continue;
            inner += pe * (double)A[(size_t)(ox * S + oy) * nk * nk + fx * nk + fy];
          }
          rsum += wd * inner;
        }
        rv = T(-rsum);
      }
    }
    sm.sc[r] = scale;
    sm.rhs[r] = rv * scale;
  }
  __syncthreads();

  // scaled patch matrix and the right-hand side row
#pragma unroll
  for (int m = 0; m < SLOTS; ++m) {
    const int I = tile_row(4 * m + W, NTILE, NT), J = tile_col(4 * m + W);
    if (I < nta) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = 16 * I + Mfma<T>::row(l, r), j = 16 * J + lc;
        if (i < p && j < p && i >= j) acc[m][r] = acc[m][r] * sm.sc[i] * sm.sc[j];
        else if (i == p && j < p) acc[m][r] = sm.rhs[j];
      }
    }
  }

  for (int P = 0; P < nta; ++P) {
    // 1. panel tiles (I, P), I >= P, to LDS
#pragma unroll
    for (int m = 0; m < SLOTS; ++m) {
      const int I = tile_row(4 * m + W, NTILE, NT), J = tile_col(4 * m + W);
      if (J == P && I < nta) {
#pragma unroll
        for (int r = 0; r < 4; ++r) sm.panel[I][Mfma<T>::row(l, r)][lc] = acc[m][r];
      }
    }
    __syncthreads();
    // 2. diagonal tile in the registers of lanes 0..15 of wavefront 0 (lane i
    //    holds row i; entries right of the diagonal are never read).  Rows
    //    from p on are not part of the SPD system: their pivots are taken as 1.
    if (W == 0) {
      T a[16];
#pragma unroll
      for (int c = 0; c < 16; ++c) a[c] = sm.panel[P][lc][c];
      int badl = 0, regl = 0;
      T rinv = T(1);   // 1 / L_PP[lc][lc]
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        T dk = Mfma<T>::lane_value(a[k], k);
        if (16 * P + k >= p) {
          dk = T(1);
        } else {
          dk = patch_pivot<T>(dk, badl, regl);
        }
        const T rk = pivot_rsqrt<T>(dk);
        const T sk = dk * rk;
        if (lc == k) rinv = rk;
        a[k] = (lc > k) ? a[k] * rk : ((lc == k) ? sk : a[k]);
#pragma unroll
        for (int c = k + 1; c < 16; ++c) a[c] -= a[k] * Mfma<T>::lane_value(a[k], c);
      }
      if (l < 16) {
#pragma unroll
        for (int c = 0; c < 16; ++c) sm.lpp[lc][c] = (c <= lc) ? a[c] : T(0);
        sm.dinv[lc] = rinv;
      }
      if (l == 0 && (badl | regl)) sm.bad |= badl | (regl << 1);
    }
    __syncthreads();
    // 3. rows of L_IP (I > P) and of L_PP^{-T}: l[c] = (a[c] - sum_{m<c} l[m] L_PP[c][m]) / L_PP[c][c]
    const int nrow = 16 * (nta - P);
    if (tid < nrow) {
      // threads 0..15 take the unit rows (their tile index is P itself, so the
      // row read is in bounds and then replaced); no divergent branch here
      const bool unit = tid < 16;
      const int I = P + (tid >> 4), i = tid & 15;
      T x[16];
#pragma unroll
      for (int c = 0; c < 16; ++c) {
        const T v = sm.panel[I][i][c];
        x[c] = unit ? ((c == i) ? T(1) : T(0)) : v;
      }
#pragma unroll
      for (int c = 0; c < 16; ++c) {
        T v = x[c];
#pragma unroll
        for (int m2 = 0; m2 < c; ++m2) v -= x[m2] * sm.lpp[c][m2];
        x[c] = v * sm.dinv[c];
      }
      T* dst = unit ? &sm.linvt[P][i][0] : &sm.panel[I][i][0];
#pragma unroll
      for (int c = 0; c < 16; ++c) dst[c] = x[c];
    }
    __syncthreads();
    // 4. keep L_IP (I >= P) in the accumulators; A_IJ -= L_IP L_JP^T for J > P
#pragma unroll
    for (int m = 0; m < SLOTS; ++m) {
      const int I = tile_row(4 * m + W, NTILE, NT), J = tile_col(4 * m + W);
      if (I < nta) {
        if (J == P) {
          if (I == P) {
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[m][r] = sm.lpp[Mfma<T>::row(l, r)][lc];
          } else {
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[m][r] = sm.panel[I][Mfma<T>::row(l, r)][lc];
          }
        } else if (J > P) {
#pragma unroll
          for (int k4 = 0; k4 < 4; ++k4) {
            const T av = -sm.panel[I][lc][4 * k4 + (l >> 4)];
            const T bv = sm.panel[J][lc][4 * k4 + (l >> 4)];
            acc[m] = Mfma<T>::mma(av, bv, acc[m]);
          }
        }
      }
    }
    __syncthreads();
  }

  // z = row p of L
#pragma unroll
  for (int m = 0; m < SLOTS; ++m) {
    const int I = tile_row(4 * m + W, NTILE, NT), J = tile_col(4 * m + W);
    if (I == p / 16) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = 16 * I + Mfma<T>::row(l, r), j = 16 * J + lc;
        if (i == p && j < p) sm.rhs[j] = acc[m][r];
      }
    }
  }
  __syncthreads();
  // back substitution L^T x = z, one column block at a time from the last
  const int ntz = (p + 15) / 16;
  for (int P = ntz - 1; P >= 0; --P) {
    // partial products L_IP^T x_I of the tiles below the diagonal
#pragma unroll
    for (int m = 0; m < SLOTS; ++m) {
      const int I = tile_row(4 * m + W, NTILE, NT), J = tile_col(4 * m + W);
      if (J == P && I > P && I < ntz) {
        T v = T(0);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = 16 * I + Mfma<T>::row(l, r);
          v += acc[m][r] * ((i < p) ? sm.rhs[i] : T(0));
        }
        v += __shfl_xor(v, 16, 64);
        v += __shfl_xor(v, 32, 64);
        if (l < 16) sm.part[I][lc] = v;
      }
    }
    __syncthreads();
    if (W == 0) {
      T y = T(0);
      const int j = 16 * P + lc;
      if (j < p) {
        y = sm.rhs[j];
        for (int I = P + 1; I < ntz; ++I) y -= sm.part[I][lc];
      }
      // x_P = L_PP^{-T} y: x_c = sum_i sm.linvt[c][i] y_i
      T xv = T(0);
#pragma unroll
      for (int i = 0; i < 16; ++i) xv += sm.linvt[P][lc][i] * __shfl(y, i, 64);
      if (l < 16 && j < p) sm.rhs[j] = xv;
    }
    __syncthreads();
  }
  if (tid == 0 && (sm.bad & 1)) atomicOr(status, kBadPivot);
  if (tid == 0 && (sm.bad & 2)) atomicOr(status, kRegularizedPivot);
  // y = sc x, then the restriction row R_i = pibar_i + sum y_j W_j
  for (int r = tid; r < p; r += 256) sm.rhs[r] *= sm.sc[r];
  __syncthreads();
  const int rw = 2 * (2 * rho + 1);
  const int ox0 = 2 * (cx - rho), oy0 = 2 * (cy - rho);
  const size_t nc2 = (size_t)nc * nc;
  T* Ri = R + ci;
  for (int e = tid; e < rw * rw; e += 256) {
    const int bx = e / rw, by = e % rw;
    const int fx = ox0 + bx, fy = oy0 + by;
    double v = 0.0;
    if (fx >= 0 && fy >= 0 && fx < nk && fy < nk) {
      const int px = fx >> 1, py = fy >> 1;
      const int d = 2 * (fx & 1) + (fy & 1);
      const int tp = parent_type(fine != 0, px, py);
      if (px == cx && py == cy) v = pibar(tp, d);
      const int lp = (px - x0) * wy + (py - y0);
      for (int tt = 0; tt < 3; ++tt) v += (double)sm.rhs[3 * lp + tt] * wcoef(tp, tt, d);
    }
    Ri[(size_t)e * nc2] = T(v);
  }
}

template <typename T, int NT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_patch_chol_mfma(
    const T* __restrict__ A, const T* __restrict__ B, const T* __restrict__ Bp, T* __restrict__ R, int nk, int s,
    int t, int rho, int fine, int* __restrict__ status) {
  __shared__ CholLds<T, NT> sm;
  switch (__builtin_amdgcn_readfirstlane(threadIdx.x >> 6)) {
    case 0: patch_chol_mfma_body<T, NT, 0>(sm, A, B, Bp, R, nk, s, t, rho, fine, status); break;
    case 1: patch_chol_mfma_body<T, NT, 1>(sm, A, B, Bp, R, nk, s, t, rho, fine, status); break;
    case 2: patch_chol_mfma_body<T, NT, 2>(sm, A, B, Bp, R, nk, s, t, rho, fine, status); break;
    default: patch_chol_mfma_body<T, NT, 3>(sm, A, B, Bp, R, nk, s, t, rho, fine, status); break;
  }
}

// ---------------------------------------------------------------------------
// Patch solves at the finest transition, band form held in registers
// (rho <= 3).  One wavefront per patch; lane d holds the d-th subdiagonal of
// the scaled patch matrix, M[c + d][c] for c = 0 .. p - 1, in registers (the
// step loop is unrolled, so every register index is static).  Step j: lane 0
// holds the pivot and every lane scales its entry of column j, giving
// L[j + d][j]; for each later column j + e of the band the column is shifted
// down one lane (DPP), its entry e is read out of lane 0's neighbourhood (lane
// read) and lane d updates M[j + e + d][j + e].  The factor stays in place.
// The right-hand side slides through the lanes so that the forward
// substitution rides along; the back substitution sums over lanes.  Same
// scaling, right-hand side and restriction row as the other patch kernels.
// ---------------------------------------------------------------------------
template <typename T>
struct WaveOps;
template <>
struct WaveOps<float> {
  template <int CTRL, int ROWM, bool BC>
  static __device__ __forceinline__ float dpp(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWM, 0xf, BC));
  }
  static __device__ __forceinline__ float lane(float v, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
  }
};
template <>
struct WaveOps<double> {
  template <int CTRL, int ROWM, bool BC>
  static __device__ __forceinline__ double dpp(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, ROWM, 0xf, BC);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROWM, 0xf, BC);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
  }
  static __device__ __forceinline__ double lane(double v, int l) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
  }
};
// Band Cholesky of the finest-level patch systems, two patches per wavefront:
// lane 32 h + d (d < 32) holds subdiagonal d of patch h in registers (the
// half-bandwidth is below 32 for rho <= 3).  The current column of L is
// passed through a small LDS buffer, so lane d reads L[j+e+d][j] and the
// broadcast L[j+e][j] at immediate offsets (several columns per read): a
// trailing-update step is one FMA and a fraction of two LDS reads, with no
// lane shifts or lane reads.  Forward substitution runs with the
// factorisation; the back substitution sums each half with row-local DPP.
template <typename T, int RHO>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 3 : 1))) void k_patch_band_pair(const T* __restrict__ A, const T* __restrict__ B,
                                                        T* __restrict__ R, int nk, int s, int* __restrict__ status) {
  constexpr int PMAX = 3 * (2 * RHO + 1) * (2 * RHO + 1);
  constexpr int BWM = 3 * (2 * RHO + 2) + 2;   // largest half-bandwidth
  static_assert(BWM < 32, "two patches per wavefront need a half-bandwidth below 32");
  constexpr int TT = 3;                        // parent stencil width at the finest level (t = 1)
  __shared__ T sb[2][PMAX + 32];               // b, then z, then x (zero beyond p)
  __shared__ T sc[2][PMAX];
  __shared__ T ld[2][PMAX];                    // diagonal of L
  __shared__ int rowinfo[2][PMAX];
  __shared__ __align__(16) T colb[2][2][64];   // [step parity][patch]: column of L, zero from entry 32 on
  const int rho = RHO;
  const int lane = threadIdx.x, h = lane >> 5, d = lane & 31;
  const int nc = nk / 2;
  const int ci = 2 * xcd_remap((int)blockIdx.x, (int)gridDim.x) + h;
  const int cx = ci / nc, cy = ci % nc;
  const int x0 = max(0, cx - rho), x1 = min(nc - 1, cx + rho);
  const int y0 = max(0, cy - rho), y1 = min(nc - 1, cy + rho);
  const int wy = y1 - y0 + 1;
  const int npar = (x1 - x0 + 1) * wy;
  const int p = 3 * npar;
  const int bw = 3 * (wy + 1) + 2;
  const int S = 2 * s + 1;
  const int ti = parent_type(true, cx, cy);

  for (int r = d; r < PMAX + 32; r += 32) {
    T scale = T(1), rv = T(0);
    if (r < p) {
      const int lp = r / 3, tt = r - 3 * lp;
      const int px = x0 + lp / wy, py = y0 + lp % wy;
      rowinfo[h][r] = (px << 20) | (py << 8) | tt;
      const T dd0 = B[b_index(TT + 1, tt * 4, px * nc + py, TT)];
      if (dd0 > T(0)) scale = T(1) / my_sqrt<T>(dd0);
      else atomicOr(status, kBadPivot);
      const int tp = parent_type(true, px, py);
      if (abs(px - cx) <= 1 && abs(py - cy) <= 1 && !is_pad_row(tp, tt)) {
        double acc = 0.0;
        for (int dd = 0; dd < 4; ++dd) {
          const double wd = wcoef(tp, tt, dd);
          if (wd == 0.0) continue;
          const int fx = 2 * px + (dd >> 1), fy = 2 * py + (dd & 1);
          double inner = 0.0;
          for (int e = 0; e < 4; ++e) {
            const double pe = pibar(ti, e);
            if (pe == 0.0) continue;
            const int gx = 2 * cx + (e >> 1), gy = 2 * cy + (e & 1);
            const int ox = gx - fx + s, oy = gy - fy + s;
            if (ox < 0 || oy < 0 || ox >= S || oy >= S) continue;
            inner += pe * (double)A[(size_t)(ox * S + oy) * nk * nk + fx * nk + fy];
          }
          acc += wd * inner;
        }
        rv = T(-acc);
      }
    }
    if (r < PMAX) sc[h][r] = scale;
    sb[h][r] = rv * scale;
  }
  colb[0][h][d] = T(0);
  colb[0][h][d + 32] = T(0);
  colb[1][h][d] = T(0);
  colb[1][h][d + 32] = T(0);
  __syncthreads();

  // this lane's subdiagonal d: M[c + d][c] (scaled to unit diagonal)
  T dg[PMAX];
#pragma clang loop unroll(full)
  for (int c = 0; c < PMAX; ++c) {
    const int r = c + d;
    T v = T(0);
    if (d <= bw && r < p) {
      const int ri = rowinfo[h][r], rj = rowinfo[h][c];
      const int rx = ri >> 20, ry = (ri >> 8) & 0xfff, trr = ri & 0xff;
      const int qx = rj >> 20, qy = (rj >> 8) & 0xfff, tcc = rj & 0xff;
      const int ox = qx - rx + 1, oy = qy - ry + 1;
      if (ox >= 0 && oy >= 0 && ox < TT && oy < TT)
        v = B[b_index(ox * TT + oy, trr * 3 + tcc, rx * nc + ry, TT)] * sc[h][r] * sc[h][c];
    }
    dg[c] = v;
  }

  int bad = 0, reg = 0;
#pragma clang loop unroll(full)
  for (int j = 0; j < PMAX; ++j) {
    T* cb = &colb[j & 1][h][0];
    const T pa = WaveOps<T>::lane(dg[j], 0), pb = WaveOps<T>::lane(dg[j], 32);
    const bool act = j < p;
    T col = T(0), inv = T(0);
    if (act) {
      const T piv = patch_pivot<T>(h ? pb : pa, bad, reg);
      inv = pivot_rsqrt<T>(piv);
      const T sq = piv * inv;
      col = (d == 0) ? sq : (d <= bw ? dg[j] * inv : T(0));
      if (d == 0) ld[h][j] = sq;
      cb[d] = col;
    }
    __syncthreads();
    if (act) {
      dg[j] = col;
      const T zj = sb[h][j] * inv;
      if (d == 0) sb[h][j] = zj;
      else if (d <= bw) sb[h][j + d] -= col * zj;
#pragma clang loop unroll(full)
      for (int e = 1; e <= BWM; ++e) {
        if (j + e < PMAX) dg[j + e] -= cb[d + e] * cb[e];
      }
    }
  }
  if (d == 0 && bad) atomicOr(status, kBadPivot);
  if (d == 0 && reg) atomicOr(status, kRegularizedPivot);
  __syncthreads();
  // back substitution L^T x = z: the sum over the half's lanes d >= 1 ends in
  // lanes 16..31 (patch 0) and 48..63 (patch 1)
#pragma clang loop unroll(full)
  for (int c = PMAX - 1; c >= 0; --c) {
    const bool act = c < p;
    T t = (act && d >= 1) ? dg[c] * sb[h][c + d] : T(0);
    t += WaveOps<T>::template dpp<0xB1, 0xf, true>(t);
    t += WaveOps<T>::template dpp<0x4E, 0xf, true>(t);
    t += WaveOps<T>::template dpp<0x141, 0xf, true>(t);
    t += WaveOps<T>::template dpp<0x140, 0xf, true>(t);
    t += WaveOps<T>::template dpp<0x142, 0xa, false>(t);
    if (act && d == 31) sb[h][c] = (sb[h][c] - t) / ld[h][c];
    __syncthreads();
  }
  for (int r = d; r < p; r += 32) sb[h][r] *= sc[h][r];
  __syncthreads();

  const int rw = 2 * (2 * rho + 1);
  const int ox0 = 2 * (cx - rho), oy0 = 2 * (cy - rho);
  const size_t nc2 = (size_t)nc * nc;
  T* Ri = R + ci;
  for (int e = d; e < rw * rw; e += 32) {
    const int bx = e / rw, by = e % rw;
    const int fx = ox0 + bx, fy = oy0 + by;
    double v = 0.0;
    if (fx >= 0 && fy >= 0 && fx < nk && fy < nk) {
      const int px = fx >> 1, py = fy >> 1;
      const int dd = 2 * (fx & 1) + (fy & 1);
      const int tp = parent_type(true, px, py);
      if (px == cx && py == cy) v = pibar(tp, dd);
      const int lp = (px - x0) * wy + (py - y0);
      for (int tt = 0; tt < 3; ++tt) v += (double)sb[h][3 * lp + tt] * wcoef(tp, tt, dd);
    }
    Ri[(size_t)e * nc2] = T(v);
  }
}

static bool band_reg_enabled() {
  const char* e = getenv("GBL_BAND_REG");
  return !(e && e[0] == '0');
}

// ---------------------------------------------------------------------------
// Patch solves at the finest transition (k = q), band form.
//
// B^(q) couples only neighbouring parents (its parent stencil is 3 x 3), so
// with the patch unknowns ordered parent row by parent row the patch matrix
// is banded with half-bandwidth bw = 3 (wy + 1) + 2.  One wavefront (one
// workgroup of 64 threads) factors one patch: the band lives in LDS as
// ab[r][d] = B_{r, r-d}; each step scales the pivot column and updates the
// trailing bw x bw triangle, the lanes sharing its entries; the forward
// substitution rides along and a column-oriented back substitution follows.
// Same scaling, right-hand side and restriction row as the dense kernel.
// ---------------------------------------------------------------------------
template <typename T, int kMaxTri>
__global__ __launch_bounds__(64) void k_patch_solve_band(const T* __restrict__ A, const T* __restrict__ B,
                                                         T* __restrict__ R, int nk, int s, int rho,
                                                         int* __restrict__ status) {
  extern __shared__ unsigned char smem_raw[];
  const int nc = nk / 2;
  const int ci = xcd_remap((int)blockIdx.x, (int)gridDim.x);
  const int cx = ci / nc, cy = ci % nc;
  const int x0 = max(0, cx - rho), x1 = min(nc - 1, cx + rho);
  const int y0 = max(0, cy - rho), y1 = min(nc - 1, cy + rho);
  const int wy = y1 - y0 + 1;
  const int npar = (x1 - x0 + 1) * wy;
  const int p = 3 * npar;
  const int bw = 3 * (wy + 1) + 2;
  const int bw1 = bw + 1;
  const int pmax = 3 * (2 * rho + 1) * (2 * rho + 1);
  const int bwmax = 3 * (2 * rho + 2) + 2;
  T* ab = reinterpret_cast<T*>(smem_raw);          // pmax * (bwmax + 1)
  T* bb = ab + (size_t)pmax * (bwmax + 1);         // pmax: right-hand side / z / x
  T* sc = bb + pmax;                               // pmax: scaling
  T* lcol = sc + pmax;                             // bwmax + 1
  const int lane = threadIdx.x;
  const int TT = 3;   // parent stencil width at the finest level (t = 1)
  const int S = 2 * s + 1;
  const size_t nc2 = (size_t)nc * nc;
  const int ti = parent_type(true, cx, cy);
  int bad = 0, reg = 0;

  // scaling and right-hand side
  for (int r = lane; r < p; r += 64) {
    const int lp = r / 3, tt = r - 3 * lp;
    const int px = x0 + lp / wy, py = y0 + lp % wy;
    const T d = B[b_index(1 * TT + 1, tt * 4, px * nc + py, TT)];
    T scale = T(1);
    if (d > T(0)) scale = T(1) / my_sqrt<T>(d);
    else bad = 1;
    const int tp = parent_type(true, px, py);
    double acc = 0.0;
    if (abs(px - cx) <= 1 && abs(py - cy) <= 1 && !is_pad_row(tp, tt)) {
      for (int dd = 0; dd < 4; ++dd) {
        const double wd = wcoef(tp, tt, dd);
        if (wd == 0.0) continue;
        const int fx = 2 * px + (dd >> 1), fy = 2 * py + (dd & 1);
        double inner = 0.0;
        for (int e = 0; e < 4; ++e) {
          const double pe = pibar(ti, e);
          if (pe == 0.0) continue;
          const int gx = 2 * cx + (e >> 1), gy = 2 * cy + (e & 1);
          const int ox = gx - fx + s, oy = gy - fy + s;
          if (ox < 0 || oy < 0 || ox >= S || oy >= S) continue;
          inner += pe * (double)A[(size_t)(ox * S + oy) * nk * nk + fx * nk + fy];
        }
        acc += wd * inner;
      }
    }
    sc[r] = scale;
    bb[r] = T(-acc) * scale;
  }
  __syncthreads();
  // band of the scaled patch matrix: ab[r][d] = B_{r, r-d}, 0 <= d <= bw
  for (int e = lane; e < p * bw1; e += 64) {
    const int r = e / bw1, d = e - r * bw1;
    const int c = r - d;
    T v = T(0);
    if (c >= 0) {
      const int lr = r / 3, trr = r - 3 * lr;
      const int lc = c / 3, tcc = c - 3 * lc;
      const int rx = x0 + lr / wy, ry = y0 + lr % wy;
      const int qx = x0 + lc / wy, qy = y0 + lc % wy;
      const int ox = qx - rx + 1, oy = qy - ry + 1;
      if (ox >= 0 && oy >= 0 && ox < TT && oy < TT)
        v = B[b_index(ox * TT + oy, trr * 3 + tcc, rx * nc + ry, TT)] * sc[r] * sc[c];
    }
    ab[e] = v;
  }
  // this lane's fixed share of the trailing triangle: entries (dr, dc),
  // 1 <= dc <= dr <= bw, enumerated column by column
  // kMaxTri = ceil(bw (bw + 1) / 2 / 64): 9 for bw <= 32 (rho <= 4), 12 for bw <= 38 (rho = 5)
  const int ntri = bw * (bw + 1) / 2;
  int tri_dr[kMaxTri], tri_dc[kMaxTri];
  {
    int dc = 1, rem = lane, len = bw;
#pragma unroll
    for (int m = 0; m < kMaxTri; ++m) {
      while (dc <= bw && rem >= len) {
        rem -= len;
        ++dc;
        --len;
      }
      const bool ok = (lane + 64 * m) < ntri;
      tri_dr[m] = ok ? dc + rem : bw + 1 + 1024;   // out of range -> skipped below
      tri_dc[m] = ok ? dc : 1;
      rem += 64;
    }
  }
  __syncthreads();

  for (int j = 0; j < p; ++j) {
    const T pv = patch_pivot<T>(ab[j * bw1], bad, reg);
    const T dj = my_sqrt<T>(pv);
    const T inv = T(1) / dj;
    const int e = lane + 1;
    if (e <= bw && j + e < p) {
      T* pe = ab + (size_t)(j + e) * bw1 + e;
      const T l = *pe * inv;
      *pe = l;
      lcol[e] = l;
    }
    const T zj = bb[j] * inv;
    __syncthreads();
    if (lane == 0) {
      ab[j * bw1] = dj;
      bb[j] = zj;
    }
    if (e <= bw && j + e < p) bb[j + e] -= lcol[e] * zj;
#pragma unroll
    for (int m = 0; m < kMaxTri; ++m) {
      const int dr = tri_dr[m], dc = tri_dc[m];
      if (j + dr < p) ab[(size_t)(j + dr) * bw1 + (dr - dc)] -= lcol[dr] * lcol[dc];
    }
    __syncthreads();
  }
  // back substitution L^T x = z, row j of L is ab[j][*]
  for (int j = p - 1; j >= 0; --j) {
    const T xj = bb[j] / ab[j * bw1];
    const int d = lane + 1;
    if (d <= bw && j - d >= 0) bb[j - d] -= ab[(size_t)j * bw1 + d] * xj;
    __syncthreads();
    if (lane == 0) bb[j] = xj;
    __syncthreads();
  }
  for (int r = lane; r < p; r += 64) bb[r] *= sc[r];
  if (bad) atomicOr(status, kBadPivot);
  if (reg && lane == 0) atomicOr(status, kRegularizedPivot);
  __syncthreads();

  const int rw = 2 * (2 * rho + 1);
  const int ox0 = 2 * (cx - rho), oy0 = 2 * (cy - rho);
  T* Ri = R + ci;
  for (int e = lane; e < rw * rw; e += 64) {
    const int bx = e / rw, by = e % rw;
    const int fx = ox0 + bx, fy = oy0 + by;
    double v = 0.0;
    if (fx >= 0 && fy >= 0 && fx < nk && fy < nk) {
      const int px = fx >> 1, py = fy >> 1;
      const int d = 2 * (fx & 1) + (fy & 1);
      const int tp = parent_type(true, px, py);
      if (px == cx && py == cy) v = pibar(tp, d);
      const int lp = (px - x0) * wy + (py - y0);
      for (int tt = 0; tt < 3; ++tt) v += (double)bb[3 * lp + tt] * wcoef(tp, tt, d);
    }
    Ri[(size_t)e * nc2] = T(v);
  }
}

template <typename T>
void launch_patch_solve_band(const LevelGeom& L, const T* A, const T* B, T* R, int* status, hipStream_t st,
                             int variant) {
  const int nc = L.nk / 2;
  const bool reg = variant == kVariantDefault ? band_reg_enabled() : variant == 1;
  if (reg && L.rho <= 3) {
    // two patches per wavefront (nc * nc is even)
    const dim3 grid(nc * nc / 2), block(64);
    if (L.rho == 3) hipLaunchKernelGGL((k_patch_band_pair<T, 3>), grid, block, 0, st, A, B, R, L.nk, L.s, status);
    else if (L.rho == 2) hipLaunchKernelGGL((k_patch_band_pair<T, 2>), grid, block, 0, st, A, B, R, L.nk, L.s, status);
    else hipLaunchKernelGGL((k_patch_band_pair<T, 1>), grid, block, 0, st, A, B, R, L.nk, L.s, status);
    return;
  }
  const int pmax = 3 * (2 * L.rho + 1) * (2 * L.rho + 1);
  const int bwmax = 3 * (2 * L.rho + 2) + 2;
  const size_t shm = ((size_t)pmax * (bwmax + 1) + 2 * (size_t)pmax + (bwmax + 1)) * sizeof(T);
  if (L.rho <= 4)
    hipLaunchKernelGGL((k_patch_solve_band<T, 9>), dim3(nc * nc), dim3(64), shm, st, A, B, R, L.nk, L.s, L.rho, status);
  else
    hipLaunchKernelGGL((k_patch_solve_band<T, 12>), dim3(nc * nc), dim3(64), shm, st, A, B, R, L.nk, L.s, L.rho,
                       status);
}

// ---------------------------------------------------------------------------
// Galerkin coarsening A^(k-1) = R^(k-1,k) A^(k) R^(k,k-1) (Theorem 4.8;
// Algorithm 2 -- the step the paper names as its complexity
// bottleneck).  One workgroup per coarse row i: first z = R_i A^(k) on the
// window of level-k slots the row can reach (staged in LDS; A is symmetric
// so z_c' is row c' of A against R_i), then every entry
// A^(k-1)_{i,i'} = z . R_{i'} of the coarse stencil.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(1024) void k_galerkin(const T* __restrict__ A, const T* __restrict__ R,
                                                  T* __restrict__ Ac, int nk, int s, int rho, int sc) {
  extern __shared__ unsigned char smem_raw[];
  T* smem = reinterpret_cast<T*>(smem_raw);
  const int nc = nk / 2;
  const int ci = xcd_remap((int)blockIdx.x, (int)gridDim.x);
  const int cx = ci / nc, cy = ci % nc;
  const int rw = 2 * (2 * rho + 1);
  const int S = 2 * s + 1;
  const int zw = rw + 2 * s;
  T* Rl = smem;              // rw * rw
  T* z = smem + rw * rw;     // zw * zw
  const int orgx = 2 * (cx - rho), orgy = 2 * (cy - rho);
  const size_t nc2 = (size_t)nc * nc;
  const size_t nk2 = (size_t)nk * nk;
  for (int e = threadIdx.x; e < rw * rw; e += blockDim.x) Rl[e] = R[e * nc2 + ci];
  __syncthreads();
  for (int e = threadIdx.x; e < zw * zw; e += blockDim.x) {
    const int zx = e / zw, zy = e % zw;
    const int fx = orgx - s + zx, fy = orgy - s + zy;
    T acc = T(0);
    if (fx >= 0 && fy >= 0 && fx < nk && fy < nk) {
      const int dx = fx - orgx, dy = fy - orgy;   // position in R coordinates
      const int oxl = max(0, s - dx), oxh = min(S - 1, s - dx + rw - 1);
      const int oyl = max(0, s - dy), oyh = min(S - 1, s - dy + rw - 1);
      const T* Arow = A + (size_t)(fx * nk + fy);
      for (int ox = oxl; ox <= oxh; ++ox) {
        const T* Ar = Arow + (size_t)ox * S * nk2;
        const T* Rr = Rl + (dx + ox - s) * rw + (dy - s);
        for (int oy = oyl; oy <= oyh; ++oy) acc += Ar[oy * nk2] * Rr[oy];
      }
    }
    z[e] = acc;
  }
  __syncthreads();
  // A^(k-1) is symmetric: this row computes the offsets (dx, dy) with dx > 0,
  // or dx = 0 and dy >= 0, and also stores each of them, mirrored, in the row
  // of the neighbour j; the other offsets are written by those neighbours,
  // except where j lies outside the level (the entry is then zero).  Every
  // location has exactly one writer.
  const int Sc = 2 * sc + 1;
  T* out = Ac + ci;   // Ac[e * nc2 + ci]
  for (int e = threadIdx.x; e < Sc * Sc; e += blockDim.x) {
    const int ox = e / Sc, oy = e % Sc;
    const int jx = cx + ox - sc, jy = cy + oy - sc;
    const bool inside = jx >= 0 && jy >= 0 && jx < nc && jy < nc;
    const bool upper = (ox > sc) || (ox == sc && oy >= sc);
    if (!upper) {
      if (!inside) out[(size_t)e * nc2] = T(0);
      continue;
    }
    T acc = T(0);
    if (inside) {
      const T* Rj = R + (jx * nc + jy);
      const int ojx = 2 * (jx - rho), ojy = 2 * (jy - rho);
      // z index of R_j entry (bx, by): (ojx + bx) - (orgx - s)
      const int shx = ojx - orgx + s, shy = ojy - orgy + s;
      const int bxl = max(0, -shx), bxh = min(rw - 1, zw - 1 - shx);
      const int byl = max(0, -shy), byh = min(rw - 1, zw - 1 - shy);
      for (int bx = bxl; bx <= bxh; ++bx) {
        const T* Rr = Rj + (size_t)bx * rw * nc2;
        const T* zr = z + (shx + bx) * zw + shy;
        for (int by = byl; by <= byh; ++by) acc += Rr[by * nc2] * zr[by];
      }
      // mirrored entry: row j, offset (-dx, -dy)
      Ac[(size_t)(Sc * Sc - 1 - e) * nc2 + (jx * nc + jy)] = acc;
    }
    out[(size_t)e * nc2] = acc;
  }
}

static bool galerkin_strip_enabled() {
  const char* e = getenv("GBL_GALERKIN_STRIP");
  return !(e && e[0] == '0');
}

// ---------------------------------------------------------------------------
// Galerkin product on strips of NS coarse rows (consecutive in y) per
// workgroup.  Neighbouring coarse rows share most of their restriction
// supports and stencil neighbours, so
//   1. the strip's R rows go to LDS, each in the frame of the union of their
//      supports (row m at y offset 2 m, zero elsewhere);
//   2. z_m = R_m A^(k) (A symmetric: z_m[c'] = sum_c A[c'][c] R_m[c]) is formed
//      over the union of the rows' windows, each A entry read once for all
//      rows; z_m comes out zero outside its own window, so all rows share one
//      frame and one index;
//   3. A^(k-1) is symmetric: only the upper half of each row's stencil is
//      formed (offsets (dx, dy) with dx > 0, or dx = 0 and dy >= 0), each
//      neighbour row R_j read once and dotted with the z of every strip row;
//   4. each entry is stored in its row and, mirrored, in the row of the
//      neighbour j; for one stencil offset both stores cover NS consecutive
//      coarse rows.  The remaining entries of the strip rows (lower offsets)
//      are written by the strips of their neighbours, or are zero where the
//      neighbour lies outside the level: every location has one writer.
// ---------------------------------------------------------------------------
constexpr int kStripThreads = 512;
// parts of the neighbour rows per phase-3 work item: enough items for the workgroup, at most 3
__host__ __device__ inline int strip_parts(int items, int threads) {
  const int p = threads / items;
  return p < 1 ? 1 : (p > 3 ? 3 : p);
}

template <typename T, int NS>
__global__ __launch_bounds__(kStripThreads) void k_galerkin_strip(const T* __restrict__ A, const T* __restrict__ R,
                                                        T* __restrict__ Ac, int nk, int s, int rho, int sc) {
  extern __shared__ unsigned char smem_raw[];
  T* smem = reinterpret_cast<T*>(smem_raw);
  const int nc = nk / 2;
  const int nstrip = nc / NS;
  const int b = xcd_remap((int)blockIdx.x, (int)gridDim.x);
  const int cx = b / nstrip, cy0 = (b - cx * nstrip) * NS;
  const int rw = 2 * (2 * rho + 1);
  const int S = 2 * s + 1;
  const int Sc = 2 * sc + 1;
  const int zw = rw + 2 * s;
  const int ry = rw + 2 * (NS - 1);   // union of the strip rows' supports (y)
  const int uy = zw + 2 * (NS - 1);   // union of their z windows (y)
  const int ho = (Sc * Sc - 1) / 2;   // centre offset; ho .. Sc*Sc-1 is the upper half
  T* Rf = smem;                       // [NS][rw][ry]
  T* zu = Rf + NS * rw * ry;          // [NS][zw][uy]
  T* ol = zu + NS * zw * uy;          // [P][Sc*Sc - ho][NS]
  const int ox0 = 2 * (cx - rho), oy0 = 2 * (cy0 - rho);   // union support origin
  const int nc2 = nc * nc;
  const size_t nk2 = (size_t)nk * nk;
  const int row0 = cx * nc + cy0;
  // 1. R rows of the strip (m fastest: the NS rows of one entry are adjacent in R)
  for (int e = threadIdx.x; e < NS * rw * ry; e += blockDim.x) {
    const int m = e % NS, r = e / NS;
    const int bx = r / ry, y = r - bx * ry, by = y - 2 * m;
    Rf[m * (rw * ry) + r] = (by >= 0 && by < rw) ? R[(size_t)(bx * rw + by) * nc2 + row0 + m] : T(0);
  }
  __syncthreads();
  // 2. z at union position (ux, u) <-> level-k slot (ox0 - s + ux, oy0 - s + u)
  const int mr = rw * ry, mz = zw * uy;
  for (int e = threadIdx.x; e < zw * uy; e += blockDim.x) {
    const int ux = e / uy, u = e - ux * uy;
    const int fx = ox0 - s + ux, fy = oy0 - s + u;
    T acc[NS];
#pragma unroll
    for (int m = 0; m < NS; ++m) acc[m] = T(0);
    if (fx >= 0 && fy >= 0 && fx < nk && fy < nk) {
      // neighbours c = (fx + ox - s, fy + oy - s) inside the union of supports
      const int dx = fx - ox0, dy = fy - oy0;
      const int oxl = max(0, s - dx), oxh = min(S - 1, s - dx + rw - 1);
      const int oyl = max(0, s - dy), oyh = min(S - 1, s - dy + ry - 1);
      const T* Arow = A + (size_t)(fx * nk + fy);
      for (int ox = oxl; ox <= oxh; ++ox) {
        const T* Ar = Arow + (size_t)ox * S * nk2;
        const T* Rb = Rf + (dx + ox - s) * ry + (dy - s);
#pragma unroll 4
        for (int oy = oyl; oy <= oyh; ++oy) {
          const T a = Ar[oy * nk2];
#pragma unroll
          for (int m = 0; m < NS; ++m) acc[m] += a * Rb[m * mr + oy];
        }
      }
    }
#pragma unroll
    for (int m = 0; m < NS; ++m) zu[m * mz + e] = acc[m];
  }
  __syncthreads();
  // 3. neighbours j = (cx + dxj, cy0 + dyj), dxj in [0, sc], dyj in [-sc, sc + NS - 1];
  //    with few neighbours per thread the rows bx of R_j are split into P parts
  //    whose partial sums are added when storing
  const int jh = 2 * sc + NS;
  const int items = (sc + 1) * jh;
  const int P = strip_parts(items, blockDim.x);
  const int nup = Sc * Sc - ho;
  for (int e = threadIdx.x; e < items * P; e += blockDim.x) {
    const int part = e / items, it = e - part * items;
    const int ejx = sc + it / jh, ejy = it - (it / jh) * jh;
    const int jx = cx + ejx - sc, jy = cy0 + ejy - sc;
    T acc[NS];
#pragma unroll
    for (int m = 0; m < NS; ++m) acc[m] = T(0);
    if (jx >= 0 && jy >= 0 && jx < nc && jy < nc) {
      // R_j entry (bx, by) sits at union position (shx + bx, shy + by)
      const int shx = 2 * (jx - rho) - ox0 + s, shy = 2 * (jy - rho) - oy0 + s;
      const int bxl = max(part * rw / P, -shx), bxh = min((part + 1) * rw / P - 1, zw - 1 - shx);
      const int byl = max(0, -shy), byh = min(rw - 1, uy - 1 - shy);
      const T* Rj = R + (jx * nc + jy);
      for (int bx = bxl; bx <= bxh; ++bx) {
        const T* Rr = Rj + (size_t)bx * rw * nc2;
        const T* zr = zu + (shx + bx) * uy + shy;
#pragma unroll 7
        for (int by = byl; by <= byh; ++by) {
          const T rv = Rr[(size_t)by * nc2];
#pragma unroll
          for (int m = 0; m < NS; ++m) acc[m] += rv * zr[m * mz + by];
        }
      }
    }
    // row m takes j at offset (ejx, ejy - m) when that offset is in the upper half
    const int oyl = ejx > sc ? 0 : sc;
#pragma unroll
    for (int m = 0; m < NS; ++m) {
      const int oy = ejy - m;
      if (oy >= oyl && oy < Sc) ol[(part * nup + ejx * Sc + oy - ho) * NS + m] = acc[m];
    }
  }
  __syncthreads();
  // 4. stores
  for (int e = threadIdx.x; e < nup * NS; e += blockDim.x) {
    const int o = ho + e / NS, m = e - (e / NS) * NS;
    T v = ol[e];
    for (int pt = 1; pt < P; ++pt) v += ol[pt * nup * NS + e];
    Ac[(size_t)o * nc2 + row0 + m] = v;
    if (o != ho) {
      const int ox = o / Sc, oy = o - ox * Sc;
      const int jx = cx + ox - sc, jy = cy0 + m + oy - sc;
      if (jx >= 0 && jy >= 0 && jx < nc && jy < nc) Ac[(size_t)(Sc * Sc - 1 - o) * nc2 + jx * nc + jy] = v;
    }
  }
  for (int e = threadIdx.x; e < ho * NS; e += blockDim.x) {
    const int o = e / NS, m = e - (e / NS) * NS;
    const int ox = o / Sc, oy = o - ox * Sc;
    const int jx = cx + ox - sc, jy = cy0 + m + oy - sc;
    if (!(jx >= 0 && jy >= 0 && jx < nc && jy < nc)) Ac[(size_t)o * nc2 + row0 + m] = T(0);
  }
}

// LDS of a strip of NS rows
static size_t strip_lds(const LevelGeom& L, const LevelGeom& C, int NS, size_t elem) {
  const size_t zw = L.rw + 2 * L.s, Sc = 2 * C.s + 1;
  const size_t ry = L.rw + 2 * (NS - 1), uy = zw + 2 * (NS - 1);
  const int P = strip_parts((C.s + 1) * (2 * C.s + NS), kStripThreads);
  return ((size_t)NS * (L.rw * ry + zw * uy) + (size_t)P * (Sc * Sc - (Sc * Sc - 1) / 2) * NS) * elem;
}

// strip height: the largest of 8, 4, 2 whose LDS staging fits 80 KB (two
// workgroups of 512 threads per compute unit) and that still gives 512
// workgroups (strips pay off only when they fill the GPU); 1 = no strips
template <typename T>
static int strip_height(const LevelGeom& L, const LevelGeom& C) {
  const int nc = L.nk / 2;
  int NS = 8;
  while (NS > 1 && (NS > nc || strip_lds(L, C, NS, sizeof(T)) > 80 * 1024 || nc * (nc / NS) < 512)) NS /= 2;
  return NS;
}

template <typename T>
bool galerkin_variant_ok(const LevelGeom& L, const LevelGeom& C, int variant) {
  return variant == 0 || (variant == 1 && strip_height<T>(L, C) >= 2);
}

template <typename T>
void launch_galerkin(const LevelGeom& L, const LevelGeom& C, const T* A, const T* R, T* Ac,
                     hipStream_t st, int variant) {
  const int nc = L.nk / 2;
  const int zw = L.rw + 2 * L.s;
  const int NS = strip_height<T>(L, C);
  const bool strips = variant == kVariantDefault ? galerkin_strip_enabled() : variant == 1;
  if (strips && NS >= 2) {
    const size_t shm = strip_lds(L, C, NS, sizeof(T));
    const dim3 grid(nc * (nc / NS)), block(kStripThreads);
    if (NS == 8)
      hipLaunchKernelGGL((k_galerkin_strip<T, 8>), grid, block, shm, st, A, R, Ac, L.nk, L.s, L.rho, C.s);
    else if (NS == 4)
      hipLaunchKernelGGL((k_galerkin_strip<T, 4>), grid, block, shm, st, A, R, Ac, L.nk, L.s, L.rho, C.s);
    else
      hipLaunchKernelGGL((k_galerkin_strip<T, 2>), grid, block, shm, st, A, R, Ac, L.nk, L.s, L.rho, C.s);
    return;
  }
  // few rows: more threads per row (the small levels are latency-bound)
  const size_t shm = (size_t)(L.rw * L.rw + zw * zw) * sizeof(T);
  const int threads = nc * nc <= 256 ? 1024 : 256;
  hipLaunchKernelGGL(k_galerkin<T>, dim3(nc * nc), dim3(threads), shm, st, A, R, Ac, L.nk, L.s, L.rho, C.s);
}

// ---------------------------------------------------------------------------
// Coarsest level: Cholesky factor of the 4 x 4 matrix A^(1) in FP64
// (coarse system of Algorithm 2).  A single thread; L1 holds the dense factor.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_coarse_factor(const T* __restrict__ A1, int s1, double* __restrict__ L1,
                                int* __restrict__ status) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int S = 2 * s1 + 1;
  double M[4][4];
  for (int i = 0; i < 4; ++i) {
    const int ix = i / 2, iy = i % 2;
    for (int j = 0; j < 4; ++j) {
      const int jx = j / 2, jy = j % 2;
      const int ox = jx - ix + s1, oy = jy - iy + s1;
      double v = 0.0;
      if (ox >= 0 && oy >= 0 && ox < S && oy < S) v = (double)A1[(ox * S + oy) * 4 + i];
      M[i][j] = v;
    }
  }
  // symmetrise (the FP32 hierarchy may carry rounding asymmetry)
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < i; ++j) M[i][j] = M[j][i] = 0.5 * (M[i][j] + M[j][i]);
  for (int j = 0; j < 4; ++j) {
    const double d0 = M[j][j];
    double d = d0;
    for (int k = 0; k < j; ++k) d -= M[j][k] * M[j][k];
    if (sizeof(T) == 4 && d0 > 0.0 && !(d > (double)kPivotFloor * d0)) {
      atomicOr(status, kRegularizedPivot);   // FP32 Galerkin rounding, as in patch_pivot
      d = (double)kPivotFloor * d0;
    } else if (!(d > 0.0)) {
      atomicOr(status, kBadPivot);
      d = 1.0;
    }
    const double l = sqrt(d);
    M[j][j] = l;
    for (int i = j + 1; i < 4; ++i) {
      double v = M[i][j];
      for (int k = 0; k < j; ++k) v -= M[i][k] * M[j][k];
      M[i][j] = v / l;
    }
  }
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) L1[i * 4 + j] = j <= i ? M[i][j] : 0.0;
}

template <typename T>
void launch_coarse_factor(const T* A1, int s1, double* L1, int* status, hipStream_t st) {
  hipLaunchKernelGGL(k_coarse_factor<T>, dim3(1), dim3(64), 0, st, A1, s1, L1, status);
}

// ---------------------------------------------------------------------------
// Upper bound of lambda_max(M B^(k)), M the inverse 3 x 3 parent blocks D_p of
// B^(k), for the Chebyshev inner iteration.  With D_p = L_p L_p^T the
// eigenvalues of M B are those of C = L^{-1} B L^{-T}, whose blocks are
// C_pq = L_p^{-1} B_pq L_q^{-T}; Gershgorin's theorem bounds them by the
// largest absolute row sum of C.  One thread per parent; the level maximum is
// kept with an integer atomic max on the bits of the non-negative float.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_chol3_inv(const T* __restrict__ B, int np, int t, T* __restrict__ Linv) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= np * np) return;
  const int TT = 2 * t + 1;
  const size_t np2 = (size_t)np * np;
  T D[3][3];
#pragma unroll
  for (int e = 0; e < 9; ++e) D[e / 3][e % 3] = B[b_index(t * TT + t, e, p, TT)];
  // D = L L^T, then the lower triangle of L^{-1}: (0,0) (1,0) (1,1) (2,0) (2,1) (2,2)
  const T l00 = my_sqrt<T>(D[0][0] > T(0) ? D[0][0] : T(1));
  const T l10 = D[1][0] / l00, l20 = D[2][0] / l00;
  const T d11 = D[1][1] - l10 * l10;
  const T l11 = my_sqrt<T>(d11 > T(0) ? d11 : T(1));
  const T l21 = (D[2][1] - l20 * l10) / l11;
  const T d22 = D[2][2] - l20 * l20 - l21 * l21;
  const T l22 = my_sqrt<T>(d22 > T(0) ? d22 : T(1));
  const T i00 = T(1) / l00, i11 = T(1) / l11, i22 = T(1) / l22;
  const T i10 = -l10 * i00 * i11;
  const T i21 = -l21 * i11 * i22;
  const T i20 = -(l20 * i00 + l21 * i10) * i22;
  Linv[0 * np2 + p] = i00;
  Linv[1 * np2 + p] = i10;
  Linv[2 * np2 + p] = i11;
  Linv[3 * np2 + p] = i20;
  Linv[4 * np2 + p] = i21;
  Linv[5 * np2 + p] = i22;
}

template <typename T>
__device__ __forceinline__ void load_linv(const T* __restrict__ Linv, size_t np2, int p, T L[3][3]) {
  L[0][0] = Linv[p];
  L[0][1] = T(0);
  L[0][2] = T(0);
  L[1][0] = Linv[np2 + p];
  L[1][1] = Linv[2 * np2 + p];
  L[1][2] = T(0);
  L[2][0] = Linv[3 * np2 + p];
  L[2][1] = Linv[4 * np2 + p];
  L[2][2] = Linv[5 * np2 + p];
}

template <typename T>
__global__ __launch_bounds__(1024) void k_gershgorin(const T* __restrict__ B, const T* __restrict__ Linv, int np,
                                                     int t, unsigned* __restrict__ out) {
  // 64 consecutive parents per workgroup, one per lane; wavefront w sums the
  // stencil rows ox = w, w + nw, ... and the row sums are added in LDS
  __shared__ T red[3][16][64];
  const int TT = 2 * t + 1;
  const size_t np2 = (size_t)np * np;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int p = blockIdx.x * 64 + lane;
  const bool live = p < np * np;
  T rs[3] = {T(0), T(0), T(0)};
  if (live) {
    const int px = p / np, py = p % np;
    T Lp[3][3];
    load_linv(Linv, np2, p, Lp);
    for (int ox = wv; ox < TT; ox += nw) {
      const int qx = px + ox - t;
      if (qx < 0 || qx >= np) continue;
      for (int oy = 0; oy < TT; ++oy) {
        const int qy = py + oy - t;
        if (qy < 0 || qy >= np) continue;
        T Bq[3][3], Lq[3][3];
#pragma unroll
        for (int e = 0; e < 9; ++e) Bq[e / 3][e % 3] = B[b_index(ox * TT + oy, e, p, TT)];
        load_linv(Linv, np2, qx * np + qy, Lq);
        // C = Lp Bq Lq^T
        T M1[3][3];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
          for (int j = 0; j < 3; ++j) M1[i][j] = Lp[i][0] * Bq[0][j] + Lp[i][1] * Bq[1][j] + Lp[i][2] * Bq[2][j];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
          for (int j = 0; j < 3; ++j) rs[i] += fabs(M1[i][0] * Lq[j][0] + M1[i][1] * Lq[j][1] + M1[i][2] * Lq[j][2]);
      }
    }
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) red[i][wv][lane] = rs[i];
  __syncthreads();
  if (wv == 0 && live) {
    T s[3] = {T(0), T(0), T(0)};
    for (int w = 0; w < nw; ++w)
#pragma unroll
      for (int i = 0; i < 3; ++i) s[i] += red[i][w][lane];
    const float g = (float)fmax(s[0], fmax(s[1], s[2]));
    if (g > 0.0f) atomicMax(out, __float_as_uint(g));
  }
}

template <typename T>
void launch_gershgorin(const LevelGeom& L, const T* B, T* scratch, unsigned* out, hipStream_t st) {
  const int np = L.nk / 2;
  const dim3 grid((np * np + 255) / 256), block(256);
  hipLaunchKernelGGL(k_chol3_inv<T>, grid, block, 0, st, B, np, L.t, scratch);
  const int TT = 2 * L.t + 1;
  hipLaunchKernelGGL(k_gershgorin<T>, dim3((np * np + 63) / 64), dim3(64 * (TT < 16 ? TT : 16)), 0, st, B, scratch,
                     np, L.t, out);
}

#define GBL_INST(T)                                                                                   \
  template void launch_assemble_fine<T>(const double*, T*, int, int*, hipStream_t);                  \
  template void launch_gershgorin<T>(const LevelGeom&, const T*, T*, unsigned*, hipStream_t);        \
  template void launch_subband_operator<T>(const LevelGeom&, const T*, T*, T*, bool, hipStream_t);   \
  template void launch_patch_solve<T>(const LevelGeom&, const T*, const T*, T*, T*, bool, int*,      \
                                      hipStream_t, int);                                             \
  template void launch_galerkin<T>(const LevelGeom&, const LevelGeom&, const T*, const T*, T*,      \
                                   hipStream_t, int);                                                \
  template bool patch_variant_ok<T>(const LevelGeom&, bool, int);                                     \
  template bool galerkin_variant_ok<T>(const LevelGeom&, const LevelGeom&, int);                      \
  template void launch_coarse_factor<T>(const T*, int, double*, int*, hipStream_t);
GBL_INST(float)
GBL_INST(double)
#undef GBL_INST

}  // namespace gbl
