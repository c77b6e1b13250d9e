// Exact (unlocalized) gamblet hierarchy: Algorithm 1 with dense level
// matrices in FP64, for small depths (the workloads of Section 5.1's example).
//
// Level k's unknowns: for k = q the interior nodes (index (i-1) m + (j-1),
// m nodes per side), for k < q the dyadic cells (index x 2^k + y).  A parent
// (level k-1) owns up to four children, listed by child position t = 2 dx + dy;
// its subband rows are the first m_p - 1 Helmert rows over its m_p children
// (Construction 4.13), stored three per parent, t-major: row t np^2 + p,
// np^2 the parents of the level; rows a parent does not have are identity
// rows of B (zero right-hand side), which changes no result.
//
// Dense kernels (row-major, leading dimensions explicit): a tiled GEMM, the
// blocked Cholesky factorization and the blocked triangular solves built on
// it, and the level operators of Algorithm 1: B = W A W^T, the right-hand
// side -W A pibar^T of D, R = pibar + D^T W, A^(k-1) = R A R^T (two GEMMs).
#include <hip/hip_runtime.h>

#include "exact_internal.hpp"

namespace gbl {

// ---------------------------------------------------------------------------
// C = alpha op(A) op(B) + beta C, FP64.  op(A)(i, k) = A[i * as0 + k * as1],
// op(B)(k, j) = B[k * bs0 + j * bs1], C(i, j) = C[i * ldc + j].  64 x 64
// output tile per workgroup (256 threads, 4 x 4 outputs each), K in slices
// of 16 staged through LDS.
// ---------------------------------------------------------------------------
constexpr int kGT = 64, kGK = 16;

__global__ __launch_bounds__(256) void k_ex_gemm(int M, int N, int K, double alpha, const double* __restrict__ A,
                                                 long as0, long as1, const double* __restrict__ B, long bs0, long bs1,
                                                 double beta, double* __restrict__ C, long ldc) {
  __shared__ double sa[kGK][kGT + 1];
  __shared__ double sb[kGK][kGT + 1];
  const int i0 = blockIdx.y * kGT, j0 = blockIdx.x * kGT;
  const int tid = threadIdx.x;
  const int ti = tid / 16, tj = tid % 16;
  double acc[4][4] = {};
  for (int k0 = 0; k0 < K; k0 += kGK) {
    for (int e = tid; e < kGK * kGT; e += 256) {
      const int kk = e / kGT, ii = e % kGT;
      const int gi = i0 + ii, gk = k0 + kk;
      sa[kk][ii] = (gi < M && gk < K) ? A[(long)gi * as0 + (long)gk * as1] : 0.0;
      const int gj = j0 + ii;
      sb[kk][ii] = (gj < N && gk < K) ? B[(long)gk * bs0 + (long)gj * bs1] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < kGK; ++kk) {
      double a[4], b[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        a[u] = sa[kk][ti + 16 * u];
        b[u] = sb[kk][tj + 16 * u];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] += a[u] * b[v];
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int gi = i0 + ti + 16 * u;
    if (gi >= M) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int gj = j0 + tj + 16 * v;
      if (gj >= N) continue;
      double* c = C + (long)gi * ldc + gj;
      *c = alpha * acc[u][v] + (beta == 0.0 ? 0.0 : beta * *c);
    }
  }
}

void ex_gemm(int M, int N, int K, double alpha, const double* A, long as0, long as1, const double* B, long bs0,
             long bs1, double beta, double* C, long ldc, hipStream_t st) {
  if (M <= 0 || N <= 0) return;
  const dim3 grid((N + kGT - 1) / kGT, (M + kGT - 1) / kGT);
  hipLaunchKernelGGL(k_ex_gemm, grid, dim3(256), 0, st, M, N, K, alpha, A, as0, as1, B, bs0, bs1, beta, C, ldc);
}

// ---------------------------------------------------------------------------
// Cholesky A = L L^T in place (lower triangle; the strict upper triangle is
// left as it was), blocks of 64: factor the diagonal block in LDS, solve the
// panel below it, update the trailing matrix with a GEMM.
// ---------------------------------------------------------------------------
constexpr int kCB = 64;

__global__ __launch_bounds__(256) void k_ex_potrf_block(double* __restrict__ A, long lda, int j0, int nb,
                                                        int* __restrict__ status) {
  __shared__ double L[kCB][kCB + 1];
  const int tid = threadIdx.x;
  for (int e = tid; e < nb * nb; e += 256) L[e / nb][e % nb] = A[(long)(j0 + e / nb) * lda + j0 + e % nb];
  __syncthreads();
  for (int c = 0; c < nb; ++c) {
    const double d = L[c][c];
    __syncthreads();
    if (!(d > 0.0)) {
      if (tid == 0) atomicOr(status, kBadPivot);
    }
    const double s = d > 0.0 ? sqrt(d) : 1.0;
    for (int i = c + tid; i < nb; i += 256) L[i][c] = (i == c) ? s : L[i][c] / s;
    __syncthreads();
    const int m = nb - 1 - c;
    for (int e = tid; e < m * m; e += 256) {
      const int i = c + 1 + e / m, j = c + 1 + e % m;
      if (j <= i) L[i][j] -= L[i][c] * L[j][c];
    }
    __syncthreads();
  }
  for (int e = tid; e < nb * nb; e += 256) {
    const int i = e / nb, j = e % nb;
    if (j <= i) A[(long)(j0 + i) * lda + j0 + j] = L[i][j];
  }
}

// rows r in [r0, n): A[r][j0..j0+nb) <- A[r][j0..] L11^-T (one thread per row)
__global__ __launch_bounds__(256) void k_ex_trsm_panel(double* __restrict__ A, long lda, int j0, int nb, int r0,
                                                       int n) {
  __shared__ double L[kCB][kCB + 1];
  const int tid = threadIdx.x;
  for (int e = tid; e < nb * nb; e += 256) L[e / nb][e % nb] = A[(long)(j0 + e / nb) * lda + j0 + e % nb];
  __syncthreads();
  const int r = r0 + blockIdx.x * 256 + tid;
  if (r >= n) return;
  // fully unrolled over the 64 panel columns (guarded by nb) so that x stays
  // in registers: a run-time index would put it in scratch memory
  double x[kCB];
  double* row = A + (long)r * lda + j0;
#pragma unroll
  for (int c = 0; c < kCB; ++c) {
    if (c < nb) {
      double v = row[c];
#pragma unroll
      for (int k = 0; k < c; ++k) v -= x[k] * L[c][k];
      x[c] = v / L[c][c];
    }
  }
#pragma unroll
  for (int c = 0; c < kCB; ++c)
    if (c < nb) row[c] = x[c];
}

void ex_cholesky(double* A, int n, long lda, int* status, hipStream_t st) {
  for (int j0 = 0; j0 < n; j0 += kCB) {
    const int nb = std::min(kCB, n - j0);
    hipLaunchKernelGGL(k_ex_potrf_block, dim3(1), dim3(256), 0, st, A, lda, j0, nb, status);
    const int r0 = j0 + nb;
    if (r0 < n) {
      hipLaunchKernelGGL(k_ex_trsm_panel, dim3((n - r0 + 255) / 256), dim3(256), 0, st, A, lda, j0, nb, r0, n);
      // A22 -= L21 L21^T
      const double* L21 = A + (long)r0 * lda + j0;
      ex_gemm(n - r0, n - r0, nb, -1.0, L21, lda, 1, L21, 1, lda, 1.0, A + (long)r0 * lda + r0, lda, st);
    }
  }
}

// ---------------------------------------------------------------------------
// Triangular solves with the factor L (lower, in A) for nrhs columns of X
// (X[i * ldx + c], overwritten): forward L Y = X, then backward L^T Z = Y.
// Blocked by 64 rows: the coupling to the rows already solved is a GEMM, the
// diagonal block is solved column by column (one thread per column).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_ex_trsv_block(const double* __restrict__ A, long lda, int i0, int nb,
                                                       double* __restrict__ X, long ldx, int nrhs, int upper) {
  __shared__ double L[kCB][kCB + 1];
  const int tid = threadIdx.x;
  for (int e = tid; e < nb * nb; e += 256) L[e / nb][e % nb] = A[(long)(i0 + e / nb) * lda + i0 + e % nb];
  __syncthreads();
  const int c = blockIdx.x * 256 + tid;
  if (c >= nrhs) return;
  // unrolled over the 64 block rows (guarded by nb): x stays in registers
  double x[kCB];
#pragma unroll
  for (int i = 0; i < kCB; ++i) x[i] = i < nb ? X[(long)(i0 + i) * ldx + c] : 0.0;
  if (!upper) {
#pragma unroll
    for (int i = 0; i < kCB; ++i) {
      if (i < nb) {
        double v = x[i];
#pragma unroll
        for (int k = 0; k < i; ++k) v -= L[i][k] * x[k];
        x[i] = v / L[i][i];
      }
    }
  } else {
#pragma unroll
    for (int i = kCB - 1; i >= 0; --i) {
      if (i < nb) {
        double v = x[i];
#pragma unroll
        for (int k = i + 1; k < kCB; ++k)
          if (k < nb) v -= L[k][i] * x[k];
        x[i] = v / L[i][i];
      }
    }
  }
#pragma unroll
  for (int i = 0; i < kCB; ++i)
    if (i < nb) X[(long)(i0 + i) * ldx + c] = x[i];
}

void ex_chol_solve(const double* A, int n, long lda, double* X, long ldx, int nrhs, hipStream_t st) {
  const dim3 g1((nrhs + 255) / 256);
  for (int i0 = 0; i0 < n; i0 += kCB) {
    const int nb = std::min(kCB, n - i0);
    if (i0 > 0)   // X[i0 block] -= L[i0 block, 0:i0] X[0:i0]
      ex_gemm(nb, nrhs, i0, -1.0, A + (long)i0 * lda, lda, 1, X, ldx, 1, 1.0, X + (long)i0 * ldx, ldx, st);
    hipLaunchKernelGGL(k_ex_trsv_block, g1, dim3(256), 0, st, A, lda, i0, nb, X, ldx, nrhs, 0);
  }
  const int last = ((n - 1) / kCB) * kCB;
  for (int i0 = last; i0 >= 0; i0 -= kCB) {
    const int nb = std::min(kCB, n - i0);
    const int r1 = i0 + nb;
    if (r1 < n)   // X[i0 block] -= L[r1:n, i0 block]^T X[r1:n]
      ex_gemm(nb, nrhs, n - r1, -1.0, A + (long)r1 * lda + i0, 1, lda, X + (long)r1 * ldx, ldx, 1, 1.0,
              X + (long)i0 * ldx, ldx, st);
    hipLaunchKernelGGL(k_ex_trsv_block, g1, dim3(256), 0, st, A, lda, i0, nb, X, ldx, nrhs, 1);
  }
}

// ---------------------------------------------------------------------------
// Matrix-vector products for up to kGvRhs right-hand sides at a time.
// y = alpha A x + beta y with A row-major (lda), x [N][nr], y [M][nr]: one
// wavefront per row, lanes striding over the row (coalesced), a wavefront
// reduction per right-hand side.  y = alpha A^T x + beta y: one lane per
// output column, looping over the rows of A (neighbouring lanes read
// neighbouring entries of a row).
// ---------------------------------------------------------------------------
constexpr int kGvRhs = 8;

__global__ __launch_bounds__(256) void k_ex_gemv(int M, int N, int nr, double alpha, const double* __restrict__ A,
                                                 long lda, const double* __restrict__ x, double beta,
                                                 double* __restrict__ y) {
  const int lane = threadIdx.x & 63;
  const long row = (long)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= M) return;
  const double* a = A + row * lda;
  for (int c0 = 0; c0 < nr; c0 += kGvRhs) {
    const int nc = min(kGvRhs, nr - c0);
    double acc[kGvRhs];
#pragma unroll
    for (int c = 0; c < kGvRhs; ++c) acc[c] = 0.0;
    for (int j = lane; j < N; j += 64) {
      const double av = a[j];
#pragma unroll
      for (int c = 0; c < kGvRhs; ++c)
        if (c < nc) acc[c] += av * x[(long)j * nr + c0 + c];
    }
#pragma unroll
    for (int c = 0; c < kGvRhs; ++c) {
      double v = acc[c];
      for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
      acc[c] = v;
    }
    if (lane < nc) {
      double v = 0.0;
#pragma unroll
      for (int c = 0; c < kGvRhs; ++c)
        if (c == lane) v = acc[c];
      double* yy = y + row * nr + c0 + lane;
      *yy = alpha * v + (beta == 0.0 ? 0.0 : beta * *yy);
    }
  }
}

__global__ __launch_bounds__(256) void k_ex_gemv_t(int M, int N, int nr, double alpha, const double* __restrict__ A,
                                                   long lda, const double* __restrict__ x, double beta,
                                                   double* __restrict__ y) {
  const long id = (long)blockIdx.x * blockDim.x + threadIdx.x;   // output column j, right-hand side c
  if (id >= (long)N * nr) return;
  const long j = id / nr;
  const int c = (int)(id % nr);
  double acc = 0.0;
  for (long i = 0; i < M; ++i) acc += A[i * lda + j] * x[i * nr + c];
  y[id] = alpha * acc + (beta == 0.0 ? 0.0 : beta * y[id]);
}

void ex_gemv(int M, int N, int nr, double alpha, const double* A, long lda, const double* x, double beta, double* y,
             hipStream_t st) {
  if (M <= 0 || nr <= 0) return;
  hipLaunchKernelGGL(k_ex_gemv, dim3((unsigned)((M + 3) / 4)), dim3(256), 0, st, M, N, nr, alpha, A, lda, x, beta, y);
}

void ex_gemv_t(int M, int N, int nr, double alpha, const double* A, long lda, const double* x, double beta, double* y,
               hipStream_t st) {
  const long tot = (long)N * nr;
  if (tot <= 0) return;
  hipLaunchKernelGGL(k_ex_gemv_t, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, M, N, nr, alpha, A, lda, x,
                     beta, y);
}

// ---------------------------------------------------------------------------
// Level operators.
// ---------------------------------------------------------------------------
__global__ void k_ex_fill(long len, double v, double* __restrict__ x) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < len) x[i] = v;
}

__global__ void k_ex_identity(long n, double* __restrict__ X) {
  const long id = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id < n * n) X[id] = (id / n == id % n) ? 1.0 : 0.0;
}

void ex_identity(long n, double* X, hipStream_t st) {
  hipLaunchKernelGGL(k_ex_identity, dim3((unsigned)((n * n + 255) / 256)), dim3(256), 0, st, n, X);
}

void ex_fill(long len, double v, double* x, hipStream_t st) {
  if (len <= 0) return;
  hipLaunchKernelGGL(k_ex_fill, dim3((unsigned)((len + 255) / 256)), dim3(256), 0, st, len, v, x);
}

// Dense Q1 stiffness over the interior nodes of an nc x nc cell grid (m =
// nc - 1 nodes per side), one thread per node row; a must be positive and
// finite (else the status bit is set).
__global__ void k_ex_assemble(const double* __restrict__ a, int nc, double* __restrict__ A, int* __restrict__ status) {
  const int m = nc - 1;
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= m * m) return;
  const int i = id / m + 1, j = id % m + 1;   // node coordinates
  const double a00 = a[(i - 1) * nc + (j - 1)], a10 = a[i * nc + (j - 1)];
  const double a01 = a[(i - 1) * nc + j], a11 = a[i * nc + j];
  if (!(a00 > 0.0 && a10 > 0.0 && a01 > 0.0 && a11 > 0.0) || !isfinite(a00 + a10 + a01 + a11))
    atomicOr(status, kBadCoefficient);
  const long N = (long)m * m;
  double* row = A + (long)id * N;
  auto put = [&](int di, int dj, double v) {
    const int ii = i + di, jj = j + dj;
    if (ii < 1 || jj < 1 || ii > m || jj > m) return;
    row[(long)(ii - 1) * m + (jj - 1)] = v;
  };
  put(0, 0, (2.0 / 3.0) * (a00 + a10 + a01 + a11));
  put(1, 0, -(a10 + a11) / 6.0);
  put(-1, 0, -(a00 + a01) / 6.0);
  put(0, 1, -(a01 + a11) / 6.0);
  put(0, -1, -(a00 + a10) / 6.0);
  put(1, 1, -a11 / 3.0);
  put(-1, -1, -a00 / 3.0);
  put(1, -1, -a10 / 3.0);
  put(-1, 1, -a01 / 3.0);
}

// B = W A W^T over the rp np2 subband rows (identity rows for rows a parent
// lacks) and C = -W A pibar^T (rp np2 x np2), one thread per entry.
__global__ void k_ex_subband(const double* __restrict__ A, long N, ExLevelTables t, double* __restrict__ B,
                             double* __restrict__ C) {
  const int cp = t.cp, rp = t.rp;
  const long nj = (long)rp * t.np2;
  const long id = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long nB = nj * nj;
  if (id < nB) {
    const int r = (int)(id / nj), s = (int)(id % nj);
    const int tr = r / t.np2, pr = r % t.np2, ts = s / t.np2, ps = s % t.np2;
    const bool rr = tr < t.nch[pr] - 1, rs = ts < t.nch[ps] - 1;
    double v = 0.0;
    if (!rr || !rs) {
      v = (r == s) ? 1.0 : 0.0;
    } else {
      for (int d = 0; d < cp; ++d) {
        const double wr = t.wc[((long)pr * rp + tr) * cp + d];
        if (wr == 0.0) continue;
        const long cr = t.child[(long)pr * cp + d];
        for (int e = 0; e < cp; ++e) {
          const double ws = t.wc[((long)ps * rp + ts) * cp + e];
          if (ws == 0.0) continue;
          v += wr * ws * A[cr * N + t.child[(long)ps * cp + e]];
        }
      }
    }
    B[id] = v;
    return;
  }
  const long id2 = id - nB;
  if (id2 >= nj * t.np2) return;
  const int r = (int)(id2 / t.np2), c = (int)(id2 % t.np2);
  const int tr = r / t.np2, pr = r % t.np2;
  double v = 0.0;
  if (tr < t.nch[pr] - 1) {
    for (int d = 0; d < cp; ++d) {
      const double wr = t.wc[((long)pr * rp + tr) * cp + d];
      if (wr == 0.0) continue;
      const long cr = t.child[(long)pr * cp + d];
      for (int e = 0; e < cp; ++e) {
        const int ce = t.child[(long)c * cp + e];
        if (ce < 0) continue;
        v += wr * A[cr * N + ce] / (double)t.nch[c];
      }
    }
  }
  C[id2] = -v;
}

// R = pibar + D^T W: R[c][b] for coarse c and level-k index b (D = the solved C, 3 np2 x np2).
__global__ void k_ex_restriction(const double* __restrict__ D, ExLevelTables t, long N, double* __restrict__ R) {
  const long id = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= (long)t.np2 * N) return;
  const int c = (int)(id / N);
  const int b = (int)(id % N);
  const int pb = t.parent[b], db = t.pos[b];
  double v = (pb == c) ? 1.0 / (double)t.nch[c] : 0.0;
  for (int tt = 0; tt < t.rp; ++tt) {
    const double w = t.wc[((long)pb * t.rp + tt) * t.cp + db];
    if (w != 0.0) v += D[((long)tt * t.np2 + pb) * t.np2 + c] * w;
  }
  R[id] = v;
}

void ex_level_operators(const double* A, long N, const ExLevelTables& t, double* B, double* C, hipStream_t st) {
  const long tot = ((long)t.rp * t.rp + t.rp) * t.np2 * t.np2;
  hipLaunchKernelGGL(k_ex_subband, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, A, N, t, B, C);
}

void ex_restriction(const double* D, const ExLevelTables& t, long N, double* R, hipStream_t st) {
  const long tot = (long)t.np2 * N;
  hipLaunchKernelGGL(k_ex_restriction, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, D, t, N, R);
}

// Entry of the bilinear element stiffness of a square cell with the constant
// symmetric tensor (a11, a12, a22), corners (dxi, dyi) and (dxj, dyj): the
// gradient components of hat_dx(x) hat_dy(y) split into 1-D factors,
// stiffness k (1 on, -1 off the diagonal), mass m (2/6 on, 1/6 off) and the
// mixed c[a][b] = int hat_a' hat_b = (a = 1 ? 1/2 : -1/2); the cell side
// cancels in two dimensions.
__device__ __forceinline__ double k_tensor2(const double* t, int dxi, int dyi, int dxj, int dyj) {
  const double kx = dxi == dxj ? 1.0 : -1.0, ky = dyi == dyj ? 1.0 : -1.0;
  const double mx = (dxi == dxj ? 2.0 : 1.0) / 6.0, my = (dyi == dyj ? 2.0 : 1.0) / 6.0;
  const double cxij = dxi == 1 ? 0.5 : -0.5, cxji = dxj == 1 ? 0.5 : -0.5;
  const double cyji = dyj == 1 ? 0.5 : -0.5, cyij = dyi == 1 ? 0.5 : -0.5;
  return t[0] * kx * my + t[2] * mx * ky + t[1] * (cxij * cyji + cxji * cyij);
}

__device__ __forceinline__ bool tensor_ok(const double* t) {
  const double det = t[0] * t[2] - t[1] * t[1];
  return t[0] > 0.0 && t[2] > 0.0 && det > 0.0 && isfinite(t[0] + t[1] + t[2]);
}

// Dense stiffness over the interior nodes of an nc x nc cell grid for a
// tensor coefficient a3[cell][3] = (a11, a12, a22), one thread per node row:
// the four cells around the node each add their element entries to the row.
__global__ void k_ex_assemble_tensor(const double* __restrict__ a3, int nc, double* __restrict__ A,
                                     int* __restrict__ status) {
  const int m = nc - 1;
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= m * m) return;
  const int i = id / m + 1, j = id % m + 1;
  const long N = (long)m * m;
  double* row = A + (long)id * N;
  for (int c = 0; c < 4; ++c) {
    const int cx = i - 1 + (c >> 1), cy = j - 1 + (c & 1);
    const double* t = a3 + ((long)cx * nc + cy) * 3;
    if (!tensor_ok(t)) atomicOr(status, kBadCoefficient);
    const int dxi = i - cx, dyi = j - cy;
    for (int lj = 0; lj < 4; ++lj) {
      const int dxj = lj >> 1, dyj = lj & 1;
      const int ii = cx + dxj, jj = cy + dyj;
      if (ii < 1 || jj < 1 || ii > m || jj > m) continue;
      row[(long)(ii - 1) * m + (jj - 1)] += k_tensor2(t, dxi, dyi, dxj, dyj);
    }
  }
}

void launch_ex_assemble_tensor(const double* a3, int nc, double* A, int* status, hipStream_t st) {
  const int m = nc - 1;
  hipLaunchKernelGGL(k_ex_assemble_tensor, dim3((m * m + 255) / 256), dim3(256), 0, st, a3, nc, A, status);
}

// Entry (li, lj) of the trilinear element stiffness of a unit cube, local
// node index 4 dx + 2 dy + dz: the gradient of a product of 1-D hats splits
// into three products of 1-D stiffness (k: 1 on, -1 off the diagonal) and
// mass (m: 2/6 on, 1/6 off) entries.
__device__ __forceinline__ double k_unit3(int li, int lj) {
  const int dx = li >> 2, dy = (li >> 1) & 1, dz = li & 1;
  const int ex = lj >> 2, ey = (lj >> 1) & 1, ez = lj & 1;
  const double kx = dx == ex ? 1.0 : -1.0, ky = dy == ey ? 1.0 : -1.0, kz = dz == ez ? 1.0 : -1.0;
  const double mx = (dx == ex ? 2.0 : 1.0) / 6.0, my = (dy == ey ? 2.0 : 1.0) / 6.0, mz = (dz == ez ? 2.0 : 1.0) / 6.0;
  return kx * my * mz + mx * ky * mz + mx * my * kz;
}

// Dense trilinear stiffness over the interior nodes of an nc^3 cell grid
// (m = nc - 1 nodes per side, node (i, j, l) -> ((i-1) m + (j-1)) m + (l-1)),
// one thread per node row: the eight cells around the node, each adding
// h a_e K_unit3 to the entries of its interior corners.
__global__ void k_ex_assemble3(const double* __restrict__ a, int nc, double* __restrict__ A,
                               int* __restrict__ status) {
  const int m = nc - 1;
  const long id = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long N = (long)m * m * m;
  if (id >= N) return;
  const int i = (int)(id / ((long)m * m)) + 1, j = (int)((id / m) % m) + 1, l = (int)(id % m) + 1;
  const double h = 1.0 / nc;
  double* row = A + id * N;
  for (int c = 0; c < 8; ++c) {
    const int cx = i - 1 + (c >> 2), cy = j - 1 + ((c >> 1) & 1), cz = l - 1 + (c & 1);   // cell
    const double ae = a[((long)cx * nc + cy) * nc + cz];
    if (!(ae > 0.0) || !isfinite(ae)) atomicOr(status, kBadCoefficient);
    const int li = ((i - cx) << 2) | ((j - cy) << 1) | (l - cz);   // the node inside the cell
    for (int lj = 0; lj < 8; ++lj) {
      const int ii = cx + (lj >> 2), jj = cy + ((lj >> 1) & 1), ll = cz + (lj & 1);
      if (ii < 1 || jj < 1 || ll < 1 || ii > m || jj > m || ll > m) continue;
      row[((long)(ii - 1) * m + (jj - 1)) * m + (ll - 1)] += h * ae * k_unit3(li, lj);
    }
  }
}

// 3-D load: mode 0 cell source ((h^3 / 8) sum of the eight cells), mode 1
// nodal source on the interior nodes (trilinear mass M g: (h/6)^3 times the
// product of the 1-D weights 4 (same) and 1 (neighbour)); then the Dirichlet
// values of u (boundary entries of [nrhs][nc+1]^3) moved to the right-hand side.
__global__ void k_ex_load3(int nc, int mode, const double* __restrict__ src, const double* __restrict__ a,
                           const double* __restrict__ u, int nrhs, double* __restrict__ b) {
  const int m = nc - 1;
  const long M3 = (long)m * m * m;
  const long id = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= M3 * nrhs) return;
  const long node = id / nrhs;
  const int c = (int)(id % nrhs);
  const int i = (int)(node / ((long)m * m)) + 1, j = (int)((node / m) % m) + 1, l = (int)(node % m) + 1;
  const double h = 1.0 / nc;
  double v = 0.0;
  if (mode == 0) {
    const double* g = src + (long)c * nc * nc * nc;
    for (int e = 0; e < 8; ++e) {
      const int cx = i - 1 + (e >> 2), cy = j - 1 + ((e >> 1) & 1), cz = l - 1 + (e & 1);
      v += g[((long)cx * nc + cy) * nc + cz];
    }
    v *= h * h * h / 8.0;
  } else {
    const double* g = src + (long)c * M3;
    for (int di = -1; di <= 1; ++di)
      for (int dj = -1; dj <= 1; ++dj)
        for (int dl = -1; dl <= 1; ++dl) {
          const int ii = i + di, jj = j + dj, ll = l + dl;
          if (ii < 1 || jj < 1 || ll < 1 || ii > m || jj > m || ll > m) continue;
          const double w = (di == 0 ? 4.0 : 1.0) * (dj == 0 ? 4.0 : 1.0) * (dl == 0 ? 4.0 : 1.0);
          v += w * g[((long)(ii - 1) * m + (jj - 1)) * m + (ll - 1)];
        }
    v *= h * h * h / 216.0;
  }
  if (i == 1 || j == 1 || l == 1 || i == m || j == m || l == m) {
    const double* uc = u + (long)c * (nc + 1) * (nc + 1) * (nc + 1);
    for (int e = 0; e < 8; ++e) {
      const int cx = i - 1 + (e >> 2), cy = j - 1 + ((e >> 1) & 1), cz = l - 1 + (e & 1);
      const double ae = a[((long)cx * nc + cy) * nc + cz];
      const int li = ((i - cx) << 2) | ((j - cy) << 1) | (l - cz);
      for (int lj = 0; lj < 8; ++lj) {
        const int ii = cx + (lj >> 2), jj = cy + ((lj >> 1) & 1), ll = cz + (lj & 1);
        if (!(ii == 0 || jj == 0 || ll == 0 || ii == nc || jj == nc || ll == nc)) continue;
        v -= h * ae * k_unit3(li, lj) * uc[((long)ii * (nc + 1) + jj) * (nc + 1) + ll];
      }
    }
  }
  b[id] = v;
}

// nodal [nrhs][(nc+1)^3] arrays and interior vectors x [N][nrhs]
__global__ void k_ex_to_nodal3(int nc, double* __restrict__ x, int nrhs, double* __restrict__ u, int back) {
  const int m = nc - 1;
  const long id = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= (long)m * m * m * nrhs) return;
  const long node = id / nrhs;
  const int c = (int)(id % nrhs);
  const int i = (int)(node / ((long)m * m)) + 1, j = (int)((node / m) % m) + 1, l = (int)(node % m) + 1;
  const long s = nc + 1;
  double* uu = u + (long)c * s * s * s + ((long)i * s + j) * s + l;
  if (back) x[id] = *uu;
  else *uu = x[id];
}

void launch_ex_assemble3(const double* a, int nc, double* A, int* status, hipStream_t st) {
  const long m = nc - 1;
  hipLaunchKernelGGL(k_ex_assemble3, dim3((unsigned)((m * m * m + 255) / 256)), dim3(256), 0, st, a, nc, A, status);
}

void ex_load3(int nc, int mode, const double* src, const double* a, const double* u, int nrhs, double* b,
              hipStream_t st) {
  const long m = nc - 1;
  const long tot = m * m * m * nrhs;
  hipLaunchKernelGGL(k_ex_load3, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, nc, mode, src, a, u, nrhs,
                     b);
}

void ex_to_nodal3(int nc, const double* x, int nrhs, double* u, bool back, hipStream_t st) {
  const long m = nc - 1;
  const long tot = m * m * m * nrhs;
  hipLaunchKernelGGL(k_ex_to_nodal3, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, nc,
                     const_cast<double*>(x), nrhs, u, back ? 1 : 0);
}

// ---------------------------------------------------------------------------
// Solve-phase vector operations (nrhs columns, vectors stored [index][nrhs]).
// ---------------------------------------------------------------------------
// Load over the interior nodes: mode 0 cell source (h^2 / 4 sum of the four
// cells), mode 1 nodal source on the interior nodes (Q1 mass M g, h^2/36 with
// weights 16, 4, 1; zero on the boundary); src is [nrhs][...].  Known
// Dirichlet values (the boundary entries of the nodal arrays u, [nrhs][nc+1]^2)
// move to the right-hand side: b_i -= sum over boundary nodes j of A_ij u_j,
// with the Q1 stiffness couplings of the cell coefficient a.
__global__ void k_ex_load(int nc, int mode, const double* __restrict__ src, const double* __restrict__ a,
                          const double* __restrict__ u, int nrhs, double* __restrict__ b, int tensor) {
  const int m = nc - 1;
  const long id = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= (long)m * m * nrhs) return;
  const int node = (int)(id / nrhs), c = (int)(id % nrhs);
  const int i = node / m + 1, j = node % m + 1;
  const double h = 1.0 / nc;
  double v = 0.0;
  if (mode == 0) {
    const double* g = src + (long)c * nc * nc;
    v = 0.25 * h * h * (g[(i - 1) * nc + (j - 1)] + g[i * nc + (j - 1)] + g[(i - 1) * nc + j] + g[i * nc + j]);
  } else {
    const double* g = src + (long)c * m * m;
    for (int di = -1; di <= 1; ++di)
      for (int dj = -1; dj <= 1; ++dj) {
        const int ii = i + di, jj = j + dj;
        if (ii < 1 || jj < 1 || ii > m || jj > m) continue;
        const double w = (di == 0 && dj == 0) ? 16.0 : ((di == 0 || dj == 0) ? 4.0 : 1.0);
        v += w * g[(ii - 1) * m + (jj - 1)];
      }
    v *= h * h / 36.0;
  }
  if (tensor && (i == 1 || j == 1 || i == m || j == m)) {
    const double* uc = u + (long)c * (nc + 1) * (nc + 1);
    for (int e = 0; e < 4; ++e) {
      const int cx = i - 1 + (e >> 1), cy = j - 1 + (e & 1);
      const double* t = a + ((long)cx * nc + cy) * 3;
      for (int lj = 0; lj < 4; ++lj) {
        const int ii = cx + (lj >> 1), jj = cy + (lj & 1);
        if (!(ii == 0 || jj == 0 || ii == nc || jj == nc)) continue;
        v -= k_tensor2(t, i - cx, j - cy, lj >> 1, lj & 1) * uc[(long)ii * (nc + 1) + jj];
      }
    }
  } else if (i == 1 || j == 1 || i == m || j == m) {
    const double a00 = a[(i - 1) * nc + (j - 1)], a10 = a[i * nc + (j - 1)];
    const double a01 = a[(i - 1) * nc + j], a11 = a[i * nc + j];
    const double* uc = u + (long)c * (nc + 1) * (nc + 1);
    for (int di = -1; di <= 1; ++di)
      for (int dj = -1; dj <= 1; ++dj) {
        const int ii = i + di, jj = j + dj;
        if (!(ii == 0 || jj == 0 || ii == nc || jj == nc)) continue;
        double kij;
        if (di == 0) kij = -(dj > 0 ? a01 + a11 : a00 + a10) / 6.0;
        else if (dj == 0) kij = -(di > 0 ? a10 + a11 : a00 + a01) / 6.0;
        else kij = -(di > 0 ? (dj > 0 ? a11 : a10) : (dj > 0 ? a01 : a00)) / 3.0;
        v -= kij * uc[(long)ii * (nc + 1) + jj];
      }
  }
  b[id] = v;
}

void ex_load(int nc, int mode, const double* src, const double* a, const double* u, int nrhs, double* b,
             bool tensor, hipStream_t st) {
  const long tot = (long)(nc - 1) * (nc - 1) * nrhs;
  hipLaunchKernelGGL(k_ex_load, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, nc, mode, src, a, u, nrhs,
                     b, tensor ? 1 : 0);
}

// y[J][c] = (W g)[J][c] (zero on the rows a parent lacks); g is level-k [N][nrhs]
__global__ void k_ex_wapply(ExLevelTables t, const double* __restrict__ g, int nrhs, double* __restrict__ y) {
  const long id = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= (long)t.rp * t.np2 * nrhs) return;
  const int r = (int)(id / nrhs), c = (int)(id % nrhs);
  const int tr = r / t.np2, pr = r % t.np2;
  double v = 0.0;
  if (tr < t.nch[pr] - 1)
    for (int d = 0; d < t.cp; ++d) {
      const double w = t.wc[((long)pr * t.rp + tr) * t.cp + d];
      if (w != 0.0) v += w * g[(long)t.child[(long)pr * t.cp + d] * nrhs + c];
    }
  y[id] = v;
}

void ex_wapply(const ExLevelTables& t, const double* g, int nrhs, double* y, hipStream_t st) {
  const long tot = (long)t.rp * t.np2 * nrhs;
  hipLaunchKernelGGL(k_ex_wapply, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, t, g, nrhs, y);
}

// v[b][c] += (W^T w)[b][c] for the level-k vector v ([N][nrhs])
__global__ void k_ex_wtadd(ExLevelTables t, long N, const double* __restrict__ w, int nrhs, double* __restrict__ v) {
  const long id = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= N * nrhs) return;
  const int b = (int)(id / nrhs), c = (int)(id % nrhs);
  const int pb = t.parent[b], db = t.pos[b];
  double acc = 0.0;
  for (int tt = 0; tt < t.rp; ++tt) {
    const double wc = t.wc[((long)pb * t.rp + tt) * t.cp + db];
    if (wc != 0.0) acc += wc * w[((long)tt * t.np2 + pb) * nrhs + c];
  }
  v[id] += acc;
}

void ex_wtadd(const ExLevelTables& t, long N, const double* w, int nrhs, double* v, hipStream_t st) {
  const long tot = N * nrhs;
  hipLaunchKernelGGL(k_ex_wtadd, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, t, N, w, nrhs, v);
}

// nodal [nrhs][(nc+1)^2] arrays and interior vectors x [N][nrhs]: write the
// interior entries of u from x (boundary untouched), or gather x from u
__global__ void k_ex_to_nodal(int nc, double* __restrict__ x, int nrhs, double* __restrict__ u, int back) {
  const int m = nc - 1;
  const long id = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= (long)m * m * nrhs) return;
  const int node = (int)(id / nrhs), c = (int)(id % nrhs);
  const int i = node / m + 1, j = node % m + 1;
  double* uu = u + (long)c * (nc + 1) * (nc + 1) + (long)i * (nc + 1) + j;
  if (back) x[id] = *uu;
  else *uu = x[id];
}

void ex_to_nodal(int nc, const double* x, int nrhs, double* u, hipStream_t st) {
  const long tot = (long)(nc - 1) * (nc - 1) * nrhs;
  hipLaunchKernelGGL(k_ex_to_nodal, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, nc, const_cast<double*>(x),
                     nrhs, u, 0);
}

void ex_from_nodal(int nc, const double* u, int nrhs, double* x, hipStream_t st) {
  const long tot = (long)(nc - 1) * (nc - 1) * nrhs;
  hipLaunchKernelGGL(k_ex_to_nodal, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, nc, x, nrhs,
                     const_cast<double*>(u), 1);
}

// y += alpha x
__global__ void k_ex_axpy(long n, double alpha, const double* __restrict__ x, double* __restrict__ y) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] += alpha * x[i];
}

void ex_axpy(long n, double alpha, const double* x, double* y, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_ex_axpy, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, alpha, x, y);
}

// the diagonal of a dense n x n matrix
__global__ void k_ex_diag(const double* __restrict__ M, long n, double* __restrict__ d) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) d[i] = M[i * n + i];
}

void ex_diag(const double* M, long n, double* d, hipStream_t st) {
  hipLaunchKernelGGL(k_ex_diag, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, M, n, d);
}

// out[i] = scale_i * in[i] with scale_i = sqrt(M[i][i]) (mode 0) or 1 / sqrt(M[i][i]) (mode 1), zero where
// the diagonal is an identity padding row (pad set) -- the normalization of the gamblet transform
__global__ void k_ex_diag_scale(const double* __restrict__ M, long n, long ld, const double* __restrict__ in,
                                double* __restrict__ out, int inverse, ExLevelTables t, int pad) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (pad) {
    const int tr = (int)(i / t.np2), pr = (int)(i % t.np2);
    if (tr >= t.nch[pr] - 1) {
      out[i] = 0.0;
      return;
    }
  }
  const double s = sqrt(M[i * ld + i]);
  out[i] = inverse ? in[i] / s : in[i] * s;
}

void ex_diag_scale(const double* M, long n, long ld, const double* in, double* out, bool inverse,
                   const ExLevelTables* t, hipStream_t st) {
  ExLevelTables z{};
  hipLaunchKernelGGL(k_ex_diag_scale, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, M, n, ld, in, out,
                     inverse ? 1 : 0, t ? *t : z, t ? 1 : 0);
}

// child sums: out[c] = sum over the children of c of in[child]  (U^(k-1) = pi U^(k))
__global__ void k_ex_child_sum(ExLevelTables t, const double* __restrict__ in, double* __restrict__ out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= t.np2) return;
  double v = 0.0;
  for (int d = 0; d < t.cp; ++d) {
    const int ch = t.child[(long)c * t.cp + d];
    if (ch >= 0) v += in[ch];
  }
  out[c] = v;
}

void ex_child_sum(const ExLevelTables& t, const double* in, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_ex_child_sum, dim3((t.np2 + 255) / 256), dim3(256), 0, st, t, in, out);
}

// w[t][p] <- sum_u G_p^-1[t][u] w[u][p], G_p = W_p W_p^T per parent (rp x rp, rp <= 7)
__global__ void k_ex_gram_solve(int np2, int rp, const double* __restrict__ gi, double* __restrict__ w) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= np2) return;
  double x[7];
  for (int a = 0; a < rp; ++a) x[a] = w[(size_t)a * np2 + p];
  const double* g = gi + (size_t)p * rp * rp;
  for (int a = 0; a < rp; ++a) {
    double v = 0.0;
    for (int b = 0; b < rp; ++b) v += g[a * rp + b] * x[b];
    w[(size_t)a * np2 + p] = v;
  }
}

void ex_gram_solve(const ExLevelTables& t, const double* gram_inv, double* w, hipStream_t st) {
  hipLaunchKernelGGL(k_ex_gram_solve, dim3((t.np2 + 255) / 256), dim3(256), 0, st, t.np2, t.rp, gram_inv, w);
}

}  // namespace gbl

namespace gbl {
void launch_ex_assemble(const double* a, int nc, double* A, int* status, hipStream_t st) {
  const int m = nc - 1;
  hipLaunchKernelGGL(k_ex_assemble, dim3((m * m + 255) / 256), dim3(256), 0, st, a, nc, A, status);
}
}  // namespace gbl
