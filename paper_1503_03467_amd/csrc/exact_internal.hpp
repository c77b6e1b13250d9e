// Exact (unlocalized) hierarchy: dense level matrices in FP64 (Algorithm 1).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>

#include "gamblet_internal.hpp"

namespace gbl {

// Tree tables of the transition from level k to level k - 1 (device pointers).
struct ExLevelTables {
  int np2 = 0;                  // parents (level k-1 unknowns)
  int cp = 4;                   // child slots per parent: 2^d
  int rp = 3;                   // subband rows per parent: 2^d - 1
  const int* nch = nullptr;     // [np2] child counts m_p
  const int* child = nullptr;   // [np2][cp] level-k index of the child at position d (by t), -1 past m_p
  const double* wc = nullptr;   // [np2][rp][cp] row t of W over parent p's child positions
  const int* parent = nullptr;  // [N_k] parent of a level-k unknown
  const int* pos = nullptr;     // [N_k] its position among the parent's children
};

void ex_gemm(int M, int N, int K, double alpha, const double* A, long as0, long as1, const double* B, long bs0,
             long bs1, double beta, double* C, long ldc, hipStream_t st);
void ex_cholesky(double* A, int n, long lda, int* status, hipStream_t st);
// y = alpha A x + beta y (A row-major M x N, x [N][nr], y [M][nr]) and its transposed form
void ex_gemv(int M, int N, int nr, double alpha, const double* A, long lda, const double* x, double beta, double* y,
             hipStream_t st);
void ex_gemv_t(int M, int N, int nr, double alpha, const double* A, long lda, const double* x, double beta, double* y,
               hipStream_t st);
void ex_chol_solve(const double* A, int n, long lda, double* X, long ldx, int nrhs, hipStream_t st);
void ex_fill(long len, double v, double* x, hipStream_t st);
void ex_identity(long n, double* X, hipStream_t st);
void ex_level_operators(const double* A, long N, const ExLevelTables& t, double* B, double* C, hipStream_t st);
void ex_restriction(const double* D, const ExLevelTables& t, long N, double* R, hipStream_t st);
void ex_load(int nc, int mode, const double* src, const double* a, const double* u, int nrhs, double* b,
             bool tensor, hipStream_t st);
void ex_wapply(const ExLevelTables& t, const double* g, int nrhs, double* y, hipStream_t st);
void ex_wtadd(const ExLevelTables& t, long N, const double* w, int nrhs, double* v, hipStream_t st);
void ex_to_nodal(int nc, const double* x, int nrhs, double* u, hipStream_t st);
void ex_from_nodal(int nc, const double* u, int nrhs, double* x, hipStream_t st);
void ex_axpy(long n, double alpha, const double* x, double* y, hipStream_t st);
void ex_diag(const double* M, long n, double* d, hipStream_t st);
void ex_diag_scale(const double* M, long n, long ld, const double* in, double* out, bool inverse,
                   const ExLevelTables* t, hipStream_t st);
void ex_child_sum(const ExLevelTables& t, const double* in, double* out, hipStream_t st);
void ex_gram_solve(const ExLevelTables& t, const double* gram_inv, double* w, hipStream_t st);
void launch_ex_assemble(const double* a, int nc, double* A, int* status, hipStream_t st);
void launch_ex_assemble_tensor(const double* a3, int nc, double* A, int* status, hipStream_t st);
void launch_ex_assemble3(const double* a, int nc, double* A, int* status, hipStream_t st);
void ex_load3(int nc, int mode, const double* src, const double* a, const double* u, int nrhs, double* b,
              hipStream_t st);
void ex_to_nodal3(int nc, const double* x, int nrhs, double* u, bool back, hipStream_t st);

}  // namespace gbl
