// Exact (unlocalized) hierarchy: host-side state and calls used by the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <string>

#include "exact_internal.hpp"

namespace gbl {

// Workspace offsets (bytes) of the exact hierarchy of depth q.
struct ExactHier {
  int q = 0, geom = 0;
  int dim = 2;     // 2 or 3
  int tensor = 0;  // 1: per-cell symmetric tensor (a11, a12, a22) in two dimensions
  int cp = 4;      // child slots per parent, 2^dim
  int rp = 3;      // subband rows per parent, 2^dim - 1
  long ncells = 0; // nc^dim
  long nnodes = 0; // (nc + 1)^dim
  long ncoef = 0;  // coefficients of the transform, 2^(dim q)
  int wkind = 0;   // 0: Construction 4.13 (Helmert), 1: Construction 4.11 (differences)
  int nc = 0;   // cells per side
  int m = 0;    // interior nodes per side
  int nr = 1;   // right-hand sides per solve pass
  long N[kMaxLevels] = {};     // unknowns of level k
  int np2[kMaxLevels] = {};    // parents of level k (unknowns of level k - 1)
  size_t offA[kMaxLevels] = {}, offB[kMaxLevels] = {}, offBL[kMaxLevels] = {}, offD[kMaxLevels] = {},
         offR[kMaxLevels] = {};
  size_t offNch[kMaxLevels] = {}, offChild[kMaxLevels] = {}, offWc[kMaxLevels] = {}, offParent[kMaxLevels] = {},
         offPos[kMaxLevels] = {}, offGinv[kMaxLevels] = {};
  size_t offG[kMaxLevels] = {}, offW[kMaxLevels] = {}, offU[kMaxLevels] = {};
  size_t offBinv[kMaxLevels] = {}, offWt[kMaxLevels] = {};
  size_t offT = 0, offB0 = 0, offX = 0, offRes = 0, offDx = 0, offL1 = 0, offStatus = 0, offSel = 0, offThr = 0;
  size_t offDot = 0, offCoef = 0;   // offCoef: a copy of the cell coefficient ([nc]^d, or [nc][nc][3])
  size_t total = 0;
  char* ws = nullptr;

  double* at(size_t off) const { return reinterpret_cast<double*>(ws + off); }
  double* A(int k) const { return at(offA[k]); }    // A^(k), N_k x N_k
  double* B(int k) const { return at(offB[k]); }    // B^(k) = W A^(k) W^T, rp np2 x rp np2
  double* BL(int k) const { return at(offBL[k]); }  // its Cholesky factor (lower)
  double* Binv(int k) const { return at(offBinv[k]); }   // B^(k)^-1 (from the factor)
  double* Wt(int k) const { return at(offWt[k]); }       // W g^(k) before the subband solve
  double* D(int k) const { return at(offD[k]); }    // D^(k,k-1), rp np2 x np2
  double* R(int k) const { return at(offR[k]); }    // R^(k-1,k), np2 x N_k
  double* G(int k) const { return at(offG[k]); }    // level-k solve vectors [N_k][nr]
  double* W(int k) const { return at(offW[k]); }    // subband vectors [rp np2][nr]
  double* U(int k) const { return at(offU[k]); }    // transform vectors [N_k]
};

int exact_layout(ExactHier& E, int q, int dim, int geom, int wkind, int tensor, int max_rhs, std::string& msg);
int exact_build(ExactHier& E, const double* a_dev, hipStream_t st, std::string& msg);
int exact_solve(ExactHier& E, int nrhs, int source, const double* src, double* u_nodal, int refine, hipStream_t st,
                std::string& msg);
int exact_transform(ExactHier& E, const double* u_nodal, double* coef, hipStream_t st);
int exact_inverse_transform(ExactHier& E, const double* coef, double* u_nodal, hipStream_t st);
int exact_energy_norm(ExactHier& E, const double* u_nodal, double* norm, hipStream_t st);
ExLevelTables exact_tables(const ExactHier& E, int k);

}  // namespace gbl
