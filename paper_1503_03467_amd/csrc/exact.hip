// Host side of the exact (unlocalized) hierarchy: Algorithm 1 on dense level
// matrices in FP64, the subband solve of Section 4.7 / Theorem 4.15 with
// every subband system solved exactly, and the gamblet transform of the
// discussion of Example 5.1 (Figures 10-11) in that basis.
//
// Geometry 0: 2^q x 2^q cells, (2^q - 1)^2 interior nodes, node (i, j) in the
// level-(q-1) cell (i / 2, j / 2) -- cells on the two low edges have one or
// two children.  Geometry 1 (the mesh of Example 5.1): (2^q + 1)^2 cells,
// 2^q x 2^q interior nodes, node (i, j) in cell ((i - 1) / 2, (j - 1) / 2),
// every parent with four children.  Levels k < q are the dyadic cells.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "exact_internal.hpp"
#include "exact_host.hpp"

namespace gbl {

namespace {

size_t al(size_t x) { return (x + 255) / 256 * 256; }

// Row t (< m - 1) of W over a parent's m children.  kind 0, Construction
// 4.13: the normalised Helmert row (1, ..., 1, -(t + 1), 0, ...) /
// sqrt((t + 1)(t + 2)) with t + 1 ones.  kind 1, Construction 4.11: the
// difference e_t - e_{t+1}.
double wrow(int kind, int m, int t, int d) {
  if (t >= m - 1 || d >= m) return 0.0;
  if (kind == 1) return d == t ? 1.0 : (d == t + 1 ? -1.0 : 0.0);
  const double s = 1.0 / std::sqrt((double)(t + 1) * (double)(t + 2));
  if (d <= t) return s;
  if (d == t + 1) return -(double)(t + 1) * s;
  return 0.0;
}

}  // namespace

int exact_layout(ExactHier& E, int q, int dim, int geom, int wkind, int tensor, int max_rhs, std::string& msg) {
  if (dim != 2 && dim != 3) { msg = "dim must be 2 or 3"; return GBL_EINVAL; }
  if (tensor && dim != 2) { msg = "tensor coefficients are built in two dimensions"; return GBL_EINVAL; }
  const int qmax = dim == 2 ? 7 : 4;
  if (q < 2 || q > qmax) {
    msg = dim == 2 ? "the exact hierarchy is built for 2 <= q <= 7" : "the exact hierarchy in 3-D is built for 2 <= q <= 4";
    return GBL_EINVAL;
  }
  if (geom != 0 && geom != 1) { msg = "geometry must be 0 or 1"; return GBL_EINVAL; }
  E = ExactHier{};
  E.q = q;
  E.dim = dim;
  E.cp = 1 << dim;
  E.rp = E.cp - 1;
  E.geom = geom;
  E.wkind = wkind;
  E.tensor = tensor ? 1 : 0;
  E.nc = geom == 0 ? (1 << q) : (1 << q) + 1;
  E.m = E.nc - 1;
  E.nr = std::max(1, std::min(max_rhs, 64));
  long mq = 1, ncd = 1, nnd = 1;
  for (int d = 0; d < dim; ++d) {
    mq *= E.m;
    ncd *= E.nc;
    nnd *= E.nc + 1;
  }
  E.ncells = ncd;
  E.nnodes = nnd;
  for (int k = 1; k <= q; ++k) E.N[k] = (k == q) ? mq : (1L << (dim * k));
  for (int k = 2; k <= q; ++k) E.np2[k] = 1 << (dim * (k - 1));
  E.ncoef = 1L << (dim * q);
  const int cp = E.cp, rp = E.rp;
  size_t b = 0;
  long most = 0;
  for (int k = 1; k <= q; ++k) {
    const long N = E.N[k];
    E.offA[k] = b; b = al(b + (size_t)N * N * 8);
    if (k >= 2) {
      const long np2 = E.np2[k], nj = (long)rp * np2;
      E.offB[k] = b; b = al(b + (size_t)nj * nj * 8);
      E.offBL[k] = b; b = al(b + (size_t)nj * nj * 8);
      E.offBinv[k] = b; b = al(b + (size_t)nj * nj * 8);
      E.offD[k] = b; b = al(b + (size_t)nj * np2 * 8);
      E.offR[k] = b; b = al(b + (size_t)np2 * N * 8);
      E.offNch[k] = b; b = al(b + (size_t)np2 * 4);
      E.offChild[k] = b; b = al(b + (size_t)np2 * cp * 4);
      E.offWc[k] = b; b = al(b + (size_t)np2 * rp * cp * 8);
      E.offParent[k] = b; b = al(b + (size_t)N * 4);
      E.offPos[k] = b; b = al(b + (size_t)N * 4);
      E.offGinv[k] = b; b = al(b + (size_t)np2 * rp * rp * 8);
      most = std::max(most, np2 * N);
      E.offW[k] = b; b = al(b + (size_t)nj * E.nr * 8);
      E.offWt[k] = b; b = al(b + (size_t)nj * E.nr * 8);
    }
    E.offG[k] = b; b = al(b + (size_t)N * E.nr * 8);
    E.offU[k] = b; b = al(b + (size_t)N * 8);
  }
  E.offT = b; b = al(b + (size_t)most * 8);
  const long Nq = E.N[q];
  E.offB0 = b; b = al(b + (size_t)Nq * E.nr * 8);
  E.offX = b; b = al(b + (size_t)Nq * E.nr * 8);
  E.offRes = b; b = al(b + (size_t)Nq * E.nr * 8);
  E.offDx = b; b = al(b + (size_t)Nq * E.nr * 8);
  E.offL1 = b; b = al(b + (size_t)cp * cp * 8);
  E.offStatus = b; b = al(b + 16);
  E.offSel = b; b = al(b + 4 * 8 + (size_t)kSelHistBins * 4);
  E.offThr = b; b = al(b + 64);
  E.offDot = b; b = al(b + (size_t)E.nr * 8);
  E.offCoef = b; b = al(b + (size_t)ncd * (E.tensor ? 3 : 1) * 8);
  E.total = b;
  return GBL_OK;
}

ExLevelTables exact_tables(const ExactHier& E, int k) {
  ExLevelTables t;
  t.np2 = E.np2[k];
  t.cp = E.cp;
  t.rp = E.rp;
  t.nch = reinterpret_cast<const int*>(E.ws + E.offNch[k]);
  t.child = reinterpret_cast<const int*>(E.ws + E.offChild[k]);
  t.wc = reinterpret_cast<const double*>(E.ws + E.offWc[k]);
  t.parent = reinterpret_cast<const int*>(E.ws + E.offParent[k]);
  t.pos = reinterpret_cast<const int*>(E.ws + E.offPos[k]);
  return t;
}

// Interior values of nodal arrays ((nc+1)^d per right-hand side) to and from
// level-q vectors ([N][nr]).
static void to_nodal(const ExactHier& E, const double* x, int nr, double* u, hipStream_t st) {
  if (E.dim == 2) ex_to_nodal(E.nc, x, nr, u, st);
  else ex_to_nodal3(E.nc, x, nr, u, false, st);
}
static void from_nodal(const ExactHier& E, const double* u, double* x, hipStream_t st) {
  if (E.dim == 2) ex_from_nodal(E.nc, u, 1, x, st);
  else ex_to_nodal3(E.nc, x, 1, const_cast<double*>(u), true, st);
}

// Tree tables of every transition, built on the host and copied (synchronously).
// Level q: the interior node with coordinates (i, j[, l]) sits in slot
// (i, j[, l]) (geometry 0) or (i - 1, j - 1[, l - 1]) (geometry 1) of the
// level's 2^q grid; levels k < q: the dyadic cells.  A slot's parent halves
// every coordinate, its child position is t = sum of the low bits, x most
// significant.
static int upload_tables(ExactHier& E, std::string& msg) {
  const int dim = E.dim, cp = E.cp, rp = E.rp;
  for (int k = 2; k <= E.q; ++k) {
    const long N = E.N[k];
    const int np2 = E.np2[k];
    const int side_par = 1 << (k - 1);
    std::vector<int> nch(np2, 0), child((size_t)cp * np2, -1), parent(N), pos(N);
    std::vector<std::vector<std::pair<int, int>>> kids(np2);   // (t, index)
    for (long b = 0; b < N; ++b) {
      int sl[3] = {0, 0, 0};   // slot coordinates on the level's 2^k grid
      long rem = b;
      for (int d = dim - 1; d >= 0; --d) {
        if (k == E.q) {
          const int c = (int)(rem % E.m) + 1;
          rem /= E.m;
          sl[d] = E.geom == 0 ? c : c - 1;
        } else {
          sl[d] = (int)(rem & ((1L << k) - 1));
          rem >>= k;
        }
      }
      int p = 0, t = 0;
      for (int d = 0; d < dim; ++d) {
        p = p * side_par + (sl[d] >> 1);
        t = 2 * t + (sl[d] & 1);
      }
      parent[b] = p;
      kids[p].push_back({t, (int)b});
    }
    std::vector<double> wc((size_t)rp * cp * np2, 0.0), gram_inv((size_t)rp * rp * np2, 0.0);
    for (int p = 0; p < np2; ++p) {
      auto& v = kids[p];
      std::sort(v.begin(), v.end());
      nch[p] = (int)v.size();
      if (v.empty() || (int)v.size() > cp) { msg = "tree construction failed"; return GBL_EINVAL; }
      for (size_t d = 0; d < v.size(); ++d) {
        child[(size_t)cp * p + d] = v[d].second;
        pos[v[d].second] = (int)d;
      }
      double* wp = &wc[(size_t)p * rp * cp];
      for (int t = 0; t < rp; ++t)
        for (int d = 0; d < cp; ++d) wp[t * cp + d] = wrow(E.wkind, nch[p], t, d);
      // (W_p W_p^T)^-1 over the parent's real rows (identity on the rows it
      // lacks), by Gauss-Jordan on the SPD Gram matrix
      const int nr = nch[p] - 1;
      double g[7][14];
      for (int a = 0; a < rp; ++a)
        for (int c = 0; c < 2 * rp; ++c) {
          double v2 = 0.0;
          if (c < rp) {
            if (a < nr && c < nr)
              for (int d = 0; d < cp; ++d) v2 += wp[a * cp + d] * wp[c * cp + d];
            else
              v2 = a == c ? 1.0 : 0.0;
          } else {
            v2 = (c - rp == a) ? 1.0 : 0.0;
          }
          g[a][c] = v2;
        }
      for (int c = 0; c < rp; ++c) {
        const double piv = g[c][c];
        for (int c2 = 0; c2 < 2 * rp; ++c2) g[c][c2] /= piv;
        for (int a = 0; a < rp; ++a)
          if (a != c) {
            const double f = g[a][c];
            for (int c2 = 0; c2 < 2 * rp; ++c2) g[a][c2] -= f * g[c][c2];
          }
      }
      for (int a = 0; a < rp; ++a)
        for (int c = 0; c < rp; ++c) gram_inv[(size_t)p * rp * rp + a * rp + c] = g[a][c + rp];
    }
    if (hipMemcpy(E.ws + E.offNch[k], nch.data(), nch.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(E.ws + E.offChild[k], child.data(), child.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(E.ws + E.offWc[k], wc.data(), wc.size() * 8, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(E.ws + E.offParent[k], parent.data(), parent.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(E.ws + E.offPos[k], pos.data(), pos.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(E.ws + E.offGinv[k], gram_inv.data(), gram_inv.size() * 8, hipMemcpyHostToDevice) != hipSuccess) {
      msg = "copy of the tree tables failed";
      return GBL_EHIP;
    }
  }
  return GBL_OK;
}

// Algorithm 1: B = W A W^T, D = -B^-1 W A pibar^T, R = pibar + D^T W,
// A^(k-1) = R A R^T for k = q .. 2, then the Cholesky factor of A^(1).
int exact_build(ExactHier& E, const double* a_dev, hipStream_t st, std::string& msg) {
  int* status = reinterpret_cast<int*>(E.ws + E.offStatus);
  ex_fill(4, 0.0, reinterpret_cast<double*>(E.ws + E.offStatus), st);   // 16 bytes: status word and spare
  if (hipStreamSynchronize(st) != hipSuccess) { msg = "stream error"; return GBL_EHIP; }
  int rc = upload_tables(E, msg);
  if (rc) return rc;
  const int q = E.q;
  double* Aq = E.A(q);
  if (hipMemcpyAsync(E.at(E.offCoef), a_dev, (size_t)E.ncells * (E.tensor ? 3 : 1) * 8, hipMemcpyDeviceToDevice,
                     st) != hipSuccess) {
    msg = "copy failed";
    return GBL_EHIP;
  }
  ex_fill(E.N[q] * E.N[q], 0.0, Aq, st);
  if (E.tensor) launch_ex_assemble_tensor(a_dev, E.nc, Aq, status, st);
  else if (E.dim == 2) launch_ex_assemble(a_dev, E.nc, Aq, status, st);
  else launch_ex_assemble3(a_dev, E.nc, Aq, status, st);
  for (int k = q; k >= 2; --k) {
    const long N = E.N[k];
    const int np2 = E.np2[k];
    const int nj = E.rp * np2;
    const ExLevelTables t = exact_tables(E, k);
    double* B = E.B(k);
    double* D = E.D(k);
    double* R = E.R(k);
    ex_level_operators(E.A(k), N, t, B, D, st);   // B and C = -W A pibar^T (into D)
    if (hipMemcpyAsync(E.BL(k), B, (size_t)nj * nj * 8, hipMemcpyDeviceToDevice, st) != hipSuccess) {
      msg = "copy failed";
      return GBL_EHIP;
    }
    ex_cholesky(E.BL(k), nj, nj, status, st);
    ex_chol_solve(E.BL(k), nj, nj, D, np2, np2, st);    // D = B^-1 C
    // B^-1 itself, for the solves: each subband system is then one
    // bandwidth-bound matrix-vector product instead of two chains of
    // dependent triangular blocks
    ex_identity(nj, E.Binv(k), st);
    ex_chol_solve(E.BL(k), nj, nj, E.Binv(k), nj, nj, st);
    ex_restriction(D, t, N, R, st);
    // A^(k-1) = R A R^T: T = R A, then T R^T
    double* T = reinterpret_cast<double*>(E.ws + E.offT);
    ex_gemm(np2, (int)N, (int)N, 1.0, R, N, 1, E.A(k), N, 1, 0.0, T, N, st);
    ex_gemm(np2, np2, (int)N, 1.0, T, N, 1, R, 1, N, 0.0, E.A(k - 1), np2, st);
  }
  // factor of A^(1) (2^d x 2^d), kept apart from A^(1)
  double* L1 = reinterpret_cast<double*>(E.ws + E.offL1);
  if (hipMemcpyAsync(L1, E.A(1), (size_t)E.cp * E.cp * 8, hipMemcpyDeviceToDevice, st) != hipSuccess) {
    msg = "copy failed";
    return GBL_EHIP;
  }
  ex_cholesky(L1, E.cp, E.cp, status, st);
  if (hipGetLastError() != hipSuccess) { msg = "launch failed"; return GBL_EHIP; }
  int h = 0;
  if (hipMemcpyAsync(&h, status, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess) {
    msg = "status read failed";
    return GBL_EHIP;
  }
  if (h & kBadCoefficient) { msg = "coefficient must be positive and finite in every cell"; return GBL_EINVAL; }
  if (h & kBadPivot) { msg = "non-positive pivot in a level matrix"; return GBL_ENOTSPD; }
  return GBL_OK;
}

// x = S y: the exact subband solve of the level-q vector y (nr columns, [N][nr])
static void subband_solve(ExactHier& E, const double* y, double* x, int nr, hipStream_t st) {
  const int q = E.q;
  // g^(q) = y, g^(k-1) = R g^(k)
  if (hipMemcpyAsync(E.G(q), y, (size_t)E.N[q] * nr * 8, hipMemcpyDeviceToDevice, st) != hipSuccess) return;
  for (int k = q; k >= 2; --k) ex_gemv(E.np2[k], (int)E.N[k], nr, 1.0, E.R(k), E.N[k], E.G(k), 0.0, E.G(k - 1), st);
  // subband systems B^(k) w = W g^(k) (w = B^-1 W g) and A^(1) U = g^(1)
  for (int k = q; k >= 2; --k) {
    const ExLevelTables t = exact_tables(E, k);
    const int nj = E.rp * E.np2[k];
    ex_wapply(t, E.G(k), nr, E.Wt(k), st);
    ex_gemv(nj, nj, nr, 1.0, E.Binv(k), nj, E.Wt(k), 0.0, E.W(k), st);
  }
  ex_chol_solve(reinterpret_cast<const double*>(E.ws + E.offL1), E.cp, E.cp, E.G(1), nr, nr, st);
  // v^(1) = U, v^(k) = R^T v^(k-1) + W^T w^(k)   (Theorem 4.15)
  for (int k = 2; k <= q; ++k) {
    double* vk = (k == q) ? x : E.G(k);
    ex_gemv_t(E.np2[k], (int)E.N[k], nr, 1.0, E.R(k), E.N[k], E.G(k - 1), 0.0, vk, st);
    ex_wtadd(exact_tables(E, k), E.N[k], E.W(k), nr, vk, st);
  }
}

// Solve for nrhs right-hand sides: u = S b plus FP64 refinement steps with the
// dense level-q operator (r = b - A u, u += S r).  The boundary entries of
// u_nodal hold the Dirichlet data on entry (lifted into b) and are kept.
int exact_solve(ExactHier& E, int nrhs, int source, const double* src, double* u_nodal, int refine, hipStream_t st,
                std::string& msg) {
  const long Nq = E.N[E.q];
  const size_t src_stride = source == 0 ? (size_t)E.ncells : (size_t)Nq;
  const size_t u_stride = (size_t)E.nnodes;
  double* b = E.at(E.offB0);
  double* x = E.at(E.offX);
  double* r = E.at(E.offRes);
  double* dx = E.at(E.offDx);
  for (int r0 = 0; r0 < nrhs; r0 += E.nr) {
    const int nr = std::min(E.nr, nrhs - r0);
    const size_t len = (size_t)Nq * nr;
    if (E.dim == 2)
      ex_load(E.nc, source, src + r0 * src_stride, E.at(E.offCoef), u_nodal + r0 * u_stride, nr, b, E.tensor != 0, st);
    else ex_load3(E.nc, source, src + r0 * src_stride, E.at(E.offCoef), u_nodal + r0 * u_stride, nr, b, st);
    subband_solve(E, b, x, nr, st);
    for (int it = 0; it < refine; ++it) {   // r = b - A u;  u += S r
      if (hipMemcpyAsync(r, b, len * 8, hipMemcpyDeviceToDevice, st) != hipSuccess) {
        msg = "copy failed";
        return GBL_EHIP;
      }
      ex_gemv((int)Nq, (int)Nq, nr, -1.0, E.A(E.q), Nq, x, 1.0, r, st);
      subband_solve(E, r, dx, nr, st);
      ex_axpy((long)len, 1.0, dx, x, st);
    }
    to_nodal(E, x, nr, u_nodal + r0 * u_stride, st);
  }
  if (hipGetLastError() != hipSuccess) { msg = "launch failed"; return GBL_EHIP; }
  if (hipStreamSynchronize(st) != hipSuccess) { msg = "stream error"; return GBL_EHIP; }
  return GBL_OK;
}

// Coefficients of a nodal u on psi^(1)/||psi^(1)||_a and chi^(k)/||chi^(k)||_a:
// U^(k-1) = pi U^(k), w^(k) = (W W^T)^-1 W (U^(k) - R^T U^(k-1)) (the Gram
// factor is the identity for the orthonormal rows of Construction 4.13),
// scaled by sqrt(A^(1)_ii), sqrt(B^(k)_jj).
int exact_transform(ExactHier& E, const double* u_nodal, double* coef, hipStream_t st) {
  const int q = E.q;
  from_nodal(E, u_nodal, E.U(q), st);
  double* d = E.at(E.offT);
  for (int k = q; k >= 2; --k) {
    const ExLevelTables t = exact_tables(E, k);
    ex_child_sum(t, E.U(k), E.U(k - 1), st);
    if (hipMemcpyAsync(d, E.U(k), (size_t)E.N[k] * 8, hipMemcpyDeviceToDevice, st) != hipSuccess) return GBL_EHIP;
    ex_gemv_t(E.np2[k], (int)E.N[k], 1, -1.0, E.R(k), E.N[k], E.U(k - 1), 1.0, d, st);   // d -= R^T U^(k-1)
    ex_wapply(t, d, 1, E.W(k), st);
    if (E.wkind != 0) ex_gram_solve(t, E.at(E.offGinv[k]), E.W(k), st);   // w = (W W^T)^-1 W d
    const int nj = E.rp * E.np2[k];
    ex_diag_scale(E.B(k), nj, nj, E.W(k), coef + E.np2[k], false, &t, st);
  }
  ex_diag_scale(E.A(1), E.cp, E.cp, E.U(1), coef, false, nullptr, st);
  return hipGetLastError() == hipSuccess ? GBL_OK : GBL_EHIP;
}

// The reconstruction of Theorem 4.15 from normalized coefficients.
int exact_inverse_transform(ExactHier& E, const double* coef, double* u_nodal, hipStream_t st) {
  const int q = E.q;
  ex_diag_scale(E.A(1), E.cp, E.cp, coef, E.U(1), true, nullptr, st);
  for (int k = 2; k <= q; ++k) {
    const ExLevelTables t = exact_tables(E, k);
    const int nj = E.rp * E.np2[k];
    ex_diag_scale(E.B(k), nj, nj, coef + E.np2[k], E.W(k), true, &t, st);
    ex_gemv_t(E.np2[k], (int)E.N[k], 1, 1.0, E.R(k), E.N[k], E.U(k - 1), 0.0, E.U(k), st);
    ex_wtadd(t, E.N[k], E.W(k), 1, E.U(k), st);
  }
  ex_fill(E.nnodes, 0.0, u_nodal, st);
  to_nodal(E, E.U(q), 1, u_nodal, st);
  return hipGetLastError() == hipSuccess ? GBL_OK : GBL_EHIP;
}

// sqrt(u^T A u) with the dense level-q operator; waits for the stream.
int exact_energy_norm(ExactHier& E, const double* u_nodal, double* norm, hipStream_t st) {
  const long Nq = E.N[E.q];
  double* x = E.at(E.offX);
  double* y = E.at(E.offRes);
  double* out = E.at(E.offDot);
  from_nodal(E, u_nodal, x, st);
  ex_gemv((int)Nq, (int)Nq, 1, 1.0, E.A(E.q), Nq, x, 0.0, y, st);   // y = A x
  ex_gemv(1, (int)Nq, 1, 1.0, x, Nq, y, 0.0, out, st);               // x . y
  double h = 0.0;
  if (hipMemcpyAsync(&h, out, 8, hipMemcpyDeviceToHost, st) != hipSuccess || hipStreamSynchronize(st) != hipSuccess)
    return GBL_EHIP;
  *norm = std::sqrt(std::max(h, 0.0));
  return GBL_OK;
}

}  // namespace gbl
