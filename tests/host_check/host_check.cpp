// Host-side check of the library's C ABI, its host code built with
// AddressSanitizer: every call below takes a path that validates
// its arguments, computes a workspace layout or releases host state without
// reaching a kernel, so it runs on a machine without a GPU.  Any out-of-bounds
// access or use after free on those paths stops the program with a report.
//
// Paths: the options validation and the workspace layout over a grid of
// depths, radii, precisions, block sizes and modes; every call with NULL or
// out-of-range arguments; the profiler's counters; the level-q and
// allocation-free entry points' argument checks; and the build's failure
// paths (the context and its resources released when the device calls fail).
#include <hip/hip_runtime_api.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "gamblet.h"

static int g_fail = 0;
#define EXPECT(cond)                                                           \
  do {                                                                         \
    if (!(cond)) {                                                             \
      std::fprintf(stderr, "host_check: %s:%d: %s\n", __FILE__, __LINE__, #cond); \
      ++g_fail;                                                                \
    }                                                                          \
  } while (0)

int main() {
  EXPECT(gbl_version() == GBL_VERSION);
  EXPECT(gbl_default_opts(nullptr) == GBL_EINVAL);
  gbl_opts o;
  EXPECT(gbl_default_opts(&o) == GBL_OK);
  size_t bytes = 0;
  EXPECT(gbl_workspace_bytes(6, &o, nullptr) == GBL_EINVAL);

  // options and layout grid
  long ok = 0, rejected = 0;
  for (int q = 0; q <= 13; ++q)
    for (int rho = 0; rho <= 6; ++rho)
      for (int rc = 0; rc <= 5; rc += 1)
        for (int prec = 0; prec <= 3; ++prec)
          for (int rhs : {0, 1, 3, 16, 17, 64, 65})
            for (int inner = 0; inner <= 3; ++inner)
              for (int mass = 0; mass <= 4; mass += 2)
                for (double wt : {0.0, 5.0, 1e3}) {
                  gbl_default_opts(&o);
                  o.rho = rho;
                  o.rho_coarse = rc;
                  o.precision = prec;
                  o.max_rhs = rhs;
                  o.inner_kind = inner;
                  o.level_q_mass = mass;
                  o.window_tol = wt;
                  const int st = gbl_workspace_bytes(q, &o, &bytes);
                  if (st == GBL_OK) {
                    ++ok;
                    EXPECT(bytes > 0);
                  } else {
                    ++rejected;
                    EXPECT(st == GBL_EINVAL);
                    EXPECT(std::strlen(gbl_last_error(nullptr)) > 0);
                  }
                }
  for (int q = 0; q <= 9; ++q)
    for (int geom = -1; geom <= 2; ++geom)
      for (int src = -1; src <= 2; ++src)
        for (int prec = 0; prec <= 3; ++prec)
          for (int rhs : {1, 7, 64, 65}) {
            gbl_default_opts(&o);
            o.exact = 1;
            o.geometry = geom;
            o.source = src;
            o.precision = prec;
            o.max_rhs = rhs;
            const int st = gbl_workspace_bytes(q, &o, &bytes);
            EXPECT(st == GBL_OK || st == GBL_EINVAL);
          }
  EXPECT(ok > 0 && rejected > 0);

  // NULL and out-of-range arguments
  gbl_default_opts(&o);
  double dummy[4] = {};
  gbl_ctx* ctx = reinterpret_cast<gbl_ctx*>(0x1);
  EXPECT(gbl_build(nullptr, 6, dummy, &o, dummy, 8, nullptr) == GBL_EINVAL);
  EXPECT(gbl_build(&ctx, 6, nullptr, &o, dummy, 8, nullptr) == GBL_EINVAL && ctx == nullptr);
  EXPECT(gbl_build(&ctx, 6, dummy, &o, nullptr, 8, nullptr) == GBL_EINVAL);
  EXPECT(gbl_build(&ctx, 6, dummy, &o, dummy, 8, nullptr) == GBL_ENOMEM);   // workspace too small
  o.exact = 1;
  o.precision = GBL_FP64;
  EXPECT(gbl_build(&ctx, 6, dummy, &o, dummy, 8, nullptr) == GBL_ENOMEM);
  gbl_default_opts(&o);
  EXPECT(gbl_solve(nullptr, 1, dummy, dummy, nullptr, nullptr) == GBL_EINVAL);
  EXPECT(gbl_adjoint(nullptr, 1, dummy, dummy, dummy, nullptr, nullptr, nullptr, nullptr) == GBL_EINVAL);
  int q3[3] = {6, 7, 1};
  const double* a3[3] = {dummy, dummy, dummy};
  void* w3[3] = {dummy, dummy, dummy};
  size_t b3[3] = {8, 8, 8};
  gbl_ctx* c3[3] = {};
  int s3[3] = {};
  EXPECT(gbl_build_batched(0, q3, a3, &o, w3, b3, c3, s3, nullptr) == GBL_EINVAL);
  EXPECT(gbl_build_batched(3, q3, a3, &o, w3, b3, c3, s3, nullptr) != GBL_OK);
  for (int i = 0; i < 3; ++i) EXPECT(c3[i] == nullptr && s3[i] != GBL_OK);
  int n3[3] = {1, 1, 1};
  const double* g3[3] = {dummy, dummy, dummy};
  double* u3[3] = {dummy, dummy, dummy};
  EXPECT(gbl_solve_batched(0, c3, n3, g3, u3, nullptr, s3, nullptr) == GBL_EINVAL);
  unsigned flags = 0;
  EXPECT(gbl_build_flags(nullptr, &flags) == GBL_EINVAL);
  gbl_level_desc d;
  EXPECT(gbl_level_layout(nullptr, 1, &d) == GBL_EINVAL);
  EXPECT(gbl_transform_size(nullptr, &bytes) == GBL_EINVAL);
  EXPECT(gbl_transform(nullptr, dummy, dummy, nullptr) == GBL_EINVAL);
  EXPECT(gbl_inverse_transform(nullptr, dummy, dummy, nullptr) == GBL_EINVAL);
  EXPECT(gbl_compress(nullptr, dummy, 1, nullptr, nullptr) == GBL_EINVAL);
  EXPECT(gbl_energy_norm(nullptr, dummy, dummy, nullptr) == GBL_EINVAL);
  EXPECT(gbl_compress_noalloc(nullptr, 4, 1, nullptr, nullptr) == GBL_EINVAL);
  EXPECT(gbl_compress_noalloc(dummy, 0, 1, nullptr, nullptr) == GBL_EINVAL);
  EXPECT(gbl_compress_noalloc(dummy, 1L << 40, 1, nullptr, nullptr) == GBL_EINVAL);
  for (int q = 0; q <= 13; ++q)
    for (int r = -1; r <= 5; ++r) {
      gbl_mass_inverse(q, r, nullptr, nullptr);
      gbl_level_q_gamblets(q, r, nullptr, dummy, nullptr);
      gbl_level_q_load(q, r, dummy, dummy, dummy, nullptr);
      gbl_level_q_operator(q, r, nullptr, dummy, dummy, nullptr);
      gbl_level_q_to_nodal(q, r, dummy, dummy, dummy, nullptr);
    }
  EXPECT(gbl_destroy(nullptr) == GBL_OK);
  EXPECT(gbl_last_error(nullptr) != nullptr);

  // On a machine without a GPU every device call fails: the builds' error
  // paths then release the context and its resources.  (Skipped where a
  // device exists: these buffers are host memory.)
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess) ndev = 0;
  if (ndev == 0) {
    for (int exact = 0; exact <= 1; ++exact) {
      gbl_default_opts(&o);
      o.exact = exact;
      if (exact) o.precision = GBL_FP64;
      size_t need = 0;
      EXPECT(gbl_workspace_bytes(4, &o, &need) == GBL_OK);
      std::vector<char> ws(need);
      std::vector<double> a(16 * 16, 1.0);
      gbl_ctx* c = reinterpret_cast<gbl_ctx*>(0x1);
      const int st = gbl_build(&c, 4, a.data(), &o, ws.data(), need, nullptr);
      EXPECT(st != GBL_OK && c == nullptr);
      std::printf("host_check: %s build without a device: status %d (%s)\n", exact ? "exact" : "localized", st,
                  gbl_last_error(nullptr));
    }
  }

  // profiler counters, including out-of-range kernel ids
  EXPECT(gbl_profile_enable(~0u) == GBL_OK);
  EXPECT(gbl_profile_reset() == GBL_OK);
  double ms = 0;
  long launches = 0;
  for (int k = -2; k <= GBL_PROF_NUM_KERNELS + 2; ++k) {
    const int st = gbl_profile_read(k, &ms, &launches);
    EXPECT((k >= 0 && k < GBL_PROF_NUM_KERNELS) ? st == GBL_OK : st == GBL_EINVAL);
  }
  EXPECT(gbl_profile_enable(0) == GBL_OK);

  std::printf("host_check: %ld layouts accepted, %ld rejected, %d failures\n", ok, rejected, g_fail);
  return g_fail ? 1 : 0;
}
