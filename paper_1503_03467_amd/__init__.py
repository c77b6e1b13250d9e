"""MI355X-native gamblet hierarchy and subband solve (HIP kernels behind a C ABI)."""
from .gamblet import (PROF_KERNELS, GambletError, GambletSolve, Hierarchy, LevelQ, LIB_PATH,  # noqa: F401
                      build_batched, compress_noalloc, lib, make_opts, profile_enable, profile_read,
                      profile_reset, solve_batched, workspace_bytes)

__all__ = ["PROF_KERNELS", "GambletError", "GambletSolve", "Hierarchy", "LevelQ", "LIB_PATH", "build_batched",
           "compress_noalloc", "lib", "make_opts", "profile_enable", "profile_read", "profile_reset",
           "solve_batched", "workspace_bytes"]
