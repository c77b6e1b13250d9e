"""MI355X-native gamblet hierarchy and subband solve (HIP kernels behind a C ABI)."""
from .gamblet import (PROF_KERNELS, GambletError, GambletSolve, Hierarchy, LIB_PATH, lib,  # noqa: F401
                      make_opts, profile_enable, profile_read, profile_reset, workspace_bytes)

__all__ = ["PROF_KERNELS", "GambletError", "GambletSolve", "Hierarchy", "LIB_PATH", "lib", "make_opts",
           "profile_enable", "profile_read", "profile_reset", "workspace_bytes"]
