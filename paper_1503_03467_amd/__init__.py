"""MI355X-native gamblet hierarchy and subband solve (HIP kernels behind a C ABI)."""
from .gamblet import (GambletError, GambletSolve, Hierarchy, LIB_PATH, lib, make_opts,  # noqa: F401
                      workspace_bytes)

__all__ = ["GambletError", "GambletSolve", "Hierarchy", "LIB_PATH", "lib", "make_opts", "workspace_bytes"]
