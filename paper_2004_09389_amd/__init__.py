"""MI355X-native HDG trace-multigrid solver for one implicit stage of the
linearised rotating shallow-water equations (arXiv:2004.09389 hot path).

The numerics live in libhdg.so (HIP, gfx950) behind the C ABI of
include/hdg.h; `paper_2004_09389_amd.hdg` is its ctypes binding.
"""
