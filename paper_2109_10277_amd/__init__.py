"""MI355X (gfx950) quasi-static PIC slice loop of HiPACE++ (arXiv:2109.10277).

The compute path is libqsp.so (hand-written HIP kernels behind the C ABI in
include/qsp.h); ``paper_2109_10277_amd.qsp`` is its ctypes binding.
"""
__all__ = ["qsp"]
