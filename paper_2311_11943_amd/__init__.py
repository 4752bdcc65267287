"""MI355X-native coded QR (Nguyen, Weissburg & Jeong, arXiv 2311.11943).

The compute path is libcqr.so: hand-written HIP kernels for gfx950 behind the C
ABI declared in include/cqr.h.  `paper_2311_11943_amd.cqr` is its ctypes
binding; importing it raises if the library has not been built
(`python -m paper_2311_11943_amd.build`).
"""
