"""MI355X (gfx950) spectral split-step Pade range march: HIP library + thin binding.

The compute path is libssp.so (csrc/, C ABI in include/ssp.h).  `ssp` is the ctypes
binding; `build` compiles the library in-tree with hipcc.
"""
