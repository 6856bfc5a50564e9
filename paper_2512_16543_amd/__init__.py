"""WB-arSVD RZF precoding on MI355X (gfx950).

The compute path lives in the HIP library `librzf.so` built from `csrc/`; the
Python module `paper_2512_16543_amd.rzf` is a thin ctypes binding over its C
ABI (see `include/rzf.h`).  `paper_2512_16543_amd.workload` draws the seeded
synthetic channel tracks.  Importing the package does not load the library.
"""
__all__ = ["workload"]
