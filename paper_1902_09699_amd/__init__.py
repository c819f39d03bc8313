"""MI355X (gfx950) PARSDMM: projections onto intersections of constraint
sets (Peters & Herrmann, arXiv:1902.09699) as hand-written HIP kernels
behind a C ABI (include/sip.h, libsip.so).

Importing the package loads nothing; ``paper_1902_09699_amd.sip`` loads
the built library on first use and raises when it is missing.
"""
__all__ = ["sip", "workloads", "build"]
