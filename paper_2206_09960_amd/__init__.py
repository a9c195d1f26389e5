"""Power-ψ on MI355X: hand-written HIP (gfx950) kernels behind a C ABI.

Importing the package loads nothing; ``paper_2206_09960_amd.api`` loads the
HIP library (``libpsi.so``) on first use and raises if it is missing.
"""
__all__ = ["api", "build"]
