"""MI355X (gfx950) Polygonal Signed Distance Function: batched PSDF values,
winning obstacle/edge and pose gradients from hand-written HIP kernels behind
a C ABI (include/psdf.h).  ``api`` holds the Python calls; ``inputs`` the
seeded synthetic workloads."""

__all__ = ["api", "inputs"]
