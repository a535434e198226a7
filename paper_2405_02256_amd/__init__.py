"""MI355X (gfx950) topological integral transforms of weighted cubical complexes.

Critical-point precompute, exact ECT and hybrid transforms (Euler-Fourier,
Euler-Laplace, Euler-Bessel) with their backward pass, behind the C ABI of
include/ect.h.  Import ``paper_2405_02256_amd.api`` for the PyTorch layer;
``workloads`` holds the seeded synthetic inputs.
"""
__all__ = ["api", "workloads", "build"]
