"""MI355X-native RKDG + compact subcell WENO (CSWENO) limiter.

Kochi & Ramakrishna, "A compact subcell WENO limiting strategy using
immediate neighbors for Runge-Kutta Discontinuous Galerkin Methods"
(arXiv 1904.11147).  The method runs in hand-written HIP kernels for gfx950
behind the C-ABI library ``libdg.so`` (declared in ``include/dg.h``);
``paper_1904_11147_amd.dg`` is the ctypes binding and
``paper_1904_11147_amd.workloads`` holds the seeded input generators.

Importing the package loads nothing; the binding is imported on use.
"""
__all__ = ["dg", "workloads"]
