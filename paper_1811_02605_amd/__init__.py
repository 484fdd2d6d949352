"""MI355X-native implicit viscous-diffusion PCG solver (HIP, gfx950).

The solve of (I - dt div(nu grad)) x = rhs on a spherical-shell grid by
point-Jacobi preconditioned CG, its single-precision-inner refined form and
its adjoint, behind the C ABI of include/mas.h.  Submodules:

  build      compile the HIP library in-tree
  _abi       ctypes binding of the C ABI (same names)
  solver     torch-facing wrappers and the autograd Function
  workloads  seeded synthetic inputs (no solver arithmetic)

The HIP library is loaded on first use of ``_abi``/``solver``; importing
the package itself does not require it.
"""
__all__ = ["build", "workloads"]
