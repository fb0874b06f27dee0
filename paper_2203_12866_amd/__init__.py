"""MI355X-native hot path of the COSEnu collective-oscillation solver
(arXiv:2203.12866): RK4 stages of the two-flavour QKE with FD4 + Kreiss-Oliger
or FV + WENO7 advection, as hand-written HIP kernels for gfx950 behind a C ABI.

Submodules:
  cosenu     ctypes binding of include/cosenu.h (Sim, Batch)
  workloads  seeded synthetic parameter sets and states
  build_lib  builds libcosenu.so in-tree with hipcc
"""
__all__ = ["cosenu", "workloads", "build_lib"]
