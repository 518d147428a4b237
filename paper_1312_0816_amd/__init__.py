"""MI355X-native basket geometry navigation.

The data-parallel hot path of "Vectorising the detector geometry to optimize
particle transport": basket-wide shape queries (Contains, Safety,
DistFromInside, DistFromOutside for box, tube and cone), the simple navigator
built on them (section 3, Fig. 1), a batched persistent form and its adjoint,
as hand-written HIP kernels behind the C ABI of ``include/geonav.h``.

Submodules:
  geonav     ctypes binding of libgeonav.so (imports torch)
  workloads  seeded synthetic inputs
  build      hipcc build of libgeonav.so
"""
