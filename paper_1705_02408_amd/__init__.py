"""MI355X-native wavefront multiobjective perception-aware search (MPAP).

Submodules:
  synth  seeded synthetic workloads (no method arithmetic)
  mpap   ctypes binding of libmpap.so (HIP kernels for gfx950)
  build  hipcc build of libmpap.so
"""
