"""MI355X (gfx950) FP64 Jacobi3D: over-decomposed sweep with on-device halo exchange.

Implements the data-parallel hot path of Choi, Richards and Kale, "Improving
Scalability with GPU-Aware Asynchronous Tasks" (arXiv 2202.11819): the
Jacobi3D proxy's 7-point update over a grid split into blocks that pack,
exchange and unpack their halo faces every iteration, with kernel fusion and
graph execution, plus a batched and a served form.

Modules:
  j3d        ctypes binding of the C ABI in include/j3d.h (libj3d.so)
  api        Solver / Batch / Pool with torch-owned device memory
  workloads  seeded synthetic inputs
  autotune   tile-shape search for the batched form
  serve      request loop (continuous batching) and its serial baseline
  build      compiles libj3d.so in-tree
"""
