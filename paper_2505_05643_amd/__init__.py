"""UltraGauss probe-plane rasterizer for AMD MI355X (gfx950).

Submodules:
  synth     seeded synthetic workloads (no method arithmetic)
  build     in-tree hipcc build of libug.so
  raster    Plan / render / backward binding of the C ABI (needs libug.so)
  autograd  torch.autograd.Function over render + adjoint
  autotune  tile shape / LDS batch / box mode search
  step      hipGraph-captured training step

Importing the package itself loads nothing native; ``raster`` and the
modules above it raise ImportError if libug.so has not been built.
"""

__all__ = ["synth", "build", "raster", "autograd"]
