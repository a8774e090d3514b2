"""MI355X-native line-by-line opacity cross-sections (gfx950 HIP kernels behind a C ABI).

Submodules:
  synth  - seeded synthetic inputs (line lists, grids, (P, T) sets, request streams)
  xsec   - ctypes binding of the C-ABI library libxsec.so (loaded on first use)
"""
