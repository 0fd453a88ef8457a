"""MI355X-native sampling-based approximate graph pattern counting (arXiv 2405.03488).

Layout:
  csrc/     HIP kernels for gfx950 and the C++ host library behind include/sgpm.h
  sgpm.py   thin ctypes binding with the C-ABI names
  synth/    seeded synthetic graph generators (inputs only)
  build.py  in-tree build of libsgpm.so
"""
