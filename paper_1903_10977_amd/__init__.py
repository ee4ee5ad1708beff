"""MI355X-native multigrid-preconditioned CG for immersed FEM / IGA.

Layout:
  csrc/       HIP kernels (gfx950) and the C-ABI solver library libimsmg.so
  gen/        host C++ generator of immersed problems, libimsmg_gen.so
  build.py    compiles both libraries in-tree
  generator.py  ctypes binding of the generator
  solver.py     ctypes binding of the solver library (same call names as the C-ABI)
"""
import os

PACKAGE_DIR = os.path.dirname(os.path.abspath(__file__))
LIB_DIR = os.path.join(PACKAGE_DIR, "lib")
ROOT_DIR = os.path.dirname(PACKAGE_DIR)
INCLUDE_DIR = os.path.join(ROOT_DIR, "include")
