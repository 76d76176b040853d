"""MI355X-native Kronecker-structured payoff-matrix gradients for poker endgames.

Submodules:
  instances - seeded synthetic endgame inputs (no method arithmetic)
  pmx       - ctypes binding of libpmx.so (HIP kernels + C ABI)
  build     - hipcc build of libpmx.so for gfx950
Importing the package has no side effects; ``pmx.lib()`` loads the library.
"""
