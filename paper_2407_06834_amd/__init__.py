"""MI355X-native (gfx950) NFFT nonlocal image denoising (arXiv 2407.06834).

Submodules:
  nld     ctypes binding of the C ABI (libnld.so, HIP kernels)
  synth   seeded synthetic images (the shared input recipe)
  build   hipcc build of libnld.so
"""
