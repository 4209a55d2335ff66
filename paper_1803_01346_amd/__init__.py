"""MI355X-native right-hand side and integrator of the FFT-based bulk
magnetization method of Prigozhin & Sokolovsky (arXiv:1803.01346).

  scfft      ctypes binding of libscfft.so (HIP kernels for gfx950)
  workloads  seeded synthetic configurations and fields (inputs only)
  build      in-tree build of libscfft.so
"""
