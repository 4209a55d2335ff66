"""Plain FP64 CPU oracle for the FFT-based bulk magnetization method of
Prigozhin & Sokolovsky, "3D simulation of superconducting magnetic shields and
lenses using the Fast Fourier Transform" (arXiv:1803.01346).

THIS PACKAGE IS TEST INFRASTRUCTURE.  Only the test suite, the smoke check and
the CPU-baseline leg of the benchmark may import it.  The product path (the
HIP library and its Python binding) never imports, calls or links anything
here, and nothing here imports the product.

Everything is float64 / complex128, written for a reader who checks it against
the paper by eye: no blocking, fusion or reordering beyond what the paper's
definitions state.  The FFT is this package's own (radix-2 plus a direct DFT);
numpy.fft / scipy.fft appear only in tests, as independent cross-checks.

Modules
  fft        discrete Fourier transform: direct definition and radix-2 FFT
  grid       uniform node grid on the box D, wavenumbers, smoothing (Sec. 2)
  operators  smoothed spectral curl, Biot-Savart operator Phi (Eqs. 4, 7)
  law        power-law current-voltage relation (Eq. 1)
  units      dimensionless scaling (Eq. 8) and applied-field drives
  geometry   voxelizer: strict-inside node masks of CSG shapes
  rhs        the right-hand side with the exterior iteration (Eq. 5)
  ode        Bogacki-Shampine 3(2) method of lines integrator
  readouts   magnetic moment, region means, probe fields
  brute      brute-force sums: direct convolution kernels, free-space fields
  adjoint    reverse-mode derivatives of the right-hand side (fixed iteration
             count, explicit warm start) and of fixed-step BS23

Parity status: every function is pinned by a CPU test (tests/test_oracle_*.py)
except where its docstring says "parity unpinned".
"""
