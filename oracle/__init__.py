"""Plain FP64 CPU oracle for the PCG-ATKM hot path.

TEST INFRASTRUCTURE ONLY. This package is a slow, obviously-correct NumPy/SciPy
implementation of what the GPU library computes. Only the test suite, the smoke
check and the benchmark's CPU-baseline leg may import it. The product path never
does, and this package imports nothing from the GPU package.

Modules (each function cites the passage of the paper it follows):
  grid       uniform grid and Fourier frequencies (Sec. 2.1)
  spectral   Fourier pseudo-spectral d/dx, Laplacian, L_z (Sec. 2.1, eq. "Laplacian")
  symbol     truncated Coulomb-kernel Fourier integral U_k (Sec. 2.2, eq. "FUk")
  dipolar    dipolar potential via ATKM (Sec. 2.2, eqs. "DDI2Cou3D", "U_TrunFour")
  energy     discrete energy, H_phi, mu, inner product (Sec. 2.3)
  pcg        Riemannian PCG, Algorithm 1 (Sec. 2.3)
  interp     spectral interpolation between grids, unit mass, phase fix (Algorithm 2, Sec. 3)
  mlp        forward pass, loss gradient and Adam step of the initial-guess network
             (project addition; BF16 rounding emulated where the library rounds)

Readings of the paper where it is silent or garbled are listed in each module's
docstring where they apply. Every function here has a pin in tests/ that does not
go through this package's own arithmetic, except where marked "parity unpinned".
"""
