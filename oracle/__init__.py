"""Plain, slow, FP64 CPU oracle for the smooth part of the single-layer potential.

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import, call or
execute this package: only the tests, the smoke check and the CPU-baseline leg
of the benchmark use it. It shares no code with the HIP library; the only
common inputs are the seeded arrays produced by `synth`.

What it computes (Exl & Schrefl, "Non-uniform FFT for the finite element
computation of the micromagnetic scalar potential"):

  phi_s(x_i) = 1/(4 pi) * sum_k w_k g_k K_F(x~_i - y~_k),
  K_F(xi)    = Re sum_{l in I_n} c_l(N_s) exp(2 pi i l . xi),

i.e. the smooth part of eq. (approx2) with the kernel replaced by its Fourier
series on the torus (eq. Fapprox, Fcoeff), the surface integral replaced by a
three-point quadrature (eq. naive_gridding) and the order of summation as in
eq. (smooth_phi). Modules:

  geometry   quadrature points/weights/normals, scaling into the torus (Sec. 2.2, 3.1)
  kernel     exponential sum for 1/r (Sec. 3.3), its truncation, the Fourier
             coefficients c_{t,q}(l) of the separable terms (eq. Fcoeff, Sec. 3.3)
  direct     R0: exact 1/(4 pi r) sum; R1: pair sum with K_F; R2: the NDFT
             route of eq. (smooth_phi)
  nufft      R3: the gridding / FFT / deconvolution / NFFT pipeline of
             Sec. 3 step by step (Gaussian window), for stage-wise comparison
  nearfield  the near-field correction of Sec. 3.4 (kernel 1/r - N_s on the
             pairs within eps), exact triangle integrals, the complete
             potential phi_s + phi_NF and the exact-integral reference
  fem        the P1 Dirichlet problem for phi_1 (Sec. 2, 2.1), its normal
             derivative on the boundary triangles, and the complete scalar
             potential phi_1 + phi_2 at every node (Alg. 1)
  integrated the paper's integrated-window gridding (Sec. 3.1, eq. gridding2,
             the matrix A): the window integrated over each triangle, and the
             closed-form Fourier transform of a triangle that pins it

Parity pins live in tests/test_oracle_*.py. Functions without an independent
pin are marked "parity unpinned" in their docstrings.
"""
from . import geometry, kernel, direct, nufft, nearfield, fem, integrated  # noqa: F401
