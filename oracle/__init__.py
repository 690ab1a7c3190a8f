"""FP64 CPU oracle for GP regression with derivatives under D-SKI / D-SKIP.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, links or
executes this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
library (no kernels, headers, tables or helpers); the only inputs both sides
consume come from the seeded generators in ``workloads``.

Each module follows one part of the paper (Eriksson, Dong, Lee, Bindel,
Wilson, "Scaling Gaussian Process Regression with Derivatives", NeurIPS 2018)
and uses a mechanism independent of the GPU design wherever one exists:
sparse CSR interpolation matrices instead of on-the-fly weights, dense
Kronecker mode products instead of FFTs, Householder QR / SVD from LAPACK
instead of Cholesky-QR, explicit Lanczos as well as CG-derived tridiagonals.

Modules:
  rng       counter-based SplitMix64 Rademacher probes (Steele et al. 2014)
  kernels   SE kernel and the exact derivative kernel k^grad (Sec. 2, App. A, App. B)
  interp    uniform grid, Keys cubic and quintic convolution weights (Sec. 3.1)
  dski      D-SKI operator [W; dW] K_UU [W; dW]^T + D, its diagonal and rows (Sec. 3.1, 3.3)
  pivchol   truncated pivoted Cholesky (Sec. 3.3)
  precond   M = D + L L^T, stable QR solve and square-root form (Sec. 3.3)
  krylov    batched PCG, CG->Lanczos tridiagonal, explicit Lanczos (Sec. 2)
  slq       stochastic Lanczos quadrature for log det (Sec. 2)
  mll       log marginal likelihood eq. (1) and its hyper-parameter gradient
  dskip     D-SKIP Hadamard operator with Lanczos compression (Sec. 3.2)
  spline    thin-plate spline kernel under D-SKI, dense K_UU (App. A, Sec. 4.3)
  mlp       the small GELU MLP log-det surrogate (FP64 reference)

Readings of points the paper leaves open are stated in each function's
docstring.  Functions without an independent pin say "parity unpinned".
"""
