"""CPU oracle for the Sdirt hot path -- TEST INFRASTRUCTURE ONLY.

A plain, slow, float64 NumPy implementation of what the dual-pixel PSF
simulator and the pixel-wise renderer compute, written from the paper
(Sec. 3.1 ray-traced DP PSF simulator, Eq. (1)-(3); Sec. 3.2 pixel-wise
rendering and the MLP, Eq. (4); Supplement S1.1 Eq. (S1), S1.3 local DP PSF
convolution, S1.4 PSF prediction network).  Only the test-suite, the smoke
check and the CPU-baseline leg of the benchmark may import it; the product
path (the HIP library and its Python binding) never does, and this package
imports nothing from the product path.

Modules
  optics   materials, paraxial system matrices, pupils, focus, object points
  pupil    counter-based jitter hash, stratified grid, concentric disk map
  trace    real-ray sequential trace (plane, sphere, even asphere, ideal)
  dp       dual-pixel split: microlens model (Eq. (1)/(2)) and sigmoid response
  psf      binning (box / tent), per-point statistics, normalisation
  render   per-pixel local DP convolution (forward and image adjoint)
  adjoint  finite-difference gradients of the traced PSFs (frozen framing)
  mlp      PSF surrogate network, loss and Adam, float64 and bf16-mirror

Parity status: every function is pinned by a `-m "not gpu"` test in
tests/test_oracle_*.py against a closed form, a printed value of the paper,
a brute-force computation or an invariant.
"""
