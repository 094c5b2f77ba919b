"""CPU oracle for the nonlinear-optimal-perturbation method (test infrastructure).

This package is a plain, slow, FP64 NumPy/SciPy restatement of the discrete
method of Keuchel & Avila, "Nonlinear optimal perturbation growth in pulsatile
pipe flow" (arXiv 2509.10103): the pseudo-spectral perturbation Navier-Stokes
step for pulsatile pipe flow (Sec. 2 and 2.3), its exact discrete adjoint
(Sec. 2, adjoint equations and compatibility condition), the gradient-ascent
update with the energy-preserving multiplier and backtracking (Sec. 2.2), and
binomial checkpoint counting (Sec. 2.4).

It exists only to check the HIP implementation.  Only ``tests/``, the smoke
entry point and the CPU-baseline leg of the benchmark may import it; the
product path never does, and this package imports nothing from the product.
"""
