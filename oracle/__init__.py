"""Plain, slow CPU oracle of the pCMD forward model (test infrastructure).

This package is the reference the GPU path is checked against.  It is test
infrastructure only: the library, its Python binding and every production code
path must never import, call or link it; only the tests, the smoke check and
the CPU-baseline leg of the benchmark use it.

Floating point is FP64 wherever the result is continuous.  Where floating point
decides an integer (the transformed-rejection Poisson sampler) the decision is
taken in IEEE single precision, operation by operation, exactly as the GPU takes
it, so that both sides reach the same integer.

Modules (each function cites the passage of Cook, Conroy, van Dokkum & Speagle,
"Measuring Star-Formation Histories, Distances, and Metallicities with Pixel
Color-Magnitude Diagrams I" (arXiv:1904.00011) it follows):

  rng       Philox4x32-10 counter-based generator (Salmon et al. 2011)
  entries   weighted age x [Fe/H] x mass discretisation (Sec. 2.1, 2.2)
  sampler   per-pixel Poisson star counts, dust split, flux sums (Sec. 2.1)
  psf       periodic PSF convolution (Sec. 2.1)
  noise     sky, shot / magnitude noise, flux -> magnitude (Sec. 2.1)
  hess      Hess diagram and mean colour / magnitude (Sec. 2.5)
  loglike   Poisson and Gaussian binned likelihoods (Sec. 2.5)
  pipeline  the whole forward model and likelihood in the paper's order
  mlp       FP64 reference of the surrogate network (forward and backward)

Parity status of each function is stated in its module header.
"""
