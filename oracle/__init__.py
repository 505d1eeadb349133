"""CPU oracle for data-driven (augmented) GMRES on the 2D FDFD Maxwell operator.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, complex128
implementation written directly from the paper ("Data-driven acceleration of
photonic simulations", Trivedi et al.).  Only the test suite, the smoke check
and the benchmark's CPU-baseline leg may import it; the product path (the HIP
library and its Python binding) never does, and shares no code with it.

Modules
  fdfd      -- stretched-coordinate PML factors and the sparse operator A (Eq. 1)
  gmres     -- restarted / unrestarted GMRES (Eq. 2)
  gmres_aug -- data-driven GMRES (Eq. 3-5 and the supplement's update rule)
  direct    -- dense and sparse direct solves
  pca       -- principal-component basis of solution snapshots
  losses    -- projection and residual losses
  cnn       -- float64 convolutional predictor: forward, backward, Adam
  eim       -- effective-index approximation of the field (the CNN's second input)
  recycle   -- harmonic Ritz vectors of a solve's last cycle carried to the next system
"""
