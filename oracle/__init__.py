"""Plain, slow FP64 CPU oracle for tiled sCOLA (Leclercq et al. 2020, arXiv:2003.04925).

This package is TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import it.  The product path (the HIP library and its
Python binding) never imports, links or executes anything here, and nothing here
imports the product.

Every function follows the paper's definitions directly, in FP64, with no blocking,
fusion or reordering beyond what the definition states.  Conventions the paper leaves
open are fixed in one place per module and each is named where it is used.

Units: lengths are measured in cells of the Lagrangian lattice (Delta q = 1) and
H0 = 1.  The box side L only enters through the initial power spectrum.

Parity status (what each function is pinned against is in tests/test_oracle_*.py):
  cosmology, LPT, DST/Poisson, deposit/interp chain, tCOLA, sCOLA step, output density
  are pinned by closed forms, invariants or brute force.  The Eisenstein-Hu no-wiggle
  fitting constants are "parity unpinned" (the paper prints no value of P(k)); only the
  k -> 0 limit and the sigma_8 normalisation are pinned.
"""
