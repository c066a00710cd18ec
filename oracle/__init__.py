"""ORACLE -- test infrastructure only.

A plain, slow, obviously correct FP64 CPU implementation of what hybrid
AB-/BA-GMRES with an unmatched backprojector computes (Bentley, Pasha, Sabate
Landman, Yang, Zhang: "Hybrid ABBA-GMRES for Unmatched Backprojectors in Large
Scale X-Ray CT").  Only the test-suite, the smoke check and the CPU-baseline
leg of the benchmark may import it; the product (the HIP library and its
Python binding) never does, and this package never imports the product.

Modules
  geometry    -- 2D parallel / 3D cone geometry tables in FP64
  operators   -- A (Joseph), A^T (exact transpose, scatter) and B (pixel /
                 voxel driven) over the plain-C definitions in projectors.c
  smallsolve  -- Givens residual, SVD, GCV / DP / fixed / none lambda rules
                 and the regularised projected solve of eq. (12)
  solver      -- hybrid AB- and BA-GMRES (Algorithms 1 and 2)
  learned     -- features, network, loss, Adam, labels and judge of the
                 learned lambda / stop-index rule
"""
from .build import build_oracle, load_oracle  # noqa: F401
