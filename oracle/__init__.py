"""CPU FP64 oracle for the PNGF pixel-flip hot path.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import, call or
execute anything in this package; only the tests, the smoke check and the
benchmark's CPU-baseline leg use it.  It shares no code with the GPU library
(no kernels, headers, helpers or generated tables); the two only consume the
same seeded input arrays from the ``workloads`` module.

What it computes is the plain definition of what the PNGF path computes:

* ``fdfd``  -- the 2D TM (Ez) finite-difference frequency-domain operator with
  a stretched-coordinate PML, and sparse direct solves of the full system
  (Methods, finite-difference discretization; Supplementary Note 2, the FDFD
  system A e = j).
* ``green`` -- the design-region numerical Green function and the output
  projection, column by column from full-system solves (Results,
  Precomputation: e_opt = B^T A^-1 B j_opt and x_obj = G_obj j + x_inc).
* ``gradient`` -- df/d eps per pixel by the adjoint method on the full
  system (Supplementary Note 5, eq. supp_grad_chainrule).
* ``dbs``   -- direct binary search in which every candidate design is scored
  by re-solving the whole sparse system (Results, Direct binary search
  optimization).  PNGF is exact at the discrete level (Results, Numerical
  Green's functions: no approximation compared to a full-wave simulation), so
  this is the reference result the low-rank GPU path must reproduce.

Pins: every function here is checked by ``tests/test_oracle_*.py`` against
closed forms, exact discrete identities, reciprocity and brute force
(see each function's docstring for which pin covers it).
"""
from .fdfd import (pml_profile, stretch, assemble, rhs, solve, Solver,
                   objective, objective_norms, field, metal_nodes, pec_system,
                   total_operator)
from .green import (green_dd, green_od, output_row, background, pngf_state,
                    equivalent_current, pec_state)
from .dbs import dbs, score_all, DBSResult
from .gradient import gradient

__all__ = ["pml_profile", "stretch", "assemble", "rhs", "solve", "Solver",
           "objective", "objective_norms", "field", "metal_nodes", "pec_system", "total_operator", "green_dd", "green_od", "output_row", "background", "pngf_state", "equivalent_current",
           "pec_state", "dbs",
           "score_all", "DBSResult", "gradient"]
