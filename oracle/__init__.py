"""CPU oracle for the tall-skinny and randomized low-rank SVD — TEST INFRASTRUCTURE ONLY.

Plain, slow, double-precision reference implementations written from the
paper (Li, Kluger, Tygert, "Randomized algorithms for distributed computation
of principal component analysis and singular value decomposition").  Only the
test-suite, the smoke check and the benchmark's CPU-baseline leg may import
this package.  The GPU library never imports it, and it imports nothing from
the GPU library: the two share no code, headers, tables or helpers.  The only
common dependency is ``synth`` (seeded input generators, no SVD arithmetic).

Modules
  tssvd_ref   Algorithms 1 and 2 (tall-skinny SVD, single / double orthonormalization)
  lowrank_ref Algorithms 5, 6 and 7 (randomized subspace iteration + direct SVD)
  gram_ref    Algorithms 3 and 4 (Gram-based tall-skinny SVD) and Algorithm 8
  lu_ref      LU with partial pivoting as the tracking basis of Algorithm 5 (Section 3)
  grad_ref    vector-Jacobian product of the low-rank forward (torch float64 autograd)
  checks      orthonormality and spectral-norm error metrics (Table "heads")
  signs       the output sign convention
  philox      Philox4x32-10 counter-based generator + Box-Muller normals

Every public function is pinned by tests under ``tests/`` against values that
do not come from the function itself (printed table values, closed forms,
50-digit brute force, invariants).  Functions without such a pin would say
"parity unpinned"; there are none at present.
"""
from .checks import gram_pairwise, maxentry_ortho, ortho_spec, spectral_residual  # noqa: F401
from .gram_ref import gram_svd_ref, lowrank_gram_ref  # noqa: F401
from .lowrank_ref import lowrank_ref  # noqa: F401
from .lu_ref import lu_basis, lu_factor_gepp  # noqa: F401
from .signs import sign_reference, apply_sign_rule  # noqa: F401
from .tssvd_ref import discard_rule, haar_mix, tssvd_ref, tsqr_ref  # noqa: F401
