"""FP64 CPU oracle for ProHD (arXiv 2511.18207) -- TEST INFRASTRUCTURE ONLY.

This package is the plain, slow reference that the HIP path is checked against.
Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import it.  The product path (``paper_2511_18207_amd``) never
imports, links or calls anything here, and this package shares no code with it:
no kernels, headers, helpers or constants.  Inputs come from the seeded
generators in ``synth/`` (which hold none of the method's arithmetic).

Contents
--------
hausdorff   exact Hausdorff distance (paper Eq. (1), Sec. II-A; per direction,
            or both directions from one pass over the distance matrix with
            the plain C loops of nnpass.c), the 1-D
            projected distance ``h_u``/``H_u`` (Sec. II-E.1) and the
            off-axis spread ``delta(u)`` (Eq. (2)).
prohd       the ProHD method: centroid axis (Alg. 1), principal directions
            (Alg. 2), per-direction extreme selection, union and the
            candidate-restricted distance (Alg. 3).
mlp         FP64 forward/backward of the learned-proposal scorer
            (an extension form, not in the paper).

Every function is FP64 on FP32 inputs upcast exactly.  Readings taken where
the paper is silent or inconsistent are listed in the module docstrings.

Parity status: every function here is pinned by ``tests/test_oracle_pins.py``
(brute force, closed forms, invariants, library reductions, hand examples);
``tests/test_oracle_mutations.py`` plants slips in a copy of this package and
checks that the pins catch each one.  None is "parity unpinned".
"""

from .hausdorff import (  # noqa: F401
    directed_hd_bruteforce,
    hd_bruteforce,
    nn_dist,
    nn_both,
    exact_hd,
    directed_hd_1d,
    hd_1d,
    hd_directions,
    delta,
    certificate,
)
from .prohd import (  # noqa: F401
    k_rule,
    centroid_direction,
    principal_directions,
    canonical_sign,
    extreme_indices,
    largest_indices,
    select,
    subset_hd,
    prohd,
    adaptive_alpha,
)
