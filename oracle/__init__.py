"""FP64 CPU oracle for randomized CP-ALS on sparse tensors.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link this package: only tests, the smoke check and the benchmark's CPU
baseline leg use it.  It shares no code with the HIP library; the only
inputs it has in common with it come from the seeded generators in
`tensorgen`.

Plain, slow, obviously correct NumPy in float64 (extended precision for the
prefix sums that define sampling boundaries).  Each function cites the
passage of the paper it follows ("Distributed-Memory Randomized Algorithms
for Sparse Tensor CP Decomposition", Bharadwaj, Malik, Murray, Buluc,
Demmel; SPAA 2024).

Readings of points the paper leaves open (all shared with the HIP path):
  * column index of mat(T, j): mode 1 varies fastest among the modes != j,
    matching the Khatri-Rao order U_N (.) ... (.) U_1 of Eq. (3);
  * a sampling row carries weight 1/sqrt(J p), so each draw adds 1/(J p) to
    S^T S; duplicate draws of a column are merged with weight count/(J p);
  * inverse CDF: index(u) = min{ i : u * Z < F(i) } for u in [0, 1); rows
    and subtrees of zero mass are never chosen;
  * the update multiplies by the pseudo-inverse of the exact Gram-Hadamard
    matrix G (Eq. 4 and 5, and step 3 of Section 4);
  * STS-CP conditions the factors in ascending mode order, with
    G_{>k} = G^+ (*) (Hadamard of the Grams of the factors drawn after k);
  * the STS-CP probability of a full draw is l_x / <G^+, G>;
  * pseudo-inverse: eigenvalues <= R * 2^-52 * lambda_max are dropped;
  * zero columns stay zero under renormalisation; zero sampling mass is an
    error.

All functions in this module are pinned by tests under tests/ (closed
forms, brute force over explicit Khatri-Rao products, library routines and
invariants); none is "parity unpinned".
"""
from .cpals import *  # noqa: F401,F403
from .cpals import __all__  # noqa: F401
