"""FP64 CPU oracle for SPED (stochastic parallelizable eigengap dilation).

TEST INFRASTRUCTURE ONLY.  Plain, slow, obviously correct numpy/scipy code in
float64 that restates what the paper defines, so that the HIP library can be
checked against it element by element.  It shares no code, header, table or
constant generator with the GPU library and imports nothing from it.  Only the
test-suite, the smoke check of the entry script and the CPU-baseline leg of the
benchmark may import it; the product path never does.

Modules
-------
laplacian  L = X^T W X from the incidence matrix (Sec. 2), the symmetric
           normalised form (Sec. 4.1), largest-component restriction.
poly       Table 2 transforms, reversal by eq. (reveig), exact p(L)V.
rng        Philox4x32-10 (Salmon et al., SC'11) and Lemire's bounded integers.
walk       The edge-chain estimator of eq. (walk_summand) with Table 1 weights:
           importance-weighted and rejection-sampled forms (Sec. 4.3).
solver     Block subspace iteration / Oja with Householder QR, Rayleigh-Ritz,
           subspace error and principal angles (Sec. 5.2).
kmeans     Lloyd's k-means with k-means++ seeding on the embedding (Sec. 1).
grad       Gradient of p_theta(L) X with respect to theta and X.
order      Node orders for gather locality (Cuthill-McKee, degree, label
           propagation with splitmix64 tie-breaks); the paper fixes none, so
           these follow their published definitions.

Parity status: every function is pinned by a `-m "not gpu"` test in
tests/test_oracle_*.py; none is "parity unpinned".
"""
from . import laplacian, poly, rng, walk, solver, kmeans, grad, order  # noqa: F401
