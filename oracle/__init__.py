"""FP64 CPU oracle for the accelerated farPCA hot path (arXiv 2506.03859).

TEST INFRASTRUCTURE ONLY. Only the test-suite, the package's smoke check and
the benchmark's CPU-baseline leg may import anything from here; the product
path (the HIP library and its Python binding) never does.

The oracle is plain, slow and written to be checked against the paper by eye:

* ``philox``  - Philox4x64-10 counter-based generator (Salmon et al., SC'11),
                written from its published definition.
* ``omega``   - the random test matrices of Definitions 2.1-2.4 (and the
                fixed-count sparse sign variant mentioned after Definition 2.2),
                materialised densely from the counter-based draws.
* ``farpca``  - Algorithm 1 (farPCA with shifted power iteration) and
                Algorithm 2 (farPCASB) in float64, in the paper's order and
                notation (Y, W, Z, T, E, eigSVD, final two eigendecompositions).

It shares no code with the HIP path; the two agree only through the written
definitions.
"""
from .philox import philox4x64_10, draws32, draws64  # noqa: F401
from .omega import (  # noqa: F401
    SKETCHES, omega_dense, bernoulli_mask, sparse_sign_fixed_mask_signs,
    threshold32, default_p, sketch_scale,
)
from .farpca import (  # noqa: F401
    FarpcaParams, farpca, eig_svd, default_block, default_maxit, projection_svd, truncation_rank,
)
