"""FP64 CPU oracle of the block incomplete LU factorization (arXiv 1908.10169).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
benchmark's CPU-baseline leg may import this package.  It shares no code
with the GPU library (``paper_1908_10169_amd``) and never imports it.
"""
from .oracle import (  # noqa: F401
    Oracle, OracleOptions, cosine_groups, ilu1t_blocks, ilu1t_sets, perturb_invert,
    fgmres_plain, sqmr_plain, load,
)
from .mwm import apply_mwm, mwm, mwm_scalings, symmetric_units  # noqa: F401
