"""Plain FP64 CPU reference ("oracle") for dual-domain convolutional sparse coding.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  The GPU library shares
no code, tables or helpers with it; both sides only share the seeded input
generator in ``synth``.

Every function follows the paper (Affara, Ghanem, Wonka, "Fast Convolutional
Sparse Coding in the Dual Domain") step by step in numpy float64; numpy's FFT
and dense linear solve are used as library primitives.
"""
from .csc import (  # noqa: F401
    pad_filters,
    filter_spectra,
    reconstruct,
    objective,
    regularizer,
    nuclear_norm,
    project_spectral_ball,
    svt,
    objective_grad,
    soft,
    code,
    code_implicit,
    learn,
    learn_dictionary,
    code_loss_grad,
)
