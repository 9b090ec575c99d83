"""Plain FP64 CPU oracle of sFFT-DT (arXiv 1407.8315) — TEST INFRASTRUCTURE.

This package exists to check the GPU path, never to stand in for it.  Only
tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may import it;
the product package (paper_1407_8315_amd) never does, and this package
imports nothing from the product.  The two share no code: the only common
module is sftgen, which draws seeded inputs and holds none of the method's
arithmetic.  Random shifts drawn by the GPU plan reach the oracle as data.

Contents
  sfft.py   syndromes, locator, grid check, amplitudes, judge, exact and
            general drivers, vote, pruning, Subspace Pursuit, metrics
  roots.py  closed-form roots for a <= 4 (the paper's Appendix, corrected)
  iterative.py  iterative sFFT-DT (Alg. 1): fold, SubFreq, SynDec, T
  mlp.py    FP64 reference network of the learned order predictor
            (forward, backward, features)

Pins (tests/test_oracle_*.py, all CPU): brute-force DFT and alias sums on
small N, the DFT shift property, the a = 1 closed form, exact recovery of
forced collisions a = 1..4 (adjacent slots and wrap-around included),
uniqueness by exhaustive search over every on-grid support for small d,
closed-form roots against an independent eigenvalue root finder, flags for
a > L, noise-free CS = syndrome decoding, SP exact recovery, finite-difference
gradients of the reference network, and the paper's printed Theorem-2 figure.
Iterative oracle (tests/test_oracle_iterative.py): folds and SubFreq against
brute-force alias sums, the Fig. 1 toy, a support-only simulation of Alg. 1,
a bin that only T brings to its decode, and the cost statement of Sec. II-F.
"""
from .sfft import (  # noqa: F401
    Result,
    Taus,
    amplitudes,
    bin_energy,
    candidate_errors,
    cs_bin,
    decode_bin,
    default_taus,
    hankel,
    hankel_singular_values,
    locator,
    noise_floor,
    rank_order,
    relative_l2,
    snr_db,
    roots_to_grid,
    sfft_exact,
    sfft_general,
    sfft_unknown_k,
    subspace_pursuit,
    support_recovery,
    syndromes,
    try_orders,
    vandermonde,
    vote,
)
from .roots import poly_roots  # noqa: F401
