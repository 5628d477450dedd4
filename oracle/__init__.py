"""CPU float64 oracle for the block-Krylov Paraexp exp-action path.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously-correct
reference used to check the HIP path.  Only the test-suite, the smoke check
(`__graft_entry__.smoke`) and the CPU-baseline leg of `bench.py` may import it;
the product library (`paper_1509_04567_amd`) never imports, links or executes
anything here, and this package imports nothing from it.

What it computes (Kooij, Botchev & Geurts, arXiv 1509.04567):
  * the exact solution of the semi-discrete problem u' = L u + g(t)
    (eq. (2.1)) on one Paraexp window, with the source replaced by its
    truncated-SVD, polynomial-in-time approximation U p(t) (eq. (2.3),
    Sec. 2.1), evaluated at the requested output times;
  * the Paraexp shift u = u0 + v with source L u0 + g (eqs. (2.5)-(2.6)), the
    window split of the source (eq. (2.7)) and the superposition sum
    (eq. (2.9));
  * the waveform-relaxation outer loop for Burgers (eqs. (2.10)-(2.18)).

Routes:
  * dense  -- builds L as an n x n matrix and exponentiates the augmented
              matrix [[L, U Pi], [0, K]] by scaling-and-squaring Pade [13/13]
              (Higham 2005), see `expm.py` and `march.py`;
  * spectral -- for constant-coefficient (circulant) L only: the same augmented
              exponential, block-diagonalised by the DFT into one
              (1+q) x (1+q) exponential per Fourier mode.

Modules: operator (S0), compress (S1-S4), expm, march (S5-S8 ground truth),
wr (S10).
"""
from .operator import dense_operator, apply_stencil, stencil_symbol  # noqa: F401
from .compress import compress, fit_time_polynomial, chebyshev_vandermonde, source_samples  # noqa: F401
from .expm import expm, pade_coefficients  # noqa: F401
from .march import (  # noqa: F401
    time_generator,
    solve_window,
    solve_windows_superposed,
    solve_sequential,
    window_model,
)
from .wr import burgers_nonlinear, burgers_jacobian, wr_burgers  # noqa: F401
