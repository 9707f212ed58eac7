"""FP64 CPU oracle for FCA and FastFCA-AS (Ito & Nakatani, arXiv 1805.09498).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or
links this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may use it.  It shares no code, header,
helper or constant with the HIP library under ``paper_1805_09498_amd/``.

Every routine is a plain, slow, complex128/float64 transcription of what the
paper defines, vectorised over frequency bins and frames with numpy; the
module ``unrolled`` restates the same steps with plain torch CPU operations so
that torch's autograd gives reference derivatives of the unrolled method, and
``stft`` holds the STFT analysis / overlap-add synthesis of the experiments.
Array layouts (the same as the C ABI of the library so that tests can feed
both the same arrays):

    x    [F][N][I]    complex   observed mixture (the paper's y(n,f))
    v    [F][N][J]    real > 0  source power spectra v_j(n,f)
    R    [F][J][I][I] complex   spatial covariance matrices S_j(f)
    lam  [F][J][I]    real > 0  diagonals of Lambda_j(f)
    P    [F][I][I]    complex   basis-transform matrices P(f), P[f][row][col]

Pinned functions are checked by ``tests/test_oracle_*.py`` against textbook
Gaussian conditioning, scipy densities, finite differences, invariances and
special cases.  Nothing here is "parity unpinned".
"""

from .fca import (
    fca_model_cov,
    fca_estep,
    fca_mstep,
    fca_em_step,
    loglik_fca,
    wiener_fca,
)
from .fastfca_as import (
    as_spatial_cov,
    as_estep,
    as_em_half_step,
    as_fpi_step,
    fastfca_as_step,
    loglik_as,
    wiener_as,
    as_wirtinger_grad,
    as_fpi_dense_vec,
    as_gradient_p_step,
    fastfca_as_step_grad,
    as_newton_p_step,
    as_newton_system,
    newton_directions,
    fastfca_as_step_newton,
    as_em_p_step,
)

__all__ = [
    "fca_model_cov", "fca_estep", "fca_mstep", "fca_em_step", "loglik_fca",
    "wiener_fca", "as_spatial_cov", "as_estep", "as_em_half_step",
    "as_fpi_step", "fastfca_as_step", "loglik_as", "wiener_as",
    "as_wirtinger_grad", "as_fpi_dense_vec", "as_gradient_p_step", "fastfca_as_step_grad",
    "as_newton_p_step", "as_newton_system", "newton_directions", "fastfca_as_step_newton", "as_em_p_step",
]
