"""Conventional full-rank spatial covariance analysis (FCA), FP64 oracle.

Test infrastructure only (see the package docstring).  Follows Section 3 of
the paper: the source model (eq. 1-2), the multichannel Wiener filter
(eq. 3), the log-likelihood L1 (eq. 5) and one EM iteration (eq. 6-10).

Readings of the paper used here:
  * M-step order: v_j is updated first with the current S_j (eq. 9), then
    S_j with the new v_j (eq. 10), as the assignments are written in
    sequence.
  * The updated S_j is made exactly Hermitian, (S + S^H)/2, and traces are
    taken as real parts; both only remove rounding.
  * The complex normal is circular: density exp(-z^H C^-1 z)/(pi^I det C).
"""

import numpy as np


def _herm(a):
    """Conjugate transpose over the last two axes."""
    return np.conj(np.swapaxes(a, -1, -2))


def fca_model_cov(v, R):
    """Per-source covariances R_j(n,f) = v_j(n,f) S_j(f)  (eq. 2).

    v [F][N][J], R [F][J][I][I]  ->  [F][N][J][I][I]
    """
    return v[:, :, :, None, None] * R[:, None, :, :, :]


def fca_estep(x, v, R):
    """E-step: posterior mean and covariance of every source image (eq. 6-8).

    mu_j  = R_j (sum_k R_k)^-1 y          (eq. 7)
    Phi_j = R_j - R_j (sum_k R_k)^-1 R_j   (eq. 8)
    Returns mu [F][N][J][I], Phi [F][N][J][I][I].
    """
    Rn = fca_model_cov(v, R)
    C = Rn.sum(axis=2)                               # [F][N][I][I]
    Cinv = np.linalg.inv(C)
    mu = np.einsum("fnjab,fnbc,fnc->fnja", Rn, Cinv, x)
    Phi = Rn - np.einsum("fnjab,fnbc,fnjcd->fnjad", Rn, Cinv, Rn)
    return mu, Phi


def fca_mstep(mu, Phi, R, N):
    """M-step (eq. 9-10) from the posterior statistics.

    v_j <- (1/I) tr(S_j^-1 (mu_j mu_j^H + Phi_j))      (eq. 9, current S_j)
    S_j <- (1/N) sum_n (mu_j mu_j^H + Phi_j) / v_j      (eq. 10, new v_j)
    """
    I = R.shape[-1]
    Rhat = np.einsum("fnja,fnjb->fnjab", mu, np.conj(mu)) + Phi
    Sinv = np.linalg.inv(R)                          # [F][J][I][I]
    v_new = np.real(np.einsum("fjab,fnjba->fnj", Sinv, Rhat)) / I
    R_new = (Rhat / v_new[:, :, :, None, None]).sum(axis=1) / N
    R_new = 0.5 * (R_new + _herm(R_new))
    return v_new, R_new


def fca_em_step(x, v, R):
    """One FCA EM iteration (Section 3.3): E-step then M-step.

    x [F][N][I] complex, v [F][N][J] > 0, R [F][J][I][I] Hermitian PD.
    Returns (v_new, R_new).
    """
    x = np.asarray(x, dtype=np.complex128)
    v = np.asarray(v, dtype=np.float64)
    R = np.asarray(R, dtype=np.complex128)
    mu, Phi = fca_estep(x, v, R)
    return fca_mstep(mu, Phi, R, x.shape[1])


def loglik_fca(x, v, R, per_bin=False):
    """Log-likelihood L1 (eq. 5): sum over (n, f) of ln CN(y; 0, sum_j v_j S_j).

    ln CN(y; 0, C) = -I ln(pi) - ln det C - y^H C^-1 y.
    Returns the total (float) or, with per_bin=True, the [F] per-bin sums.
    """
    x = np.asarray(x, dtype=np.complex128)
    I = x.shape[-1]
    C = fca_model_cov(np.asarray(v, np.float64), np.asarray(R, np.complex128)).sum(axis=2)
    sign, logdet = np.linalg.slogdet(C)
    z = np.linalg.solve(C, x[..., None])[..., 0]
    quad = np.real(np.einsum("fna,fna->fn", np.conj(x), z))
    terms = -I * np.log(np.pi) - logdet - quad       # [F][N]
    per_f = terms.sum(axis=1)
    return per_f if per_bin else float(per_f.sum())


def wiener_fca(x, v, R):
    """Multichannel Wiener filter (eq. 3): x_j = R_j (sum_k R_k)^-1 y.

    Returns the source images in the layout [J][F][N][I].
    """
    x = np.asarray(x, dtype=np.complex128)
    Rn = fca_model_cov(np.asarray(v, np.float64), np.asarray(R, np.complex128))
    C = Rn.sum(axis=2)
    z = np.linalg.solve(C, x[..., None])[..., 0]     # C^-1 y
    s = np.einsum("fnjab,fnb->jfna", Rn, z)
    return s
