"""Independent reference computations used to pin the oracle.

Nothing here calls the oracle's arithmetic: these are textbook definitions
written generically (joint-Gaussian conditioning of a stacked vector, the
expected complete-data log-likelihood, real-valued Gaussian densities).
"""

import numpy as np


def cn(rng, shape):
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / np.sqrt(2.0)


def rand_hpd(rng, I, ridge=0.2):
    A = cn(rng, (I, I))
    return A @ A.conj().T / I + ridge * np.eye(I)


def stacked_posterior(x_n, covs):
    """Posterior of s = [s_1; ...; s_J] given x = sum_j s_j, s_j ~ CN(0, covs[j]).

    Joint-Gaussian conditioning of [s; x] with x = H s, H = [I I ... I]:
        E[s|x]   = Sigma H^H (H Sigma H^H)^-1 x
        Cov[s|x] = Sigma - Sigma H^H (H Sigma H^H)^-1 H Sigma
    Returns per-source means [J][I] and covariances [J][I][I].
    """
    J = len(covs)
    I = covs[0].shape[0]
    Sigma = np.zeros((I * J, I * J), dtype=np.complex128)
    for j in range(J):
        Sigma[j * I:(j + 1) * I, j * I:(j + 1) * I] = covs[j]
    H = np.hstack([np.eye(I)] * J)
    G = Sigma @ H.conj().T @ np.linalg.inv(H @ Sigma @ H.conj().T)
    m = G @ x_n
    V = Sigma - G @ H @ Sigma
    mus = np.stack([m[j * I:(j + 1) * I] for j in range(J)])
    Phis = np.stack([V[j * I:(j + 1) * I, j * I:(j + 1) * I] for j in range(J)])
    return mus, Phis


def q_function(v, S, mus, Phis):
    """Expected complete-data log-likelihood for one bin,

        sum_{n,j} E[ln CN(s_j(n); 0, v_j(n) S_j)]
          = sum_{n,j} -I ln pi - ln det(v S_j) - tr((v S_j)^-1 (mu mu^H + Phi)).

    v [N][J], S [J][I][I], mus [N][J][I], Phis [N][J][I][I].
    """
    N, J = v.shape
    I = S.shape[-1]
    total = 0.0
    for n in range(N):
        for j in range(J):
            Rj = v[n, j] * S[j]
            stat = np.outer(mus[n, j], mus[n, j].conj()) + Phis[n, j]
            total += (-I * np.log(np.pi) - np.log(np.linalg.det(Rj).real)
                      - np.trace(np.linalg.solve(Rj, stat)).real)
    return total


def real_form_logpdf(z, C):
    """ln density of a circular complex Gaussian CN(0, C) evaluated through
    the real 2I-dimensional Gaussian of [Re z; Im z] (scipy)."""
    from scipy.stats import multivariate_normal
    Cr = 0.5 * np.block([[C.real, -C.imag], [C.imag, C.real]])
    return multivariate_normal(mean=np.zeros(2 * len(z)), cov=Cr).logpdf(
        np.concatenate([z.real, z.imag]))
