"""Pins of the oracle's E-steps (FCA eq. 6-8, FastFCA-AS eq. 15-17) and of the
joint-diagonalisation parameterisation (eq. 11-12) against textbook
joint-Gaussian conditioning of the stacked source vector."""

import numpy as np
import pytest

import oracle
from tests.oracle_helpers import cn, rand_hpd, stacked_posterior


def _as_params(rng, F, I, J):
    P = np.eye(I) + 0.3 * cn(rng, (F, I, I))
    lam = rng.uniform(0.2, 2.0, size=(F, J, I))
    return P, lam


@pytest.mark.parametrize("I,J", [(1, 2), (2, 2), (2, 3), (3, 3), (3, 4), (3, 1)])
def test_fca_estep_equals_stacked_conditioning(I, J):
    rng = np.random.default_rng(10 + 7 * I + J)
    F, N = 2, 4
    x = cn(rng, (F, N, I))
    v = rng.gamma(0.7, 1.0, size=(F, N, J)) + 0.05
    R = np.stack([[rand_hpd(rng, I) for _ in range(J)] for _ in range(F)])
    mu, Phi = oracle.fca_estep(x, v, R)
    for f in range(F):
        for n in range(N):
            m_ref, P_ref = stacked_posterior(x[f, n], [v[f, n, j] * R[f, j] for j in range(J)])
            np.testing.assert_allclose(mu[f, n], m_ref, rtol=1e-10, atol=1e-12)
            np.testing.assert_allclose(Phi[f, n], P_ref, rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("I,J", [(2, 2), (2, 3), (3, 3), (3, 5)])
def test_as_spatial_cov_is_jointly_diagonalised(I, J):
    """eq. 12 solved from eq. 11: P^H S_j P must equal Lambda_j exactly."""
    rng = np.random.default_rng(100 + I * J)
    P, lam = _as_params(rng, 3, I, J)
    S = oracle.as_spatial_cov(P, lam)
    for f in range(3):
        for j in range(J):
            np.testing.assert_allclose(P[f].conj().T @ S[f, j] @ P[f], np.diag(lam[f, j]),
                                       atol=1e-12)
            np.testing.assert_allclose(S[f, j], S[f, j].conj().T, atol=1e-13)


@pytest.mark.parametrize("I,J", [(1, 3), (2, 2), (2, 3), (3, 3), (3, 4)])
def test_as_estep_equals_stacked_conditioning(I, J):
    """With R_j = v_j P^-H Lambda_j P^-1 the diagonal posterior of eq. 16-17 is
    the transformed full posterior: P^H mu_j = mu~_j and P^H Phi_j P =
    diag(phi~_j) with vanishing off-diagonal entries."""
    rng = np.random.default_rng(200 + 7 * I + J)
    F, N = 2, 5
    x = cn(rng, (F, N, I))
    v = rng.gamma(0.5, 1.0, size=(F, N, J)) + 0.01
    P, lam = _as_params(rng, F, I, J)
    S = oracle.as_spatial_cov(P, lam)
    yt, mut, phit = oracle.as_estep(x, v, lam, P)
    for f in range(F):
        PH = P[f].conj().T
        for n in range(N):
            np.testing.assert_allclose(yt[f, n], PH @ x[f, n], atol=1e-12)
            m_ref, Phi_ref = stacked_posterior(x[f, n], [v[f, n, j] * S[f, j] for j in range(J)])
            for j in range(J):
                np.testing.assert_allclose(mut[f, n, j], PH @ m_ref[j], rtol=1e-9, atol=1e-11)
                np.testing.assert_allclose(PH @ Phi_ref[j] @ P[f], np.diag(phit[f, n, j]),
                                           rtol=1e-9, atol=1e-11)


def test_as_estep_single_source_passes_everything():
    """J = 1: the Wiener gain is 1 and the posterior variance is 0."""
    rng = np.random.default_rng(3)
    F, N, I = 2, 6, 3
    x = cn(rng, (F, N, I))
    v = rng.gamma(0.5, 1.0, size=(F, N, 1)) + 0.1
    P, lam = _as_params(rng, F, I, 1)
    yt, mut, phit = oracle.as_estep(x, v, lam, P)
    np.testing.assert_allclose(mut[:, :, 0], yt, atol=1e-12)
    np.testing.assert_allclose(phit, 0.0, atol=1e-12)
