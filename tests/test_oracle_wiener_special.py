"""Pins of the oracle's multichannel Wiener filter (eq. 3) and special cases.

* The estimated images sum to the mixture (the filters sum to identity).
* The filter output is the posterior mean of textbook conditioning, and in
  the transformed basis it is P^-H mu~_j (eq. 16).
* J = 1: the v-update reduces to (1/I) sum_i |(P^H y)_i|^2 / lambda_i.
* J = 2: the generalised eigenvectors of (S_1, S_2) jointly diagonalise any
  FCA pair (Section 4.1), so L1(S) = L2(P_gevd, Lambda_gevd).
"""

import numpy as np
import pytest
import scipy.linalg

import oracle
from paper_1805_09498_amd import synth
from tests.oracle_helpers import cn, rand_hpd, stacked_posterior


@pytest.mark.parametrize("I,J", [(2, 3), (3, 3), (3, 5), (4, 2)])
def test_wiener_sums_to_mixture_and_is_posterior_mean(I, J):
    rng = np.random.default_rng(31 + I * J)
    F, N = 2, 5
    x = cn(rng, (F, N, I))
    v = rng.gamma(0.5, 1.0, size=(F, N, J)) + 0.02
    R = np.stack([[rand_hpd(rng, I) for _ in range(J)] for _ in range(F)])
    s = oracle.wiener_fca(x, v, R)
    assert s.shape == (J, F, N, I)
    np.testing.assert_allclose(s.sum(axis=0), x, atol=1e-12)
    for f in range(F):
        for n in range(N):
            m, _ = stacked_posterior(x[f, n], [v[f, n, j] * R[f, j] for j in range(J)])
            np.testing.assert_allclose(s[:, f, n], m, rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("I,J", [(2, 3), (3, 3), (3, 4)])
def test_wiener_as_in_transformed_basis(I, J):
    p = synth.make_problem(I, J, 3, 7, seed=41 + I * J)
    s = oracle.wiener_as(p.x, p.v0, p.lam0, p.P0)
    np.testing.assert_allclose(s.sum(axis=0), p.x, atol=1e-12)
    _, mut, _ = oracle.as_estep(p.x, p.v0, p.lam0, p.P0)
    PinvH = np.conj(np.swapaxes(np.linalg.inv(p.P0), -1, -2))
    ref = np.einsum("fab,fnjb->jfna", PinvH, mut)
    np.testing.assert_allclose(s, ref, rtol=1e-10, atol=1e-12)


def test_single_source_v_update():
    rng = np.random.default_rng(8)
    F, N, I = 2, 9, 3
    x = cn(rng, (F, N, I))
    v = rng.gamma(0.5, 1.0, size=(F, N, 1)) + 0.1
    P = np.eye(I) + 0.3 * cn(rng, (F, I, I))
    lam = rng.uniform(0.5, 1.5, size=(F, 1, I))
    v_new, _ = oracle.as_em_half_step(x, v, lam, P)
    y = np.einsum("fki,fnk->fni", np.conj(P), x)
    np.testing.assert_allclose(v_new[:, :, 0], (np.abs(y) ** 2 / lam[:, None, 0, :]).mean(axis=2),
                               rtol=1e-12)


@pytest.mark.parametrize("I", [2, 3, 4])
def test_two_sources_generalised_eigenvectors(I):
    rng = np.random.default_rng(90 + I)
    F, N = 2, 6
    S = np.stack([[rand_hpd(rng, I) for _ in range(2)] for _ in range(F)])
    x = cn(rng, (F, N, I))
    v = rng.gamma(0.5, 1.0, size=(F, N, 2)) + 0.05
    P = np.empty((F, I, I), dtype=np.complex128)
    lam = np.empty((F, 2, I))
    for f in range(F):
        w, W = scipy.linalg.eigh(S[f, 0], S[f, 1])    # W^H S1 W = diag(w), W^H S2 W = I
        P[f] = W
        lam[f, 0], lam[f, 1] = w, 1.0
    np.testing.assert_allclose(oracle.as_spatial_cov(P, lam), S, rtol=1e-9, atol=1e-11)
    assert oracle.loglik_as(x, v, lam, P) == pytest.approx(oracle.loglik_fca(x, v, S), rel=1e-10)
