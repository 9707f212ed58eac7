"""Pins of the oracle's M-steps: FCA eq. 9-10 and FastFCA-AS eq. 19-20.

* Each update is the conditional maximiser of the expected complete-data
  log-likelihood (the Q-function of eq. 18), checked by central finite
  differences of a generic Q built from textbook posterior moments.
* Under R_j = P^-H Lambda_j P^-1 the AS and FCA v-updates coincide, and the AS
  Lambda-update is the diagonal of P^H R'_j P with R'_j the FCA update.
"""

import numpy as np
import pytest

import oracle
from tests.oracle_helpers import cn, q_function, rand_hpd, stacked_posterior


def _setup(seed, I, J, N=6):
    rng = np.random.default_rng(seed)
    x = cn(rng, (1, N, I))
    v = rng.gamma(0.6, 1.0, size=(1, N, J)) + 0.05
    P = np.eye(I) + 0.3 * cn(rng, (1, I, I))
    lam = rng.uniform(0.3, 2.0, size=(1, J, I))
    return rng, x, v, P, lam


def _posteriors(x, v, S):
    N, J = v.shape[1], v.shape[2]
    mus, Phis = [], []
    for n in range(N):
        m, Ph = stacked_posterior(x[0, n], [v[0, n, j] * S[j] for j in range(J)])
        mus.append(m)
        Phis.append(Ph)
    return np.array(mus), np.array(Phis)


@pytest.mark.parametrize("I,J", [(2, 2), (2, 3), (3, 3), (3, 4)])
def test_fca_mstep_is_conditional_argmax_of_q(I, J):
    rng, x, v, _, _ = _setup(11 * I + J, I, J)
    S = np.stack([rand_hpd(rng, I) for _ in range(J)])
    v_new, S_new = oracle.fca_em_step(x, v, S[None])
    mus, Phis = _posteriors(x, v, S)
    h = 1e-5
    # v-update: stationary in every v_j(n) with the current S (eq. 9).
    base = q_function(v_new[0], S, mus, Phis)
    for n in range(v.shape[1]):
        for j in range(J):
            vp = v_new[0].copy(); vp[n, j] *= 1 + h
            vm = v_new[0].copy(); vm[n, j] *= 1 - h
            qp, qm = q_function(vp, S, mus, Phis), q_function(vm, S, mus, Phis)
            assert abs(qp - qm) / (2 * h) < 1e-6 * (1 + abs(base))
            assert qp <= base + 1e-9 and qm <= base + 1e-9
    # S-update: stationary along Hermitian directions with the new v (eq. 10).
    base = q_function(v_new[0], S_new[0], mus, Phis)
    for j in range(J):
        for _ in range(3):
            E = cn(rng, (I, I)); E = E + E.conj().T
            Sp = S_new[0].copy(); Sp[j] = Sp[j] + h * E
            Sm = S_new[0].copy(); Sm[j] = Sm[j] - h * E
            qp = q_function(v_new[0], Sp, mus, Phis)
            qm = q_function(v_new[0], Sm, mus, Phis)
            assert abs(qp - qm) / (2 * h) < 1e-5 * (1 + abs(base))
            assert qp <= base + 1e-8 and qm <= base + 1e-8


@pytest.mark.parametrize("I,J", [(2, 2), (2, 3), (3, 3), (3, 4), (1, 3)])
def test_as_mstep_is_conditional_argmax_of_q(I, J):
    rng, x, v, P, lam = _setup(300 + 11 * I + J, I, J)
    Pinv = np.linalg.inv(P[0])

    def spatial(lmb):
        return np.stack([Pinv.conj().T @ np.diag(lmb[j]) @ Pinv for j in range(J)])

    v_new, lam_new = oracle.as_em_half_step(x, v, lam, P)
    mus, Phis = _posteriors(x, v, spatial(lam[0]))
    h = 1e-5
    base = q_function(v_new[0], spatial(lam[0]), mus, Phis)     # eq. 19, current Lambda
    for n in range(v.shape[1]):
        for j in range(J):
            vp = v_new[0].copy(); vp[n, j] *= 1 + h
            vm = v_new[0].copy(); vm[n, j] *= 1 - h
            qp = q_function(vp, spatial(lam[0]), mus, Phis)
            qm = q_function(vm, spatial(lam[0]), mus, Phis)
            assert abs(qp - qm) / (2 * h) < 1e-6 * (1 + abs(base))
    base = q_function(v_new[0], spatial(lam_new[0]), mus, Phis)  # eq. 20, new v
    for j in range(J):
        for i in range(I):
            lp = lam_new[0].copy(); lp[j, i] *= 1 + h
            lm = lam_new[0].copy(); lm[j, i] *= 1 - h
            qp = q_function(v_new[0], spatial(lp), mus, Phis)
            qm = q_function(v_new[0], spatial(lm), mus, Phis)
            assert abs(qp - qm) / (2 * h) < 1e-6 * (1 + abs(base))
            assert qp <= base + 1e-9 and qm <= base + 1e-9


@pytest.mark.parametrize("I,J", [(2, 3), (3, 3), (3, 4), (4, 2)])
def test_as_mstep_matches_fca_mstep_componentwise(I, J):
    rng = np.random.default_rng(77 + I * J)
    F, N = 3, 20
    x = cn(rng, (F, N, I))
    v = rng.gamma(0.5, 1.0, size=(F, N, J)) + 0.01
    P = np.eye(I) + 0.3 * cn(rng, (F, I, I))
    lam = rng.uniform(0.3, 2.0, size=(F, J, I))
    S = oracle.as_spatial_cov(P, lam)
    v_as, lam_as = oracle.as_em_half_step(x, v, lam, P)
    v_em, S_em = oracle.fca_em_step(x, v, S)
    np.testing.assert_allclose(v_as, v_em, rtol=1e-10)
    for f in range(F):
        for j in range(J):
            M = P[f].conj().T @ S_em[f, j] @ P[f]
            np.testing.assert_allclose(np.real(np.diag(M)), lam_as[f, j], rtol=1e-10)
