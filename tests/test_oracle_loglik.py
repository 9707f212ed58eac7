"""Pins of the oracle's log-likelihoods L1 (eq. 5) and L2 (eq. 14), and of
EM monotonicity (the EM steps of Sections 3.3 and 4.4.1 never decrease the
likelihood)."""

import numpy as np
import pytest

import oracle
from paper_1805_09498_amd import synth
from tests.oracle_helpers import cn, rand_hpd, real_form_logpdf


@pytest.mark.parametrize("I,J", [(1, 2), (2, 3), (3, 3)])
def test_loglik_terms_equal_real_gaussian_density(I, J):
    rng = np.random.default_rng(5 + I * J)
    F, N = 2, 3
    x = cn(rng, (F, N, I))
    v = rng.gamma(0.5, 1.0, size=(F, N, J)) + 0.05
    R = np.stack([[rand_hpd(rng, I) for _ in range(J)] for _ in range(F)])
    ref = 0.0
    for f in range(F):
        for n in range(N):
            C = sum(v[f, n, j] * R[f, j] for j in range(J))
            ref += real_form_logpdf(x[f, n], C)
    assert oracle.loglik_fca(x, v, R) == pytest.approx(ref, rel=1e-12)
    per_bin = oracle.loglik_fca(x, v, R, per_bin=True)
    assert per_bin.shape == (F,)
    assert per_bin.sum() == pytest.approx(ref, rel=1e-12)


@pytest.mark.parametrize("I,J", [(2, 2), (3, 3), (3, 4)])
def test_loglik_as_equals_density_and_diagonal_form(I, J):
    """L2 evaluated as a density of y equals the real-form scipy density, and
    equals the per-point diagonal form
    -I ln pi + 2 ln|det P| - sum_i ln d_i - sum_i |(P^H y)_i|^2 / d_i."""
    rng = np.random.default_rng(50 + I * J)
    F, N = 2, 4
    x = cn(rng, (F, N, I))
    v = rng.gamma(0.5, 1.0, size=(F, N, J)) + 0.05
    P = np.eye(I) + 0.4 * cn(rng, (F, I, I))
    lam = rng.uniform(0.3, 2.0, size=(F, J, I))
    L = oracle.loglik_as(x, v, lam, P)
    ref = 0.0
    diag_form = 0.0
    for f in range(F):
        Pinv = np.linalg.inv(P[f])
        for n in range(N):
            d = (v[f, n, :, None] * lam[f]).sum(axis=0)
            C = Pinv.conj().T @ np.diag(d) @ Pinv
            ref += real_form_logpdf(x[f, n], C)
            y = P[f].conj().T @ x[f, n]
            diag_form += (-I * np.log(np.pi) + 2 * np.log(abs(np.linalg.det(P[f])))
                          - np.log(d).sum() - (np.abs(y) ** 2 / d).sum())
    assert L == pytest.approx(ref, rel=1e-11)
    assert L == pytest.approx(diag_form, rel=1e-11)


def test_fca_em_is_monotone():
    p = synth.make_problem(3, 3, 6, 40, seed=9)
    R = synth.random_hpd(1, 6, 3, 3)
    v = p.v0
    prev = oracle.loglik_fca(p.x, v, R)
    for _ in range(8):
        v, R = oracle.fca_em_step(p.x, v, R)
        cur = oracle.loglik_fca(p.x, v, R)
        assert cur >= prev - 1e-12 * abs(prev)
        prev = cur


@pytest.mark.parametrize("I,J", [(2, 3), (3, 3), (4, 2)])
def test_as_em_half_step_is_monotone(I, J):
    """The EM half-step on (Lambda, v) never lowers L2 (the fixed-point P step
    carries no such guarantee and is not asserted)."""
    p = synth.make_problem(I, J, 5, 40, seed=19 + I)
    v, lam, P = p.v0, p.lam0, p.P0
    for _ in range(6):
        before = oracle.loglik_as(p.x, v, lam, P)
        v, lam = oracle.as_em_half_step(p.x, v, lam, P)
        after = oracle.loglik_as(p.x, v, lam, P)
        assert after >= before - 1e-12 * abs(before)
        P = oracle.as_fpi_step(p.x, v, lam, P)
