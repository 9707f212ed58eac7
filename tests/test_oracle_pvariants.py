"""Pins of the oracle's remaining P updates of Section 4.5:

* Newton's step (as_newton_p_step): its reduced Hessian equals central
  finite differences of the gradient of eq. 21 (pinned elsewhere), the
  resulting step equals the Newton step built from those differences, it
  converges quadratically to a stationary point of L2, and it vanishes
  there;
* EM with P in the M-step (as_em_p_step): every column update maximises a
  generic expected complete-data log-likelihood (built from textbook
  Gaussian conditioning, not from the oracle) over that column, the P
  update never lowers it, and the log-likelihood L2 never decreases over
  whole iterations (a generalised EM algorithm).
"""

import numpy as np
import pytest
from scipy.optimize import minimize

import oracle
from oracle.fastfca_as import newton_directions
from tests.oracle_helpers import cn, q_function, stacked_posterior


def _problem(seed, I, J, N=40, F=2, spread=0.3):
    rng = np.random.default_rng(seed)
    x = cn(rng, (F, N, I))
    v = rng.gamma(0.8, 1.0, size=(F, N, J)) + 0.05
    P = np.eye(I) + spread * cn(rng, (F, I, I))
    lam = rng.uniform(0.3, 2.0, size=(F, J, I))
    return x, v, lam, P


def _df(x, v, lam, P, E):
    """Directional derivative of L2 / N along E from eq. 21: 2 Re tr(g^H E)."""
    N = x.shape[1]
    g = oracle.as_wirtinger_grad(x, v, lam, P[None])[0] / N
    return 2.0 * np.real(np.trace(np.conj(g).T @ E))


@pytest.mark.parametrize("I,J", [(1, 2), (2, 2), (3, 3)])
def test_newton_step_from_finite_differences_of_eq21(I, J):
    x, v, lam, P = _problem(60 + I, I, J, F=1)
    P0 = P[0]
    dirs = [P0 @ U for U in newton_directions(I)]
    h = 1e-6
    H = np.empty((len(dirs), len(dirs)))
    for l, El in enumerate(dirs):
        for k, Ek in enumerate(dirs):
            H[k, l] = (_df(x, v, lam, P0 + h * El, Ek) - _df(x, v, lam, P0 - h * El, Ek)) / (2 * h)
    g = np.array([_df(x, v, lam, P0, E) for E in dirs])
    s = np.linalg.solve(0.5 * (H + H.T), -g)
    expected = P0 + sum(w * E for w, E in zip(s, dirs))
    np.testing.assert_allclose(oracle.as_newton_p_step(x, v, lam, P)[0], expected, rtol=1e-6, atol=1e-7)


@pytest.mark.parametrize("I,J", [(2, 3), (3, 2)])
def test_newton_converges_quadratically(I, J):
    """From near a stationary point of L2 (v, Lambda held), the gradient norm
    falls quadratically; at the limit the step is zero."""
    x, v, lam, P0 = _problem(70 + I, I, J, F=1, N=60)
    N = x.shape[1]

    def unpack(z):
        return (z[:I * I] + 1j * z[I * I:]).reshape(1, I, I)

    def negL(z):
        return -oracle.loglik_as(x, v, lam, unpack(z))

    def negG(z):
        g = oracle.as_wirtinger_grad(x, v, lam, unpack(z))[0].reshape(-1)
        return -np.concatenate([2 * g.real, 2 * g.imag])

    # a stationary point found by an independent maximiser (BFGS), then a
    # small perturbation of it
    z0 = np.concatenate([P0[0].real.reshape(-1), P0[0].imag.reshape(-1)])
    Ps = unpack(minimize(negL, z0, jac=negG, method="BFGS", options=dict(gtol=1e-11, maxiter=5000)).x)
    P = Ps + 1e-3 * cn(np.random.default_rng(1), Ps.shape)
    iterates = [P]
    for _ in range(6):
        iterates.append(oracle.as_newton_p_step(x, v, lam, iterates[-1]))
    lim = iterates[-1]

    def dist(A, B):   # distance up to the columns' phases, which L2 ignores
        ph = np.sum(np.conj(B[0]) * A[0], axis=0)
        return np.linalg.norm(A[0] - B[0] * (ph / np.abs(ph))[None, :])

    e = [dist(Pk, lim) for Pk in iterates]
    assert e[0] > 1e-4
    assert e[1] < 20 * e[0] ** 2 and e[2] < 20 * e[1] ** 2 and e[3] < 1e-12
    np.testing.assert_allclose(oracle.as_newton_p_step(x, v, lam, lim), lim, rtol=1e-10, atol=1e-11)
    assert np.linalg.norm(oracle.as_wirtinger_grad(x, v, lam, lim)) / N < 1e-11
    assert dist(lim, Ps) < 1e-6       # the stationary point BFGS found


def _q_bin(v_new, lam_new, P, mus, Phis):
    """The generic Q-function of one bin at (v_new, S_j = P^-H Lambda_j P^-1)."""
    S = oracle.as_spatial_cov(P[None], lam_new[None])[0]
    return q_function(v_new, S, mus, Phis)


def _posterior(x, v, lam, P):
    S = oracle.as_spatial_cov(P, lam)[0]
    N, J = v.shape[1], v.shape[2]
    out = [stacked_posterior(x[0, n], [v[0, n, j] * S[j] for j in range(J)]) for n in range(N)]
    return np.array([m for m, _ in out]), np.array([c for _, c in out])


@pytest.mark.parametrize("I,J", [(2, 2), (2, 3), (3, 2)])
def test_em_p_last_column_is_a_conditional_maximiser(I, J):
    x, v, lam, P = _problem(80 + 10 * I + J, I, J, F=1, N=12)
    mus, Phis = _posterior(x, v, lam, P)
    v_new, lam_new, P_new = oracle.as_em_p_step(x, v, lam, P)
    base = _q_bin(v_new[0], lam_new[0], P_new[0], mus, Phis)
    rng = np.random.default_rng(3)
    h = 1e-5
    for _ in range(4):
        d = cn(rng, (I,))
        Pp = P_new[0].copy(); Pp[:, I - 1] += h * d
        Pm = P_new[0].copy(); Pm[:, I - 1] -= h * d
        qp = _q_bin(v_new[0], lam_new[0], Pp, mus, Phis)
        qm = _q_bin(v_new[0], lam_new[0], Pm, mus, Phis)
        assert abs(qp - qm) / (2 * h) < 1e-6 * (1 + abs(base))
        assert qp <= base + 1e-9 and qm <= base + 1e-9


@pytest.mark.parametrize("I,J", [(2, 3), (3, 3), (4, 2)])
def test_em_p_step_raises_the_q_function(I, J):
    x, v, lam, P = _problem(90 + I, I, J, F=1, N=15)
    mus, Phis = _posterior(x, v, lam, P)
    v_new, lam_new, P_new = oracle.as_em_p_step(x, v, lam, P)
    q_old = _q_bin(v[0], lam[0], P[0], mus, Phis)
    q_vl = _q_bin(v_new[0], lam_new[0], P[0], mus, Phis)        # after eq. 19-20
    q_all = _q_bin(v_new[0], lam_new[0], P_new[0], mus, Phis)   # after the P update
    assert q_vl >= q_old - 1e-9 * abs(q_old)
    assert q_all >= q_vl - 1e-9 * abs(q_vl)
    assert q_all > q_old


def test_em_p_sweeps_reach_a_stationary_point_of_q():
    I, J = 3, 2
    x, v, lam, P = _problem(97, I, J, F=1, N=15)
    mus, Phis = _posterior(x, v, lam, P)
    v_new, lam_new, P_new = oracle.as_em_p_step(x, v, lam, P, sweeps=5000)
    base = _q_bin(v_new[0], lam_new[0], P_new[0], mus, Phis)
    rng = np.random.default_rng(4)
    h = 1e-5
    for _ in range(5):
        E = cn(rng, (I, I))
        qp = _q_bin(v_new[0], lam_new[0], P_new[0] + h * E, mus, Phis)
        qm = _q_bin(v_new[0], lam_new[0], P_new[0] - h * E, mus, Phis)
        assert abs(qp - qm) / (2 * h) < 1e-6 * (1 + abs(base))


@pytest.mark.parametrize("I,J,seed", [(2, 2, 1), (3, 3, 2), (4, 3, 3), (3, 5, 4)])
def test_em_p_log_likelihood_never_decreases(I, J, seed):
    x, v, lam, P = _problem(seed, I, J, F=3, N=50, spread=0.5)
    L = [oracle.loglik_as(x, v, lam, P)]
    for _ in range(10):
        v, lam, P = oracle.as_em_p_step(x, v, lam, P)
        L.append(oracle.loglik_as(x, v, lam, P))
    for a, b in zip(L, L[1:]):
        assert b >= a - 1e-10 * abs(a), L
    assert L[-1] > L[0]
