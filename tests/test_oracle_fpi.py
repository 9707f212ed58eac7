"""Pins of the oracle's fixed-point update of P(f) (Section 4.3.2, eq. 21-23).

* eq. 21 equals a central finite-difference Wirtinger derivative of L2.
* The column-wise update (eq. 23) equals the dense vectorised solve (eq. 22).
* A stationary point of L2 in P, found by an independent quasi-Newton
  maximiser, is left in place by the update, and there p_i^H Q_i p_i = 1.
* I = 1 closed form: p <- 1 / (q conj(p)).
"""

import numpy as np
import pytest
from scipy.optimize import minimize

import oracle
from tests.oracle_helpers import cn


def _problem(seed, I, J, N=30, F=1):
    rng = np.random.default_rng(seed)
    x = cn(rng, (F, N, I))
    v = rng.gamma(0.8, 1.0, size=(F, N, J)) + 0.05
    P = np.eye(I) + 0.3 * cn(rng, (F, I, I))
    lam = rng.uniform(0.3, 2.0, size=(F, J, I))
    return rng, x, v, lam, P


@pytest.mark.parametrize("I,J", [(1, 2), (2, 2), (3, 3), (3, 4)])
def test_wirtinger_gradient_matches_finite_differences(I, J):
    _, x, v, lam, P = _problem(40 + I * J, I, J)
    G = oracle.as_wirtinger_grad(x, v, lam, P)[0]
    h = 1e-6
    for a in range(I):
        for b in range(I):
            E = np.zeros((1, I, I), dtype=np.complex128); E[0, a, b] = 1.0
            d_re = (oracle.loglik_as(x, v, lam, P + h * E) - oracle.loglik_as(x, v, lam, P - h * E)) / (2 * h)
            d_im = (oracle.loglik_as(x, v, lam, P + 1j * h * E)
                    - oracle.loglik_as(x, v, lam, P - 1j * h * E)) / (2 * h)
            # dL/dP* = (dL/dRe + i dL/dIm) / 2 for real L.
            ref = 0.5 * (d_re + 1j * d_im)
            assert abs(G[a, b] - ref) < 1e-5 * (1 + abs(ref))


@pytest.mark.parametrize("I,J", [(1, 3), (2, 2), (2, 3), (3, 3), (3, 2)])
def test_columnwise_update_equals_dense_vec_solve(I, J):
    _, x, v, lam, P = _problem(60 + I * J, I, J, N=12, F=2)
    np.testing.assert_allclose(oracle.as_fpi_step(x, v, lam, P),
                               oracle.as_fpi_dense_vec(x, v, lam, P), rtol=1e-9, atol=1e-11)


@pytest.mark.parametrize("I,J", [(2, 2), (2, 3), (3, 3)])
def test_stationary_point_is_a_fixed_point(I, J):
    _, x, v, lam, P0 = _problem(80 + I * J, I, J, N=40)

    def unpack(z):
        return (z[:I * I] + 1j * z[I * I:]).reshape(1, I, I)

    def negL(z):
        return -oracle.loglik_as(x, v, lam, unpack(z))

    def negG(z):
        g = oracle.as_wirtinger_grad(x, v, lam, unpack(z))[0].reshape(-1)
        # dL/dRe = 2 Re(dL/dP*), dL/dIm = 2 Im(dL/dP*)
        return -np.concatenate([2 * g.real, 2 * g.imag])

    z0 = np.concatenate([P0[0].real.reshape(-1), P0[0].imag.reshape(-1)])
    res = minimize(negL, z0, jac=negG, method="BFGS", options=dict(gtol=1e-11, maxiter=5000))
    Ps = unpack(res.x)
    gnorm = np.abs(oracle.as_wirtinger_grad(x, v, lam, Ps)).max()
    assert gnorm < 1e-7
    Pn = oracle.as_fpi_step(x, v, lam, Ps)
    np.testing.assert_allclose(Pn, Ps, rtol=1e-6, atol=1e-7)
    Q = oracle.fastfca_as.as_weighted_covs(x, v, lam)
    for i in range(I):
        p = Ps[0, :, i]
        assert (p.conj() @ Q[0, i] @ p).real == pytest.approx(1.0, abs=1e-7)


def test_single_microphone_closed_form():
    rng, x, v, lam, P = _problem(7, 1, 3, N=25, F=3)
    Pn = oracle.as_fpi_step(x, v, lam, P)
    d = (v * lam[:, None, :, 0]).sum(axis=2)                  # [F][N]
    q = (np.abs(x[:, :, 0]) ** 2 / d).mean(axis=1)
    np.testing.assert_allclose(Pn[:, 0, 0], 1.0 / (q * np.conj(P[:, 0, 0])), rtol=1e-12)


def test_inner_iterations_reuse_weighted_covariances():
    """K = 2 inner steps equal two K = 1 steps at fixed (v, Lambda)."""
    _, x, v, lam, P = _problem(91, 3, 3, N=20, F=2)
    P1 = oracle.as_fpi_step(x, v, lam, P)
    np.testing.assert_allclose(oracle.as_fpi_step(x, v, lam, P, K=2),
                               oracle.as_fpi_step(x, v, lam, P1), rtol=1e-12)


def test_operation_counts_quoted_in_the_paper():
    """Sections 3.4 and 4.4: (J+N)F inversions and 2JNF multiplications per FCA
    iteration, (I+1)FK inversions per FastFCA-AS iteration."""
    I = J = 3; N = 249; F = 512; K = 1
    assert (J + N) * F == 129024
    assert 2 * J * N * F == 764928
    assert (I + 1) * F * K == 2048
