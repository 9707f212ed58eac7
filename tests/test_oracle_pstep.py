"""Pins of the gradient-type P updates of the oracle (as_gradient_p_step):
the step's first-order gain in L2 equals the closed form of a directional
derivative, the natural step is equivariant to mixing (the plain one is
not), both vanish at a stationary point, and the kernels' closed form of
the gradient, (1/N) dL2/dP* = P^-H (1 - Gamma) with Gamma_ki = (P^H Q_i P)_ki,
equals eq. 21."""

import numpy as np
import pytest
from scipy.optimize import minimize

import oracle
from oracle.fastfca_as import as_weighted_covs
from tests.oracle_helpers import cn


def _problem(seed, I, J, N=30, F=2):
    rng = np.random.default_rng(seed)
    x = cn(rng, (F, N, I))
    v = rng.gamma(0.8, 1.0, size=(F, N, J)) + 0.05
    P = np.eye(I) + 0.3 * cn(rng, (F, I, I))
    lam = rng.uniform(0.3, 2.0, size=(F, J, I))
    return x, v, lam, P


@pytest.mark.parametrize("I,J", [(1, 2), (2, 3), (3, 3), (4, 2)])
def test_gradient_closed_form_in_the_basis_of_y(I, J):
    x, v, lam, P = _problem(10 + I, I, J)
    N = x.shape[1]
    g = oracle.as_wirtinger_grad(x, v, lam, P) / N
    Q = as_weighted_covs(x, v, lam)
    Gam = np.stack([np.einsum("fab,fbc,fc->fa", np.conj(np.swapaxes(P, 1, 2)), Q[:, i], P[:, :, i])
                    for i in range(I)], axis=2)               # column i: P^H Q_i p_i = G_i e_i
    alt = np.einsum("fba,fbc->fac", np.conj(np.linalg.inv(P)), np.eye(I) - Gam)
    np.testing.assert_allclose(g, alt, rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("natural", [False, True])
@pytest.mark.parametrize("I,J", [(2, 2), (3, 3)])
def test_first_order_gain(I, J, natural):
    x, v, lam, P = _problem(20 + I, I, J, F=1)
    N = x.shape[1]
    g = oracle.as_wirtinger_grad(x, v, lam, P) / N
    D = (P @ np.conj(np.swapaxes(P, 1, 2)) @ g) if natural else g
    mu = 1e-6
    gain = (oracle.loglik_as(x, v, lam, oracle.as_gradient_p_step(x, v, lam, P, mu, natural))
            - oracle.loglik_as(x, v, lam, P)) / mu
    # dL = 2 Re <dL/dP*, dP> = 2 N Re <g, D>
    expected = 2 * N * np.sum((np.conj(g) * D).real)
    assert expected > 0
    assert abs(gain - expected) <= 1e-4 * expected


def test_natural_step_is_equivariant_and_the_plain_one_is_not():
    I, J = 3, 2
    x, v, lam, P = _problem(31, I, J)
    rng = np.random.default_rng(5)
    A = np.eye(I) + 0.5 * cn(rng, (I, I))
    xA = np.einsum("ab,fnb->fna", A, x)
    PA = np.einsum("ba,fbc->fac", np.conj(np.linalg.inv(A)), P)    # A^-H P
    AinvH = np.conj(np.linalg.inv(A)).T
    for natural, equal in ((True, True), (False, False)):
        lhs = oracle.as_gradient_p_step(xA, v, lam, PA, 0.3, natural)
        rhs = np.einsum("ab,fbc->fac", AinvH, oracle.as_gradient_p_step(x, v, lam, P, 0.3, natural))
        assert np.allclose(lhs, rhs, rtol=1e-10, atol=1e-12) == equal


@pytest.mark.parametrize("natural", [False, True])
def test_steps_vanish_at_a_stationary_point(natural):
    I, J = 2, 3
    x, v, lam, P0 = _problem(41, I, J, N=40, F=1)

    def unpack(z):
        return (z[:I * I] + 1j * z[I * I:]).reshape(1, I, I)

    def negL(z):
        return -oracle.loglik_as(x, v, lam, unpack(z))

    def negG(z):
        g = oracle.as_wirtinger_grad(x, v, lam, unpack(z))[0].reshape(-1)
        return -np.concatenate([2 * g.real, 2 * g.imag])

    z0 = np.concatenate([P0[0].real.reshape(-1), P0[0].imag.reshape(-1)])
    Ps = unpack(minimize(negL, z0, jac=negG, method="BFGS", options=dict(gtol=1e-11, maxiter=5000)).x)
    np.testing.assert_allclose(oracle.as_gradient_p_step(x, v, lam, Ps, 0.5, natural), Ps, rtol=1e-7, atol=1e-8)
