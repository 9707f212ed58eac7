"""Equivariance pins of whole iterations of the oracle.

* Scale gauge: (c v_j, Lambda_j / c) and (P D, Lambda |D|^2) describe the same
  model (eq. 12, 15); one FastFCA-AS iteration maps them to the correspondingly
  transformed outputs.
* Mixing: x -> A x with P -> A^-H P (AS) or S_j -> A S_j A^H (FCA) leaves v,
  Lambda unchanged, maps the updated P to A^-H P', and shifts the
  log-likelihood by -2 N F ln|det A| (change of variables in eq. 5 / 14).
Transposition and conjugation mistakes in eq. 16-23 break these.
"""

import numpy as np
import pytest

import oracle
from paper_1805_09498_amd import synth
from tests.oracle_helpers import cn


@pytest.fixture(scope="module")
def prob():
    return synth.make_problem(3, 3, 4, 30, seed=123)


def test_source_scale_gauge(prob):
    c = np.array([0.5, 3.0, 1.7])
    v1, l1, P1 = oracle.fastfca_as_step(prob.x, prob.v0, prob.lam0, prob.P0)
    v2, l2, P2 = oracle.fastfca_as_step(prob.x, prob.v0 * c, prob.lam0 / c[None, :, None], prob.P0)
    np.testing.assert_allclose(v2, v1 * c, rtol=1e-11)
    np.testing.assert_allclose(l2, l1 / c[None, :, None], rtol=1e-11)
    np.testing.assert_allclose(P2, P1, rtol=1e-10, atol=1e-12)


def test_basis_column_gauge(prob):
    rng = np.random.default_rng(2)
    F, I = prob.P0.shape[:2]
    D = cn(rng, (F, I)) + 0.5
    P0D = prob.P0 * D[:, None, :]
    lamD = prob.lam0 * (np.abs(D) ** 2)[:, None, :]
    v1, l1, P1 = oracle.fastfca_as_step(prob.x, prob.v0, prob.lam0, prob.P0)
    v2, l2, P2 = oracle.fastfca_as_step(prob.x, prob.v0, lamD, P0D)
    np.testing.assert_allclose(v2, v1, rtol=1e-10)
    np.testing.assert_allclose(l2, l1 * (np.abs(D) ** 2)[:, None, :], rtol=1e-10)
    np.testing.assert_allclose(P2, P1 * D[:, None, :], rtol=1e-9, atol=1e-11)


def test_mixing_equivariance_as(prob):
    rng = np.random.default_rng(3)
    F, N, I = prob.x.shape
    A = np.eye(I) + 0.5 * cn(rng, (F, I, I))
    AinvH = np.conj(np.swapaxes(np.linalg.inv(A), -1, -2))
    xA = np.einsum("fab,fnb->fna", A, prob.x)
    PA = AinvH @ prob.P0
    v1, l1, P1 = oracle.fastfca_as_step(prob.x, prob.v0, prob.lam0, prob.P0)
    v2, l2, P2 = oracle.fastfca_as_step(xA, prob.v0, prob.lam0, PA)
    np.testing.assert_allclose(v2, v1, rtol=1e-9)
    np.testing.assert_allclose(l2, l1, rtol=1e-9)
    np.testing.assert_allclose(P2, AinvH @ P1, rtol=1e-8, atol=1e-10)
    shift = -2 * N * np.log(np.abs(np.linalg.det(A))).sum()
    assert oracle.loglik_as(xA, v2, l2, P2) == pytest.approx(
        oracle.loglik_as(prob.x, v1, l1, P1) + shift, rel=1e-10)


def test_mixing_equivariance_fca(prob):
    rng = np.random.default_rng(4)
    F, N, I = prob.x.shape
    A = np.eye(I) + 0.5 * cn(rng, (F, I, I))
    R = synth.random_hpd(5, F, 3, I)
    xA = np.einsum("fab,fnb->fna", A, prob.x)
    RA = np.einsum("fab,fjbc,fdc->fjad", A, R, np.conj(A))
    v1, R1 = oracle.fca_em_step(prob.x, prob.v0, R)
    v2, R2 = oracle.fca_em_step(xA, prob.v0, RA)
    np.testing.assert_allclose(v2, v1, rtol=1e-9)
    np.testing.assert_allclose(R2, np.einsum("fab,fjbc,fdc->fjad", A, R1, np.conj(A)),
                               rtol=1e-9, atol=1e-11)
