"""GPU parity of the conventional FCA EM baseline (Section 3.3), its
log-likelihood (eq. 5) and Wiener filter (eq. 3) against the FP64 oracle."""

import numpy as np
import pytest

import oracle
from paper_1805_09498_amd import synth
from tests.gpu_common import (TOL_LOGLIK, TOL_PARAM, oracle_em, params, problem, rel, sub_problem,
                              to_dev)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ff():
    import torch
    assert torch.cuda.is_available()
    from paper_1805_09498_amd import fastfca
    return fastfca


def c64(a):
    return a.astype(np.complex64).astype(np.complex128)


def run_em(ff, p, n_iter, R0=None, path=0):
    t = to_dev(p, R0)
    ctx = ff.fca_init(ff.FCA_METHOD_EM, t["x"], t["v0"], t["lam0"], t["P0"], t.get("R0"))
    ff.fca_set_option(ctx, "path", path)
    ff.fca_em_iterate(ctx, n_iter)
    return ctx


@pytest.mark.parametrize("cfg", [dict(I=3, J=3, F=129, N=100, seed=1000),
                                 dict(I=3, J=3, F=513, N=626, seed=2000)], ids=["small", "speech10s"])
@pytest.mark.parametrize("path", [1, 2], ids=["resident", "streaming"])
def test_one_iteration_from_as_start(ff, cfg, path):
    """EM context started at S_j = P^-H diag(lambda_j) P^-1, formed on the device."""
    p = problem(**cfg)
    ctx = run_em(ff, p, 1, path=path)
    v, _, R = params(ff, ctx)
    v_ref, R_ref = oracle_em(p, oracle.as_spatial_cov(p.P0, p.lam0), 1)
    print(rel(v, v_ref), rel(R, R_ref))
    assert rel(v, v_ref) <= TOL_PARAM
    assert rel(R, R_ref) <= TOL_PARAM


def test_one_iteration_given_covariances(ff):
    p = problem(3, 4, 65, 150, seed=21)
    R0 = c64(synth.random_hpd(3, 65, 4, 3))
    ctx = run_em(ff, p, 1, R0=R0)
    v, _, R = params(ff, ctx)
    v_ref, R_ref = oracle_em(p, R0, 1)
    assert rel(v, v_ref) <= TOL_PARAM
    assert rel(R, R_ref) <= TOL_PARAM


@pytest.mark.parametrize("cfg", [dict(I=3, J=3, F=129, N=100, seed=1000),
                                 dict(I=3, J=3, F=513, N=626, seed=2000)], ids=["small", "speech10s"])
@pytest.mark.parametrize("path", [1, 2], ids=["resident", "streaming"])
def test_ten_iterations_loglik(ff, cfg, path):
    p = problem(**cfg)
    ctx = run_em(ff, p, 10, path=path)
    L = ff.fca_loglik(ctx)
    v_ref, R_ref = oracle_em(p, oracle.as_spatial_cov(p.P0, p.lam0), 10)
    L_ref = oracle.loglik_fca(p.x, v_ref, R_ref)
    print(L, L_ref, abs(L - L_ref) / abs(L_ref))
    assert abs(L - L_ref) <= TOL_LOGLIK * abs(L_ref)


def test_same_start_as_fastfca(ff):
    """Both methods start from the same model: equal initial log-likelihood,
    and the first v updates coincide (the AS E-step is the FCA E-step under
    eq. 12)."""
    p = problem(3, 3, 64, 120, seed=22)
    t = to_dev(p)
    a = ff.fca_init(ff.FCA_METHOD_AS, t["x"], t["v0"], t["lam0"], t["P0"])
    e = ff.fca_init(ff.FCA_METHOD_EM, t["x"], t["v0"], t["lam0"], t["P0"])
    assert ff.fca_loglik(a) == pytest.approx(ff.fca_loglik(e), rel=1e-5)
    ff.fastfca_as_iterate(a, 1)
    ff.fca_em_iterate(e, 1)
    va = params(ff, a)[0]
    ve = params(ff, e)[0]
    assert rel(va, ve) <= TOL_PARAM


def test_wiener(ff):
    p = problem(3, 3, 40, 100, seed=23)
    ctx = run_em(ff, p, 2)
    v, _, R = params(ff, ctx)
    s = ff.fca_wiener_separate(ctx).cpu().numpy().astype(np.complex128)
    assert rel(s.sum(axis=0), p.x) <= 1e-5
    assert rel(s, oracle.wiener_fca(p.x, v, R)) <= TOL_PARAM


def test_full_size_long_array_sampled_bins(ff):
    """I=6, J=4, F=1025, N=3750: one FCA EM iteration, sampled bins."""
    p = problem(6, 4, 1025, 3750, seed=3000, spatial="ula", psd="lognormal")
    ctx = run_em(ff, p, 1)
    v, _, R = params(ff, ctx)
    bins = np.array([0, 3, 400, 1024])
    sp = sub_problem(p, bins)
    v_ref, R_ref = oracle_em(sp, oracle.as_spatial_cov(sp.P0, sp.lam0), 1)
    assert rel(v[bins], v_ref) <= TOL_PARAM
    assert rel(R[bins], R_ref) <= TOL_PARAM
