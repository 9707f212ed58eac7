"""GPU parity of the P updates other than the fixed point (option
"p_update": 1 gradient, 2 natural gradient with the real option "p_step";
3 Newton's step; 4 EM with P in the M-step) against the oracle
(oracle.fastfca_as_step_grad), on both execution paths, after 1 and 3
iterations, at the parameter tolerance of the fixed-point update and entry
by entry within the summed first-order rounding bounds of the iterations."""

import numpy as np
import pytest
import torch

import oracle
from tests.gpu_common import TOL_PARAM, check, check_as_params, oracle_as_bounded, params, problem, rel, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ff():
    assert torch.cuda.is_available()
    from paper_1805_09498_amd import fastfca
    return fastfca


def run(ff, p, n_iter, p_update, mu, path):
    t = to_dev(p)
    ctx = ff.fca_init(ff.FCA_METHOD_AS, t["x"], t["v0"], t["lam0"], t["P0"])
    ff.fca_set_option(ctx, "path", path)
    ff.fca_set_option(ctx, "p_update", p_update)
    ff.fca_set_option_f64(ctx, "p_step", mu)
    ff.fastfca_as_iterate(ctx, n_iter)
    return ctx


@pytest.mark.parametrize("p_update,mu", [(1, 0.05), (2, 0.1)])
@pytest.mark.parametrize("I,J", [(1, 2), (2, 3), (3, 3), (4, 2), (6, 4)])
def test_gradient_type_steps_match_oracle(ff, p_update, mu, I, J):
    p = problem(I, J, 9, 150, seed=70 + I)
    paths = (0, 2) if (p_update == 1 and I > 4) else (0, 1, 2)
    for n_iter in (1, 3):
        ref = oracle_as_bounded(p, n_iter, p_update=p_update, mu=mu)
        for path in paths:
            ctx = run(ff, p, n_iter, p_update, mu, path)
            check_as_params(params(ff, ctx), ref, tag=f" p_update {p_update} I{I} J{J} it {n_iter} path {path}")
    if p_update == 1 and I > 4:
        with pytest.raises(ff.FcaError):
            run(ff, p, 1, p_update, mu, 1)             # the resident kernels take it up to I = 4


def test_step_options(ff):
    p = problem(2, 2, 3, 40, seed=77)
    t = to_dev(p)
    ctx = ff.fca_init(ff.FCA_METHOD_AS, t["x"], t["v0"], t["lam0"], t["P0"])
    assert ff.fca_get_option(ctx, "p_update") == 0
    assert ff.fca_get_option_f64(ctx, "p_step") == pytest.approx(0.1)
    ff.fca_set_option_f64(ctx, "p_step", 0.25)
    assert ff.fca_get_option_f64(ctx, "p_step") == pytest.approx(0.25)
    for bad in (0.0, -1.0, float("nan"), 1e4):
        with pytest.raises(ff.FcaError):
            ff.fca_set_option_f64(ctx, "p_step", bad)
    with pytest.raises(ff.FcaError):
        ff.fca_set_option(ctx, "p_update", 5)
    with pytest.raises(ff.FcaError):
        ff.fca_set_option_f64(ctx, "nope", 1.0)
    ff.fca_set_option(ctx, "p_update", 2)
    with pytest.raises(ff.FcaError):
        ff.fastfca_as_forward(ctx, 2, 1)             # the recorded run is for the fixed-point step
    em = ff.fca_init(ff.FCA_METHOD_EM, t["x"], t["v0"], t["lam0"], t["P0"])
    with pytest.raises(ff.FcaError):
        ff.fca_set_option(em, "p_update", 1)


@pytest.mark.parametrize("p_update", [3, 4], ids=["newton", "em_with_P"])
@pytest.mark.parametrize("I,J,N", [(1, 2, 150), (2, 3, 150), (3, 3, 1100), (4, 2, 150), (6, 4, 150), (8, 6, 90)])
def test_newton_and_em_p_updates_match_oracle(ff, p_update, I, J, N):
    """Newton's P step (3) and EM with P in the M-step (4), Section 4.5: the
    streaming kernels (the automatic path picks them; forcing the resident
    kernels is refused) against the oracle after 1 and 3 iterations, within
    the per-tensor tolerance and the summed per-bin rounding bounds
    (N = 1100 spans two tiles)."""
    p = problem(I, J, 7, N, seed=170 + 10 * I + J)
    for n_iter in (1, 3):
        ref = oracle_as_bounded(p, n_iter, p_update=p_update)
        ctx = run(ff, p, n_iter, p_update, 0.1, 0)
        assert ff.fca_get_option(ctx, "last_waves") == 0
        # the benchmark spec's tolerance is stated for the fixed-point update; the
        # P of these steps carries its own derived bounds (cond of the Newton
        # system, of H_i and of A)
        check_as_params(params(ff, ctx), ref, tag=f" p_update {p_update} I{I} J{J} N{N} it {n_iter}", tol_P=None)
    with pytest.raises(ff.FcaError):
        run(ff, p, 1, p_update, 0.1, 1)


def test_em_p_update_raises_the_log_likelihood_on_the_gpu(ff):
    """EM with P in the M-step is a generalised EM algorithm: the GPU's
    log-likelihood never decreases over 15 iterations (slack: the FP32
    evaluation, 1e-6 relative)."""
    p = problem(3, 3, 20, 300, seed=190)
    t = to_dev(p)
    ctx = ff.fca_init(ff.FCA_METHOD_AS, t["x"], t["v0"], t["lam0"], t["P0"])
    ff.fca_set_option(ctx, "p_update", 4)
    L = [ff.fca_loglik(ctx)]
    for _ in range(15):
        ff.fastfca_as_iterate(ctx, 1)
        L.append(ff.fca_loglik(ctx))
    for a, b in zip(L, L[1:]):
        assert b >= a - 1e-6 * abs(a), L
    assert L[-1] > L[0]
