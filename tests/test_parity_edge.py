"""GPU parity on edge and degenerate cases: every (I, J) corner of the
instantiated range, ragged N (not a multiple of a wave or a tile), the
minimum N = I, a single bin, a single source, a single microphone, more
sources than microphones, and errors raised through the ABI."""

import numpy as np
import pytest

import oracle
from tests import error_bounds as EB
from tests.gpu_common import (TOL_LOGLIK, TOL_PARAM, check, check_as_params, check_loglik_bins, oracle_as,
                              oracle_as_bounded, oracle_em, params, problem, rel, run_as, to_dev)
from tests.test_parity_em import em_bounds

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ff():
    import torch
    assert torch.cuda.is_available()
    from paper_1805_09498_amd import fastfca
    return fastfca


CASES = [
    (1, 1, 3, 5), (1, 2, 4, 7), (2, 1, 5, 33), (2, 2, 3, 64), (2, 3, 7, 65),
    (3, 1, 4, 100), (3, 3, 1, 3), (3, 5, 9, 1025), (4, 4, 6, 257), (5, 2, 5, 130),
    (6, 4, 4, 300), (6, 7, 3, 2049), (7, 3, 3, 150), (8, 1, 2, 40), (8, 6, 3, 1100),
    (8, 9, 2, 700), (4, 9, 5, 8),
]


@pytest.mark.parametrize("I,J,F,N", CASES)
def test_as_edge_shapes(ff, I, J, F, N):
    p = problem(I, J, F, N, seed=100 * I + 10 * J + F)
    ref = oracle_as_bounded(p, 1)
    for path in (0, 2):
        ctx = run_as(ff, p, 1, path=path)
        check_as_params(params(ff, ctx), ref, tag=f" edge I{I} J{J} F{F} N{N} path {path}")


@pytest.mark.parametrize("I,J,F,N", CASES)
def test_em_edge_shapes(ff, I, J, F, N):
    p = problem(I, J, F, N, seed=100 * I + 10 * J + F)
    S0 = oracle.as_spatial_cov(p.P0, p.lam0)
    v_ref, R_ref = oracle_em(p, S0, 1)
    b = em_bounds(p.x, p.v0, S0)
    for path in (0, 2):
        t = to_dev(p)
        ctx = ff.fca_init(ff.FCA_METHOD_EM, t["x"], t["v0"], t["lam0"], t["P0"])
        ff.fca_set_option(ctx, "path", path)
        ff.fca_em_iterate(ctx, 1)
        v, _, R = params(ff, ctx)
        check(f"em v edge I{I} J{J} F{F} N{N} path {path}", v, v_ref, b["v"], TOL_PARAM)
        check(f"em S edge I{I} J{J} F{F} N{N} path {path}", R, R_ref, b["S"], TOL_PARAM)


@pytest.mark.parametrize("I,J,F,N", [(1, 2, 4, 7), (2, 3, 7, 65), (8, 9, 2, 700), (8, 6, 3, 333), (6, 7, 3, 2049)])
def test_loglik_and_wiener_edge(ff, I, J, F, N):
    p = problem(I, J, F, N, seed=7 * I + J)
    ctx = run_as(ff, p, 2)
    v, lam, P = params(ff, ctx)
    L = ff.fca_loglik(ctx)
    assert abs(L - oracle.loglik_as(p.x, v, lam, P)) <= TOL_LOGLIK * abs(L)
    # on the GPU's own parameters the only error is the evaluation's rounding
    check(f"loglik_bins edge I{I} J{J}", ff.fca_loglik_bins(ctx).cpu().numpy(),
          oracle.loglik_as(p.x, v, lam, P, per_bin=True), EB.loglik_bin_bounds(p.x, v, lam, P))
    s = ff.fca_wiener_separate(ctx).cpu().numpy().astype(np.complex128)
    assert rel(s.sum(axis=0), p.x) <= 1e-5
    check(f"wiener edge I{I} J{J}", s, oracle.wiener_as(p.x, v, lam, P), EB.as_wiener_bounds(p.x, v, lam, P),
          TOL_PARAM, axis=1)


@pytest.mark.parametrize("method", ["as", "em"])
def test_loglik_device_matches_the_host_call(ff, method):
    """fca_loglik_device queues the same sum as fca_loglik into device memory
    without a host round trip: two queued values (after 1 and after 3
    iterations) equal the synchronous calls bitwise; a NULL destination is an
    argument error."""
    import torch
    p = problem(3, 3, 6, 130, seed=55)
    t = to_dev(p)
    m = ff.FCA_METHOD_AS if method == "as" else ff.FCA_METHOD_EM
    iterate = ff.fastfca_as_iterate if method == "as" else ff.fca_em_iterate
    ctx = ff.fca_init(m, t["x"], t["v0"], t["lam0"], t["P0"])
    iterate(ctx, 1)
    a = ff.fca_loglik_device(ctx)
    ref_a = ff.fca_loglik(ctx)
    iterate(ctx, 2)
    b = torch.empty((1,), dtype=torch.float64, device="cuda")
    ff.fca_loglik_device(ctx, b)
    ref_b = ff.fca_loglik(ctx)
    torch.cuda.synchronize()
    assert float(a.item()) == ref_a and float(b.item()) == ref_b
    assert ref_a != ref_b
    assert ff.lib.fca_loglik_device(ctx.handle, None) == ff.FCA_ERR_ARG


@pytest.mark.parametrize("I,J,F,N", [(3, 3, 5, 1100), (6, 4, 7, 300), (2, 2, 1, 70)])
def test_split_streams_same_bits(ff, I, J, F, N):
    """The streaming iterations with the bins split over 2, 3 or 4 streams
    give the same bits as on one stream, the bins being independent (F not a
    multiple of the parts, fewer bins than parts, F = 1), and match the oracle
    after one iteration."""
    p = problem(I, J, F, N, seed=500 + 10 * I + F)
    ref = oracle_as_bounded(p, 1)
    runs = []
    for split in (1, 2, 3, 4):
        t = to_dev(p)
        ctx = ff.fca_init(ff.FCA_METHOD_AS, t["x"], t["v0"], t["lam0"], t["P0"])
        ff.fca_set_option(ctx, "path", 2)
        ff.fca_set_option(ctx, "split_streams", split)
        assert ff.fca_get_option(ctx, "split_streams") == split
        ff.fastfca_as_iterate(ctx, 1)
        check_as_params(params(ff, ctx), ref, tag=f" split {split} I{I}")
        ff.fastfca_as_iterate(ctx, 4)
        runs.append(params(ff, ctx))
    for other in runs[1:]:
        for a, b in zip(runs[0], other):
            assert np.array_equal(a, b)


@pytest.mark.parametrize("I,J,F,N", [(8, 6, 5, 1100), (5, 3, 3, 3000)])
def test_streaming_bin_solve_over_iterations(ff, I, J, F, N):
    """Above I = 4: iterations one call at a time on the streaming path (2
    and 3 tiles per bin, the last ragged; the bins split over two streams;
    the row-parallel per-bin solve) against the oracle after each."""
    p = problem(I, J, F, N, seed=700 + 10 * I + J)
    ctx = run_as(ff, p, 0, path=2)
    for it in range(3):
        ff.fastfca_as_iterate(ctx, 1)
        ref = oracle_as_bounded(p, it + 1)
        check_as_params(params(ff, ctx), ref, tol=TOL_PARAM if it == 0 else None,
                        tag=f" streaming solve I{I} it {it + 1}")


@pytest.mark.parametrize("sums_mfma", [1, 2], ids=["mfma16x16x4", "mfma4x4x1"])
@pytest.mark.parametrize("I,J", [(5, 2), (6, 4), (7, 3), (8, 6)])
def test_streaming_sums_on_matrix_cores(ff, I, J, sums_mfma):
    """Pass B's eq. 23 sums on the matrix cores (both tile forms) at every I
    they serve: two tiles per bin, the second ragged, two iterations one call
    at a time against the oracle."""
    p = problem(I, J, 4, 1100, seed=900 + 10 * I + J)
    ctx = run_as(ff, p, 0, path=2)
    ff.fca_set_option(ctx, "sums_mfma", sums_mfma)
    for it in range(2):
        ff.fastfca_as_iterate(ctx, 1)
        ref = oracle_as_bounded(p, it + 1)
        check_as_params(params(ff, ctx), ref, tol=TOL_PARAM if it == 0 else None,
                        tag=f" sums_mfma {sums_mfma} I{I}J{J} it {it + 1}")


@pytest.mark.parametrize("J", [1, 2, 3])
def test_long_run_ragged_frames_stay_finite(ff, J):
    """Lanes past N (padding) must stay finite over long in-kernel runs: 300
    iterations in one call, N not a multiple of the lane count, all shapes.
    Compared with the oracle on the log-likelihood after the run."""
    p = problem(2, J, 5, 70, seed=31 + J)
    v, lam, P = oracle_as(p, 300)
    L_ref = oracle.loglik_as(p.x, v, lam, P)
    for waves, bpw in ((1, 1), (2, 1), (4, 1), (4, 2)):
        ctx = run_as(ff, p, 300, path=1, waves=waves, bpw=bpw)
        vg, lg, Pg = params(ff, ctx)
        assert np.isfinite(vg).all() and np.isfinite(lg).all() and np.isfinite(Pg).all()
        L = ff.fca_loglik(ctx)
        assert abs(L - L_ref) <= 1e-3 * abs(L_ref), (waves, bpw, L, L_ref)


def test_method_mismatch_and_options(ff):
    p = problem(3, 3, 4, 20, seed=1)
    ctx = run_as(ff, p, 0)
    with pytest.raises(ff.FcaError) as e:
        ff.fca_em_iterate(ctx, 1)
    assert e.value.status == ff.FCA_ERR_STATE
    for key, val in [("K", 0), ("K", 65), ("path", 3), ("waves", 3), ("bins_per_wg", 3), ("autotune", 2),
                     ("split_streams", 0), ("split_streams", 5), ("nope", 1)]:
        with pytest.raises(ff.FcaError) as e:
            ff.fca_set_option(ctx, key, val)
        assert e.value.status == ff.FCA_ERR_ARG
    with pytest.raises(ff.FcaError):
        ff.fastfca_as_iterate(ctx, -1)


def test_nonfinite_input_detected(ff):
    """A NaN in the mixture propagates to the parameters and is reported when
    the opt-in finiteness check is on (it is a host-forced condition: every
    kernel still runs to completion)."""
    p = problem(3, 3, 8, 40, seed=2)
    p.x[3, 5, 1] = np.nan
    t = to_dev(p)
    ctx = ff.fca_init(ff.FCA_METHOD_AS, t["x"], t["v0"], t["lam0"], t["P0"])
    ff.fca_set_option(ctx, "check_finite", 1)
    with pytest.raises(ff.FcaError) as e:
        ff.fastfca_as_iterate(ctx, 1)
    assert e.value.status == ff.FCA_ERR_NONFINITE


@pytest.mark.parametrize("case", ["lambda_zero", "v_negative", "v_nan", "P_zero_column"])
def test_parameter_check_on_the_device(ff, case):
    """With "check_finite", the first iterate call after fca_init (or
    fca_set_params) checks the parameters the model requires on the device
    (host-forced invalid values; every kernel runs to completion):
    non-positive or non-finite v / lambda give FCA_ERR_ARG, a singular P(f)
    FCA_ERR_SINGULAR, and nothing is iterated.  Valid parameters set
    afterwards pass."""
    p = problem(3, 3, 6, 80, seed=3)
    good = to_dev(p)
    if case == "lambda_zero":
        p.lam0[2, 1, 0] = 0.0
    elif case == "v_negative":
        p.v0[4, 7, 2] = -1.0
    elif case == "v_nan":
        p.v0[1, 79, 0] = np.nan
    else:
        p.P0[3, :, 1] = 0.0
    t = to_dev(p)
    ctx = ff.fca_init(ff.FCA_METHOD_AS, t["x"], t["v0"], t["lam0"], t["P0"])
    ff.fca_set_option(ctx, "check_finite", 1)
    with pytest.raises(ff.FcaError) as e:
        ff.fastfca_as_iterate(ctx, 1)
    assert e.value.status == (ff.FCA_ERR_SINGULAR if case == "P_zero_column" else ff.FCA_ERR_ARG), case
    ff.fca_set_params(ctx, good["v0"], good["lam0"], good["P0"])
    ff.fastfca_as_iterate(ctx, 1)


@pytest.mark.parametrize("path", [1, 2], ids=["resident", "streaming"])
def test_zero_bin_reports_a_singular_solve(ff, path):
    """A bin whose mixture is zero at every frame makes the weighted
    covariances of eq. 23 zero: with "check_finite" the iterate call reports
    FCA_ERR_SINGULAR (the kernels still complete; that bin's P is not
    finite), without it the call succeeds and the other bins are updated
    as usual."""
    p = problem(3, 3, 5, 90, seed=4)
    p.x[2] = 0.0
    t = to_dev(p)
    ctx = ff.fca_init(ff.FCA_METHOD_AS, t["x"], t["v0"], t["lam0"], t["P0"])
    ff.fca_set_option(ctx, "path", path)
    ff.fca_set_option(ctx, "check_finite", 1)
    with pytest.raises(ff.FcaError) as e:
        ff.fastfca_as_iterate(ctx, 1)
    assert e.value.status == ff.FCA_ERR_SINGULAR
    other = np.array([0, 1, 3, 4])
    ref = oracle_as_bounded(synth_sub(p, other), 1)
    v, lam, P = params(ff, ctx)
    check_as_params((v[other], lam[other], P[other]), ref, tag=f" zero bin path {path}")


def synth_sub(p, bins):
    from tests.gpu_common import sub_problem
    return sub_problem(p, bins)


@pytest.mark.parametrize("case", ["S_negative", "S_zero", "v_zero"])
def test_em_parameter_check_on_the_device(ff, case):
    """FCA EM contexts: v > 0 and every S_j(f) positive definite, checked on
    the device by the first iterate call with "check_finite"."""
    p = problem(3, 2, 4, 60, seed=5)
    S0 = oracle.as_spatial_cov(p.P0, p.lam0)
    if case == "S_negative":
        S0[2, 1] = -np.eye(3)
    elif case == "S_zero":
        S0[0, 0] = 0.0
    else:
        p.v0[3, 10, 1] = 0.0
    t = to_dev(p, S0)
    ctx = ff.fca_init(ff.FCA_METHOD_EM, t["x"], t["v0"], t["lam0"], t["P0"], t["R0"])
    ff.fca_set_option(ctx, "check_finite", 1)
    with pytest.raises(ff.FcaError) as e:
        ff.fca_em_iterate(ctx, 1)
    assert e.value.status == (ff.FCA_ERR_ARG if case == "v_zero" else ff.FCA_ERR_SINGULAR), case
