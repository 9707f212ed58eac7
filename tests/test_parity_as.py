"""GPU parity of FastFCA-AS (Section 4.3) against the FP64 oracle, through
the C ABI, on both execution paths (frequency-resident and streaming).

Every comparison asserts the per-tensor spec tolerance and, entry by
entry, the first-order rounding bound of an FP32 run (tests/error_bounds.py,
computed before the run from the oracle's state; for P it scales with the
condition number of each eq. 23 matrix)."""

import numpy as np
import pytest

import oracle
from tests import error_bounds as EB
from tests.gpu_common import (TOL_LOGLIK, TOL_PARAM, as_loglik_bin_bound, check, check_as_params,
                              check_loglik_bins, oracle_as_bounded, params, problem, rel, run_as, sub_problem,
                              to_dev)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ff():
    import torch
    assert torch.cuda.is_available()
    from paper_1805_09498_amd import fastfca
    return fastfca


SMALL = dict(I=3, J=3, F=129, N=100, seed=1000)          # small oracle-scale case
SPEECH = dict(I=3, J=3, F=513, N=626, seed=2000)         # 10 s speech scale
PAPER = dict(I=3, J=3, F=512, N=249, seed=1500)          # the shape of the paper's experiments


@pytest.mark.parametrize("cfg", [SMALL, PAPER, SPEECH], ids=["small", "paper", "speech10s"])
@pytest.mark.parametrize("path", [1, 2], ids=["resident", "streaming"])
def test_one_iteration_params(ff, cfg, path):
    p = problem(**cfg)
    ref = oracle_as_bounded(p, 1)
    ctx = run_as(ff, p, 1, path=path)
    check_as_params(params(ff, ctx), ref, tag=f" {cfg['F']}x{cfg['N']} path {path}")


@pytest.mark.parametrize("cfg,n_iter", [(SMALL, 10), (PAPER, 20), (SPEECH, 10)], ids=["small", "paper", "speech10s"])
@pytest.mark.parametrize("path", [1, 2], ids=["resident", "streaming"])
def test_loglik_after_iterations(ff, cfg, n_iter, path):
    """The log-likelihood after the configuration's iterations (10; the
    paper shape runs its 20), in total and per bin."""
    p = problem(**cfg)
    ctx = run_as(ff, p, n_iter, path=path)
    L = ff.fca_loglik(ctx)
    Lb = ff.fca_loglik_bins(ctx).cpu().numpy()
    ref = oracle_as_bounded(p, n_iter, rho_every=2)
    Lb_ref = oracle.loglik_as(p.x, *ref[:3], per_bin=True)
    L_ref = float(Lb_ref.sum())
    print(cfg, path, L, L_ref, abs(L - L_ref) / abs(L_ref))
    assert abs(L - L_ref) <= TOL_LOGLIK * abs(L_ref)
    assert abs(Lb.sum() - L) <= 1e-9 * abs(L)
    check_loglik_bins(Lb, Lb_ref, as_loglik_bin_bound(p, ref), tag=f" {cfg['F']}x{cfg['N']} {n_iter} iterations path {path}")


def test_loglik_headline_run(ff):
    """The benchmark's job at the 10 s speech shape: 100 iterations, then the
    log-likelihood, against 100 oracle iterations (total and per bin)."""
    p = problem(**SPEECH)
    ctx = run_as(ff, p, 100)
    L = ff.fca_loglik(ctx)
    Lb = ff.fca_loglik_bins(ctx).cpu().numpy()
    ref = oracle_as_bounded(p, 100, rho_every=10)
    Lb_ref = oracle.loglik_as(p.x, *ref[:3], per_bin=True)
    L_ref = float(Lb_ref.sum())
    print("100 iterations", L, L_ref, abs(L - L_ref) / abs(L_ref))
    assert abs(L - L_ref) <= TOL_LOGLIK * abs(L_ref)
    check_loglik_bins(Lb, Lb_ref, as_loglik_bin_bound(p, ref), tag=" speech10s 100 iterations")


def test_loglik_at_initial_point(ff):
    p = problem(**SMALL)
    ctx = run_as(ff, p, 0)
    L = ff.fca_loglik(ctx)
    Lb_ref = oracle.loglik_as(p.x, p.v0, p.lam0, p.P0, per_bin=True)
    assert abs(L - Lb_ref.sum()) <= TOL_LOGLIK * abs(Lb_ref.sum())
    # at the initial point the only error is the evaluation's own rounding
    bound = EB.loglik_bin_bounds(p.x, p.v0, p.lam0, p.P0)
    check("loglik_bins initial point", ff.fca_loglik_bins(ctx).cpu().numpy(), Lb_ref, bound)


@pytest.mark.parametrize("waves,bpw", [(1, 1), (2, 1), (4, 1), (2, 2), (4, 2)])
def test_resident_launch_shapes_agree(ff, waves, bpw):
    p = problem(**SPEECH)          # F = 513: the last workgroup of a 2-bin shape holds one bin
    ref = oracle_as_bounded(p, 1)
    ctx = run_as(ff, p, 1, path=1, waves=waves, bpw=bpw)
    check_as_params(params(ff, ctx), ref, tag=f" w{waves}b{bpw}")


@pytest.mark.parametrize("I,J,N", [(3, 3, 100), (3, 3, 200), (3, 3, 300), (3, 3, 600), (3, 3, 700), (3, 3, 850),
                                   (2, 4, 250), (4, 2, 690)])
def test_resident_exact_slot_counts(ff, I, J, N):
    """The plain step at I <= 4 launches the kernel compiled for the exact
    number of 64-frame slots per lane (4 waves, 2 bins: 128 lanes per bin, so
    N = 100 .. 850 needs 1, 2, 3, 5, 6 and 7 slots).  Where every slot of a
    wave holds frames the wave runs phases A and B without a test per slot
    (both waves at N = 100, 200, 600, 850; one at 300, 700), elsewhere the
    tested form; with F = 9 the last workgroup holds one bin on 4 waves (256
    lanes) and takes the tested form.  Two iterations: the second E-step
    starts from the weights kept by the first iteration's phase B."""
    p = problem(I=I, J=J, F=9, N=N, seed=2100 + N)
    ref = oracle_as_bounded(p, 2)
    ctx = run_as(ff, p, 2, path=1, waves=4, bpw=2)
    check_as_params(params(ff, ctx), ref, tag=f" I{I} J{J} N{N}")


def test_inner_fixed_point_steps(ff):
    p = problem(3, 3, 33, 90, seed=5)
    ref = oracle_as_bounded(p, 1, K=3)
    for path in (1, 2):
        ctx = run_as(ff, p, 1, path=path, K=3)
        check_as_params(params(ff, ctx), ref, tag=f" K3 path {path}")


@pytest.mark.parametrize("I,J", [(4, 3), (6, 4)])
def test_inner_fixed_point_steps_larger_I(ff, I, J):
    """K = 3 at I = 4 (resident and streaming kernels) and I = 6 (streaming
    only: the automatic path picks it, forcing the resident one is refused)."""
    p = problem(I, J, 9, 70, seed=6)
    ref = oracle_as_bounded(p, 1, K=3)
    for path in ((0, 1, 2) if I <= 4 else (0, 2)):
        ctx = run_as(ff, p, 1, path=path, K=3)
        check_as_params(params(ff, ctx), ref, tag=f" K3 I{I} path {path}")
    if I > 4:
        with pytest.raises(ff.FcaError):
            run_as(ff, p, 1, path=1, K=3)


@pytest.mark.parametrize("I,J,N", [(3, 2, 617), (6, 7, 1200)])
def test_ill_conditioned_low_bins_over_iterations(ff, I, J, N):
    """Plane waves in a diffuse field on a uniform array: near DC the weighted
    covariances of eq. 23 reach condition numbers of 1e3 - 1e4.  Parameters
    after 1, 2 and 3 iterations against the oracle, every entry of every
    bin, within the sum of the iterations' first-order rounding bounds
    (each computed from the condition numbers at the oracle's state before
    that iteration; printed)."""
    p = problem(I, J, 9, N, seed=17, spatial="ula")
    ctx = run_as(ff, p, 0)
    for it in range(3):
        ff.fastfca_as_iterate(ctx, 1)
        ref = oracle_as_bounded(p, it + 1)
        print("iteration", it + 1, "largest eq. 23 condition number %.3g" % ref[4])
        # the benchmark spec's tolerance is stated for one iteration; later ones
        # carry the derived bounds only
        check_as_params(params(ff, ctx), ref, tol=TOL_PARAM if it == 0 else None, tag=f" ula I{I} it {it + 1}")


def test_wiener_sums_to_mixture_and_matches_oracle(ff):
    p = problem(**SMALL)
    ctx = run_as(ff, p, 3)
    v, lam, P = params(ff, ctx)
    s = ff.fca_wiener_separate(ctx).cpu().numpy().astype(np.complex128)
    assert rel(s.sum(axis=0), p.x) <= 1e-5
    s_ref = oracle.wiener_as(p.x, v, lam, P)   # oracle on the GPU's own parameters
    check("wiener", s, s_ref, EB.as_wiener_bounds(p.x, v, lam, P), TOL_PARAM, axis=1)


def test_resume_is_bitwise(ff):
    """10 iterations equal 5 + get/set round trip + 5, bit for bit."""
    p = problem(3, 3, 40, 200, seed=11)
    a = run_as(ff, p, 10)
    va, la, Pa = params(ff, a)
    b = run_as(ff, p, 5)
    v5, l5, P5 = ff.fca_get_params(b)
    t = to_dev(p)
    c = ff.fca_init(ff.FCA_METHOD_AS, t["x"], t["v0"], t["lam0"], t["P0"])
    ff.fca_set_params(c, v5, l5, P5)
    ff.fastfca_as_iterate(c, 5)
    vc, lc, Pc = params(ff, c)
    np.testing.assert_array_equal(va, vc)
    np.testing.assert_array_equal(la, lc)
    np.testing.assert_array_equal(Pa, Pc)


def test_deterministic(ff):
    p = problem(3, 3, 40, 300, seed=13)
    outs = [params(ff, run_as(ff, p, 4)) for _ in range(2)]
    for a, b in zip(*outs):
        np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("sums_mfma", [0, 1, 2], ids=["valu", "mfma16x16x4", "mfma4x4x1"])
@pytest.mark.parametrize("I,J,seed,bins", [(8, 6, 3001, [0, 1, 137, 512, 800, 1024]),
                                           (6, 4, 3000, [0, 2, 250, 700, 1024])], ids=["long8x6", "long6x4"])
def test_full_size_long_array_sampled_bins(ff, I, J, seed, bins, sums_mfma):
    """The 60 s workloads (F=1025, N=3750, plane-wave + diffuse covariances,
    sparse log-normal spectra): one iteration on the whole problem in the
    launch configuration the benchmark uses, compared bin by bin on sampled
    bins with the oracle run on those bins alone; pass B's eq. 23 sums on the
    vector units (the default) and on the matrix cores in both tile forms
    (option sums_mfma)."""
    p = problem(I, J, 1025, 3750, seed=seed, spatial="ula", psd="lognormal")
    t = to_dev(p)
    ctx = ff.fca_init(ff.FCA_METHOD_AS, t["x"], t["v0"], t["lam0"], t["P0"])
    ff.fca_set_option(ctx, "sums_mfma", sums_mfma)
    assert ff.fca_get_option(ctx, "sums_mfma") == sums_mfma
    ff.fastfca_as_iterate(ctx, 1)
    v, lam, P = params(ff, ctx)
    bins = np.array(bins)
    ref = oracle_as_bounded(sub_problem(p, bins), 1)
    check_as_params((v[bins], lam[bins], P[bins]), ref, tag=f" long{I}x{J} sampled")
