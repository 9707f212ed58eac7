"""GPU test of the allocation-free run (fastfca_as_run_noalloc), through the
C ABI: its results against the context path (fca_init + fastfca_as_iterate
+ fca_get_params, and fca_loglik_device) forced to the same launch shape,
bit for bit, on calls in a row on the same device array (each later call
with a smaller problem than the one before), on the frequency-resident and
the streaming kernels."""

import numpy as np
import pytest
import torch

from tests.gpu_common import params, problem, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ff():
    assert torch.cuda.is_available()
    from paper_1805_09498_amd import fastfca
    return fastfca


def context_run(ff, p, n_iter, waves, bpw):
    t = to_dev(p)
    ctx = ff.fca_init(ff.FCA_METHOD_AS, t["x"], t["v0"], t["lam0"], t["P0"])
    ff.fca_set_option(ctx, "autotune", 0)
    if waves == 0:
        ff.fca_set_option(ctx, "path", 2)
        ff.fca_set_option(ctx, "split_streams", 1)
    else:
        ff.fca_set_option(ctx, "path", 1)
        ff.fca_set_option(ctx, "waves", waves)
        ff.fca_set_option(ctx, "bins_per_wg", bpw)
    ff.fastfca_as_iterate(ctx, n_iter)
    L = ff.fca_loglik_device(ctx)
    v, lam, P = params(ff, ctx)
    assert ff.fca_get_option(ctx, "last_waves") == waves
    return v, lam, P, float(L.item())


def noalloc_run(ff, p, n_iter):
    t = to_dev(p)
    v, lam, P = t["v0"].clone(), t["lam0"].clone(), t["P0"].clone()
    L = torch.full((1,), np.nan, dtype=torch.float64, device="cuda")
    ff.fastfca_as_run_noalloc(t["x"], v, lam, P, n_iter, L)
    torch.cuda.synchronize()
    return (v.cpu().numpy().astype(np.float64), lam.cpu().numpy().astype(np.float64),
            P.cpu().numpy().astype(np.complex128), float(L.item()))


# (I, J, F, N, iterations, launch shape the entry point picks): calls in a
# row, each problem smaller than the previous one
CALLS = [
    (3, 3, 40, 3500, 3, 0),     # streaming kernels (N beyond the resident kernels)
    (3, 3, 33, 300, 5, 4),      # resident, 4 waves, 2 bins per workgroup, odd F
    (2, 2, 6, 70, 4, 4),        # smaller again, ragged N
]


def test_noalloc_equals_context_path_on_consecutive_calls(ff):
    for I, J, F, N, T, waves in CALLS:
        p = problem(I, J, F, N, seed=900 + I + F)
        got = noalloc_run(ff, p, T)
        ref = context_run(ff, p, T, waves, 2 if waves else 0)
        print("noalloc", (I, J, F, N, T), "loglik", got[3], ref[3])
        for a, b in zip(got[:3], ref[:3]):
            np.testing.assert_array_equal(a, b)
        assert got[3] == ref[3]


def test_noalloc_twice_in_a_row_same_results(ff):
    """The array keeps the previous call's contents: a second identical call
    after a larger one gives the same bits as the first."""
    big = problem(3, 3, 40, 3500, seed=901)
    small = problem(2, 3, 9, 130, seed=902)
    a = noalloc_run(ff, small, 3)
    noalloc_run(ff, big, 2)
    b = noalloc_run(ff, small, 3)
    for x, y in zip(a[:3], b[:3]):
        np.testing.assert_array_equal(x, y)
    assert a[3] == b[3]


def test_noalloc_rejects_a_problem_beyond_its_array(ff):
    p = problem(8, 6, 2, 16, seed=903)
    t = to_dev(p)
    F, N = 1500, 4000                 # 4 (2I + J) F ceil64(N) bytes > 64 MiB
    st = ff.lib.fastfca_as_run_noalloc(F, N, 8, 6, t["x"].data_ptr(), t["v0"].data_ptr(), t["lam0"].data_ptr(),
                                       t["P0"].data_ptr(), 1, None, None)
    assert st == ff.FCA_ERR_ARG
    assert "working storage" in ff.fca_last_error()
