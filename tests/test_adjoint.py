"""GPU tests of the reverse-mode derivatives of unrolled FastFCA-AS
(fastfca_as_forward / fastfca_as_backward and the torch.autograd.Function
on top), against the FP64 PyTorch oracle's autograd (oracle/unrolled.py,
itself pinned to finite differences).

Tolerance (relative Frobenius error, for each gradient tensor on its own and
for each bin of it): grad_tol(p, T) = (T + 1) kappa gamma(c), derived
before the runs from an FP32 error model:

* each of the T iterations' adjoints, and the Wiener filter's, is one chain
  of at most c = 16 I + 8 J + 2 ceil(log2 N) + 32 roundings per value (the
  per-point adjoint arithmetic, the per-bin sums over the frames and the
  per-bin solves), i.e. a relative error gamma(c) of its own;
* the per-bin solves with the eq. 23 matrices (and the forward states they
  use, which carry the same order of error) amplify relative errors by at
  most kappa, the largest condition number of those matrices along the
  oracle's trajectory (computed here, typically 5 - 13);
* the T + 1 contributions add (first order).
"""

import math

import numpy as np
import pytest
import torch

from oracle import unrolled as U
from paper_1805_09498_amd import synth
from tests import error_bounds as EB
from tests.gpu_common import check, oracle_as_bounded, problem, rel, to_dev

pytestmark = pytest.mark.gpu


def grad_tol(p, n_iter):
    F, N, I = p.x.shape
    J = p.v0.shape[2]
    kmax = oracle_as_bounded(p, max(n_iter, 1))[4]
    c = 16 * I + 8 * J + 2 * math.ceil(math.log2(max(N, 2))) + 32
    return (n_iter + 1) * kmax * EB.gamma(c)


def check_grads(tag, grads, refs, tol):
    for name, g, r in zip(("x", "v0", "lam0", "P0"), grads, refs):
        check(f"grad {name} {tag}", g, r, tol=tol, bin_tol=tol)


@pytest.fixture(scope="module")
def ff():
    assert torch.cuda.is_available()
    from paper_1805_09498_amd import fastfca
    return fastfca


def grad_out_for(p, seed):
    rng = np.random.default_rng(seed)
    F, N, I = p.x.shape
    J = p.v0.shape[2]
    g = (rng.standard_normal((J, F, N, I)) + 1j * rng.standard_normal((J, F, N, I))).astype(np.complex64)
    return g.astype(np.complex128)


def run_gpu(ff, p, n_iter, every, g, path=0):
    t = to_dev(p)
    ctx = ff.fca_init(ff.FCA_METHOD_AS, t["x"], t["v0"], t["lam0"], t["P0"])
    ff.fca_set_option(ctx, "path", path)
    out = ff.fastfca_as_forward(ctx, n_iter, every)
    grads = ff.fastfca_as_backward(ctx, torch.from_numpy(g.astype(np.complex64)).cuda())
    torch.cuda.synchronize()
    return ctx, out.cpu().numpy(), [a.cpu().numpy() for a in grads]


def reference(p, n_iter, g):
    _, s_hat, gx, gv, gl, gP = U.unrolled_grads(p.x, p.v0, p.lam0, p.P0, n_iter, grad_out=g)
    return s_hat.numpy(), [a.numpy() for a in (gx, gv, gl, gP)]


@pytest.mark.parametrize("n_iter,every", [(0, 1), (1, 1), (3, 1), (3, 2), (3, 5)])
def test_gradients_match_oracle(ff, n_iter, every):
    p = problem(3, 3, 9, 70, seed=31)          # N = 70: one full wave and a ragged one per workgroup stride
    g = grad_out_for(p, 1)
    _, out, grads = run_gpu(ff, p, n_iter, every, g)
    s_ref, gref = reference(p, n_iter, g)
    assert rel(out, s_ref) <= 1e-4
    check_grads(f"T{n_iter} every {every}", grads, gref, grad_tol(p, n_iter))


@pytest.mark.parametrize("I,J,N", [(3, 3, 70), (2, 2, 1500)])
def test_gradients_streaming_path(ff, I, J, N):
    """The streaming kernels (path 2): segments are rebuilt one iteration at a
    time and the adjoint sums the eq. 23 terms itself; N = 1500 spans two
    tiles of the streaming kernels."""
    p = problem(I, J, 5, N, seed=36)
    g = grad_out_for(p, 4)
    _, out, grads = run_gpu(ff, p, 3, 2, g, path=2)
    s_ref, gref = reference(p, 3, g)
    assert rel(out, s_ref) <= 1e-4
    check_grads(f"streaming I{I} J{J} N{N}", grads, gref, grad_tol(p, 3))


@pytest.mark.parametrize("I,J", [(1, 2), (2, 3), (4, 2), (6, 4)])
def test_gradients_other_sizes(ff, I, J):
    p = problem(I, J, 5, 41, seed=32 + I)
    g = grad_out_for(p, 2)
    _, out, grads = run_gpu(ff, p, 2, 1, g)
    s_ref, gref = reference(p, 2, g)
    assert rel(out, s_ref) <= 1e-4
    check_grads(f"I{I} J{J}", grads, gref, grad_tol(p, 2))


def test_checkpoint_interval_does_not_change_gradients(ff):
    """The segments are rebuilt bitwise, so every interval gives the same bits."""
    p = problem(3, 3, 7, 90, seed=33)
    g = grad_out_for(p, 3)
    res = [run_gpu(ff, p, 6, every, g)[2] for every in (1, 2, 4, 6)]
    for other in res[1:]:
        for a, b in zip(res[0], other):
            np.testing.assert_array_equal(a, b)


def test_autograd_function_mse(ff):
    from paper_1805_09498_amd.autograd import unrolled_separate
    p = synth.make_problem(3, 3, 8, 48, seed=34, with_sources=True).rounded_c64()
    t = to_dev(p)
    leaves = [t[k].clone().requires_grad_(True) for k in ("x", "v0", "lam0", "P0")]
    s_hat = unrolled_separate(*leaves, n_iter=3, ckpt_every=2)
    s_true = torch.from_numpy(p.s.astype(np.complex64)).cuda()
    loss = (s_hat - s_true).abs().pow(2).mean()
    loss.backward()
    _, _, gx, gv, gl, gP = U.unrolled_grads(p.x, p.v0, p.lam0, p.P0, 3, s_ref=p.s)
    check_grads("autograd MSE", [l.grad.cpu().numpy() for l in leaves], [r.numpy() for r in (gx, gv, gl, gP)],
                grad_tol(p, 3))


def test_unrolled_workload_full_size(ff):
    """The unrolled workload: I = J = 3, F = 257, N = 500, 20 iterations, a
    checkpoint every 5, MSE against the seeded true images."""
    p = synth.make_config("unrolled", with_sources=True).rounded_c64()
    t = to_dev(p)
    from paper_1805_09498_amd.autograd import unrolled_separate
    leaves = [t[k].clone().requires_grad_(True) for k in ("x", "v0", "lam0", "P0")]
    s_hat = unrolled_separate(*leaves, n_iter=20, ckpt_every=5)
    s_true = torch.from_numpy(p.s.astype(np.complex64)).cuda()
    loss = (s_hat - s_true).abs().pow(2).mean()
    loss.backward()
    _, s_ref, gx, gv, gl, gP = U.unrolled_grads(p.x, p.v0, p.lam0, p.P0, 20, s_ref=p.s)
    assert rel(s_hat.detach().cpu().numpy(), s_ref.numpy()) <= 1e-4
    check_grads("unrolled workload", [l.grad.cpu().numpy() for l in leaves], [r.numpy() for r in (gx, gv, gl, gP)],
                grad_tol(p, 20))


def test_derivative_call_errors(ff):
    p = problem(2, 2, 3, 20, seed=35)
    t = to_dev(p)
    ctx = ff.fca_init(ff.FCA_METHOD_AS, t["x"], t["v0"], t["lam0"], t["P0"])
    g = torch.zeros((2, 3, 20, 2), dtype=torch.complex64, device="cuda")
    with pytest.raises(ff.FcaError):
        ff.fastfca_as_backward(ctx, g)                 # nothing recorded
    ff.fastfca_as_forward(ctx, 2, 1)
    ff.fastfca_as_backward(ctx, g)
    ff.fastfca_as_iterate(ctx, 1)
    with pytest.raises(ff.FcaError):
        ff.fastfca_as_backward(ctx, g)                 # the state moved on
    ff.fastfca_as_forward(ctx, 2, 1)
    ff.fca_set_option(ctx, "K", 2)
    with pytest.raises(ff.FcaError):
        ff.fastfca_as_backward(ctx, g)                 # the recorded run was for K = 1
    with pytest.raises(ff.FcaError):
        ff.fastfca_as_forward(ctx, 2, 1)               # K > 1 has no adjoint
    with pytest.raises(ff.FcaError):
        ff.fastfca_as_forward(ctx, 2, 0)


@pytest.mark.parametrize("key,value", [("K", 2), ("p_update", 2)])
def test_backward_refused_after_a_p_step_option_changes(ff, key, value):
    """A recorded run on the streaming kernels (path 2 rebuilds segments
    with the current options) is refused once K or the P update changed."""
    p = problem(2, 2, 3, 20, seed=35)
    t = to_dev(p)
    ctx = ff.fca_init(ff.FCA_METHOD_AS, t["x"], t["v0"], t["lam0"], t["P0"])
    ff.fca_set_option(ctx, "path", 2)
    g = torch.zeros((2, 3, 20, 2), dtype=torch.complex64, device="cuda")
    ff.fastfca_as_forward(ctx, 2, 1)
    ff.fca_set_option(ctx, key, value)
    with pytest.raises(ff.FcaError) as e:
        ff.fastfca_as_backward(ctx, g)
    assert e.value.status == ff.FCA_ERR_STATE
