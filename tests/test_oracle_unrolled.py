"""Pins of the PyTorch oracle of the unrolled method (oracle/unrolled.py):
its forward equals the numpy oracle, and its autograd derivatives equal FP64
central finite differences (F = 8, N = 16) in random directions of every
input, which also fixes the complex-gradient convention."""

import numpy as np
import pytest
import torch

import oracle
from oracle import unrolled as U
from paper_1805_09498_amd import synth


def prob(I, J, F, N, seed, **kw):
    return synth.make_problem(I, J, F, N, seed, **kw)


@pytest.mark.parametrize("I,J", [(1, 2), (2, 3), (3, 3), (4, 2)])
def test_step_and_wiener_equal_numpy_oracle(I, J):
    p = prob(I, J, 5, 24, seed=50 + I)
    v, lam, P = p.v0, p.lam0, p.P0
    tv, tl, tP = (torch.from_numpy(a) for a in (v, lam, P))
    x = torch.from_numpy(p.x)
    for _ in range(3):
        v, lam, P = oracle.fastfca_as_step(p.x, v, lam, P)
        tv, tl, tP = U.as_step(x, tv, tl, tP)
        for a, b in ((tv, v), (tl, lam), (tP, P)):
            np.testing.assert_allclose(a.numpy(), b, rtol=1e-11, atol=1e-12 * np.abs(b).max())
    np.testing.assert_allclose(U.wiener(x, tv, tl, tP).numpy(), oracle.wiener_as(p.x, v, lam, P),
                               rtol=1e-10, atol=1e-11 * np.abs(p.x).max())


def _loss(p, s_ref, x, v0, lam0, P0, n_iter):
    with torch.no_grad():
        return float(U.mse(U.unrolled(torch.from_numpy(x), torch.from_numpy(v0), torch.from_numpy(lam0),
                                      torch.from_numpy(P0), n_iter), torch.from_numpy(s_ref)))


@pytest.mark.parametrize("I,J,n_iter", [(3, 3, 2), (2, 3, 3)])
def test_gradients_equal_finite_differences(I, J, n_iter):
    p = prob(I, J, 8, 16, seed=60 + I, with_sources=True)
    s_ref = p.s                                       # [J][F][N][I] seeded true images
    loss, _, gx, gv, gl, gP = U.unrolled_grads(p.x, p.v0, p.lam0, p.P0, n_iter, s_ref=s_ref)
    rng = np.random.default_rng(7)
    base = dict(x=p.x, v0=p.v0, lam0=p.lam0, P0=p.P0)
    grads = dict(x=gx.numpy(), v0=gv.numpy(), lam0=gl.numpy(), P0=gP.numpy())
    for name in ("x", "v0", "lam0", "P0"):
        a = base[name]
        for _ in range(2):
            if np.iscomplexobj(a):
                d = rng.standard_normal(a.shape) + 1j * rng.standard_normal(a.shape)
            else:
                d = rng.standard_normal(a.shape) * a        # relative steps keep v, lam > 0
            h = 1e-6
            kw_p = dict(base); kw_p[name] = a + h * d
            kw_m = dict(base); kw_m[name] = a - h * d
            fd = (_loss(p, s_ref, n_iter=n_iter, **kw_p) - _loss(p, s_ref, n_iter=n_iter, **kw_m)) / (2 * h)
            an = float(np.sum((np.conj(grads[name]) * d).real))   # Re <grad, d>
            assert abs(fd - an) <= 1e-6 * max(abs(an), abs(fd), 1e-3 * float(loss)), (name, fd, an)
