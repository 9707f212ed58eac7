"""Helpers of the GPU parity tests: move a seeded problem to the device, run
the library through the C ABI, compare with the FP64 oracle.

Tolerances: per-tensor relative Frobenius error |a - b| / |b| <= 1e-4 for
v, lambda, P (or S) after one iteration; <= 1e-5 relative on the
log-likelihood after ten iterations.  The oracle always runs on the
single-precision-rounded inputs widened to FP64, so input rounding is not
charged to the GPU.
"""

import numpy as np
import torch

import oracle
from paper_1805_09498_amd import synth

TOL_PARAM = 1e-4
TOL_LOGLIK = 1e-5


def rel(a, b):
    a = np.asarray(a); b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def problem(I, J, F, N, seed, **kw):
    return synth.make_problem(I, J, F, N, seed, **kw).rounded_c64()


def to_dev(p, R0=None):
    dev = torch.device("cuda:0")
    t = dict(
        x=torch.from_numpy(p.x.astype(np.complex64)).to(dev),
        v0=torch.from_numpy(p.v0.astype(np.float32)).to(dev),
        lam0=torch.from_numpy(p.lam0.astype(np.float32)).to(dev),
        P0=torch.from_numpy(p.P0.astype(np.complex64)).to(dev),
    )
    if R0 is not None:
        t["R0"] = torch.from_numpy(R0.astype(np.complex64)).to(dev)
    return t


def run_as(ff, p, n_iter, path=0, waves=0, K=1, bpw=0):
    t = to_dev(p)
    ctx = ff.fca_init(ff.FCA_METHOD_AS, t["x"], t["v0"], t["lam0"], t["P0"])
    ff.fca_set_option(ctx, "path", path)
    ff.fca_set_option(ctx, "waves", waves)
    ff.fca_set_option(ctx, "bins_per_wg", bpw)
    ff.fca_set_option(ctx, "K", K)
    ff.fastfca_as_iterate(ctx, n_iter)
    return ctx


def params(ff, ctx):
    v, lam, M = ff.fca_get_params(ctx)
    torch.cuda.synchronize()
    return (v.cpu().numpy().astype(np.float64),
            None if lam is None else lam.cpu().numpy().astype(np.float64),
            M.cpu().numpy().astype(np.complex128))


def oracle_as(p, n_iter, K=1):
    v, lam, P = p.v0, p.lam0, p.P0
    for _ in range(n_iter):
        v, lam, P = oracle.fastfca_as_step(p.x, v, lam, P, K=K)
    return v, lam, P


def oracle_em(p, R, n_iter):
    v = p.v0
    for _ in range(n_iter):
        v, R = oracle.fca_em_step(p.x, v, R)
    return v, R


def sub_problem(p, bins):
    """The bins `bins` of a problem (bins are independent in both methods)."""
    return synth.Problem(x=p.x[bins], v0=p.v0[bins], lam0=p.lam0[bins], P0=p.P0[bins])
