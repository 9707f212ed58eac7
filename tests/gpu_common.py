"""Helpers of the GPU parity tests: move a seeded problem to the device, run
the library through the C ABI, compare with the FP64 oracle.

Two kinds of bounds are asserted:

* per tensor, the relative Frobenius error |a - b| / |b| <= 1e-4 for v,
  lambda, P (or S) after one iteration and <= 1e-5 relative on the
  log-likelihood after ten iterations;
* per entry, |a - b| <= a first-order bound on the rounding error of the
  single-precision evaluation, computed in FP64 from the state the step
  starts from (tests/error_bounds.py; for P it scales with the condition
  number of each eq. 23 matrix).

``check`` also reports the worst per-bin relative error and the largest
elementwise relative error over the entries above 1e-6 of their bin's
largest magnitude.  The oracle always runs on the single-precision-rounded
inputs widened to FP64, so input rounding is not charged to the GPU.
"""

import json
import os

import numpy as np
import torch

import oracle
from paper_1805_09498_amd import synth

TOL_PARAM = 1e-4
TOL_LOGLIK = 1e-5
ELEM_FLOOR = 1e-6


def rel(a, b):
    a = np.asarray(a); b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def _bin_errors(a, b, axis=0):
    """Relative Frobenius error of every bin (axis `axis`)."""
    a = np.moveaxis(np.asarray(a), axis, 0)
    b = np.moveaxis(np.asarray(b), axis, 0)
    F = b.shape[0]
    num = np.linalg.norm((a - b).reshape(F, -1), axis=1)
    den = np.linalg.norm(b.reshape(F, -1), axis=1)
    return num / np.where(den > 0, den, 1.0)


def per_bin_rel(a, b, axis=0):
    """The largest relative Frobenius error over the bins (axis `axis`)."""
    return float(np.max(_bin_errors(a, b, axis)))


def elem_rel(a, b, axis=0, floor=ELEM_FLOOR):
    """The largest |a - b| / |b| over the entries with |b| above `floor` times
    the largest |b| of their bin (axis `axis`)."""
    a = np.moveaxis(np.asarray(a), axis, 0)
    b = np.moveaxis(np.asarray(b), axis, 0)
    F = b.shape[0]
    ab = np.abs(b).reshape(F, -1)
    err = np.abs(a - b).reshape(F, -1)
    keep = ab > floor * ab.max(axis=1, keepdims=True)
    if not keep.any():
        return 0.0
    return float(np.max(err[keep] / ab[keep]))


def check(name, got, ref, bound=None, tol=None, axis=0, bin_tol=None):
    """Compare a HIP result with the oracle's: every entry within `bound`
    (absolute, broadcastable to `ref`), the tensor within `tol` (relative
    Frobenius) and every bin (axis `axis`) within `bin_tol` (relative
    Frobenius per bin), whichever are given.  Returns the measures; when
    FASTFCA_PARITY_LOG names a file they are appended to it as a JSON line."""
    got = np.asarray(got)
    ref = np.asarray(ref)
    assert got.shape == ref.shape, (name, got.shape, ref.shape)
    assert np.isfinite(got).all(), f"{name}: non-finite entries"
    m = {"name": name, "rel": rel(got, ref), "bin_rel": per_bin_rel(got, ref, axis),
         "elem_rel": elem_rel(got, ref, axis)}
    if bound is not None:
        bound = np.broadcast_to(np.asarray(bound, np.float64), ref.shape)
        err = np.abs(got - ref)
        m["err_over_bound"] = float(np.max(err / np.where(bound > 0, bound, np.inf))) if err.size else 0.0
    log = os.environ.get("FASTFCA_PARITY_LOG")
    if log:
        with open(log, "a") as fh:
            fh.write(json.dumps(m) + "\n")
    print("parity", json.dumps(m))
    if bound is not None:
        assert np.all(err <= bound), f"{name}: error above the rounding bound {m}"
    if tol is not None:
        assert m["rel"] <= tol, f"{name}: relative error above {tol} {m}"
    if bin_tol is not None:
        bins = _bin_errors(got, ref, axis)
        bt = np.broadcast_to(np.asarray(bin_tol, np.float64), bins.shape)
        m["bin_rel_over_tol"] = float(np.max(bins / bt))
        if log:
            with open(log, "a") as fh:
                fh.write(json.dumps(dict(m, name=m["name"] + " [bins]")) + "\n")
        assert np.all(bins <= bt), f"{name}: a bin's relative error above its bound {m}"
    return m


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


def _bin_rel(bound, ref):
    """Per-bin relative Frobenius size of an absolute bound (axis 0 = bin)."""
    F = ref.shape[0]
    num = np.linalg.norm(np.asarray(bound).reshape(F, -1), axis=1)
    den = np.linalg.norm(np.asarray(ref).reshape(F, -1), axis=1)
    return num / np.where(den > 0, den, 1.0)


def oracle_as_bounded(p, n_iter, K=1, p_update=0, mu=0.1, rho_every=1):
    """The oracle's (v, lam, P) after n_iter iterations from the problem's
    start, with the bounds an FP32 run is checked against:

    * n_iter = 1: per-entry first-order bounds of the iteration's rounding
      (tests/error_bounds.py), in b["v"], b["lam"], b["P"];
    * always, per-bin relative bounds b["bin_rel"] [F]: the sum over the
      iterations of rho_m(f), the largest per-bin relative size of iteration
      m's own first-order bound (of v, lambda or P, evaluated at the
      oracle's state before that iteration).  This takes a relative error
      carried into an iteration not to grow (the iteration map treated as
      non-expansive; worst-case propagation through the eq. 23 solves
      multiplies by their condition numbers every iteration and bounds
      nothing after two); the comparisons check that assumption.  With
      rho_every = k the bound is evaluated every k-th iteration and counted
      k times.

    Returns (v, lam, P, bounds dict, largest eq. 23 condition number)."""
    from tests import error_bounds as EB
    v, lam, P = p.v0, p.lam0, p.P0
    kmax = 1.0
    first = None
    rho = np.zeros(p.x.shape[0])
    for m in range(n_iter):
        if m % rho_every == 0:
            b = EB.as_step_bounds(p.x, v, lam, P, K=K, p_update=p_update if p_update < 3 else 0, mu=mu)
            if p_update >= 3:
                b = dict(b, P=EB.as_variant_p_bounds(p.x, v, lam, P, p_update))
            kmax = max(kmax, float(np.max(b["kappa"])))
            if first is None:
                first = b
        if p_update == 0:
            vn, ln, Pn = oracle.fastfca_as_step(p.x, v, lam, P, K=K)
        elif p_update == 3:
            vn, ln, Pn = oracle.fastfca_as_step_newton(p.x, v, lam, P)
        elif p_update == 4:
            vn, ln, Pn = oracle.as_em_p_step(p.x, v, lam, P)
        else:
            vn, ln, Pn = oracle.fastfca_as_step_grad(p.x, v, lam, P, mu, natural=(p_update == 2))
        if m % rho_every == 0:
            rho += rho_every * np.max(np.stack([_bin_rel(b["v"], vn), _bin_rel(b["lam"], ln),
                                                _bin_rel(b["P"], Pn)]), axis=0)
        v, lam, P = vn, ln, Pn
    bounds = {k: first[k] for k in ("v", "lam", "P")} if n_iter == 1 else {}
    bounds["bin_rel"] = rho
    return v, lam, P, bounds, kmax


def check_as_params(got, ref_and_bounds, tol=TOL_PARAM, tag="", tol_P="same"):
    """v, lambda, P of a FastFCA-AS run against oracle_as_bounded's result:
    per entry after one iteration, per bin after several; the per-tensor
    tolerance `tol` when given (`tol_P` for P, by default the same)."""
    v, lam, P = got
    v_ref, lam_ref, P_ref, b, _ = ref_and_bounds
    for name, g, r in (("v", v, v_ref), ("lam", lam, lam_ref), ("P", P, P_ref)):
        t = tol if (name != "P" or tol_P == "same") else tol_P
        if name in b:
            check(name + tag, g, r, b[name], t)
        else:
            check(name + tag, g, r, tol=t, bin_tol=b["bin_rel"])


def check_loglik_bins(Lb, Lb_ref, bound, tag=""):
    """Per-bin log-likelihoods within an absolute bound per bin."""
    return check("loglik_bins" + tag, np.asarray(Lb, np.float64), np.asarray(Lb_ref, np.float64), bound)


def as_loglik_bin_bound(p, ref_and_bounds):
    """Bound of the per-bin L2 of an FP32 run after the iterations that
    oracle_as_bounded followed: the accumulated per-bin relative state bound
    times the log-likelihood's sensitivity, plus the evaluation's own
    rounding at the final state."""
    from tests import error_bounds as EB
    v, lam, P, b, _ = ref_and_bounds
    return b["bin_rel"] * EB.loglik_bin_sensitivity(p.x, v, lam, P) + EB.loglik_bin_bounds(p.x, v, lam, P)


def oracle_em_bounded(p, S0, n_iter):
    """The FCA EM analogue of oracle_as_bounded: the oracle's (v, S) after
    n_iter iterations, the per-entry bounds of the first iteration and the
    accumulated per-bin relative bound rho [F]."""
    from tests import error_bounds as EB
    v, S = p.v0, S0
    first = None
    rho = np.zeros(p.x.shape[0])
    for _ in range(n_iter):
        b = EB.em_step_bounds(p.x, v, S)
        first = b if first is None else first
        vn, Sn = oracle.fca_em_step(p.x, v, S)
        rho += np.maximum(_bin_rel(b["v"], vn), _bin_rel(b["S"], Sn))
        v, S = vn, Sn
    return v, S, first, rho


def oracle_em(p, R, n_iter):
    v = p.v0
    for _ in range(n_iter):
        v, R = oracle.fca_em_step(p.x, v, R)
    return v, R


def sub_problem(p, bins):
    """The bins `bins` of a problem (bins are independent in both methods)."""
    return synth.Problem(x=p.x[bins], v0=p.v0[bins], lam0=p.lam0[bins], P0=p.P0[bins])
