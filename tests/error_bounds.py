"""First-order bounds on the rounding error of a single-precision evaluation
of the method, computed in FP64 from the state the evaluation starts from.

The GPU parity tests use them to bound every entry of a result (not only a
norm per tensor).  These functions return error bounds, never expected
values: expected values always come from the oracle.

Error model (running error analysis, as in Higham, "Accuracy and Stability
of Numerical Algorithms", ch. 3):

* u = 2^-24 is the unit roundoff of FP32; gamma(k) = k u / (1 - k u).
* A quantity q that k floating-point operations form from exact operands
  carries an absolute error of at most gamma(k) * M_q, where M_q is q
  evaluated with every term replaced by its absolute value.
* Errors inherited from inexact operands are carried to first order by the
  partial derivatives (written out per step below).
* Sums over the frames of a bin are a few sequential additions per lane,
  then tree sums over lanes, waves and tiles: at most ceil(log2 N) + 8
  roundings per term.
* Reciprocals use the hardware reciprocal (1 ulp): two roundings each.
* A linear solve G a = b by a Cholesky or LDL^H factorisation is backward
  stable: the computed a solves (G + dG) a = b with ||dG|| <= I gamma(3I + 1)
  ||G||, so ||da|| <= kappa(G) (eps_G + I gamma(3I + 1)) ||a|| to first order,
  where eps_G is the relative error of G itself.

The operation counts are generous upper counts of the kernels' evaluation
order (per point: y = P^H x, the diagonal variances d, e = (|y|^2/d - 1)/d,
W = 1 + (v/I) sum_i lambda_i e_i, r = 1 + v lambda e; per bin: the frame
sums, one solve per column of eq. 23 in the basis of y, one product with P).

Shapes follow the oracle: x [F][N][I], v [F][N][J], lam [F][J][I],
P [F][I][I], S [F][J][I][I].
"""

import math

import numpy as np

import oracle

U = 2.0 ** -24


def gamma(k):
    return k * U / (1.0 - k * U)


def _levels(N):
    return int(math.ceil(math.log2(max(N, 2)))) + 8


def _herm(a):
    return np.conj(np.swapaxes(a, -1, -2))


def _solve_bound(G, a, epsG, I):
    """||da|| for G a = b solved in FP32 with G known to relative error epsG
    (per matrix); inf where the first-order bound does not apply."""
    kap = np.linalg.cond(G)
    eps = epsG + I * gamma(3 * I + 1)
    den = 1.0 - kap * eps
    with np.errstate(divide="ignore", invalid="ignore"):
        out = np.where(den > 0.0, kap * eps * np.linalg.norm(a, axis=-1) / np.where(den > 0, den, 1.0), np.inf)
    return out, kap


def as_point_stats(x, v, lam, P, dv_in=0.0, dlam_in=0.0, dP_in=0.0):
    """Per-point quantities of the E-step and the v update, with first-order
    absolute error bounds of their FP32 evaluation from inputs (v, lam, P)
    that carry absolute errors dv_in, dlam_in, dP_in (0: exact inputs).
    Returns a dict of arrays."""
    x = np.asarray(x, np.complex128)
    v = np.asarray(v, np.float64)
    lam = np.asarray(lam, np.float64)
    P = np.asarray(P, np.complex128)
    I = x.shape[2]
    J = v.shape[2]
    dv_in = np.broadcast_to(np.asarray(dv_in, np.float64), v.shape)
    dlam_in = np.broadcast_to(np.asarray(dlam_in, np.float64), lam.shape)
    dP_in = np.broadcast_to(np.asarray(dP_in, np.float64), P.shape)
    ax = np.abs(x)
    y = np.einsum("fki,fnk->fni", np.conj(P), x)
    ay = np.abs(y)
    dy = gamma(4 * I) * np.einsum("fki,fnk->fni", np.abs(P), ax) + np.einsum("fki,fnk->fni", dP_in, ax)
    q = ay ** 2
    dq = 2.0 * ay * dy + dy ** 2 + gamma(3) * q
    d = np.einsum("fnj,fji->fni", v, lam)
    dd = gamma(J + 1) * d + np.einsum("fnj,fji->fni", dv_in, lam) + np.einsum("fnj,fji->fni", v, dlam_in)
    # 1/d by the hardware reciprocal: relative error of d plus two roundings
    rel_d = dd / d + gamma(2)
    h = q / d - 1.0
    dh = dq / d + q / d * rel_d + gamma(1) * (q / d + 1.0)
    e = h / d
    de = dh / d + np.abs(h) / d * rel_d + gamma(1) * np.abs(e)
    W = 1.0 + np.einsum("fnj,fji,fni->fnj", v, lam, e) / I
    MW = 1.0 + np.einsum("fnj,fji,fni->fnj", v, lam, np.abs(e)) / I
    dW = (np.einsum("fnj,fji,fni->fnj", v, lam, de) + np.einsum("fnj,fji,fni->fnj", dv_in, lam, np.abs(e))
          + np.einsum("fnj,fji,fni->fnj", v, dlam_in, np.abs(e))) / I + gamma(I + 6) * MW
    v_new = v * W
    dv = v * dW + dv_in * np.abs(W) + gamma(1) * np.abs(v_new)
    vl = v[:, :, :, None] * lam[:, None, :, :]                                # [F][N][J][I]
    dvl = dv_in[:, :, :, None] * lam[:, None, :, :] + v[:, :, :, None] * dlam_in[:, None, :, :]
    r = 1.0 + vl * e[:, :, None, :]
    Mr = 1.0 + vl * np.abs(e)[:, :, None, :]
    dr = vl * de[:, :, None, :] + dvl * np.abs(e)[:, :, None, :] + gamma(3) * Mr
    return dict(y=y, ay=ay, dy=dy, q=q, dq=dq, d=d, dd=dd, e=e, de=de, W=W, dW=dW, v_new=v_new, dv=dv, r=r,
                dr=dr)


def as_em_bounds(x, v, lam, P, dv_in=0.0, dlam_in=0.0, dP_in=0.0):
    """Bounds of the EM half-step (eq. 16-20): returns (dv [F][N][J],
    dlam [F][J][I], stats) for the FP32 evaluation from inputs carrying the
    given absolute errors.  The kernels sum eq. 20 in two parts per bin,
    S0_j = sum_n 1/W_j and S1_ji = sum_n (v_j/W_j) e_i, and form
    lambda' = lambda (S0 + lambda S1) / N."""
    st = as_point_stats(x, v, lam, P, dv_in, dlam_in, dP_in)
    v = np.asarray(v, np.float64)
    lam = np.asarray(lam, np.float64)
    dv_in = np.broadcast_to(np.asarray(dv_in, np.float64), v.shape)
    dlam_in = np.broadcast_to(np.asarray(dlam_in, np.float64), lam.shape)
    N = st["y"].shape[1]
    L = _levels(N)
    W = st["W"]
    rW = 1.0 / W
    drW = np.abs(rW) * (st["dW"] / np.abs(W) + gamma(2))
    m = v * rW
    dm = v * drW + dv_in * np.abs(rW) + gamma(1) * np.abs(m)
    e, de = st["e"], st["de"]
    me = m[..., None] * e[:, :, None, :]                                       # [F][N][J][I]
    dme = np.abs(m)[..., None] * de[:, :, None, :] + dm[..., None] * np.abs(e)[:, :, None, :] + gamma(1) * np.abs(me)
    S0 = rW.sum(axis=1)                                                       # [F][J]
    dS0 = drW.sum(axis=1) + gamma(L) * np.abs(rW).sum(axis=1)
    S1 = me.sum(axis=1)                                                       # [F][J][I]
    dS1 = dme.sum(axis=1) + gamma(L) * np.abs(me).sum(axis=1)
    dlam = (lam / N) * (dS0[..., None] + lam * dS1) + (dlam_in / N) * np.abs(S0[..., None] + 2.0 * lam * S1) \
        + gamma(3) * (lam / N) * (S0[..., None] + lam * np.abs(S1))
    return st["dv"], dlam, st


def as_step_bounds(x, v, lam, P, K=1, p_update=0, mu=0.1, dv_in=0.0, dlam_in=0.0, dP_in=0.0):
    """First-order absolute error bounds of one hybrid iteration (Section 4.3)
    evaluated in FP32 from the state (v, lam, P), which may carry absolute
    errors dv_in, dlam_in, dP_in from earlier iterations (0: exact):
    returns dict(v=[F][N][J], lam=[F][J][I], P=[F][I][I], kappa=[F][I],
    epsG=[F][I]), kappa being the condition numbers of the eq. 23 matrices
    in the basis of y (G_c = P^H Q_c P), whose solves dominate the bound on
    P, and epsG the relative error of those matrices.

    p_update 0: K fixed-point steps (eq. 23); 1: gradient step P + mu g;
    2: natural-gradient step P + mu P P^H g, with g = (1/N) dL2/dP* (eq. 21).
    """
    x = np.asarray(x, np.complex128)
    P = np.asarray(P, np.complex128)
    F, N, I = x.shape
    dP_in = np.broadcast_to(np.asarray(dP_in, np.float64), P.shape)
    dv, dlam, st = as_em_bounds(x, v, lam, P, dv_in, dlam_in, dP_in)
    v_new, lam_new = oracle.as_em_half_step(x, v, lam, P)
    J = v_new.shape[2]
    y, ay, dy = st["y"], st["ay"], st["dy"]
    dp = np.einsum("fnj,fji->fni", v_new, lam_new)
    ddp = np.einsum("fnj,fji->fni", dv, lam_new) + np.einsum("fnj,fji->fni", v_new, dlam) + gamma(J) * dp
    w = 1.0 / dp
    G = np.einsum("fnc,fna,fnb->fcab", w, y, np.conj(y)) / N                 # [F][c][I][I]
    Gabs = np.einsum("fnc,fna,fnb->fcab", w, ay, ay) / N
    dG = (np.einsum("fnc,fna,fnb->fcab", w, dy, ay) + np.einsum("fnc,fna,fnb->fcab", w, ay, dy)
          + np.einsum("fnc,fna,fnb->fcab", ddp * w ** 2, ay, ay)) / N + gamma(_levels(N) + 3) * Gabs
    nG = np.linalg.norm(G, ord=2, axis=(-2, -1))
    epsG = np.linalg.norm(dG, axis=(-2, -1)) / nG                            # [F][c]
    absP = np.abs(P)
    eye = np.broadcast_to(np.eye(I), (F, I, I))
    kap = np.linalg.cond(G)
    if p_update == 0:
        # A_1 columns solve G_c a = e_c; later steps G_c a = [A^-H]_c.
        A = np.eye(I, dtype=np.complex128)[None].repeat(F, 0)
        dA = np.zeros((F, I))                                                # ||delta a_c||
        for _ in range(K):
            B = _herm(np.linalg.inv(A))                                      # A^-H
            nAinv = np.linalg.norm(np.linalg.inv(A), ord=2, axis=(-2, -1))
            kA = np.linalg.cond(A)
            # error of column c of A^-H: inherited through the inverse, plus its own rounding
            dB = (nAinv ** 2)[:, None] * dA.max(axis=1, keepdims=True) + \
                (I * gamma(3 * I + 1) * kA * nAinv)[:, None] * np.linalg.norm(B, axis=1)
            An = np.empty_like(A)
            dAn = np.empty((F, I))
            for c in range(I):
                a = np.linalg.solve(G[:, c], B[:, :, c, None])[..., 0]
                da, _ = _solve_bound(G[:, c], a, epsG[:, c], I)
                Ginv_norm = 1.0 / np.linalg.svd(G[:, c], compute_uv=False)[:, -1]
                An[:, :, c] = a
                dAn[:, c] = da + Ginv_norm * dB[:, c]
            A, dA = An, dAn
        dP = (np.einsum("fkl->fk", absP)[:, :, None] * dA[:, None, :]
              + gamma(2 * I + 2) * np.einsum("fkl,flc->fkc", absP, np.abs(A))
              + np.einsum("fkl,flc->fkc", dP_in, np.abs(A)))
    else:
        # Gamma's column c is G_c e_c; natural: A = 1 + mu (1 - Gamma), P A;
        # gradient: P + mu P^-H (1 - Gamma).
        Gam = np.stack([G[:, c, :, c] for c in range(I)], axis=-1)           # [F][a][c]
        dGam = np.stack([np.linalg.norm(dG[:, c], axis=(-2, -1)) for c in range(I)], axis=-1)  # per column
        if p_update == 2:
            A = eye + mu * (eye - Gam)
            dA = mu * dGam + gamma(3) * (1.0 + mu * (1.0 + np.linalg.norm(Gam, axis=1)))
            dP = (np.einsum("fkl->fk", absP)[:, :, None] * dA[:, None, :]
                  + gamma(2 * I + 2) * np.einsum("fkl,flc->fkc", absP, np.abs(A))
                  + np.einsum("fkl,flc->fkc", dP_in, np.abs(A)))
        else:
            Pinv = np.linalg.inv(P)
            B = _herm(Pinv)
            nPinv = np.linalg.norm(Pinv, ord=2, axis=(-2, -1))
            kP = np.linalg.cond(P)
            M = eye - Gam
            g = np.einsum("fab,fbc->fac", B, M)
            dM = dGam + gamma(2)
            nMcol = np.linalg.norm(M, axis=1)
            dg = nPinv[:, None] * dM + (I * gamma(3 * I + 1) * kP * nPinv)[:, None] * nMcol \
                + gamma(2 * I + 2) * np.linalg.norm(np.einsum("fab,fbc->fac", np.abs(B), np.abs(M)), axis=1) \
                + (nPinv ** 2 * np.linalg.norm(dP_in, axis=(-2, -1)))[:, None] * nMcol
            dP = mu * dg[:, None, :] + gamma(2) * (absP + mu * np.abs(g)) + dP_in
    return dict(v=dv, lam=dlam, P=dP, kappa=kap, epsG=epsG)


def as_wiener_bounds(x, v, lam, P):
    """Bounds of the Wiener filter s_j = P^-H (g_j o y), g_ji = v_j lam_ji / d_i
    (eq. 3 with eq. 15-16), [J][F][N][I]."""
    x = np.asarray(x, np.complex128)
    P = np.asarray(P, np.complex128)
    v = np.asarray(v, np.float64)
    lam = np.asarray(lam, np.float64)
    F, N, I = x.shape
    J = v.shape[2]
    st = as_point_stats(x, v, lam, P)
    g = v[:, :, :, None] * lam[:, None, :, :] / st["d"][:, :, None, :]          # [F][N][J][I]
    z = g * st["y"][:, :, None, :]
    dz = g * st["dy"][:, :, None, :] + gamma(J + 4) * np.abs(z)
    Pinv = np.linalg.inv(P)
    B = _herm(Pinv)
    nPinv = np.linalg.norm(Pinv, ord=2, axis=(-2, -1))
    kP = np.linalg.cond(P)
    absB = np.abs(B)
    nz = np.linalg.norm(z, axis=-1)
    ds = np.einsum("fab,fnjb->fnja", absB, dz) \
        + (I * gamma(3 * I + 1) * kP * nPinv)[:, None, None, None] * nz[..., None] \
        + gamma(2 * I + 2) * np.einsum("fab,fnjb->fnja", absB, np.abs(z))
    return np.transpose(ds, (2, 0, 1, 3))


def em_step_bounds(x, v, S):
    """Bounds of one conventional FCA EM iteration (eq. 6-10) in FP32 from
    the exact state (v, S): dict(v=[F][N][J], S=[F][J][I][I] (per entry),
    kappa_C=[F][N]).  Per point the error is driven by the condition of
    C = sum_j v_j S_j (inverted per point) and of S_j (inverted per bin)."""
    x = np.asarray(x, np.complex128)
    v = np.asarray(v, np.float64)
    S = np.asarray(S, np.complex128)
    F, N, I = x.shape
    J = v.shape[2]
    C = np.einsum("fnj,fjab->fnab", v, S)
    Cinv = np.linalg.inv(C)
    kC = np.linalg.cond(C)                                                    # [F][N]
    nCinv = np.linalg.norm(Cinv, ord=2, axis=(-2, -1))
    nS = np.linalg.norm(S, ord=2, axis=(-2, -1))                              # [F][J]
    kS = np.linalg.cond(S)
    nx = np.linalg.norm(x, axis=-1)
    epsC = gamma(2 * J + 2) + I * gamma(3 * I + 1)
    # ||delta C^-1|| <= kappa(C) eps ||C^-1||; the statistics mu mu^H + Phi of
    # source j are v^2 S C^-1 x x^H C^-1 S + v S - v^2 S C^-1 S.
    dCinv = kC * epsC * nCinv                                                 # [F][N]
    vS = v * nS[:, None, :]                                                   # ||v_j S_j||
    Mstat = vS ** 2 * (nCinv ** 2 * nx ** 2)[..., None] + vS + vS ** 2 * nCinv[..., None]
    dstat = vS ** 2 * ((2.0 * nCinv * nx ** 2 + 1.0) * dCinv)[..., None] + gamma(6 * I + 4) * Mstat
    v_new, S_new = oracle.fca_em_step(x, v, S)
    nSinv = 1.0 / np.linalg.svd(S, compute_uv=False)[..., -1]                 # ||S_j^-1||
    dv = (nSinv[:, None, :] * dstat + (kS * I * gamma(3 * I + 1) * nSinv)[:, None, :] * Mstat) \
        + gamma(2 * I + 2) * nSinv[:, None, :] * Mstat
    dv = np.minimum(dv, np.inf)
    vn = v_new
    dS = ((dstat / vn + Mstat * dv / vn ** 2).mean(axis=1) + gamma(_levels(N) + 2) * (Mstat / vn).mean(axis=1))
    return dict(v=dv, S=np.broadcast_to(dS[..., None, None], S_new.shape).copy(), kappa_C=kC)


def em_wiener_bounds(x, v, S):
    """Bounds of the FCA Wiener filter s_j = v_j S_j C^-1 x (eq. 3),
    [J][F][N][I] per entry (norm-wise per point)."""
    x = np.asarray(x, np.complex128)
    v = np.asarray(v, np.float64)
    S = np.asarray(S, np.complex128)
    F, N, I = x.shape
    J = v.shape[2]
    C = np.einsum("fnj,fjab->fnab", v, S)
    kC = np.linalg.cond(C)
    nCinv = np.linalg.norm(np.linalg.inv(C), ord=2, axis=(-2, -1))
    nS = np.linalg.norm(S, ord=2, axis=(-2, -1))
    nx = np.linalg.norm(x, axis=-1)
    eps = kC * (gamma(2 * J + 2) + I * gamma(3 * I + 1)) + gamma(4 * I + 4)
    ds = (v * nS[:, None, :]) * (nCinv * nx * eps)[..., None]                # [F][N][J]
    return np.broadcast_to(np.transpose(ds, (2, 0, 1))[..., None], (J, F, N, I)).copy()


def loglik_bin_bounds(x, v, lam, P):
    """Bound of the per-bin log-likelihood L2 (eq. 14) [F], evaluated in FP32
    per point (the hardware logarithm: at most 2^-21 absolute error per
    logarithm) and summed over the frames in FP64, plus 2 N |delta ln|det P||
    from an FP32 LU of P."""
    x = np.asarray(x, np.complex128)
    P = np.asarray(P, np.complex128)
    F, N, I = x.shape
    st = as_point_stats(x, v, lam, P)
    d, dd, q, dq = st["d"], st["dd"], st["q"], st["dq"]
    point = dd / d + 2.0 ** -21 + dq / d + q * dd / d ** 2 + gamma(3 * I + 4) * (np.abs(np.log(d)) + q / d + 1.0)
    kP = np.linalg.cond(P)
    dlogdet = I * I * gamma(3 * I + 1) * kP
    return point.sum(axis=(1, 2)) + 2.0 * N * dlogdet + gamma(4) * N * I * math.log(math.pi)


def as_variant_p_bounds(x, v, lam, P, p_update, dv_in=0.0, dlam_in=0.0, dP_in=0.0):
    """Bounds on P after one hybrid iteration whose P update is Newton's
    step (p_update 3) or EM with P in the M-step (p_update 4), norm-wise per
    bin and broadcast to every entry of the bin's P [F][I][I].

    Both updates are P_new = P (1 + X) or P A with per-bin small solves:
    * Newton: the reduced (2I^2 - I)-square real system M s = -g (the
      oracle's as_newton_system at the new v, lambda), whose entries carry
      the relative error eps_G of the eq. 23 sums; Gaussian elimination
      adds n gamma(3n) (backward error), both amplified by cond(M);
    * EM with P: each column solves H_i a = A^-H e_i (cond(H_i), and
      cond(A) for A^-H), H_i carrying the error of sums like eps_G plus
      J I roundings per term; the columns are swept in order, so an error
      in earlier columns reaches later ones through A^-H (factor
      1 + cond(A)).
    """
    x = np.asarray(x, np.complex128)
    P = np.asarray(P, np.complex128)
    F, N, I = x.shape
    base = as_step_bounds(x, v, lam, P, dv_in=dv_in, dlam_in=dlam_in, dP_in=dP_in)
    epsG = np.max(base["epsG"], axis=1)                                      # [F]
    nPin = np.linalg.norm(np.broadcast_to(np.asarray(dP_in, np.float64), P.shape), axis=(-2, -1))
    v_new, lam_new = oracle.as_em_half_step(x, v, lam, P)
    J = v_new.shape[2]
    nP = np.linalg.norm(P, ord=2, axis=(-2, -1))
    if p_update == 3:
        n = 2 * I * I - I
        bound = np.empty(F)
        for f, (H, g) in enumerate(oracle.as_newton_system(x, v_new, lam_new, P)):
            s = np.linalg.solve(H, -g)
            kM = np.linalg.cond(H)
            dX = kM * (epsG[f] + n * gamma(3 * n)) * (np.linalg.norm(s) + 1.0)
            bound[f] = nP[f] * dX + (gamma(2 * I + 2) * nP[f] + nPin[f]) * (1.0 + np.linalg.norm(s))
    else:
        mu, Phi = oracle.fca_estep(x, np.asarray(v, np.float64), oracle.as_spatial_cov(P, lam))
        M = np.einsum("fnja,fnjb->fnjab", mu, np.conj(mu)) + Phi
        V = np.einsum("fnjab,fnj,fji->fiab", M, 1.0 / v_new, 1.0 / lam_new) / (N * J)
        H = np.einsum("fka,fikl,flb->fiab", np.conj(P), V, P)                  # P^H V_i P
        P_new = oracle.as_em_p_step(x, v, lam, P)[2]
        A = np.linalg.solve(P, P_new)
        kA = np.linalg.cond(A)
        kH = np.linalg.cond(H)                                                # [F][I]
        na = np.linalg.norm(A, axis=1)                                        # column norms [F][I]
        epsH = epsG + gamma(J * I + 8)
        per_col = na * (kH * (epsH[:, None] + I * gamma(3 * I + 1)) + (kA * I * gamma(3 * I + 1))[:, None]
                        + gamma(2 * I + 4))
        dA = (1.0 + kA) * per_col.sum(axis=1)
        bound = nP * dA + (gamma(2 * I + 2) * nP + nPin) * np.linalg.norm(A, ord=2, axis=(-2, -1))
    return np.broadcast_to(bound[:, None, None], P.shape).copy()


def loglik_bin_sensitivity(x, v, lam, P):
    """First-order size of the change of each bin's L2 (eq. 14) [F] per unit
    relative error of the state: a relative error e of d_i moves each term
    -ln d_i - |y_i|^2 / d_i by at most e (1 + |y_i|^2 / d_i); one of P moves
    |y_i|^2 by 2 e |y_i|^2 and ln|det P| by I cond(P) e."""
    x = np.asarray(x, np.complex128)
    P = np.asarray(P, np.complex128)
    F, N, I = x.shape
    st = as_point_stats(x, v, lam, P)
    q_d = st["q"] / st["d"]
    return (1.0 + 3.0 * q_d).sum(axis=(1, 2)) + 2.0 * N * I * np.linalg.cond(P)


def em_loglik_bin_sensitivity(x, v, S):
    """The same for L1 (eq. 5) of FCA: a relative error e of the model
    covariance C = sum_j v_j S_j moves -ln det C - x^H C^-1 x by at most
    cond(C) e (I + x^H C^-1 x)."""
    x = np.asarray(x, np.complex128)
    C = np.einsum("fnj,fjab->fnab", np.asarray(v, np.float64), np.asarray(S, np.complex128))
    quad = np.real(np.einsum("fna,fna->fn", np.conj(x), np.linalg.solve(C, x[..., None])[..., 0]))
    return (np.linalg.cond(C) * (C.shape[-1] + quad)).sum(axis=1)
