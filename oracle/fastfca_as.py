"""FastFCA-AS (Section 4 of the paper), FP64 oracle.

Test infrastructure only (see the package docstring).  One hybrid iteration
is the two steps of Section 4.3: an EM update of (Lambda_j, v_j) with P(f)
held fixed (Section 4.3.1, eq. 15-20), then the fixed-point update of P(f)
(Section 4.3.2, eq. 21-23).

Readings of the paper used here:
  * v_j is updated first with the current Lambda_j (eq. 19) and Lambda_j then
    uses the new v_j (eq. 20), the order in which the updates are written.
  * The fixed-point step uses the (v, Lambda) produced by the EM step of the
    same iteration, and updates every column of P(f) from the same current
    P(f)^-H (all columns at once).  With K > 1 inner steps the weighted
    covariances of eq. 23 stay fixed and only P(f)^-H is recomputed.
  * No normalisation of the scale ambiguities (v_j c, Lambda_j / c) or
    (P D, Lambda |D|^2) is applied; the paper applies none.
"""

import numpy as np

from .fca import fca_model_cov, loglik_fca, wiener_fca


def _herm(a):
    return np.conj(np.swapaxes(a, -1, -2))


def as_spatial_cov(P, lam):
    """Spatial covariances under the joint-diagonalisation model (eq. 12).

    S_j(f) = (P(f)^-1)^H Lambda_j(f) P(f)^-1.
    P [F][I][I], lam [F][J][I]  ->  R [F][J][I][I]
    """
    P = np.asarray(P, dtype=np.complex128)
    Pinv = np.linalg.inv(P)                          # [F][I][I]
    PinvH = _herm(Pinv)
    return np.einsum("fab,fjb,fbc->fjac", PinvH, np.asarray(lam, np.float64), Pinv)


def as_estep(x, v, lam, P):
    """E-step in the transformed basis (eq. 15-17).

    y~    = P^H y                                        (eq. 16, right)
    mu~_j = v_j Lambda_j (sum_k v_k Lambda_k)^-1 y~      (eq. 16)
    Phi~_j = v_j Lambda_j - v_j Lambda_j (sum_k v_k Lambda_k)^-1 v_j Lambda_j
                                                        (eq. 17, diagonal)
    Returns y~ [F][N][I], mu~ [F][N][J][I], diag(Phi~) [F][N][J][I].
    """
    x = np.asarray(x, dtype=np.complex128)
    v = np.asarray(v, dtype=np.float64)
    lam = np.asarray(lam, dtype=np.float64)
    P = np.asarray(P, dtype=np.complex128)
    yt = np.einsum("fki,fnk->fni", np.conj(P), x)     # (P^H y)_i = sum_k conj(P_ki) y_k
    vl = v[:, :, :, None] * lam[:, None, :, :]       # v_j Lambda_j     [F][N][J][I]
    D = vl.sum(axis=2)                               # sum_k v_k Lambda_k  [F][N][I]
    mut = vl / D[:, :, None, :] * yt[:, :, None, :]
    phit = vl - vl * vl / D[:, :, None, :]
    return yt, mut, phit


def as_em_half_step(x, v, lam, P):
    """Step 1 of the hybrid algorithm: one EM iteration on (Lambda, v).

    v_j      <- (1/I) tr(Lambda_j^-1 (diag|mu~_j|^2 + Phi~_j))     (eq. 19)
    Lambda_j <- (1/N) sum_n (diag|mu~_j|^2 + Phi~_j) / v_j          (eq. 20)
    Returns (v_new [F][N][J], lam_new [F][J][I]).
    """
    _, mut, phit = as_estep(x, v, lam, P)
    stat = np.abs(mut) ** 2 + phit                   # diagonal of the bracket
    I = stat.shape[-1]
    N = stat.shape[1]
    v_new = (stat / np.asarray(lam, np.float64)[:, None, :, :]).sum(axis=3) / I
    lam_new = (stat / v_new[:, :, :, None]).sum(axis=1) / N
    return v_new, lam_new


def as_weighted_covs(x, v, lam):
    """The matrices inverted in eq. 23, one per column index i:

    Q_i(f) = (1/N) sum_n y y^H / (sum_j v_j(n,f) [Lambda_j(f)]_ii).
    Returns Q [F][I][I][I] with Q[f, i] the I x I matrix of column i.
    """
    x = np.asarray(x, dtype=np.complex128)
    D = np.einsum("fnj,fji->fni", np.asarray(v, np.float64), np.asarray(lam, np.float64))
    N = x.shape[1]
    return np.einsum("fni,fna,fnb->fiab", 1.0 / D, x, np.conj(x)) / N


def as_fpi_step(x, v, lam, P, K=1):
    """Step 2 of the hybrid algorithm: fixed-point update of P(f) (eq. 23).

    [P]_i <- Q_i^-1 [(P^-1)^H]_i for every column i, all columns computed
    from the same current P.  K inner steps reuse the same Q_i.
    """
    P = np.asarray(P, dtype=np.complex128).copy()
    Q = as_weighted_covs(x, v, lam)
    F, I = P.shape[0], P.shape[1]
    for _ in range(K):
        B = _herm(np.linalg.inv(P))                  # (P^-1)^H
        Pn = np.empty_like(P)
        for f in range(F):
            for i in range(I):
                Pn[f, :, i] = np.linalg.solve(Q[f, i], B[f, :, i])
        P = Pn
    return P


def as_gradient_p_step(x, v, lam, P, mu, natural=False):
    """A gradient-type update of P(f) in place of the fixed-point step (the
    alternatives Section 4.5 names).  With g = (1/N) dL2/dP* (eq. 21) at the
    given v, Lambda:

      gradient ascent:               P <- P + mu g
      natural (relative) gradient:   P <- P + mu P P^H g

    The second is the steepest-ascent direction under the metric that makes
    the step equivariant to x -> A x, P -> A^-H P.
    """
    P = np.asarray(P, dtype=np.complex128)
    N = np.asarray(x).shape[1]
    g = as_wirtinger_grad(x, v, lam, P) / N
    if natural:
        return P + mu * np.einsum("fab,fcb,fcd->fad", P, np.conj(P), g)
    return P + mu * g


def fastfca_as_step_grad(x, v, lam, P, mu, natural=False):
    """A hybrid iteration with the gradient-type P update: the EM step on
    (Lambda, v), then as_gradient_p_step with the new (v, Lambda)."""
    v_new, lam_new = as_em_half_step(x, v, lam, P)
    return v_new, lam_new, as_gradient_p_step(x, v_new, lam_new, P, mu, natural)


def fastfca_as_step(x, v, lam, P, K=1):
    """One hybrid iteration of FastFCA-AS (Section 4.3): EM on (Lambda, v),
    then the fixed-point update of P with the new (Lambda, v).

    Returns (v_new, lam_new, P_new).
    """
    v_new, lam_new = as_em_half_step(x, v, lam, P)
    P_new = as_fpi_step(x, v_new, lam_new, P, K=K)
    return v_new, lam_new, P_new


def loglik_as(x, v, lam, P, per_bin=False):
    """Log-likelihood L2 (eq. 14): the Gaussian log-likelihood of y with
    covariance sum_j v_j (P^-1)^H Lambda_j P^-1, i.e. L1 with eq. 12."""
    return loglik_fca(x, v, as_spatial_cov(P, lam), per_bin=per_bin)


def wiener_as(x, v, lam, P):
    """Multichannel Wiener filter (eq. 3) with the covariances of eq. 15.
    Returns [J][F][N][I]."""
    return wiener_fca(x, v, as_spatial_cov(P, lam))


def as_wirtinger_grad(x, v, lam, P):
    """Wirtinger derivative of L2 with respect to conj(P(f)) (eq. 21):

    dL2/dP* = N (P^-1)^H - sum_n y y^H P (sum_j v_j Lambda_j)^-1.
    Returns [F][I][I].
    """
    x = np.asarray(x, dtype=np.complex128)
    P = np.asarray(P, dtype=np.complex128)
    N = x.shape[1]
    D = np.einsum("fnj,fji->fni", np.asarray(v, np.float64), np.asarray(lam, np.float64))
    yyH_P = np.einsum("fna,fnb,fbc->fnac", x, np.conj(x), P)
    return N * _herm(np.linalg.inv(P)) - (yyH_P / D[:, :, None, :]).sum(axis=1)


def as_fpi_dense_vec(x, v, lam, P):
    """The vectorised stationarity condition (eq. 22) used as an update:

    vec(P) <- [ (1/N) sum_n D_n^-1 (kron) y y^H ]^-1 vec((P^-1)^H),
    with vec stacking columns and D_n = sum_j v_j Lambda_j.  A dense
    I^2 x I^2 solve per bin; meant for small I only.
    """
    x = np.asarray(x, dtype=np.complex128)
    P = np.asarray(P, dtype=np.complex128)
    F, N, I = x.shape
    D = np.einsum("fnj,fji->fni", np.asarray(v, np.float64), np.asarray(lam, np.float64))
    out = np.empty_like(P)
    for f in range(F):
        M = np.zeros((I * I, I * I), dtype=np.complex128)
        for n in range(N):
            M += np.kron(np.diag(1.0 / D[f, n]), np.outer(x[f, n], np.conj(x[f, n])))
        M /= N
        rhs = _herm(np.linalg.inv(P[f])).reshape(-1, order="F")
        out[f] = np.linalg.solve(M, rhs).reshape(I, I, order="F")
    return out
