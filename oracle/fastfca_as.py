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


def as_newton_p_step(x, v, lam, P):
    """Newton's method in place of the fixed-point P update (an alternative
    Section 4.5 names): one full Newton step on L2 (eq. 14) as a function of
    P(f) alone, v and Lambda held, no damping or line search.

    Per bin, with Q_i the matrices of eq. 23, L2 / N equals, up to terms free
    of P,  f(P) = 2 ln|det P| - sum_i p_i^H Q_i p_i.  Its derivatives along
    complex directions E, F (I x I) are
      df[E]      = 2 Re tr(G^H E),   G = P^-H - [Q_1 p_1, ..., Q_I p_I]
                                        = (1/N) dL2/dP*  (eq. 21),
      d2f[E, F]  = -2 Re tr(P^-1 E P^-1 F) - 2 sum_i Re(E_i^H Q_i F_i).
    f does not change when a column of P is multiplied by a unit complex
    number, so the Hessian is singular along E = P i D (D real diagonal).
    The step is taken in the relative form P + P X (the form of the other P
    updates) over the real directions U of X other than the imaginary
    diagonal entries (the columns' phases are left alone to first order):
    with E_k = P U_k the reduced Hessian H_kl = d2f[E_k, E_l] and gradient
    g_k = df[E_k] are formed entry by entry, H s = -g is solved densely and
    P + P sum_k s_k U_k is returned.
    """
    P = np.asarray(P, dtype=np.complex128)
    basis = newton_directions(P.shape[1])
    out = np.empty_like(P)
    for f, (H, grad) in enumerate(as_newton_system(x, v, lam, P)):
        step = np.linalg.solve(H, -grad)
        X = sum(w * U for w, U in zip(step, basis))
        out[f] = P[f] + P[f] @ X
    return out


def as_newton_system(x, v, lam, P):
    """The reduced Hessian and gradient of Newton's P step (see
    as_newton_p_step), one (H, g) pair per bin, over the directions
    P U_k with U_k from newton_directions."""
    x = np.asarray(x, dtype=np.complex128)
    P = np.asarray(P, dtype=np.complex128)
    F, I = P.shape[0], P.shape[1]
    Q = as_weighted_covs(x, v, lam)                      # [F][i][I][I]
    basis = newton_directions(I)
    systems = []
    for f in range(F):
        Pinv = np.linalg.inv(P[f])
        G = _herm(Pinv) - np.stack([Q[f, i] @ P[f, :, i] for i in range(I)], axis=1)
        dirs = [P[f] @ U for U in basis]
        grad = np.array([2.0 * np.real(np.trace(_herm(G) @ E)) for E in dirs])
        H = np.empty((len(dirs), len(dirs)))
        for k, E in enumerate(dirs):
            for l, Fd in enumerate(dirs):
                quad = sum(np.real(np.conj(E[:, i]) @ Q[f, i] @ Fd[:, i]) for i in range(I))
                H[k, l] = -2.0 * np.real(np.trace(Pinv @ E @ Pinv @ Fd)) - 2.0 * quad
        systems.append((H, grad))
    return systems


def newton_directions(I):
    """The real directions of X in Newton's P step: a unit real entry at
    every (a, c), a unit imaginary entry at every (a, c) with a != c."""
    basis = []
    for part in (1.0, 1j):
        for a in range(I):
            for c in range(I):
                if part == 1j and a == c:
                    continue
                U = np.zeros((I, I), dtype=np.complex128)
                U[a, c] = part
                basis.append(U)
    return basis


def as_em_p_step(x, v, lam, P, sweeps=1):
    """The normal EM algorithm with P in the M-step (named in Section 4.5):
    the E-step at (v, Lambda, P) gives the posterior moments of every source
    image in the basis of x (eq. 7-8 with the covariances of eq. 12); the
    M-step raises the Q-function (eq. 18) over v and Lambda (eq. 19-20 with
    the current P) and then over P with the new v, Lambda.

    As a function of P, Q is  2NJ ln|det P| - NJ sum_i p_i^H V_i p_i + const
    with V_i = (1/(NJ)) sum_{n,j} (mu_j mu_j^H + Phi_j) / (v_j lambda_ji)
    (new v, Lambda).  The column update p_i <- V_i^-1 [P^-H]_i rescaled to
    p_i^H V_i p_i = 1 maximises Q over p_i with the other columns held
    (iterative projection); `sweeps` passes over i = 1..I, each column using
    the P that the previous columns left.  Every step raises Q, so the
    iteration is a generalised EM algorithm.  Returns (v, Lambda, P).
    """
    from .fca import fca_estep
    x = np.asarray(x, dtype=np.complex128)
    P = np.asarray(P, dtype=np.complex128).copy()
    F, N, I = x.shape
    mu, Phi = fca_estep(x, np.asarray(v, np.float64), as_spatial_cov(P, lam))
    v_new, lam_new = as_em_half_step(x, v, lam, P)
    J = v_new.shape[2]
    M = np.einsum("fnja,fnjb->fnjab", mu, np.conj(mu)) + Phi
    V = np.einsum("fnjab,fnj,fji->fiab", M, 1.0 / v_new, 1.0 / lam_new) / (N * J)
    for _ in range(sweeps):
        for i in range(I):
            b = _herm(np.linalg.inv(P))[:, :, i]
            p = np.linalg.solve(V[:, i], b[..., None])[..., 0]
            scale = np.sqrt(np.real(np.einsum("fa,fab,fb->f", np.conj(p), V[:, i], p)))
            P[:, :, i] = p / scale[:, None]
    return v_new, lam_new, P


def fastfca_as_step_newton(x, v, lam, P):
    """A hybrid iteration with Newton's P update: the EM step on (Lambda, v),
    then as_newton_p_step with the new (v, Lambda)."""
    v_new, lam_new = as_em_half_step(x, v, lam, P)
    return v_new, lam_new, as_newton_p_step(x, v_new, lam_new, P)


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
