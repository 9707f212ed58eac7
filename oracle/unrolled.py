"""Unrolled FastFCA-AS in plain PyTorch (complex128 / float64 on the CPU), the
reference for reverse-mode derivatives.

Test infrastructure only (see the package docstring).  The same steps as
``fastfca_as.py`` (Section 4.3: the EM update of eq. 15-20, then the
fixed-point update of eq. 23) and the multichannel Wiener filter (eq. 3 with
the covariances of eq. 12 and eq. 15), written with torch operations so that
torch's autograd gives the derivative of a loss on the separated images
with respect to the mixture and the initial parameters.  For complex tensors
torch returns dL/dRe z + i dL/dIm z for a real loss L.

Layouts as in the package docstring; the Wiener output is [J][F][N][I].
"""

import torch

C128 = torch.complex128
F64 = torch.float64


def _h(a):
    return a.conj().transpose(-1, -2)


def as_step(x, v, lam, P):
    """One hybrid iteration (Section 4.3), K = 1.

    E-step in the basis y~ = P^H y (eq. 16-17, diagonal), v update (eq. 19)
    with the current Lambda, Lambda update (eq. 20) with the new v, then every
    column of P from the same current P: p_i <- Q_i^-1 [P^-H]_i with
    Q_i = (1/N) sum_n y y^H / (sum_j v_j Lambda_j)_ii (eq. 23).
    """
    N = x.shape[1]
    I = x.shape[2]
    yt = torch.einsum("fki,fnk->fni", P.conj(), x)            # P^H y
    vl = v[:, :, :, None] * lam[:, None, :, :]                # v_j Lambda_j [F][N][J][I]
    D = vl.sum(dim=2)                                         # sum_k v_k Lambda_k
    gain = vl / D[:, :, None, :]
    mu2 = (gain * gain) * (yt.abs() ** 2)[:, :, None, :]      # |mu~_j|^2 (eq. 16)
    phi = vl - vl * gain                                      # diag Phi~_j (eq. 17)
    stat = mu2 + phi
    v_new = (stat / lam[:, None, :, :]).sum(dim=3) / I        # eq. 19
    lam_new = (stat / v_new[:, :, :, None]).sum(dim=1) / N    # eq. 20
    D_new = torch.einsum("fnj,fji->fni", v_new, lam_new)
    Q = torch.einsum("fni,fna,fnb->fiab", (1.0 / D_new).to(C128), x, x.conj()) / N
    B = _h(torch.linalg.inv(P))                               # (P^-1)^H
    cols = [torch.linalg.solve(Q[:, i], B[:, :, i]) for i in range(I)]
    P_new = torch.stack(cols, dim=2)
    return v_new, lam_new, P_new


def spatial_cov(P, lam):
    """S_j = P^-H Lambda_j P^-1 (eq. 12).  [F][J][I][I]"""
    Pinv = torch.linalg.inv(P)
    return torch.einsum("fab,fjb,fbc->fjac", _h(Pinv), lam.to(C128), Pinv)


def wiener(x, v, lam, P):
    """Multichannel Wiener filter (eq. 3): s^_j = v_j S_j C^-1 x with
    C = sum_j v_j S_j and S_j from eq. 12.  Returns [J][F][N][I]."""
    S = spatial_cov(P, lam)
    C = torch.einsum("fnj,fjab->fnab", v.to(C128), S)
    Cx = torch.linalg.solve(C, x.unsqueeze(-1)).squeeze(-1)   # C^-1 x
    s = torch.einsum("fnj,fjab,fnb->jfna", v.to(C128), S, Cx)
    return s


def unrolled(x, v0, lam0, P0, n_iter):
    """n_iter hybrid iterations from (v0, lam0, P0), then the Wiener filter of
    the final parameters.  Returns the images [J][F][N][I]."""
    v, lam, P = v0, lam0, P0
    for _ in range(n_iter):
        v, lam, P = as_step(x, v, lam, P)
    return wiener(x, v, lam, P)


def mse(s_hat, s_ref):
    """Mean squared error over all entries of the images."""
    return (s_hat - s_ref).abs().pow(2).mean()


def unrolled_grads(x, v0, lam0, P0, n_iter, s_ref=None, grad_out=None):
    """Reference derivatives of the unrolled separation.  With s_ref the loss
    is mse(images, s_ref); with grad_out (a tensor of the images' shape) the
    loss is the real inner product Re <grad_out, images>, whose derivative
    with respect to the images is grad_out itself.  Inputs are numpy or torch
    arrays; returns (loss, images, dx, dv0, dlam0, dP0) as torch tensors."""
    x = torch.as_tensor(x).to(C128).clone().requires_grad_(True)
    v0 = torch.as_tensor(v0).to(F64).clone().requires_grad_(True)
    lam0 = torch.as_tensor(lam0).to(F64).clone().requires_grad_(True)
    P0 = torch.as_tensor(P0).to(C128).clone().requires_grad_(True)
    s_hat = unrolled(x, v0, lam0, P0, n_iter)
    if grad_out is not None:
        g = torch.as_tensor(grad_out).to(C128)
        loss = (g.conj() * s_hat).real.sum()
    else:
        loss = mse(s_hat, torch.as_tensor(s_ref).to(C128))
    loss.backward()
    return loss.detach(), s_hat.detach(), x.grad, v0.grad, lam0.grad, P0.grad
