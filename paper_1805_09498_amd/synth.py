"""Seeded synthetic STFT-domain workloads for FCA / FastFCA-AS.

This module draws inputs only: it holds none of the estimation arithmetic
(no covariance models of the method, no E/M steps, no likelihoods).  Both the
HIP library's callers and the FP64 oracle are fed the arrays it returns.

Generative model (Section 3.1 of the paper, eq. 1-2): each source image is
s_j(n,f) ~ CN(0, v_j(n,f) R_j(f)), independent over (j, n, f), and the mixture
is x(n,f) = sum_j s_j(n,f).  The paper's speech recordings and measured room
impulse responses are not available; these draws stand in for them:

  * ``rank1``:  R_j(f) = a a^H + 0.1 I with a = g/|g|, g ~ CN(0, I) drawn
    independently per (j, f).
  * ``ula``:    R_j(f) = a_j(f) a_j(f)^H + 0.2 Gamma(f) + 1e-3 I, with a_j(f) a
    far-field plane wave on a uniform linear array (4 cm spacing, c = 343 m/s,
    16 kHz sampling, direction of arrival ~ U[-80, 80] degrees per source) and
    Gamma_ab(f) = sin(w d_ab / c) / (w d_ab / c) the diffuse-field coherence.
  * ``gamma`` PSD:     v_j(n,f) ~ Gamma(shape 0.5, scale 1), i.i.d.
  * ``lognormal`` PSD: v_j(n,f) = exp(1.5 g), g ~ N(0,1), then 30 % of the
    entries set to zero (sparse, heavy-tailed spectra).

Initial parameters (the paper initialises from masks of another method,
which is not available): P(f) = I + 0.1 G with G_ab ~ CN(0,1);
lambda_{jf,i} ~ U[0.5, 1.5]; v_j(n,f) = (|x(n,f)|^2/I + 1e-3 mean_n |x|^2/I)
* U[0.5, 1.5].  All are strictly positive / non-singular with probability 1.

Random streams: ``numpy.random.SeedSequence(seed).spawn(4)`` gives the child
streams (steering, psd, noise, init) in that order.

Layouts (the library's ABI layouts):
    x [F][N][I] complex, v [F][N][J], lam [F][J][I], P [F][I][I] (row-major),
    s [J][F][N][I] complex (ground-truth images, optional).
"""

import dataclasses

import numpy as np

FS_HZ = 16000.0
SOUND_SPEED = 343.0
ULA_SPACING = 0.04


@dataclasses.dataclass
class Problem:
    x: np.ndarray        # [F][N][I] complex128
    v0: np.ndarray       # [F][N][J] float64
    lam0: np.ndarray     # [F][J][I] float64
    P0: np.ndarray       # [F][I][I] complex128
    s: np.ndarray = None  # [J][F][N][I] complex128 (optional)
    v_true: np.ndarray = None   # [F][N][J]
    R_true: np.ndarray = None   # [F][J][I][I]

    @property
    def shape(self):
        F, N, I = self.x.shape
        return F, N, I, self.v0.shape[2]

    def rounded_c64(self):
        """The same problem rounded to complex64/float32 and widened back to
        FP64, i.e. exactly the values a single-precision consumer sees."""
        return Problem(
            x=self.x.astype(np.complex64).astype(np.complex128),
            v0=self.v0.astype(np.float32).astype(np.float64),
            lam0=self.lam0.astype(np.float32).astype(np.float64),
            P0=self.P0.astype(np.complex64).astype(np.complex128),
            s=None if self.s is None else self.s.astype(np.complex64).astype(np.complex128),
            v_true=self.v_true, R_true=self.R_true)


def _cn(rng, shape):
    """Circular complex normal CN(0, 1) samples."""
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / np.sqrt(2.0)


def spatial_rank1(rng, F, J, I):
    g = _cn(rng, (F, J, I))
    a = g / np.linalg.norm(g, axis=-1, keepdims=True)
    return np.einsum("fja,fjb->fjab", a, np.conj(a)) + 0.1 * np.eye(I)


def spatial_ula(rng, F, J, I):
    doa = np.deg2rad(rng.uniform(-80.0, 80.0, size=J))
    f_hz = np.arange(F) * FS_HZ / (2.0 * max(F - 1, 1))
    m = np.arange(I)
    delay = m[None, :] * ULA_SPACING * np.sin(doa)[:, None] / SOUND_SPEED    # [J][I]
    a = np.exp(-2j * np.pi * f_hz[:, None, None] * delay[None, :, :])       # [F][J][I]
    dist = np.abs(m[:, None] - m[None, :]) * ULA_SPACING                    # [I][I]
    coh = np.sinc(2.0 * f_hz[:, None, None] * dist[None] / SOUND_SPEED)      # sin(wd/c)/(wd/c)
    return (np.einsum("fja,fjb->fjab", a, np.conj(a))
            + 0.2 * coh[:, None, :, :] + 1e-3 * np.eye(I))


def psd_gamma(rng, F, N, J):
    return rng.gamma(shape=0.5, scale=1.0, size=(F, N, J))


def psd_lognormal_sparse(rng, F, N, J):
    v = np.exp(1.5 * rng.standard_normal((F, N, J)))
    v[rng.uniform(size=(F, N, J)) < 0.3] = 0.0
    return v


def make_problem(I, J, F, N, seed, spatial="rank1", psd="gamma",
                 with_sources=False, chunk=32):
    """Draw one mixture and its initial parameters (see the module docstring)."""
    if min(I, J, F, N) < 1:
        raise ValueError("I, J, F, N must be positive")
    ss = np.random.SeedSequence(seed).spawn(4)
    rng_steer, rng_psd, rng_noise, rng_init = (np.random.default_rng(s) for s in ss)
    R = {"rank1": spatial_rank1, "ula": spatial_ula}[spatial](rng_steer, F, J, I)
    v = {"gamma": psd_gamma, "lognormal": psd_lognormal_sparse}[psd](rng_psd, F, N, J)
    L = np.linalg.cholesky(R)                                  # R = L L^H
    x = np.zeros((F, N, I), dtype=np.complex128)
    s = np.zeros((J, F, N, I), dtype=np.complex128) if with_sources else None
    for f0 in range(0, F, chunk):
        f1 = min(F, f0 + chunk)
        z = _cn(rng_noise, (f1 - f0, N, J, I))
        sj = np.sqrt(v[f0:f1, :, :, None]) * np.einsum("fjab,fnjb->fnja", L[f0:f1], z)
        x[f0:f1] = sj.sum(axis=2)
        if with_sources:
            s[:, f0:f1] = np.moveaxis(sj, 2, 0)
    v0, lam0, P0 = init_params(x, J, rng_init)
    return Problem(x=x, v0=v0, lam0=lam0, P0=P0, s=s, v_true=v, R_true=R)


def init_params(x, J, rng_or_seed):
    """Seeded initial parameters for a mixture x [F][N][I] (no estimation):
    P = 1 + 0.1 G with G complex normal, lambda ~ U[0.5, 1.5], and
    v = (|x|^2 / I + 1e-3 mean_n |x|^2 / I) U[0.5, 1.5].  Returns (v0, lam0, P0)."""
    rng = np.random.default_rng(rng_or_seed)
    F, N, I = x.shape
    P0 = np.eye(I) + 0.1 * _cn(rng, (F, I, I))
    lam0 = rng.uniform(0.5, 1.5, size=(F, J, I))
    pw = (np.abs(x) ** 2).sum(axis=2) / I                      # [F][N]
    base = pw + 1e-3 * pw.mean(axis=1, keepdims=True)
    base = np.where(base > 0, base, 1e-6)
    v0 = base[:, :, None] * rng.uniform(0.5, 1.5, size=(F, N, J))
    return v0, lam0, P0


def random_hpd(rng_or_seed, F, J, I, ridge=0.1):
    """Random Hermitian positive-definite matrices A A^H + ridge*I, [F][J][I][I]
    (an initial S_j for FCA drawn independently of any P, lambda)."""
    rng = np.random.default_rng(rng_or_seed)
    A = _cn(rng, (F, J, I, I))
    return np.einsum("fjab,fjcb->fjac", A, np.conj(A)) / I + ridge * np.eye(I)


# Named workloads.  ``iters`` is the iteration count each is run for.
CONFIGS = {
    "small":      dict(I=3, J=3, F=129, N=100, iters=10, spatial="rank1", psd="gamma", seed=1000),
    "paper":      dict(I=3, J=3, F=512, N=249, iters=20, spatial="rank1", psd="gamma", seed=1500),
    "speech10s":  dict(I=3, J=3, F=513, N=626, iters=100, spatial="rank1", psd="gamma", seed=2000),
    "long6x4":    dict(I=6, J=4, F=1025, N=3750, iters=50, spatial="ula", psd="lognormal", seed=3000),
    "long8x6":    dict(I=8, J=6, F=1025, N=3750, iters=50, spatial="ula", psd="lognormal", seed=3001),
    "unrolled":   dict(I=3, J=3, F=257, N=500, iters=20, spatial="rank1", psd="gamma", seed=5000),
}


def make_config(name, **override):
    cfg = dict(CONFIGS[name])
    cfg.update(override)
    cfg.pop("iters")
    return make_problem(cfg.pop("I"), cfg.pop("J"), cfg.pop("F"), cfg.pop("N"),
                        cfg.pop("seed"), **cfg)


def make_batch(n_mix=64, F=513, seed=4000, n_range=(200, 2000), i_choices=(2, 3, 4, 6)):
    """Uneven batch: N ~ U[200, 2000], I in {2,3,4,6}, J ~ U[2, I+1] per
    mixture, Gamma(0.5) PSDs and plane-wave + diffuse spatial covariances."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n_mix):
        I = int(rng.choice(i_choices))
        J = int(rng.integers(2, I + 2))
        N = int(rng.integers(n_range[0], n_range[1] + 1))
        out.append(make_problem(I, J, F, N, seed=seed * 1000 + k, spatial="ula", psd="gamma"))
    return out


def make_waveforms(I, J, L, seed, rir_len=256, fs=16000):
    """Multichannel mixture waveforms: J sources (white noise under a slow
    random envelope, a stand-in for speech), each filtered by I random room
    responses (exponentially decaying noise, rir_len taps, a direct path at
    tap 0) and summed.  Returns (mix [I][L], images [J][I][L]) in float64."""
    rng = np.random.default_rng(np.random.SeedSequence(seed).spawn(1)[0])
    t = np.arange(L) / fs
    images = np.zeros((J, I, L))
    for j in range(J):
        env = np.zeros(L)
        for k in range(4):                        # a few slow modulations per source
            env += rng.uniform(0.2, 1.0) * (1 + np.sin(2 * np.pi * rng.uniform(0.5, 4.0) * t + rng.uniform(0, 2 * np.pi)))
        src = rng.standard_normal(L) * env
        for i in range(I):
            h = rng.standard_normal(rir_len) * np.exp(-np.arange(rir_len) / (rir_len / 6.0))
            h[0] = 1.0
            images[j, i] = np.convolve(src, h)[:L]
    return images.sum(axis=0), images
