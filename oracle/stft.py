"""STFT analysis and overlap-add synthesis (the front and back end of the
experiments, Table 1 of the paper: 16 kHz, frames of 1024 samples, shift 512,
square root of a Hann window for analysis and synthesis), FP64 numpy.

Test infrastructure only (see the package docstring).

Framing (a reading: the paper gives frame length, shift and window only):
frame n covers samples n*H - (W - H) ... n*H - (W - H) + W - 1, samples
outside [0, L) are zero, and N = floor((L - 1 + W - H) / H) + 1, so that
every sample is covered by W / H frames.  The window is the periodic Hann
window's square root, w[t] = sin(pi t / W).  Bins f = 0 .. W/2 (F = W/2 + 1)
of X(n, f) = sum_t w[t] s[n H - (W - H) + t] exp(-2 pi i f t / W).

Synthesis: s[t] = (2H / W) sum_n w[t - n H + (W - H)] * irfft(X(n, .))[...],
the inverse of the analysis for H = W / R, R >= 2 (the squared window of
consecutive frames sums to W / (2H)).

Layouts: waveforms [C][L]; spectra [F][N][C] complex (the mixture layout of
the package docstring).
"""

import numpy as np


def stft_shape(L, W, H):
    """(F, N) of an L-sample signal."""
    return W // 2 + 1, (L - 1 + W - H) // H + 1


def window(W):
    return np.sin(np.pi * np.arange(W) / W)


def stft(wav, W, H):
    """wav [C][L] real -> X [F][N][C] complex128."""
    wav = np.asarray(wav, dtype=np.float64)
    C, L = wav.shape
    F, N = stft_shape(L, W, H)
    pad0 = W - H
    total = (N - 1) * H + W
    buf = np.zeros((C, total))
    buf[:, pad0:pad0 + L] = wav
    w = window(W)
    frames = np.stack([buf[:, n * H:n * H + W] * w for n in range(N)], axis=1)   # [C][N][W]
    X = np.fft.rfft(frames, axis=-1)                                              # [C][N][F]
    return np.transpose(X, (2, 1, 0))


def istft(X, W, H, L):
    """X [F][N][C] complex -> wav [C][L] real (the inverse of stft)."""
    X = np.asarray(X, dtype=np.complex128)
    F, N, C = X.shape
    assert F == W // 2 + 1
    frames = np.fft.irfft(np.transpose(X, (2, 1, 0)), n=W, axis=-1)            # [C][N][W]
    w = window(W)
    total = (N - 1) * H + W
    buf = np.zeros((C, total))
    for n in range(N):
        buf[:, n * H:n * H + W] += frames[:, n] * w
    pad0 = W - H
    return buf[:, pad0:pad0 + L] * (2.0 * H / W)


def separate_waveforms(images, W, H, L):
    """Separated images [J][F][N][I] -> waveforms [J][I][L]."""
    return np.stack([istft(images[j], W, H, L) for j in range(images.shape[0])])
