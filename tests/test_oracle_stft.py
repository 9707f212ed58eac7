"""Pins of the STFT front and back end of the oracle (oracle/stft.py):
analysis against a brute-force DFT sum, the window's overlap sum in closed
form, frame coverage, and perfect reconstruction."""

import numpy as np
import pytest

from oracle import stft as S


@pytest.mark.parametrize("W,H", [(16, 8), (16, 4), (32, 4)])
def test_analysis_equals_direct_dft(W, H):
    rng = np.random.default_rng(W + H)
    L = 3 * W + 5
    wav = rng.standard_normal((2, L))
    X = S.stft(wav, W, H)
    F, N = S.stft_shape(L, W, H)
    assert X.shape == (F, N, 2)
    w = np.array([np.sin(np.pi * t / W) for t in range(W)])
    for c in range(2):
        for n in range(N):
            for f in range(F):
                acc = 0j
                for t in range(W):
                    k = n * H - (W - H) + t
                    if 0 <= k < L:
                        acc += w[t] * wav[c, k] * np.exp(-2j * np.pi * f * t / W)
                assert abs(X[f, n, c] - acc) <= 1e-10 * max(1.0, abs(acc))


@pytest.mark.parametrize("W,R", [(16, 2), (64, 4), (1024, 2), (2048, 8)])
def test_squared_window_overlap_sum(W, R):
    H = W // R
    w = S.window(W)
    for t in range(0, H):
        assert abs(sum(w[t + m * H] ** 2 for m in range(R)) - W / (2 * H)) <= 1e-12


@pytest.mark.parametrize("L,W,H", [(1000, 64, 32), (1024, 64, 16), (16000, 1024, 512), (16001, 2048, 256)])
def test_every_sample_covered_by_w_over_h_frames(L, W, H):
    F, N = S.stft_shape(L, W, H)
    cover = np.zeros(L, dtype=int)
    for n in range(N):
        a = n * H - (W - H)
        cover[max(a, 0):min(a + W, L)] += 1
    assert (cover == W // H).all()


@pytest.mark.parametrize("L,W,H", [(777, 16, 8), (5000, 64, 16), (16000, 1024, 512), (20000, 2048, 256)])
def test_perfect_reconstruction(L, W, H):
    rng = np.random.default_rng(L)
    wav = rng.standard_normal((3, L))
    back = S.istft(S.stft(wav, W, H), W, H, L)
    assert np.max(np.abs(back - wav)) <= 1e-11
