"""GPU tests of the STFT front and back end (fca_stft / fca_istft) against
the FP64 oracle (oracle/stft.py), and of the whole waveform-to-waveform
separation (STFT, FastFCA-AS iterations, Wiener filter, overlap-add).

Tolerance: relative Frobenius error <= 1e-5 for the transforms (a radix-2
FP32 FFT of length W loses ~log2(W) * 6e-8 relative; W <= 2048 gives
<= 7e-7) and <= 1e-4 after the separation, the parameter tolerance of the
iterations.  Entry by entry: a radix-2 FFT of length W has a norm-wise
relative error of at most log2(W) (gamma(4) (sqrt 2 + mu) + mu), mu the
twiddles' error (Higham, ch. 24); per frame that bounds every bin of the
analysis by gamma(8 log2 W + 8) sqrt(2) |X_frame| (Parseval over the half
spectrum), and every synthesised sample by
2 gamma(8 log2 W + 12) sqrt(2 / W) max_frame |S_frame| (W / hop frames
overlap, each scaled by 2 hop / W)."""

import numpy as np
import pytest
import torch

import oracle
from oracle import stft as S
from paper_1805_09498_amd import synth
from tests import error_bounds as EB
from tests.gpu_common import check, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ff():
    assert torch.cuda.is_available()
    from paper_1805_09498_amd import fastfca
    return fastfca


def f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


@pytest.mark.parametrize("C,L,W,H", [(3, 16000, 1024, 512), (2, 20001, 2048, 256), (1, 777, 16, 8), (4, 5000, 64, 16)])
def test_stft_matches_oracle(ff, C, L, W, H):
    rng = np.random.default_rng(L)
    wav = f32(rng.standard_normal((C, L)))
    X = ff.fca_stft(torch.from_numpy(wav.astype(np.float32)).cuda(), W, H)
    torch.cuda.synchronize()
    ref = S.stft(wav, W, H)
    assert X.shape == ref.shape
    bound = EB.gamma(8 * int(np.log2(W)) + 8) * np.sqrt(2.0) * np.linalg.norm(ref, axis=0, keepdims=True)
    check(f"stft C{C} L{L} W{W} H{H}", X.cpu().numpy(), ref, bound, 1e-5)


@pytest.mark.parametrize("J,C,L,W,H", [(3, 3, 16000, 1024, 512), (2, 2, 9000, 2048, 256), (1, 1, 100, 16, 4)])
def test_istft_matches_oracle(ff, J, C, L, W, H):
    F, N = S.stft_shape(L, W, H)
    rng = np.random.default_rng(W + L)
    spec = (rng.standard_normal((J, F, N, C)) + 1j * rng.standard_normal((J, F, N, C))).astype(np.complex64)
    out = ff.fca_istft(torch.from_numpy(spec).cuda(), L, W, H)
    torch.cuda.synchronize()
    ref = np.stack([S.istft(spec[j].astype(np.complex128), W, H, L) for j in range(J)])
    smax = np.linalg.norm(spec.astype(np.complex128), axis=1).max(axis=1)          # [J][C]
    bound = 2.0 * EB.gamma(8 * int(np.log2(W)) + 12) * np.sqrt(2.0 / W) * smax[:, :, None]
    check(f"istft J{J} C{C} L{L} W{W} H{H}", out.cpu().numpy(), ref, bound, 1e-5)


@pytest.mark.parametrize("W,H", [(1024, 512), (2048, 256)])
def test_round_trip(ff, W, H):
    mix, _ = synth.make_waveforms(3, 2, 12345, seed=3)
    wav = torch.from_numpy(mix.astype(np.float32)).cuda()
    back = ff.fca_istft(ff.fca_stft(wav, W, H).unsqueeze(0), mix.shape[1], W, H)[0]
    torch.cuda.synchronize()
    assert rel(back.cpu().numpy(), wav.cpu().numpy()) <= 1e-5


def test_waveform_separation_pipeline(ff):
    """Waveforms in, separated waveforms out: 2 s of a 3-microphone, 3-source
    mixture (16 kHz, frame 1024, shift 512), 5 FastFCA-AS iterations, Wiener
    filter, overlap-add; against the same pipeline in the oracle, and the
    separated waveforms sum to the input."""
    I, J, L, W, H, T = 3, 3, 32000, 1024, 512, 5
    mix, _ = synth.make_waveforms(I, J, L, seed=11)
    wav = f32(mix)
    X = ff.fca_stft(torch.from_numpy(wav.astype(np.float32)).cuda(), W, H)
    x64 = S.stft(wav, W, H)
    v0, lam0, P0 = synth.init_params(X.cpu().numpy().astype(np.complex128), J, 12)
    v0, lam0, P0 = f32(v0), f32(lam0), np.asarray(P0, np.complex64).astype(np.complex128)
    ctx = ff.fca_init(ff.FCA_METHOD_AS, X, torch.from_numpy(v0.astype(np.float32)).cuda(),
                      torch.from_numpy(lam0.astype(np.float32)).cuda(),
                      torch.from_numpy(P0.astype(np.complex64)).cuda())
    ff.fastfca_as_iterate(ctx, T)
    out = ff.fca_istft(ff.fca_wiener_separate(ctx), L, W, H)
    torch.cuda.synchronize()
    got = out.cpu().numpy().astype(np.float64)
    assert rel(got.sum(axis=0), wav) <= 1e-5
    xr = X.cpu().numpy().astype(np.complex128)       # the oracle separates the GPU's spectrum
    assert rel(xr, x64) <= 1e-5
    v, lam, P = v0, lam0, P0
    for _ in range(T):
        v, lam, P = oracle.fastfca_as_step(xr, v, lam, P)
    ref = S.separate_waveforms(oracle.wiener_as(xr, v, lam, P), W, H, L)
    assert rel(got, ref) <= 1e-4
