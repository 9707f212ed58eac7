"""The seeded generator draws from the model of eq. 1-2 (statistical checks),
is deterministic per seed, and returns positive, well-formed initial values."""

import numpy as np
import pytest

from paper_1805_09498_amd import synth


def test_deterministic_per_seed():
    a = synth.make_problem(3, 3, 4, 10, seed=5)
    b = synth.make_problem(3, 3, 4, 10, seed=5)
    c = synth.make_problem(3, 3, 4, 10, seed=6)
    np.testing.assert_array_equal(a.x, b.x)
    np.testing.assert_array_equal(a.P0, b.P0)
    assert not np.array_equal(a.x, c.x)


def test_mixture_is_sum_of_images_and_shapes():
    p = synth.make_problem(3, 4, 5, 12, seed=1, with_sources=True)
    assert p.x.shape == (5, 12, 3) and p.v0.shape == (5, 12, 4)
    assert p.lam0.shape == (5, 4, 3) and p.P0.shape == (5, 3, 3)
    np.testing.assert_allclose(p.s.sum(axis=0), p.x, atol=1e-12)
    assert (p.v0 > 0).all() and (p.lam0 > 0).all()


@pytest.mark.parametrize("spatial", ["rank1", "ula"])
def test_image_covariance_is_v_times_R(spatial):
    """(1/N) sum_n s s^H / v -> R_j(f)  as N grows (eq. 2)."""
    p = synth.make_problem(3, 2, 2, 40000, seed=3, spatial=spatial, with_sources=True)
    for j in range(2):
        for f in range(2):
            s = p.s[j, f]
            w = 1.0 / np.sqrt(p.v_true[f, :, j])
            emp = np.einsum("na,nb->ab", s * w[:, None], np.conj(s * w[:, None])) / s.shape[0]
            np.testing.assert_allclose(emp, p.R_true[f, j], atol=0.03)


def test_gamma_psd_moments():
    rng = np.random.default_rng(0)
    v = synth.psd_gamma(rng, 4, 50000, 2)
    assert v.mean() == pytest.approx(0.5, rel=0.02)
    assert v.var() == pytest.approx(0.5, rel=0.05)


def test_lognormal_psd_sparsity():
    rng = np.random.default_rng(0)
    v = synth.psd_lognormal_sparse(rng, 4, 50000, 2)
    assert (v == 0).mean() == pytest.approx(0.3, abs=0.01)
    nz = np.log(v[v > 0])
    assert nz.mean() == pytest.approx(0.0, abs=0.02)
    assert nz.std() == pytest.approx(1.5, rel=0.02)


def test_ula_covariances_are_hermitian_pd_with_unit_diffuse_diagonal():
    rng = np.random.default_rng(1)
    R = synth.spatial_ula(rng, 9, 3, 6)
    np.testing.assert_allclose(R, np.conj(np.swapaxes(R, -1, -2)), atol=1e-14)
    assert (np.linalg.eigvalsh(R) > 0).all()
    np.testing.assert_allclose(np.real(np.diagonal(R, axis1=-2, axis2=-1)), 1.0 + 0.2 + 1e-3)


def test_uneven_batch_ranges():
    mixes = synth.make_batch(n_mix=12, F=9)
    for p in mixes:
        F, N, I, J = p.shape
        assert I in (2, 3, 4, 6) and 2 <= J <= I + 1 and 200 <= N <= 2000 and F == 9


def test_waveform_mixture_is_the_sum_of_images_and_seeded():
    mix, images = synth.make_waveforms(3, 2, 4000, seed=5, rir_len=64)
    assert mix.shape == (3, 4000) and images.shape == (2, 3, 4000)
    np.testing.assert_allclose(mix, images.sum(axis=0), rtol=0, atol=1e-12)
    mix2, _ = synth.make_waveforms(3, 2, 4000, seed=5, rir_len=64)
    np.testing.assert_array_equal(mix, mix2)
