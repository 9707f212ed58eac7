"""GPU tests of the on-disk launch-shape cache (FASTFCA_TUNE_CACHE): the
tuner appends what it measured, and a later lookup takes a stored shape
without measuring again."""

import os

import pytest

from tests.gpu_common import problem, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture()
def cache_file(tmp_path):
    path = tmp_path / "tune.txt"
    old = os.environ.get("FASTFCA_TUNE_CACHE")
    os.environ["FASTFCA_TUNE_CACHE"] = str(path)
    yield path
    if old is None:
        del os.environ["FASTFCA_TUNE_CACHE"]
    else:
        os.environ["FASTFCA_TUNE_CACHE"] = old


def lines_with(path, needle):
    if not path.exists():
        return []
    return [l for l in path.read_text().splitlines() if needle in l]


def iterate_once(ff, I, J, F, N, seed):
    t = to_dev(problem(I, J, F, N, seed))
    ctx = ff.fca_init(ff.FCA_METHOD_AS, t["x"], t["v0"], t["lam0"], t["P0"])
    ff.fastfca_as_iterate(ctx, 1)
    return ctx


def test_measured_shape_is_stored_and_reused(cache_file):
    from paper_1805_09498_amd import fastfca as ff
    # shapes no other test tunes, so the in-process cache is empty for them
    iterate_once(ff, 2, 2, 7, 53, seed=41)
    stored = lines_with(cache_file, " as I=2 J=2 F=7 N=53 ")
    assert len(stored) == 1
    key, val = stored[0].split("\t")
    # plant an entry for another shape (the same key with J = 3); the tuner
    # must take it as it is
    other = key.replace(" J=2 ", " J=3 ")
    with open(cache_file, "a") as f:
        f.write(f"{other}\t4 2\n")
    ctx = iterate_once(ff, 2, 3, 7, 53, seed=42)
    assert ff.fca_get_option(ctx, "last_waves") == 4
    assert ff.fca_get_option(ctx, "last_bins_per_wg") == 2
    assert len(lines_with(cache_file, " as I=2 J=3 F=7 N=53 ")) == 1   # not measured again


def test_entry_that_does_not_fit_is_measured(cache_file):
    from paper_1805_09498_amd import fastfca as ff
    iterate_once(ff, 1, 2, 5, 61, seed=43)
    key = lines_with(cache_file, " as I=1 J=2 F=5 N=61 ")[0].split("\t")[0]
    other = key.replace(" J=2 ", " J=3 ")
    with open(cache_file, "a") as f:
        f.write(f"{other}\t1 2\n")   # 2 bins per workgroup need >= 2 waves
    ctx = iterate_once(ff, 1, 3, 5, 61, seed=44)
    assert (ff.fca_get_option(ctx, "last_waves"), ff.fca_get_option(ctx, "last_bins_per_wg")) != (1, 2)
    assert len(lines_with(cache_file, " as I=1 J=3 F=5 N=61 ")) == 2   # measured and appended
