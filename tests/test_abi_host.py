"""CPU-side checks of the C ABI: the built library loads, exports every
function that include/fastfca.h declares, and rejects bad arguments on the
host before touching any device (no GPU is needed for these calls)."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fastfca.h")
LIB = os.path.join(ROOT, "paper_1805_09498_amd", "libfastfca.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libfastfca.so not built")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(f[a-z_0-9]+)\s*\(", text, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    L = ctypes.CDLL(LIB)
    vp, i = ctypes.c_void_p, ctypes.c_int
    L.fca_init.argtypes = [ctypes.POINTER(vp), i, i, i, i, i, vp, vp, vp, vp, vp, vp]
    L.fca_init.restype = i
    L.fca_last_error.argtypes = [vp]
    L.fca_last_error.restype = ctypes.c_char_p
    L.fca_set_option.argtypes = [vp, ctypes.c_char_p, ctypes.c_longlong]
    L.fca_set_option.restype = i
    for name in ("fastfca_as_iterate", "fca_em_iterate"):
        getattr(L, name).argtypes = [vp, i]
        getattr(L, name).restype = i
    L.fca_loglik.argtypes = [vp, ctypes.POINTER(ctypes.c_double)]
    L.fca_loglik.restype = i
    L.fca_destroy.argtypes = [vp]
    L.fca_destroy.restype = None
    return L


def test_header_declares_the_expected_calls():
    assert declared_functions() == sorted([
        "fca_init", "fastfca_as_iterate", "fca_em_iterate", "fca_wiener_separate",
        "fca_loglik", "fca_loglik_device", "fca_loglik_bins", "fca_get_params", "fca_set_params", "fca_set_option",
        "fca_get_option", "fca_set_option_f64", "fca_get_option_f64", "fca_last_error", "fca_destroy",
        "fca_batch_init", "fca_batch_iterate", "fca_batch_context", "fca_batch_set_option",
        "fca_batch_get_option", "fca_batch_last_error", "fca_batch_destroy",
        "fastfca_as_forward", "fastfca_as_backward", "fca_stft_shape", "fca_stft", "fca_istft",
        "fastfca_as_run_noalloc"])


def test_every_declared_function_is_exported(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_loglik_device_rejects_a_null_context_on_the_host(lib):
    lib.fca_loglik_device.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    lib.fca_loglik_device.restype = ctypes.c_int
    assert lib.fca_loglik_device(None, FAKE) == -1


FAKE = 0x10000  # aligned, never dereferenced: every case below fails validation first


def _init(lib, method=0, F=4, N=8, I=3, J=3, x=FAKE, v=FAKE, lam=FAKE, P=FAKE, R=None):
    h = ctypes.c_void_p(123)
    st = lib.fca_init(ctypes.byref(h), method, F, N, I, J, x, v, lam, P, R, None)
    return st, h.value


@pytest.mark.parametrize("kw,code", [
    (dict(I=9), -2), (dict(J=10), -2), (dict(I=0), -1), (dict(F=0), -1),
    (dict(N=2, I=3), -1), (dict(x=None), -1), (dict(P=None), -1),
    (dict(x=FAKE + 4), -1), (dict(v=FAKE + 2), -1), (dict(method=7), -1),
    (dict(R=FAKE), -1),                      # AS contexts take no R0
    (dict(F=1 << 20, N=1 << 12), -1),        # size limit
])
def test_init_rejects_bad_arguments_on_the_host(lib, kw, code):
    st, h = _init(lib, **kw)
    assert st == code
    assert h is None
    assert len(lib.fca_last_error(None)) > 0


def test_null_context_calls(lib):
    assert lib.fastfca_as_iterate(None, 1) == -1
    assert lib.fca_em_iterate(None, 1) == -1
    assert lib.fca_set_option(None, b"K", 1) == -1
    d = ctypes.c_double()
    assert lib.fca_loglik(None, ctypes.byref(d)) == -1
    lib.fca_destroy(None)
    assert lib.fca_init(None, 0, 1, 1, 1, 1, FAKE, FAKE, FAKE, FAKE, None, None) == -1


def test_batch_init_rejects_bad_arguments(lib):
    lib.fca_batch_init.restype = ctypes.c_int
    h = ctypes.c_void_p(5)
    assert lib.fca_batch_init(ctypes.byref(h), 0, None, None, None, None, None, None, None, None, None) == -1
    assert h.value is None
    n = 2
    ints = (ctypes.c_int * n)(4, 4)
    bad_i = (ctypes.c_int * n)(3, 9)        # I = 9 unsupported for mixture 1
    ptr = (ctypes.c_void_p * n)(FAKE, FAKE)
    st = lib.fca_batch_init(ctypes.byref(h), n, ints, (ctypes.c_int * n)(2, 2), (ctypes.c_int * n)(3, 3), ints,
                            ptr, ptr, ptr, ptr, None)
    assert st == -1   # N = 2 < I = 3 for mixture 0: rejected before any device work
    lib.fca_batch_last_error.restype = ctypes.c_char_p
    lib.fca_batch_last_error.argtypes = [ctypes.c_void_p]
    assert b"mixture 0" in lib.fca_batch_last_error(None)
    st = lib.fca_batch_init(ctypes.byref(h), n, ints, (ctypes.c_int * n)(8, 8), bad_i, ints,
                            ptr, ptr, ptr, ptr, None)
    assert st == -2   # I = 9 in mixture 1: every mixture is checked before any device work
    assert b"mixture 1" in lib.fca_batch_last_error(None)


def test_null_context_derivative_calls(lib):
    vp = ctypes.c_void_p
    lib.fastfca_as_forward.argtypes = [vp, ctypes.c_int, ctypes.c_int, vp]
    lib.fastfca_as_backward.argtypes = [vp, vp, vp, vp, vp, vp]
    assert lib.fastfca_as_forward(None, 3, 1, None) == -1
    assert lib.fastfca_as_backward(None, FAKE, None, None, None, None) == -1


def test_binding_has_no_fallback():
    """The Python binding loads the HIP library or fails: there is no CPU
    path and no import of the oracle."""
    for name in ("fastfca.py", "autograd.py"):
        src = open(os.path.join(ROOT, "paper_1805_09498_amd", name)).read()
        assert "oracle" not in src and "numpy" not in src, name
    import paper_1805_09498_amd.fastfca as ff
    assert ff.lib._name == ff.LIB_PATH


@pytest.mark.parametrize("L,W,H", [(160000, 1024, 512), (1, 16, 8), (16001, 2048, 256), (5000, 64, 16)])
def test_stft_shape_matches_the_framing_rule(lib, L, W, H):
    ip = ctypes.POINTER(ctypes.c_int)
    lib.fca_stft_shape.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ip, ip]
    F, N = ctypes.c_int(), ctypes.c_int()
    assert lib.fca_stft_shape(L, W, H, ctypes.byref(F), ctypes.byref(N)) == 0
    assert (F.value, N.value) == (W // 2 + 1, (L - 1 + W - H) // H + 1)


@pytest.mark.parametrize("W,H", [(1000, 500), (8, 4), (8192, 4096), (1024, 1024), (1024, 300), (1024, 0)])
def test_stft_rejects_bad_frames_on_the_host(lib, W, H):
    ip = ctypes.POINTER(ctypes.c_int)
    lib.fca_stft_shape.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ip, ip]
    F, N = ctypes.c_int(), ctypes.c_int()
    assert lib.fca_stft_shape(1000, W, H, ctypes.byref(F), ctypes.byref(N)) == -1
    vp, i = ctypes.c_void_p, ctypes.c_int
    lib.fca_stft.argtypes = [vp, i, i, i, i, vp, vp]
    assert lib.fca_stft(FAKE, 2, 1000, W, H, FAKE, None) == -1
    lib.fca_istft.argtypes = [vp, i, i, i, i, i, i, vp, vp]
    assert lib.fca_istft(FAKE, 2, 2, 3, W, H, 1000, FAKE, None) == -1


def test_noalloc_run_rejects_on_the_host(lib):
    """The allocation-free run checks its arguments and the size of its
    working storage before any device call (fake, never dereferenced
    pointers)."""
    vp, i = ctypes.c_void_p, ctypes.c_int
    lib.fastfca_as_run_noalloc.argtypes = [i, i, i, i, vp, vp, vp, vp, i, vp, vp]
    lib.fastfca_as_run_noalloc.restype = i
    fake = vp(1 << 20)
    run = lambda F, N, I, J, n_iter=1, ll=None: lib.fastfca_as_run_noalloc(F, N, I, J, fake, fake, fake, fake,
                                                                          n_iter, ll, None)
    assert run(1500, 4000, 8, 6) == -1                     # needs more than FCA_NOALLOC_SCRATCH_BYTES
    assert b"working storage" in lib.fca_last_error(None)
    assert run(4, 10, 3, 3, n_iter=-1) == -1
    assert run(4, 2, 3, 3) == -1                           # N < I
    assert run(4, 10, 9, 3) == -2                          # I outside the instantiated range
    assert run(4, 10, 3, 3, ll=vp((1 << 20) + 4)) == -1    # misaligned log-likelihood pointer
    lib.fastfca_as_run_noalloc.argtypes = [i, i, i, i, vp, vp, vp, vp, i, vp, vp]
    assert lib.fastfca_as_run_noalloc(4, 10, 3, 3, None, fake, fake, fake, 1, None, None) == -1


def test_status_codes_of_header_and_binding_agree():
    """Every fca_status of the header, with its value, is a constant of the
    Python binding (FCA_ERR_SINGULAR included)."""
    text = open(HEADER).read()
    codes = dict((k, int(v)) for k, v in re.findall(r"\b(FCA_(?:OK|ERR_[A-Z]+))\s*=\s*(-?\d+)", text))
    assert codes["FCA_ERR_SINGULAR"] == -6 and len(codes) == 7
    from paper_1805_09498_amd import fastfca
    for k, v in codes.items():
        assert getattr(fastfca, k) == v, k
