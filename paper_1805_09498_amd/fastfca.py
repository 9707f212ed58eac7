"""Python binding of libfastfca (ctypes).  Argument marshalling only: every
step of FCA / FastFCA-AS runs in the library's HIP kernels.

The functions carry the names of the C ABI (include/fastfca.h):
``fca_init``, ``fastfca_as_iterate``, ``fca_em_iterate``,
``fca_wiener_separate``, ``fca_loglik``, ``fca_loglik_device``, ``fca_loglik_bins``,
``fca_get_params``,
``fca_set_params``, ``fca_set_option``, ``fca_get_option``, ``fca_last_error``,
``fca_destroy``, the batch calls ``fca_batch_*`` and the derivative calls
``fastfca_as_forward`` / ``fastfca_as_backward`` (``autograd.py`` wraps them
in a ``torch.autograd.Function``) and the STFT calls ``fca_stft_shape``,
``fca_stft``, ``fca_istft``, and ``fastfca_as_run_noalloc`` (no context, no
device allocation).
Arrays are torch tensors on the GPU in the ABI layouts (complex64 /
float32, C-contiguous); PyTorch provides the device memory and the stream.

If the shared library has not been built, importing this module raises
ImportError: there is no fallback implementation.
"""

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfastfca.so")

FCA_OK = 0
FCA_ERR_ARG = -1
FCA_ERR_UNSUPPORTED = -2
FCA_ERR_HIP = -3
FCA_ERR_STATE = -4
FCA_ERR_NONFINITE = -5
FCA_ERR_SINGULAR = -6

FCA_METHOD_AS = 0
FCA_METHOD_EM = 1

EXPORTED = ("fca_init", "fastfca_as_iterate", "fca_em_iterate", "fca_wiener_separate",
            "fca_loglik", "fca_loglik_device", "fca_loglik_bins", "fca_get_params", "fca_set_params", "fca_set_option",
            "fca_get_option", "fca_set_option_f64", "fca_get_option_f64", "fca_last_error", "fca_destroy",
            "fca_batch_init", "fca_batch_iterate", "fca_batch_context", "fca_batch_set_option",
            "fca_batch_get_option", "fca_batch_last_error", "fca_batch_destroy",
            "fastfca_as_forward", "fastfca_as_backward", "fca_stft_shape", "fca_stft", "fca_istft",
            "fastfca_as_run_noalloc")


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it first (python -c 'import __graft_entry__ as g; g.build()')")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i, c = ctypes.c_void_p, ctypes.c_int, ctypes.c_char_p
    lib.fca_init.argtypes = [ctypes.POINTER(vp), i, i, i, i, i, vp, vp, vp, vp, vp, vp]
    lib.fca_init.restype = i
    lib.fastfca_as_iterate.argtypes = [vp, i]
    lib.fastfca_as_iterate.restype = i
    lib.fca_em_iterate.argtypes = [vp, i]
    lib.fca_em_iterate.restype = i
    lib.fca_wiener_separate.argtypes = [vp, vp]
    lib.fca_wiener_separate.restype = i
    lib.fca_loglik.argtypes = [vp, ctypes.POINTER(ctypes.c_double)]
    lib.fca_loglik.restype = i
    lib.fca_loglik_device.argtypes = [vp, vp]
    lib.fca_loglik_device.restype = i
    lib.fca_loglik_bins.argtypes = [vp, vp]
    lib.fca_loglik_bins.restype = i
    lib.fca_get_params.argtypes = [vp, vp, vp, vp]
    lib.fca_get_params.restype = i
    lib.fca_set_params.argtypes = [vp, vp, vp, vp]
    lib.fca_set_params.restype = i
    lib.fca_set_option.argtypes = [vp, c, ctypes.c_longlong]
    lib.fca_set_option.restype = i
    lib.fca_get_option.argtypes = [vp, c, ctypes.POINTER(ctypes.c_longlong)]
    lib.fca_get_option.restype = i
    lib.fca_set_option_f64.argtypes = [vp, c, ctypes.c_double]
    lib.fca_set_option_f64.restype = i
    lib.fca_get_option_f64.argtypes = [vp, c, ctypes.POINTER(ctypes.c_double)]
    lib.fca_get_option_f64.restype = i
    lib.fca_last_error.argtypes = [vp]
    lib.fca_last_error.restype = c
    lib.fca_destroy.argtypes = [vp]
    lib.fca_destroy.restype = None
    ip = ctypes.POINTER(ctypes.c_int)
    pp = ctypes.POINTER(vp)
    lib.fca_batch_init.argtypes = [pp, i, ip, ip, ip, ip, pp, pp, pp, pp, vp]
    lib.fca_batch_init.restype = i
    lib.fca_batch_iterate.argtypes = [vp, i]
    lib.fca_batch_iterate.restype = i
    lib.fca_batch_context.argtypes = [vp, i, pp]
    lib.fca_batch_context.restype = i
    lib.fca_batch_set_option.argtypes = [vp, c, ctypes.c_longlong]
    lib.fca_batch_set_option.restype = i
    lib.fca_batch_get_option.argtypes = [vp, c, i, ctypes.POINTER(ctypes.c_longlong)]
    lib.fca_batch_get_option.restype = i
    lib.fca_batch_last_error.argtypes = [vp]
    lib.fca_batch_last_error.restype = c
    lib.fca_batch_destroy.argtypes = [vp]
    lib.fca_batch_destroy.restype = None
    lib.fastfca_as_forward.argtypes = [vp, i, i, vp]
    lib.fastfca_as_forward.restype = i
    lib.fastfca_as_backward.argtypes = [vp, vp, vp, vp, vp, vp]
    lib.fastfca_as_backward.restype = i
    lib.fca_stft_shape.argtypes = [i, i, i, ip, ip]
    lib.fca_stft_shape.restype = i
    lib.fca_stft.argtypes = [vp, i, i, i, i, vp, vp]
    lib.fca_stft.restype = i
    lib.fca_istft.argtypes = [vp, i, i, i, i, i, i, vp, vp]
    lib.fca_istft.restype = i
    lib.fastfca_as_run_noalloc.argtypes = [i, i, i, i, vp, vp, vp, vp, i, vp, vp]
    lib.fastfca_as_run_noalloc.restype = i
    return lib


lib = _load()


class FcaError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"libfastfca status {status}: {message}")
        self.status = status


def fca_last_error(ctx=None):
    return lib.fca_last_error(ctx.handle if ctx is not None else None).decode()


def _check(status, ctx=None):
    if status != FCA_OK:
        raise FcaError(status, fca_last_error(ctx))


def _ptr(t, dtype, shape, name):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise ValueError(f"{name} must be a CUDA/HIP torch tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _stream_handle(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream), s


class FcaContext:
    """An opaque libfastfca context (one mixture, one method)."""

    def __init__(self, handle, method, F, N, I, J, stream, keep, owned=True):
        self.handle = handle
        self.method = method
        self.F, self.N, self.I, self.J = F, N, I, J
        self.stream = stream
        self._keep = keep   # inputs stay referenced until the stream has consumed them
        self.owned = owned  # False for the contexts of a batch

    def __del__(self):
        try:
            if self.owned:
                fca_destroy(self)
        except Exception:
            pass


def fca_init(method, x, v0, lam0, P0, R0=None, stream=None):
    """fca_init: x [F][N][I] complex64, v0 [F][N][J] float32, lam0 [F][J][I]
    float32, P0 [F][I][I] complex64, R0 [F][J][I][I] complex64 or None."""
    if x.dim() != 3 or v0.dim() != 3:
        raise ValueError("x must be [F][N][I] and v0 [F][N][J]")
    F, N, I = x.shape
    J = v0.shape[2]
    args = [
        _ptr(x, torch.complex64, (F, N, I), "x"),
        _ptr(v0, torch.float32, (F, N, J), "v0"),
        _ptr(lam0, torch.float32, (F, J, I), "lam0"),
        _ptr(P0, torch.complex64, (F, I, I), "P0"),
        _ptr(R0, torch.complex64, (F, J, I, I), "R0"),
    ]
    sh, s = _stream_handle(stream)
    h = ctypes.c_void_p()
    _check(lib.fca_init(ctypes.byref(h), int(method), F, N, I, J, *args, sh))
    return FcaContext(h, int(method), F, N, I, J, s, (x, v0, lam0, P0, R0))


def fastfca_as_iterate(ctx, n_iter):
    _check(lib.fastfca_as_iterate(ctx.handle, int(n_iter)), ctx)


def fca_em_iterate(ctx, n_iter):
    _check(lib.fca_em_iterate(ctx.handle, int(n_iter)), ctx)


def fca_wiener_separate(ctx, out=None):
    """Returns (or fills) out [J][F][N][I] complex64."""
    if out is None:
        with torch.cuda.stream(ctx.stream):
            out = torch.empty((ctx.J, ctx.F, ctx.N, ctx.I), dtype=torch.complex64, device="cuda")
    p = _ptr(out, torch.complex64, (ctx.J, ctx.F, ctx.N, ctx.I), "out")
    _check(lib.fca_wiener_separate(ctx.handle, p), ctx)
    return out


def fca_loglik(ctx):
    out = ctypes.c_double()
    _check(lib.fca_loglik(ctx.handle, ctypes.byref(out)), ctx)
    return out.value


def fca_loglik_device(ctx, out=None):
    """Enqueues the log-likelihood into a one-element float64 device tensor
    (allocated if not given) without synchronising; returns the tensor."""
    if out is None:
        with torch.cuda.stream(ctx.stream):
            out = torch.empty((1,), dtype=torch.float64, device="cuda")
    _check(lib.fca_loglik_device(ctx.handle, _ptr(out, torch.float64, (1,), "out")), ctx)
    return out


def fca_loglik_bins(ctx, out=None):
    """Enqueues the per-bin log-likelihood into a float64 device tensor [F]
    (allocated if not given) without synchronising; returns the tensor."""
    if out is None:
        with torch.cuda.stream(ctx.stream):
            out = torch.empty((ctx.F,), dtype=torch.float64, device="cuda")
    _check(lib.fca_loglik_bins(ctx.handle, _ptr(out, torch.float64, (ctx.F,), "out")), ctx)
    return out


def fca_get_params(ctx):
    """AS: (v [F][N][J], lam [F][J][I], P [F][I][I]); EM: (v, None, R [F][J][I][I])."""
    F, N, I, J = ctx.F, ctx.N, ctx.I, ctx.J
    with torch.cuda.stream(ctx.stream):
        v = torch.empty((F, N, J), dtype=torch.float32, device="cuda")
        if ctx.method == FCA_METHOD_AS:
            lam = torch.empty((F, J, I), dtype=torch.float32, device="cuda")
            M = torch.empty((F, I, I), dtype=torch.complex64, device="cuda")
        else:
            lam = None
            M = torch.empty((F, J, I, I), dtype=torch.complex64, device="cuda")
    _check(lib.fca_get_params(ctx.handle, ctypes.c_void_p(v.data_ptr()),
                              None if lam is None else ctypes.c_void_p(lam.data_ptr()),
                              ctypes.c_void_p(M.data_ptr())), ctx)
    return v, lam, M


def fca_set_params(ctx, v=None, lam=None, P_or_R=None):
    F, N, I, J = ctx.F, ctx.N, ctx.I, ctx.J
    mshape = (F, I, I) if ctx.method == FCA_METHOD_AS else (F, J, I, I)
    _check(lib.fca_set_params(ctx.handle, _ptr(v, torch.float32, (F, N, J), "v"),
                              _ptr(lam, torch.float32, (F, J, I), "lam"),
                              _ptr(P_or_R, torch.complex64, mshape, "P_or_R")), ctx)
    ctx._keep_set = (v, lam, P_or_R)   # referenced until the next call


def fca_set_option(ctx, key, value):
    _check(lib.fca_set_option(ctx.handle, key.encode(), int(value)), ctx)


def fca_get_option(ctx, key):
    out = ctypes.c_longlong()
    _check(lib.fca_get_option(ctx.handle, key.encode(), ctypes.byref(out)), ctx)
    return out.value


def fca_set_option_f64(ctx, key, value):
    _check(lib.fca_set_option_f64(ctx.handle, key.encode(), float(value)), ctx)


def fca_get_option_f64(ctx, key):
    out = ctypes.c_double()
    _check(lib.fca_get_option_f64(ctx.handle, key.encode(), ctypes.byref(out)), ctx)
    return out.value


def fastfca_as_forward(ctx, n_iter, ckpt_every=5, out=None):
    """n_iter recorded iterations, then the Wiener filter; returns (or fills)
    out [J][F][N][I] complex64."""
    if out is None:
        with torch.cuda.stream(ctx.stream):
            out = torch.empty((ctx.J, ctx.F, ctx.N, ctx.I), dtype=torch.complex64, device="cuda")
    p = _ptr(out, torch.complex64, (ctx.J, ctx.F, ctx.N, ctx.I), "out")
    _check(lib.fastfca_as_forward(ctx.handle, int(n_iter), int(ckpt_every), p), ctx)
    return out


def fastfca_as_backward(ctx, grad_out, need=(True, True, True, True)):
    """Derivatives of the last fastfca_as_forward for dL/d(out) = grad_out:
    returns (dx [F][N][I], dv0 [F][N][J], dlam0 [F][J][I], dP0 [F][I][I]),
    None where need is False."""
    F, N, I, J = ctx.F, ctx.N, ctx.I, ctx.J
    g = _ptr(grad_out, torch.complex64, (J, F, N, I), "grad_out")
    shapes = (((F, N, I), torch.complex64), ((F, N, J), torch.float32), ((F, J, I), torch.float32),
              ((F, I, I), torch.complex64))
    outs = []
    with torch.cuda.stream(ctx.stream):
        for want, (shp, dt) in zip(need, shapes):
            outs.append(torch.empty(shp, dtype=dt, device="cuda") if want else None)
    ptrs = [None if o is None else ctypes.c_void_p(o.data_ptr()) for o in outs]
    _check(lib.fastfca_as_backward(ctx.handle, g, *ptrs), ctx)
    ctx._keep_grad = grad_out   # referenced until the stream has consumed it
    return tuple(outs)


def fca_destroy(ctx):
    if not ctx.owned:
        raise ValueError("the contexts of a batch are released by fca_batch_destroy")
    if ctx.handle is not None and ctx.handle.value:
        lib.fca_destroy(ctx.handle)
    ctx.handle = ctypes.c_void_p()


class FcaBatch:
    """An opaque libfastfca batch of FastFCA-AS mixtures."""

    def __init__(self, handle, shapes, stream, keep):
        self.handle = handle
        self.shapes = shapes          # [(F, N, I, J)] per mixture
        self.stream = stream
        self._keep = keep

    def __del__(self):
        try:
            fca_batch_destroy(self)
        except Exception:
            pass


def fca_batch_last_error(batch=None):
    return lib.fca_batch_last_error(batch.handle if batch is not None else None).decode()


def _bcheck(status, batch=None):
    if status != FCA_OK:
        raise FcaError(status, fca_batch_last_error(batch))


def fca_batch_init(mixtures, stream=None):
    """mixtures: sequence of (x, v0, lam0, P0) device tensors in the layouts of
    fca_init (complex64 / float32)."""
    n = len(mixtures)
    Fs, Ns, Is, Js, ptrs = [], [], [], [], [[], [], [], []]
    for k, (x, v0, lam0, P0) in enumerate(mixtures):
        F, N, I = x.shape
        J = v0.shape[2]
        Fs.append(F); Ns.append(N); Is.append(I); Js.append(J)
        for lst, t, dt, shp, nm in ((ptrs[0], x, torch.complex64, (F, N, I), "x"),
                                    (ptrs[1], v0, torch.float32, (F, N, J), "v0"),
                                    (ptrs[2], lam0, torch.float32, (F, J, I), "lam0"),
                                    (ptrs[3], P0, torch.complex64, (F, I, I), "P0")):
            lst.append(_ptr(t, dt, shp, f"mixture {k} {nm}"))
    ia = lambda a: (ctypes.c_int * n)(*a)
    pa = lambda a: (ctypes.c_void_p * n)(*[p.value for p in a])
    sh, s = _stream_handle(stream)
    h = ctypes.c_void_p()
    _bcheck(lib.fca_batch_init(ctypes.byref(h), n, ia(Fs), ia(Ns), ia(Is), ia(Js),
                               pa(ptrs[0]), pa(ptrs[1]), pa(ptrs[2]), pa(ptrs[3]), sh))
    return FcaBatch(h, list(zip(Fs, Ns, Is, Js)), s, tuple(mixtures))


def fca_batch_iterate(batch, n_iter):
    _bcheck(lib.fca_batch_iterate(batch.handle, int(n_iter)), batch)


def fca_batch_context(batch, m):
    out = ctypes.c_void_p()
    _bcheck(lib.fca_batch_context(batch.handle, int(m), ctypes.byref(out)), batch)
    F, N, I, J = batch.shapes[m]
    return FcaContext(out, FCA_METHOD_AS, F, N, I, J, batch.stream, (batch,), owned=False)


def fca_batch_set_option(batch, key, value):
    _bcheck(lib.fca_batch_set_option(batch.handle, key.encode(), int(value)), batch)


def fca_batch_get_option(batch, key, group=0):
    out = ctypes.c_longlong()
    _bcheck(lib.fca_batch_get_option(batch.handle, key.encode(), int(group), ctypes.byref(out)), batch)
    return out.value


def fca_batch_destroy(batch):
    if batch.handle is not None and batch.handle.value:
        lib.fca_batch_destroy(batch.handle)
    batch.handle = ctypes.c_void_p()


def fca_stft_shape(L, frame=1024, hop=512):
    F, N = ctypes.c_int(), ctypes.c_int()
    _check(lib.fca_stft_shape(int(L), int(frame), int(hop), ctypes.byref(F), ctypes.byref(N)))
    return F.value, N.value


def fca_stft(wav, frame=1024, hop=512, stream=None):
    """wav [C][L] float32 (GPU) -> X [F][N][C] complex64, the mixture layout."""
    if wav.dim() != 2:
        raise ValueError("wav must be [C][L]")
    C, L = wav.shape
    F, N = fca_stft_shape(L, frame, hop)
    sh, s = _stream_handle(stream)
    with torch.cuda.stream(s):
        X = torch.empty((F, N, C), dtype=torch.complex64, device="cuda")
    _check(lib.fca_stft(_ptr(wav, torch.float32, (C, L), "wav"), C, L, int(frame), int(hop),
                        ctypes.c_void_p(X.data_ptr()), sh))
    return X


def fca_istft(S, L, frame=1024, hop=512, stream=None):
    """S [J][F][N][C] complex64 (GPU) -> waveforms [J][C][L] float32."""
    if S.dim() != 4:
        raise ValueError("S must be [J][F][N][C]")
    J, F, N, C = S.shape
    sh, s = _stream_handle(stream)
    with torch.cuda.stream(s):
        wav = torch.empty((J, C, int(L)), dtype=torch.float32, device="cuda")
    _check(lib.fca_istft(_ptr(S, torch.complex64, (J, F, N, C), "S"), J, C, N, int(frame), int(hop), int(L),
                         ctypes.c_void_p(wav.data_ptr()), sh))
    return wav


def fastfca_as_run_noalloc(x, v, lam, P, n_iter, loglik=None, stream=None):
    """n_iter iterations on the caller's (v, lam, P) in place, no context and
    no device allocation by the library: x [F][N][I] complex64, v [F][N][J]
    float32, lam [F][J][I] float32, P [F][I][I] complex64; loglik None or a
    one-element float64 tensor that receives L2 of the final state."""
    if x.dim() != 3 or v.dim() != 3:
        raise ValueError("x must be [F][N][I] and v [F][N][J]")
    F, N, I = x.shape
    J = v.shape[2]
    sh, _ = _stream_handle(stream)
    _check(lib.fastfca_as_run_noalloc(
        F, N, I, J, _ptr(x, torch.complex64, (F, N, I), "x"), _ptr(v, torch.float32, (F, N, J), "v"),
        _ptr(lam, torch.float32, (F, J, I), "lam"), _ptr(P, torch.complex64, (F, I, I), "P"), int(n_iter),
        _ptr(loglik, torch.float64, (1,), "loglik"), sh))
