/*
 * libfastfca -- FastFCA-AS and conventional FCA EM on one AMD Instinct MI355X
 * (gfx950), C ABI.
 *
 * Method: N. Ito and T. Nakatani, "FastFCA-AS: joint diagonalization based
 * acceleration of full-rank spatial covariance analysis for separating any
 * number of sources" (arXiv 1805.09498).  Section numbers and equation
 * numbers below refer to that paper.
 *
 * Notation.  The observed STFT mixture at I microphones is x(n,f) in C^I
 * (the paper's y(n,f), Section 2), n = 0..N-1 frames, f = 0..F-1 bins; J
 * sources.  The FCA model (Section 3.1, eq. 1-2) gives source image j the
 * covariance v_j(n,f) S_j(f).  FastFCA-AS constrains
 * S_j(f) = P(f)^-H diag(lambda_j(f)) P(f)^-1 (eq. 12).
 *
 * Array layouts (all row-major, C order; complex values are interleaved
 * (re, im) float pairs, the layout of torch.complex64):
 *   x    [F][N][I]      complex  mixture
 *   v    [F][N][J]      float    v_j(n,f) > 0
 *   lam  [F][J][I]      float    lambda_{j,i}(f) > 0, the diagonal of Lambda_j(f)
 *   P    [F][I][I]      complex  P[f][r][c] = P(f)_{rc}
 *   R    [F][J][I][I]   complex  S_j(f), Hermitian positive definite
 *   out  [J][F][N][I]   complex  separated source images
 *
 * Memory: every array argument is a device pointer owned by the caller,
 * except the host scalar of fca_loglik.  fca_init copies what it needs into
 * library-owned device memory, so the caller may free its inputs once
 * fca_init has returned and the stream has reached that point.  The library
 * owns its state until fca_destroy.
 *
 * Streams: all work is enqueued on the hipStream_t given to fca_init and is
 * asynchronous unless stated.  A context is not thread-safe; separate
 * contexts are independent.
 *
 * Errors: every call returns an fca_status; nothing else crosses the ABI.
 * Host-side argument checks happen before any device work is enqueued.
 * fca_last_error gives a message for the last failure on a context (or,
 * with NULL, for the last failed fca_init of the calling thread).
 *
 * Supported sizes: 1 <= I <= 8 microphones, 1 <= J <= 9 sources, N >= I
 * frames (below that the weighted covariances of eq. 23 are singular),
 * F >= 1 bins, N*F*max(I,J) < 2^31.
 */
#ifndef FASTFCA_H
#define FASTFCA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  float re, im;
} fca_c64;

typedef struct fca_ctx fca_ctx;

typedef enum {
  FCA_OK = 0,
  FCA_ERR_ARG = -1,         /* bad pointer, size or option */
  FCA_ERR_UNSUPPORTED = -2, /* (I, J) outside the instantiated range */
  FCA_ERR_HIP = -3,         /* a HIP runtime call failed; see fca_last_error */
  FCA_ERR_STATE = -4,       /* call does not match the context's method */
  FCA_ERR_NONFINITE = -5,   /* non-finite parameters after an update
                               (check_finite=1) */
  FCA_ERR_SINGULAR = -6     /* check_finite=1: P(f) singular or S_j(f) not
                               positive definite in the given parameters, or
                               a pivot <= 0 in an update's solves (a weighted
                               covariance of eq. 23, or C / S_j of FCA EM) */
} fca_status;

typedef enum {
  FCA_METHOD_AS = 0, /* FastFCA-AS: state (v, lambda, P), Section 4 */
  FCA_METHOD_EM = 1, /* conventional FCA EM: state (v, S), Section 3.3 */
  /* not a method: widens the enum to every non-negative int, so that a
   * caller's out-of-range value is a defined value the library rejects */
  FCA_METHOD_MAX_ENUM = 0x7fffffff
} fca_method;

/* Create a context for one mixture (Section 2: estimate the J source images
 * from x).  x, v0, lam0 and P0 are device pointers in the layouts above.
 *   FCA_METHOD_AS: the state is (v0, lam0, P0); R0 must be NULL.
 *   FCA_METHOD_EM: the state is (v0, S); S = R0 when R0 is not NULL, else
 *                  S_j(f) = P0(f)^-H diag(lam0_j(f)) P0(f)^-1 (eq. 12) is
 *                  formed on the device, so both methods can start from the
 *                  same point.
 * hip_stream is a hipStream_t (NULL = the default stream).
 * Returns FCA_ERR_ARG for NULL/misaligned pointers (8-byte alignment for
 * complex, 4 for float) or bad sizes, FCA_ERR_UNSUPPORTED outside the
 * (I, J) range, FCA_ERR_HIP if device allocation fails.  On failure *out is
 * set to NULL. */
fca_status fca_init(fca_ctx **out, fca_method method, int F, int N, int I, int J,
                    const fca_c64 *x, const float *v0, const float *lam0,
                    const fca_c64 *P0, const fca_c64 *R0, void *hip_stream);

/* Run n_iter hybrid iterations of FastFCA-AS (Section 4.3): the EM update of
 * v and lambda (eq. 15-20), then K fixed-point updates of every P(f) (eq. 23,
 * K from the "K" option, default 1) with the new v and lambda.
 * n_iter >= 0.  FCA_ERR_STATE on an EM context.  Asynchronous. */
fca_status fastfca_as_iterate(fca_ctx *ctx, int n_iter);

/* Run n_iter iterations of the conventional FCA EM algorithm (Section 3.3,
 * eq. 6-10): per time-frequency point an I x I inverse and 2J I x I products.
 * FCA_ERR_STATE on an AS context.  Asynchronous. */
fca_status fca_em_iterate(fca_ctx *ctx, int n_iter);

/* Multichannel Wiener filter (eq. 3) with the current parameters: for the
 * AS method R_j(n,f) follows eq. 15.  out is a device array [J][F][N][I]
 * complex.  The J estimates sum to x.  Asynchronous. */
fca_status fca_wiener_separate(fca_ctx *ctx, fca_c64 *out);

/* Log-likelihood of the current parameters, L1 (eq. 5) for EM contexts, L2
 * (eq. 14) for AS contexts, including the -I ln(pi) constant of the complex
 * normal density, summed over all N*F points.  out is a HOST pointer.
 * Synchronises the context's stream. */
fca_status fca_loglik(fca_ctx *ctx, double *out);

/* The same log-likelihood (eq. 5 / eq. 14), written to a DEVICE double:
 * out_dev (8-byte aligned device pointer, owned by the caller) holds L once
 * the context's stream has passed this call.  Asynchronous: nothing waits,
 * so a caller can queue job after job and read the values later.
 * FCA_ERR_ARG for a NULL or misaligned out_dev. */
fca_status fca_loglik_device(fca_ctx *ctx, double *out_dev);

/* The log-likelihood of each frequency bin (the sum over n of eq. 5 / eq. 14
 * for one f, constant term included), written to out_dev [F] (device
 * doubles, 8-byte aligned, owned by the caller).  The bins' values add up to
 * fca_loglik's total up to the order of the FP64 additions.  Asynchronous.
 * FCA_ERR_ARG for a NULL or misaligned out_dev. */
fca_status fca_loglik_bins(fca_ctx *ctx, double *out_dev);

/* Copy the current parameters to caller-owned device arrays in the ABI
 * layouts.  AS: v [F][N][J], lam [F][J][I], P_or_R = P [F][I][I].
 * EM: v [F][N][J], lam ignored (may be NULL), P_or_R = S [F][J][I][I].
 * Any pointer may be NULL to skip it.  Asynchronous. */
fca_status fca_get_params(fca_ctx *ctx, float *v, float *lam, fca_c64 *P_or_R);

/* Overwrite the current parameters from device arrays in the same layouts
 * as fca_get_params (NULL skips).  Asynchronous. */
fca_status fca_set_params(fca_ctx *ctx, const float *v, const float *lam,
                          const fca_c64 *P_or_R);

/* Options: "K" (fixed-point steps per hybrid iteration, 1..64, default 1),
 * "p_update" (FastFCA-AS only; how step 2 of a hybrid iteration updates P --
 * the fixed-point update and the alternatives named in Section 4.5:
 * 0 = the fixed-point update of eq. 23 (default), 1 = gradient ascent
 * P + mu g, 2 = natural (relative) gradient P + mu P P^H g, with
 * g = (1/N) dL2/dP* of eq. 21 at the new v, lambda and mu the real option
 * "p_step" (default 0.1), 3 = one Newton step on L2 (eq. 14) in P with
 * v, lambda held (the columns' phases, which L2 ignores, unchanged to first
 * order), 4 = EM with P in the M-step: after the E-step at the current
 * parameters, eq. 19-20 and then one sweep of column-wise maximisations of
 * the Q-function (eq. 18) over P, p_i <- V_i^-1 [P^-H]_i scaled to
 * p_i^H V_i p_i = 1; K applies to the fixed-point update only; 3 and 4 run
 * on the streaming kernels),
 * "check_finite" (0/1, default 0.  With 1, iterate calls synchronise and
 * check on the device: (a) once after fca_init or fca_set_params, before
 * iterating, the parameters the model requires (Section 3.1, eq. 12):
 * v(n,f) > 0 and finite for every frame, lambda > 0 and finite, P(f)
 * non-singular to single precision (an LU pivot's modulus above
 * I 2^-23 times the largest entry's), or for EM every S_j(f) positive
 * definite -- FCA_ERR_ARG for v / lambda, FCA_ERR_SINGULAR for P / S, and
 * nothing is iterated; (b) after the iterations, FCA_ERR_SINGULAR if a
 * solve met a pivot <= 0 (a weighted covariance of eq. 23, or C / S_j of
 * FCA EM; e.g. a bin whose mixture is zero), else FCA_ERR_NONFINITE if a
 * parameter is NaN/Inf), "path" (0 = automatic,
 * 1 = force the frequency-resident kernels, 2 = force the streaming
 * kernels; K > 1 or the gradient P step at I > 4 always use the streaming
 * kernels), "waves"
 * (64-lane waves per workgroup of the frequency-resident
 * kernels: 0 = automatic, 1, 2 or 4), "bins_per_wg" (frequency bins per
 * workgroup of the frequency-resident FastFCA-AS kernel: 0 = automatic, 1 or
 * 2; 2 needs at least 2 waves), "autotune" (1 = default: unless a shape is
 * forced by the options above, the first iterate call of a context times
 * every launch shape that fits on a saved copy of the state, restores it and
 * caches the fastest for the process under (method, I, J, F, N, K); this call
 * synchronises the stream.  0 = fixed preference order), "split_streams"
 * (FastFCA-AS on the streaming kernels: the bins are split into this many
 * parts, 1..4, default 3, that iterate on the context's stream and on
 * streams the library owns, forked and joined with events; 1 = one stream),
 * "sums_mfma" (FastFCA-AS on the streaming kernels above I = 4: where the
 * eq. 23 sums of pass B run; 0 = vector units, 1 = FP32 matrix cores in
 * 16x16x4 tiles, 2 = FP32 matrix cores in 16-block 4x4x1 tiles (I <= 8),
 * -1 = default: 2 at I = 8, where it measured fastest, else 0; results
 * agree to rounding).  When the
 * environment variable FASTFCA_TUNE_CACHE names a writable file, measured
 * shapes are also appended to it and read back by later processes (keyed by
 * GPU architecture, compute-unit count and library build; unreadable or
 * unwritable files only cost a re-measurement).  Unknown keys or
 * values out of range give FCA_ERR_ARG; a forced shape that cannot hold N
 * frames per bin makes the iterate call return FCA_ERR_ARG.  Results are
 * bitwise reproducible for a given launch shape. */
fca_status fca_set_option(fca_ctx *ctx, const char *key, long long value);

/* Real-valued options: "p_step" (step size mu of the gradient-type P
 * updates, in (0, 1000], default 0.1).  FCA_ERR_ARG for unknown keys or
 * values out of range. */
fca_status fca_set_option_f64(fca_ctx *ctx, const char *key, double value);
fca_status fca_get_option_f64(fca_ctx *ctx, const char *key, double *value);

/* Read an option ("K", "p_update", "check_finite", "path", "waves", "bins_per_wg",
 * "autotune", "split_streams", "sums_mfma": the configured values) or the launch shape the last iterate
 * call used ("last_waves": waves per workgroup, 0 = streaming kernels, -1 =
 * no call yet; "last_bins_per_wg").  value is a host pointer.  Unknown keys
 * give FCA_ERR_ARG. */
fca_status fca_get_option(fca_ctx *ctx, const char *key, long long *value);

/* Human-readable message for the last error on ctx, or for the calling
 * thread's last failed fca_init when ctx is NULL.  Never NULL. */
const char *fca_last_error(const fca_ctx *ctx);

/* Release all device memory of the context (after synchronising its stream).
 * NULL is ignored. */
void fca_destroy(fca_ctx *ctx);

/* ------------------------------------------------------------------------
 * Batched FastFCA-AS: many mixtures of different (F, N, I, J) advanced
 * together.  Each mixture is an ordinary FCA_METHOD_AS context owned by the
 * batch; mixtures of equal (I, J) advance in one launch per batch step over a
 * table of (mixture, bin) tiles ordered by decreasing N.  One batch step is
 * recorded once per iteration count as a HIP graph and replayed (when the
 * stream is not NULL and the "graph" option is on).
 * ------------------------------------------------------------------------ */
typedef struct fca_batch fca_batch;

/* n_mix mixtures; F, N, I, J are HOST arrays of n_mix sizes; x, v0, lam0, P0
 * are HOST arrays of n_mix DEVICE pointers in the layouts of fca_init.  The
 * same checks as fca_init apply per mixture (error message names it).  The
 * caller may free the inputs once the stream has passed this call. */
fca_status fca_batch_init(fca_batch **out, int n_mix, const int *F, const int *N, const int *I,
                          const int *J, const fca_c64 *const *x, const float *const *v0,
                          const float *const *lam0, const fca_c64 *const *P0, void *hip_stream);

/* n_iter hybrid iterations of every mixture (Section 4.3).  The first call
 * times the candidate launch shapes per (I, J) group (synchronising the
 * stream; the state is restored; FASTFCA_TUNE_CACHE as for fca_set_option's
 * "autotune").  Asynchronous otherwise. */
fca_status fca_batch_iterate(fca_batch *b, int n_iter);

/* The context of mixture m (owned by the batch: do not destroy it) for
 * fca_loglik, fca_wiener_separate, fca_get_params, fca_set_params. */
fca_status fca_batch_context(fca_batch *b, int m, fca_ctx **ctx);

/* "graph" (1 = default: replay a recorded HIP graph per batch step; 0 =
 * launch directly), "queue" (0 = default: one workgroup per (mixture, bin)
 * tile in the table's order; 1 = a persistent grid of as many workgroups as
 * fit on the device that take tiles from a device counter, for the groups
 * whose queue kernel needs no scratch memory, the first form for the others;
 * the results are bitwise the same), "autotune" (1 = default, 0 = smallest fitting shape),
 * "waves" (0 = automatic, 1, 2 or 4), "K" (fixed-point steps, 1..64, applied
 * to every mixture). */
fca_status fca_batch_set_option(fca_batch *b, const char *key, long long value);

/* "groups" (number of (I, J) groups; group ignored), per group index:
 * "group_I", "group_J", "group_tiles", "group_waves" (waves per workgroup
 * chosen, 0 = streaming kernels, -1 = not tuned yet), "group_queued" (1 if
 * the group's last launch took the work-queue form); "queue" (group
 * ignored).  value: host pointer. */
fca_status fca_batch_get_option(fca_batch *b, const char *key, int group, long long *value);

/* Message for the last error on b, or for the calling thread's last failed
 * fca_batch_init when b is NULL.  Never NULL. */
const char *fca_batch_last_error(const fca_batch *b);

/* Synchronise the stream and release the batch and its contexts. */
void fca_batch_destroy(fca_batch *b);

/* ------------------------------------------------------------------------
 * Derivatives of the unrolled method (reverse mode): a recorded run of
 * hybrid iterations (Section 4.3) followed by the Wiener filter (eq. 3 with
 * eq. 15), and the derivative of a real loss on its output with respect to
 * the mixture and the starting parameters.
 * ------------------------------------------------------------------------ */

/* Run n_iter hybrid iterations (K = 1) from the context's current state, as
 * fastfca_as_iterate does, recording the state every ckpt_every iterations,
 * then write the Wiener estimates of the final state into out [J][F][N][I]
 * (device, may be NULL).  The recording lives in library-owned device memory
 * (ceil(n_iter / ckpt_every) + ckpt_every + 1 copies of (v, lambda, P), plus
 * the adjoint buffers) until the next call of this function or
 * fca_destroy.  n_iter >= 0, ckpt_every >= 1.  FCA_ERR_UNSUPPORTED unless the
 * "K" option is 1 and "p_update" is 0.  Asynchronous (a context's first iterations may run
 * the launch-shape tuner, see "autotune"). */
fca_status fastfca_as_forward(fca_ctx *ctx, int n_iter, int ckpt_every, fca_c64 *out);

/* Reverse-mode derivative of the last fastfca_as_forward of ctx.  grad_out
 * [J][F][N][I] is dL/d(out) for a real loss L; the call writes dL/dx
 * [F][N][I], dL/dv0 [F][N][J], dL/dlam0 [F][J][I] and dL/dP0 [F][I][I],
 * where x is the context's mixture and (v0, lam0, P0) the state the recorded
 * run started from.  A complex entry z receives dL/dRe z + i dL/dIm z (the
 * convention of PyTorch's autograd).  All pointers are device pointers; any
 * output may be NULL.  The iterations of each checkpoint segment are rebuilt
 * with the recorded launch shape (bitwise the recorded states) and their
 * adjoints run in reverse order.  FCA_ERR_STATE if the state changed since
 * the recorded run (an iterate or set_params call).  The call may be
 * repeated with other grad_out.  Asynchronous. */
fca_status fastfca_as_backward(fca_ctx *ctx, const fca_c64 *grad_out, fca_c64 *grad_x, float *grad_v0,
                               float *grad_lam0, fca_c64 *grad_P0);

/* ------------------------------------------------------------------------
 * STFT front and back end (the analysis and synthesis settings of the
 * paper's experiments, Table 1: 16 kHz, frame 1024, shift 512, square root
 * of a Hann window for both), so that multichannel waveforms go in and
 * separated waveforms come out.  frame: a power of two in 16..4096; hop:
 * divides frame, at most frame / 2.  Frame n covers samples
 * n hop - (frame - hop) .. n hop - (frame - hop) + frame - 1 (zero outside
 * the signal), so every sample lies in frame / hop frames; the window is
 * w[t] = sin(pi t / frame); bins f = 0 .. frame / 2.  Errors: FCA_ERR_ARG
 * (message in fca_last_error(NULL)), FCA_ERR_HIP.
 * ------------------------------------------------------------------------ */

/* Spectrum shape of an L-sample signal: *F = frame / 2 + 1,
 * *N = floor((L - 1 + frame - hop) / hop) + 1.  Host only. */
fca_status fca_stft_shape(int L, int frame, int hop, int *F, int *N);

/* Analysis of C channels: wav [C][L] float (device) -> X [F][N][C] complex
 * (device; the mixture layout of fca_init).  Asynchronous. */
fca_status fca_stft(const float *wav, int C, int L, int frame, int hop, fca_c64 *X, void *hip_stream);

/* Synthesis of J signals of C channels each: S [J][F][N][C] complex (device;
 * the layout of fca_wiener_separate) -> wav [J][C][L] float (device), the
 * inverse of fca_stft (overlap-add of windowed inverse transforms, scaled by
 * 2 hop / frame; only the real parts of bins 0 and frame / 2 are used).  N
 * must be the frame count of an L-sample signal.  Allocates J*C*N*frame
 * floats of stream-ordered scratch for the call.  Asynchronous. */
fca_status fca_istft(const fca_c64 *S, int J, int C, int N, int frame, int hop, int L, float *wav,
                     void *hip_stream);

/* ------------------------------------------------------------------------
 * Allocation-free run, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  It allocates nothing: the working storage (the repacked
 * mixture and v, the per-tile partial sums, the log-likelihood partials)
 * lives in a library array of FCA_NOALLOC_SCRATCH_BYTES per device, held
 * from the first call on a device until the process ends.
 * ------------------------------------------------------------------------ */
#define FCA_NOALLOC_SCRATCH_BYTES (64ull << 20)

/* n_iter FastFCA-AS hybrid iterations (K = 1, the fixed-point P update),
 * as fca_init + fastfca_as_iterate + fca_get_params would run them, on the
 * caller's parameters in place: x [F][N][I] (device, read), v [F][N][J],
 * lam [F][J][I], P [F][I][I] (device, read and overwritten with the state
 * after the iterations).  loglik: NULL, or a device double that receives L2
 * (eq. 14) of the final state.  The launch shape is fixed (the first
 * frequency-resident shape of (4 waves, 2 bins), (4, 1), (2, 1), (1, 1) that
 * holds N frames, else the streaming kernels on hip_stream alone), so the
 * results equal those of a context forced to the same shape.  Checks as
 * fca_init, and FCA_ERR_ARG when the working storage,
 * 4 (2I + J) F ceil64(N) bytes plus the partial sums, exceeds
 * FCA_NOALLOC_SCRATCH_BYTES; messages in fca_last_error(NULL).  Calls
 * overlapping on one device share the array and race: serialise them (one
 * stream, or events).  Asynchronous; calls no allocating routine. */
fca_status fastfca_as_run_noalloc(int F, int N, int I, int J, const fca_c64 *x, float *v, float *lam,
                                  fca_c64 *P, int n_iter, double *loglik, void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* FASTFCA_H */
