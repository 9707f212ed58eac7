// C ABI of libfastfca (declared in include/fastfca.h): argument checks,
// context and device-memory ownership, dispatch to the (I, J) kernel sets.
#include "fastfca.h"

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <tuple>

#include "fca_state.h"

namespace fca {
#define FCA_DECL_J(I_, J_) const KernelSet* kernel_set_I##I_##_J##J_();
#define FCA_DECL_I(I_)                                                                     \
  FCA_DECL_J(I_, 1) FCA_DECL_J(I_, 2) FCA_DECL_J(I_, 3) FCA_DECL_J(I_, 4) FCA_DECL_J(I_, 5) \
  FCA_DECL_J(I_, 6) FCA_DECL_J(I_, 7) FCA_DECL_J(I_, 8) FCA_DECL_J(I_, 9)
FCA_DECL_I(1) FCA_DECL_I(2) FCA_DECL_I(3) FCA_DECL_I(4)
FCA_DECL_I(5) FCA_DECL_I(6) FCA_DECL_I(7) FCA_DECL_I(8)

const KernelSet* kernel_set(int I, int J) {
#define FCA_ROW(I_)                                                                         \
  { &kernel_set_I##I_##_J1, &kernel_set_I##I_##_J2, &kernel_set_I##I_##_J3,                 \
    &kernel_set_I##I_##_J4, &kernel_set_I##I_##_J5, &kernel_set_I##I_##_J6,                 \
    &kernel_set_I##I_##_J7, &kernel_set_I##I_##_J8, &kernel_set_I##I_##_J9 }
  static const KernelSet* (*const table[8][9])() = {FCA_ROW(1), FCA_ROW(2), FCA_ROW(3), FCA_ROW(4),
                                                    FCA_ROW(5), FCA_ROW(6), FCA_ROW(7), FCA_ROW(8)};
  if (I < 1 || I > 8 || J < 1 || J > 9) return nullptr;
  return table[I - 1][J - 1]();
}
}  // namespace fca

#include "fca_internal.h"

using fca::DevState;
using fca::KernelSet;

namespace {

thread_local std::string g_init_error;

fca_status fail(fca_ctx* c, fca_status st, const std::string& msg) {
  if (c) c->err = msg; else g_init_error = msg;
  return st;
}

fca_status hip_fail(fca_ctx* c, hipError_t e, const char* where) {
  return fail(c, FCA_ERR_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

struct Arena {
  size_t off = 0;
  template <class T>
  size_t take(size_t count) {
    const size_t at = align_up(off, 256);
    off = at + count * sizeof(T);
    return at;
  }
};

// ---------------------------------------------------------------------------
// Launch shapes and the tuner.
//
// A shape is (waves per workgroup, bins per workgroup) of a frequency-resident
// kernel, or the streaming path (waves = 0).  Which one is fastest depends on
// F (bins against the 256 CUs: the dispatcher spreads 4-wave workgroups one
// per CU but can double 2-wave ones up on a SIMD), N (frames per lane) and
// (I, J) (registers).  With "autotune" on (the default) and no shape forced
// by options, the first iterate call of a context times every shape that
// fits on a saved copy of the state, restores the state and caches the
// winner for the process under (method, I, J, F, N).
// ---------------------------------------------------------------------------
struct Shape {
  int waves, bpw;  // waves == 0: streaming kernels
};

std::mutex g_tune_mu;
std::map<std::tuple<int, int, int, int, int, int, int>, Shape> g_tuned;  // (method, I, J, F, N, K, P step)

bool shape_fits(const fca_ctx* c, Shape sh) {
  if (sh.waves == 0) return true;
  if (c->method == FCA_METHOD_AS && (c->s.K > 1 || c->s.p_update == 1) && c->I > fca::kResMaxIK) return false;
  if (c->method == FCA_METHOD_AS && c->s.p_update >= 3) return false;  // Newton / EM with P: streaming kernels
  return c->method == FCA_METHOD_AS ? c->ks->as_resident_fits(c->N, sh.waves, sh.bpw) != 0
                                    : (sh.bpw == 1 && c->ks->em_resident_fits(c->N, sh.waves) != 0);
}

// Bins f0 .. f0 + nf - 1 of a FastFCA-AS context as a problem of their own:
// every array the streaming iteration touches is bin-major.
DevState bin_view(const fca_ctx* c, int f0, int nf) {
  const DevState& s = c->s;
  const size_t f = (size_t)f0, I = c->I, J = c->J, Np = s.Npad;
  DevState v = s;
  v.F = nf;
  v.xs = s.xs + f * 2 * I * Np;
  v.vs = s.vs + f * J * Np;
  v.lam = s.lam + f * J * I;
  v.P = s.P + f * I * I;
  v.partA = s.partA + f * s.nchunk * J * (I + 1);
  v.partB = s.partB + f * s.nchunk * I * I * I;
  v.partE = s.partE + f * s.nchunk * J * (I * I + I);
  v.partL = s.partL + f * (s.nchunk > s.nchunk_em ? s.nchunk : s.nchunk_em);
  v.llf = s.llf + f;
  return v;
}

// The split's streams and events, created once per context (default
// priority, non-blocking).
hipError_t ensure_side_streams(fca_ctx* c) {
  if (c->side[0]) return hipSuccess;
  hipStream_t st[3] = {nullptr, nullptr, nullptr};
  hipEvent_t fork = nullptr, join[3] = {nullptr, nullptr, nullptr};
  hipError_t e = hipEventCreateWithFlags(&fork, hipEventDisableTiming);
  for (int k = 0; k < 3 && e == hipSuccess; ++k) {
    e = hipStreamCreateWithFlags(&st[k], hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&join[k], hipEventDisableTiming);
  }
  if (e != hipSuccess) {
    for (int k = 0; k < 3; ++k) {
      if (join[k]) (void)hipEventDestroy(join[k]);
      if (st[k]) (void)hipStreamDestroy(st[k]);
    }
    if (fork) (void)hipEventDestroy(fork);
    return e;
  }
  for (int k = 0; k < 3; ++k) { c->side[k] = st[k]; c->ev_join[k] = join[k]; }
  c->ev_fork = fork;
  return hipSuccess;
}

// Streaming FastFCA-AS iterations with the bins split into c->split parts on
// as many streams (the bins never interact): one part's HBM-bound pass A can
// share the CUs with another part's VALU-bound pass B.  Fork and join are
// events, so the call can be captured into a graph.
hipError_t launch_stream_split(fca_ctx* c, int n_iter) {
  hipError_t e = ensure_side_streams(c);
  if (e != hipSuccess) return e;
  const int parts = c->split < c->F ? c->split : c->F;
  if ((e = hipEventRecord(c->ev_fork, c->stream)) != hipSuccess) return e;
  for (int k = 1; k < parts; ++k)
    if ((e = hipStreamWaitEvent(c->side[k - 1], c->ev_fork, 0)) != hipSuccess) return e;
  for (int k = 0; k < parts; ++k) {
    const int f0 = (int)((long long)c->F * k / parts), f1 = (int)((long long)c->F * (k + 1) / parts);
    const DevState h = bin_view(c, f0, f1 - f0);
    hipStream_t st = k == 0 ? c->stream : c->side[k - 1];
    for (int it = 0; it < n_iter && e == hipSuccess; ++it) e = c->ks->as_iter_stream(h, st);
    if (e != hipSuccess) return e;
  }
  for (int k = 1; k < parts; ++k) {
    if ((e = hipEventRecord(c->ev_join[k - 1], c->side[k - 1])) != hipSuccess) return e;
    if ((e = hipStreamWaitEvent(c->stream, c->ev_join[k - 1], 0)) != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_shape(fca_ctx* c, Shape sh, int n_iter) {
  if (sh.waves == 0 && c->method == FCA_METHOD_AS && c->split > 1 && c->F >= 2) return launch_stream_split(c, n_iter);
  if (sh.waves == 0) {
    for (int it = 0; it < n_iter; ++it) {
      hipError_t e = c->method == FCA_METHOD_AS ? c->ks->as_iter_stream(c->s, c->stream)
                                                : c->ks->em_iter(c->s, c->stream);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  for (int done = 0; done < n_iter;) {
    const int step = (n_iter - done) > 1024 ? 1024 : (n_iter - done);
    hipError_t e = c->method == FCA_METHOD_AS ? c->ks->as_iter_resident(c->s, c->stream, step, sh.waves, sh.bpw)
                                              : c->ks->em_iter_resident(c->s, c->stream, step, sh.waves);
    if (e != hipSuccess) return e;
    done += step;
  }
  return hipSuccess;
}

// Byte sizes of the iterated state (backup layout: vs, then lam and P for
// AS, R and Rinv for EM).
size_t state_bytes_v(const fca_ctx* c) { return sizeof(float) * (size_t)c->F * c->J * c->s.Npad; }
size_t state_bytes_p(const fca_ctx* c) {
  return c->method == FCA_METHOD_AS ? sizeof(float2) * (size_t)c->F * c->I * c->I : 0;
}

hipError_t copy_one(fca_ctx* c, void* dev, char* bk, size_t n, bool save) {
  return save ? hipMemcpyAsync(bk, dev, n, hipMemcpyDeviceToDevice, c->stream)
              : hipMemcpyAsync(dev, bk, n, hipMemcpyDeviceToDevice, c->stream);
}

// Save the iterated state to the backup region or restore it from there.
hipError_t copy_state(fca_ctx* c, bool save) {
  char* b = reinterpret_cast<char*>(c->backup);
  const size_t nv = state_bytes_v(c);
  hipError_t e = copy_one(c, c->s.vs, b, nv, save);
  if (c->method == FCA_METHOD_AS) {
    const size_t nl = sizeof(float) * (size_t)c->F * c->J * c->I;
    if (e == hipSuccess) e = copy_one(c, c->s.lam, b + nv, nl, save);
    if (e == hipSuccess) e = copy_one(c, c->s.P, b + nv + nl, state_bytes_p(c), save);
  } else {
    const size_t nr = sizeof(float2) * (size_t)c->F * c->J * c->I * c->I;
    if (e == hipSuccess) e = copy_one(c, c->s.R, b + nv, nr, save);
    if (e == hipSuccess) e = copy_one(c, c->s.Rinv, b + nv + nr, nr, save);
  }
  return e;
}

// The launch shape for the next iterate call (may run the tuner).
fca_status choose_shape(fca_ctx* c, int n_iter_hint, Shape* out) {
  static const Shape as_cands[] = {{1, 1}, {2, 1}, {4, 1}, {2, 2}, {4, 2}, {0, 0}};
  static const Shape em_cands[] = {{1, 1}, {2, 1}, {4, 1}, {0, 0}};
  const bool as = c->method == FCA_METHOD_AS;
  const Shape* cands = as ? as_cands : em_cands;
  const int ncand = as ? 6 : 4;
  // Forced choices first.
  if (c->path == 2) { *out = Shape{0, 0}; return FCA_OK; }
  if (c->path == 1) {
    bool any = false;
    for (int k = 0; k < ncand; ++k) any = any || (cands[k].waves > 0 && shape_fits(c, cands[k]));
    if (!any)
      return fail(c, FCA_ERR_ARG, "the frequency-resident path does not fit this problem (N, K > 1 or the gradient "
                                  "P step at I > 4, or Newton's / the EM P update, which use the streaming kernels)");
  }
  const bool forced = c->waves > 0 || c->bpw > 0;
  if (forced || !c->autotune) {
    for (int k = 0; k < ncand; ++k) {
      Shape sh = cands[k];
      if (sh.waves == 0) continue;
      if (c->waves > 0) sh.waves = c->waves;
      if (c->bpw > 0) sh.bpw = c->bpw;
      if (shape_fits(c, sh)) { *out = sh; return FCA_OK; }
    }
    if (c->path == 1)
      return fail(c, FCA_ERR_ARG, "the frequency-resident path does not fit this problem with this launch shape");
    *out = Shape{0, 0};
    return FCA_OK;
  }
  const auto key = std::make_tuple((int)c->method, c->I, c->J, c->F, c->N, c->s.K, c->s.p_update);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tuned.find(key);
    if (it != g_tuned.end() && (c->path == 0 || it->second.waves > 0) && shape_fits(c, it->second)) {
      *out = it->second;
      return FCA_OK;
    }
  }
  const std::string disk_key = fca::tune_key_prefix() + (c->method == FCA_METHOD_AS ? " as" : " em") +
                               " I=" + std::to_string(c->I) + " J=" + std::to_string(c->J) +
                               " F=" + std::to_string(c->F) + " N=" + std::to_string(c->N) +
                               " K=" + std::to_string(c->s.K) + " pstep=" + std::to_string(c->s.p_update);
  {
    Shape sh{0, 0};
    if (c->path == 0 && fca::tune_cache_get(disk_key, &sh.waves, &sh.bpw) && shape_fits(c, sh)) {
      std::lock_guard<std::mutex> lk(g_tune_mu);
      g_tuned[key] = sh;
      *out = sh;
      return FCA_OK;
    }
  }
  // Tune: for each fitting shape, the marginal cost per iteration
  // (T(n1 + n2) - T(n1)) / n2 (best of two trials each, from the saved state)
  // projected to a call of max(n_iter, 20) iterations plus the fixed cost.
  hipEvent_t e0, e1;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e != hipSuccess) return hip_fail(c, e, "tuner events");
  if ((e = copy_state(c, true)) != hipSuccess) return hip_fail(c, e, "tuner save");
  const int n1 = 8, n2 = 32;
  const int nref = n_iter_hint > 20 ? n_iter_hint : 20;
  float best = 1e30f;
  Shape best_sh{0, 0};
  for (int k = 0; k < ncand && e == hipSuccess; ++k) {
    const Shape sh = cands[k];
    if (!shape_fits(c, sh) || (c->path == 1 && sh.waves == 0)) continue;
    float t[2] = {1e30f, 1e30f};
    for (int len = 0; len < 2 && e == hipSuccess; ++len) {
      for (int trial = 0; trial < 2 && e == hipSuccess; ++trial) {
        if ((e = copy_state(c, false)) != hipSuccess) break;
        if ((e = hipEventRecord(e0, c->stream)) != hipSuccess) break;
        if ((e = launch_shape(c, sh, len ? n1 + n2 : n1)) != hipSuccess) break;
        if ((e = hipEventRecord(e1, c->stream)) != hipSuccess) break;
        if ((e = hipEventSynchronize(e1)) != hipSuccess) break;
        float ms = 0.f;
        if ((e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) break;
        if (ms < t[len]) t[len] = ms;
      }
    }
    if (e != hipSuccess) break;
    float per = (t[1] - t[0]) / (float)n2;
    if (per < 0.f) per = 0.f;
    const float fixed = t[0] - n1 * per;
    const float cost = fixed + nref * per;
    if (cost < best) { best = cost; best_sh = sh; }
  }
  if (e == hipSuccess) e = copy_state(c, false);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess) return hip_fail(c, e, "tuner run");
  if (c->path == 0) {
    {
      std::lock_guard<std::mutex> lk(g_tune_mu);
      g_tuned[key] = best_sh;
    }
    fca::tune_cache_put(disk_key, best_sh.waves, best_sh.bpw);
  }
  *out = best_sh;
  return FCA_OK;
}

// The device flag after the work queued so far (synchronises the stream).
fca_status read_flag(fca_ctx* c, int* h) {
  hipError_t e = hipMemcpyAsync(h, c->s.flag, sizeof(int), hipMemcpyDeviceToHost, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "hipMemcpyAsync");
  if ((e = hipStreamSynchronize(c->stream)) != hipSuccess) return hip_fail(c, e, "hipStreamSynchronize");
  return FCA_OK;
}

fca_status pre_check(fca_ctx* c) {
  if (!c->check_finite) return FCA_OK;
  const DevState& s = c->s;
  const bool as = c->method == FCA_METHOD_AS;
  hipError_t e = fca::launch_set_flag(s.flag, 0, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "flag reset");
  if (c->params_checked) return FCA_OK;
  e = fca::launch_check_positive(s.vs, c->F, c->J, c->N, s.Npad, as ? s.lam : nullptr,
                                 as ? (long long)c->F * c->J * c->I : 0, s.flag, c->stream);
  if (e == hipSuccess) e = c->ks->check_matrices(s, c->stream, as ? 0 : 1);
  if (e != hipSuccess) return hip_fail(c, e, "parameter check");
  int h = 0;
  fca_status st = read_flag(c, &h);
  if (st != FCA_OK) return st;
  if (h & fca::kFlagNonPositive) return fail(c, FCA_ERR_ARG, as ? "v or lambda is not positive and finite" : "v is not positive and finite");
  if (h & fca::kFlagSingularParam)
    return fail(c, FCA_ERR_SINGULAR, as ? "P(f) is singular (to single precision) in some bin"
                                        : "S_j(f) is not positive definite in some bin");
  c->params_checked = 1;
  return FCA_OK;
}

fca_status post_check(fca_ctx* c) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(c, e, "kernel launch");
  if (!c->check_finite) return FCA_OK;
  const DevState& s = c->s;
  e = fca::launch_check_finite(s.vs, (long long)c->F * c->J * s.Npad, s.flag, c->stream);
  if (e == hipSuccess && c->method == FCA_METHOD_AS) {
    e = fca::launch_check_finite(s.lam, (long long)c->F * c->J * c->I, s.flag, c->stream);
    if (e == hipSuccess)
      e = fca::launch_check_finite(reinterpret_cast<const float*>(s.P), 2LL * c->F * c->I * c->I, s.flag, c->stream);
  } else if (e == hipSuccess) {
    e = fca::launch_check_finite(reinterpret_cast<const float*>(s.R), 2LL * c->F * c->J * c->I * c->I, s.flag, c->stream);
  }
  if (e != hipSuccess) return hip_fail(c, e, "finiteness check");
  int h = 0;
  fca_status st = read_flag(c, &h);
  if (st != FCA_OK) return st;
  if (h & fca::kFlagSingular)
    return fail(c, FCA_ERR_SINGULAR, c->method == FCA_METHOD_AS
                                         ? "a weighted covariance of eq. 23 is not positive definite (pivot <= 0)"
                                         : "a model covariance C or an S_j is not positive definite (pivot <= 0)");
  if (h) return fail(c, FCA_ERR_NONFINITE, "non-finite parameter values after the update");
  return FCA_OK;
}

}  // namespace

namespace fca {
hipError_t copy_state(fca_ctx* c, bool save) { return ::copy_state(c, save); }

fca_status ctx_fail(fca_ctx* c, fca_status st, const std::string& msg) { return fail(c, st, msg); }
fca_status ctx_hip_fail(fca_ctx* c, hipError_t e, const char* where) { return hip_fail(c, e, where); }

fca_status as_iterate_chosen(fca_ctx* c, int n_iter, int* waves, int* bpw) {
  Shape sh;
  fca_status st = choose_shape(c, n_iter, &sh);
  if (st != FCA_OK) return st;
  c->last_waves = sh.waves; c->last_bpw = sh.bpw;
  *waves = sh.waves; *bpw = sh.bpw;
  ++c->version;
  hipError_t e = launch_shape(c, sh, n_iter);
  if (e != hipSuccess) return hip_fail(c, e, "FastFCA-AS iteration");
  return FCA_OK;
}

fca_status as_iterate_chosen_trace(fca_ctx* c, int n_iter, const Trace& tr, int* waves, int* bpw, bool* recorded) {
  Shape sh;
  fca_status st = choose_shape(c, n_iter, &sh);
  if (st != FCA_OK) return st;
  c->last_waves = sh.waves; c->last_bpw = sh.bpw;
  *waves = sh.waves; *bpw = sh.bpw;
  ++c->version;
  *recorded = sh.waves > 0 && n_iter <= 1024;
  hipError_t e = *recorded ? c->ks->as_iter_resident_trace(c->s, c->stream, n_iter, sh.waves, sh.bpw, tr)
                           : launch_shape(c, sh, n_iter);
  if (e != hipSuccess) return hip_fail(c, e, "FastFCA-AS iteration");
  return FCA_OK;
}

hipError_t as_iterate_view(fca_ctx* c, const DevState& s, int waves, int bpw, int n_iter) {
  if (waves == 0) {
    for (int it = 0; it < n_iter; ++it) {
      hipError_t e = c->ks->as_iter_stream(s, c->stream);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  for (int done = 0; done < n_iter;) {
    const int step = (n_iter - done) > 1024 ? 1024 : (n_iter - done);
    hipError_t e = c->ks->as_iter_resident(s, c->stream, step, waves, bpw);
    if (e != hipSuccess) return e;
    done += step;
  }
  return hipSuccess;
}

fca_status pre_iterate(fca_ctx* c) { return pre_check(c); }
fca_status post_iterate(fca_ctx* c) { return post_check(c); }

fca_status validate_init(fca_method method, int F, int N, int I, int J, const void* x, const void* v0,
                         const void* lam0, const void* P0, const void* R0, std::string* msg) {
  auto bad = [&](fca_status st, const char* m) { *msg = m; return st; };
  if (method != FCA_METHOD_AS && method != FCA_METHOD_EM) return bad(FCA_ERR_ARG, "unknown method");
  if (F < 1 || N < 1 || I < 1 || J < 1) return bad(FCA_ERR_ARG, "F, N, I, J must be positive");
  if (I > 8 || J > 9) return bad(FCA_ERR_UNSUPPORTED, "supported sizes are 1 <= I <= 8, 1 <= J <= 9");
  if (N < I) return bad(FCA_ERR_ARG, "N must be at least I (the weighted covariances are singular otherwise)");
  const long long Npad = ((long long)N + 63) / 64 * 64;
  const int mx = I > J ? I : J;
  // in double: exact below 2^53, and no overflow for any int arguments
  if ((double)F * (double)Npad * 2.0 * mx >= 2147483648.0)
    return bad(FCA_ERR_ARG, "problem too large (N*F*max(I,J) >= 2^31)");
  if (!x || !v0 || !lam0 || !P0) return bad(FCA_ERR_ARG, "x, v0, lam0 and P0 must be non-NULL device pointers");
  if (!aligned(x, 8) || !aligned(P0, 8) || !aligned(v0, 4) || !aligned(lam0, 4) || (R0 && !aligned(R0, 8)))
    return bad(FCA_ERR_ARG, "misaligned pointer (complex arrays need 8-byte, float arrays 4-byte alignment)");
  if (method == FCA_METHOD_AS && R0) return bad(FCA_ERR_ARG, "R0 must be NULL for FCA_METHOD_AS");
  return FCA_OK;
}
}  // namespace fca

extern "C" {

fca_status fca_init(fca_ctx** out, fca_method method, int F, int N, int I, int J, const fca_c64* x,
                    const float* v0, const float* lam0, const fca_c64* P0, const fca_c64* R0,
                    void* hip_stream) {
  if (!out) return fail(nullptr, FCA_ERR_ARG, "out is NULL");
  *out = nullptr;
  {
    std::string msg;
    const fca_status st = fca::validate_init(method, F, N, I, J, x, v0, lam0, P0, R0, &msg);
    if (st != FCA_OK) return fail(nullptr, st, msg);
  }
  const long long Npad = ((long long)N + 63) / 64 * 64;
  const KernelSet* ks = fca::kernel_set(I, J);
  if (!ks) return fail(nullptr, FCA_ERR_UNSUPPORTED, "(I, J) not instantiated");

  fca_ctx* c = new (std::nothrow) fca_ctx();
  if (!c) return fail(nullptr, FCA_ERR_HIP, "host allocation failed");
  c->method = method; c->F = F; c->N = N; c->I = I; c->J = J;
  c->stream = reinterpret_cast<hipStream_t>(hip_stream);
  c->ks = ks; c->check_finite = 0; c->params_checked = 0; c->path = 0; c->waves = 0; c->bpw = 0; c->autotune = 1;
  c->split = 3; c->ev_fork = nullptr;
  for (int k = 0; k < 3; ++k) { c->side[k] = nullptr; c->ev_join[k] = nullptr; }
  c->backup = nullptr; c->arena = nullptr; c->last_waves = -1; c->last_bpw = -1;
  c->version = 0; c->tape = nullptr; c->tape_bytes = 0; c->tape_iters = 0; c->tape_every = 0;
  c->tape_waves = 0; c->tape_bpw = 0; c->tape_last_rec = 0; c->tape_version = ~0ULL;

  DevState& s = c->s;
  s.F = F; s.N = N; s.Npad = (int)Npad; s.K = 1;
  s.p_update = 0; s.p_step = 0.1f; s.sums_mfma = -1;
  s.nchunk = (N + fca::kChunk - 1) / fca::kChunk;
  s.nchunk_em = (N + fca::kChunkEm - 1) / fca::kChunkEm;
  const size_t FJI = (size_t)F * J * I, FII = (size_t)F * I * I, FJII = (size_t)F * J * I * I;
  Arena a;
  const size_t o_xs = a.take<float>((size_t)F * 2 * I * Npad);
  const size_t o_vs = a.take<float>((size_t)F * J * Npad);
  const size_t o_lam = a.take<float>(FJI);
  const size_t o_P = a.take<float2>(FII);
  const bool em = method == FCA_METHOD_EM;
  const size_t o_R = em ? a.take<float2>(FJII) : 0;
  const size_t o_Ri = em ? a.take<float2>(FJII) : 0;
  size_t nA = (size_t)F * s.nchunk * J * (I + 1);  // eq. 20 sums S0 (J) and S1 (J I) per tile
  if (em) nA = (size_t)F * s.nchunk_em * J * I * I;
  const size_t o_pA = a.take<float>(nA);
  const size_t o_pB = em ? 0 : a.take<float>((size_t)F * s.nchunk * I * I * I);
  const size_t o_pE = em ? 0 : a.take<float>((size_t)F * s.nchunk * J * (I * I + I));
  const size_t o_pL = a.take<double>((size_t)F * (s.nchunk > s.nchunk_em ? s.nchunk : s.nchunk_em));
  const size_t o_llf = a.take<double>(F);
  const size_t o_ll = a.take<double>(1);
  const size_t o_flag = a.take<int>(1);
  // state backup for the tuner: vs, then lam (AS) or R and Rinv (EM), then P
  const size_t o_bk = a.take<char>(sizeof(float) * (size_t)F * J * Npad +
                                   (em ? 2 * sizeof(float2) * FJII : sizeof(float) * FJI + sizeof(float2) * FII));
  hipError_t e = hipMalloc(&c->arena, a.off);
  if (e != hipSuccess) {
    delete c;
    return hip_fail(nullptr, e, "hipMalloc");
  }
  char* base = static_cast<char*>(c->arena);
  s.xs = reinterpret_cast<float*>(base + o_xs);
  s.vs = reinterpret_cast<float*>(base + o_vs);
  s.lam = reinterpret_cast<float*>(base + o_lam);
  s.P = reinterpret_cast<float2*>(base + o_P);
  s.R = em ? reinterpret_cast<float2*>(base + o_R) : nullptr;
  s.Rinv = em ? reinterpret_cast<float2*>(base + o_Ri) : nullptr;
  s.partA = reinterpret_cast<float*>(base + o_pA);
  s.partB = em ? nullptr : reinterpret_cast<float*>(base + o_pB);
  s.partE = em ? nullptr : reinterpret_cast<float*>(base + o_pE);
  s.partL = reinterpret_cast<double*>(base + o_pL);
  s.llf = reinterpret_cast<double*>(base + o_llf);
  s.ll = reinterpret_cast<double*>(base + o_ll);
  s.flag = reinterpret_cast<int*>(base + o_flag);
  c->backup = reinterpret_cast<float*>(base + o_bk);

  hipStream_t st = c->stream;
  if ((e = fca::launch_pack_x(reinterpret_cast<const float2*>(x), const_cast<float*>(s.xs), F, N, I, s.Npad, st)) != hipSuccess ||
      (e = fca::launch_pack_v(v0, s.vs, F, N, J, s.Npad, st)) != hipSuccess ||
      (e = hipMemcpyAsync(s.lam, lam0, FJI * sizeof(float), hipMemcpyDeviceToDevice, st)) != hipSuccess ||
      (e = hipMemcpyAsync(s.P, P0, FII * sizeof(float2), hipMemcpyDeviceToDevice, st)) != hipSuccess) {
    fca_status r = hip_fail(nullptr, e, "fca_init upload");
    (void)hipFree(c->arena);
    delete c;
    return r;
  }
  if (em) {
    if (R0) {
      e = hipMemcpyAsync(s.R, R0, FJII * sizeof(float2), hipMemcpyDeviceToDevice, st);
      if (e == hipSuccess) e = ks->em_rinv(s, st);
    } else {
      e = ks->em_from_as(s, st);
    }
    if (e != hipSuccess) {
      fca_status r = hip_fail(nullptr, e, "fca_init covariance setup");
      (void)hipFree(c->arena);
      delete c;
      return r;
    }
  }
  *out = c;
  return FCA_OK;
}

fca_status fastfca_as_iterate(fca_ctx* c, int n_iter) {
  if (!c) return fail(nullptr, FCA_ERR_ARG, "NULL context");
  if (c->method != FCA_METHOD_AS) return fail(c, FCA_ERR_STATE, "fastfca_as_iterate on an FCA EM context");
  if (n_iter < 0) return fail(c, FCA_ERR_ARG, "n_iter must be >= 0");
  if (n_iter == 0) return FCA_OK;
  fca_status st = pre_check(c);
  if (st != FCA_OK) return st;
  int w = 0, b = 0;
  st = fca::as_iterate_chosen(c, n_iter, &w, &b);
  if (st != FCA_OK) return st;
  return post_check(c);
}

fca_status fca_em_iterate(fca_ctx* c, int n_iter) {
  if (!c) return fail(nullptr, FCA_ERR_ARG, "NULL context");
  if (c->method != FCA_METHOD_EM) return fail(c, FCA_ERR_STATE, "fca_em_iterate on a FastFCA-AS context");
  if (n_iter < 0) return fail(c, FCA_ERR_ARG, "n_iter must be >= 0");
  if (n_iter == 0) return FCA_OK;
  fca_status st = pre_check(c);
  if (st != FCA_OK) return st;
  Shape sh;
  st = choose_shape(c, n_iter, &sh);
  if (st != FCA_OK) return st;
  c->last_waves = sh.waves; c->last_bpw = sh.bpw;
  ++c->version;
  hipError_t e = launch_shape(c, sh, n_iter);
  if (e != hipSuccess) return hip_fail(c, e, "FCA EM iteration");
  return post_check(c);
}

fca_status fca_wiener_separate(fca_ctx* c, fca_c64* out) {
  if (!c) return fail(nullptr, FCA_ERR_ARG, "NULL context");
  if (!out || !aligned(out, 8)) return fail(c, FCA_ERR_ARG, "out must be an 8-byte aligned device pointer");
  hipError_t e = c->method == FCA_METHOD_AS ? c->ks->as_wiener(c->s, c->stream, reinterpret_cast<float2*>(out))
                                            : c->ks->em_wiener(c->s, c->stream, reinterpret_cast<float2*>(out));
  if (e != hipSuccess) return hip_fail(c, e, "Wiener filter");
  return FCA_OK;
}

fca_status fca_loglik(fca_ctx* c, double* out) {
  if (!c) return fail(nullptr, FCA_ERR_ARG, "NULL context");
  if (!out) return fail(c, FCA_ERR_ARG, "out is NULL");
  hipError_t e = c->method == FCA_METHOD_AS ? c->ks->as_loglik(c->s, c->stream) : c->ks->em_loglik(c->s, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "log-likelihood");
  double h = 0.0;
  if ((e = hipMemcpyAsync(&h, c->s.ll, sizeof(double), hipMemcpyDeviceToHost, c->stream)) != hipSuccess)
    return hip_fail(c, e, "hipMemcpyAsync");
  if ((e = hipStreamSynchronize(c->stream)) != hipSuccess) return hip_fail(c, e, "hipStreamSynchronize");
  *out = h;
  return FCA_OK;
}

fca_status fca_loglik_device(fca_ctx* c, double* out_dev) {
  if (!c) return fail(nullptr, FCA_ERR_ARG, "NULL context");
  if (!out_dev || !aligned(out_dev, 8)) return fail(c, FCA_ERR_ARG, "out_dev must be an 8-byte aligned device pointer");
  DevState s = c->s;
  s.ll = out_dev;  // the final sum writes the caller's double directly
  hipError_t e = c->method == FCA_METHOD_AS ? c->ks->as_loglik(s, c->stream) : c->ks->em_loglik(s, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "log-likelihood");
  return FCA_OK;
}

fca_status fca_loglik_bins(fca_ctx* c, double* out_dev) {
  if (!c) return fail(nullptr, FCA_ERR_ARG, "NULL context");
  if (!out_dev || !aligned(out_dev, 8)) return fail(c, FCA_ERR_ARG, "out_dev must be an 8-byte aligned device pointer");
  const DevState& s = c->s;
  const bool as = c->method == FCA_METHOD_AS;
  hipError_t e = as ? c->ks->as_loglik(s, c->stream) : c->ks->em_loglik(s, c->stream);
  if (e == hipSuccess) {
    if (as && c->I > fca::kLoglikDetInTileMaxI)
      e = hipMemcpyAsync(out_dev, s.llf, sizeof(double) * c->F, hipMemcpyDeviceToDevice, c->stream);
    else
      e = fca::launch_sum_chunks(s.partL, c->F, as ? s.nchunk : s.nchunk_em, out_dev, c->stream);
  }
  if (e != hipSuccess) return hip_fail(c, e, "per-bin log-likelihood");
  return FCA_OK;
}

fca_status fca_get_params(fca_ctx* c, float* v, float* lam, fca_c64* P_or_R) {
  if (!c) return fail(nullptr, FCA_ERR_ARG, "NULL context");
  if ((v && !aligned(v, 4)) || (lam && !aligned(lam, 4)) || (P_or_R && !aligned(P_or_R, 8)))
    return fail(c, FCA_ERR_ARG, "misaligned pointer");
  const DevState& s = c->s;
  hipError_t e = hipSuccess;
  if (v) e = fca::launch_unpack_v(s.vs, v, c->F, c->N, c->J, s.Npad, c->stream);
  if (e == hipSuccess && lam && c->method == FCA_METHOD_AS)
    e = hipMemcpyAsync(lam, s.lam, sizeof(float) * c->F * c->J * c->I, hipMemcpyDeviceToDevice, c->stream);
  if (e == hipSuccess && P_or_R) {
    if (c->method == FCA_METHOD_AS)
      e = hipMemcpyAsync(P_or_R, s.P, sizeof(float2) * c->F * c->I * c->I, hipMemcpyDeviceToDevice, c->stream);
    else
      e = hipMemcpyAsync(P_or_R, s.R, sizeof(float2) * c->F * c->J * c->I * c->I, hipMemcpyDeviceToDevice, c->stream);
  }
  if (e != hipSuccess) return hip_fail(c, e, "fca_get_params");
  return FCA_OK;
}

fca_status fca_set_params(fca_ctx* c, const float* v, const float* lam, const fca_c64* P_or_R) {
  if (!c) return fail(nullptr, FCA_ERR_ARG, "NULL context");
  if ((v && !aligned(v, 4)) || (lam && !aligned(lam, 4)) || (P_or_R && !aligned(P_or_R, 8)))
    return fail(c, FCA_ERR_ARG, "misaligned pointer");
  const DevState& s = c->s;
  hipError_t e = hipSuccess;
  ++c->version;
  c->params_checked = 0;
  if (v && c->method == FCA_METHOD_AS && (lam || P_or_R)) {
    // v, lambda and P in one launch (a NULL lambda or P is skipped)
    e = fca::launch_pack_v_copy2(v, s.vs, c->F, c->N, c->J, s.Npad, s.lam, lam,
                                 lam ? (long long)c->F * c->J * c->I : 0, reinterpret_cast<float*>(s.P),
                                 reinterpret_cast<const float*>(P_or_R), P_or_R ? 2LL * c->F * c->I * c->I : 0,
                                 c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "fca_set_params");
    return FCA_OK;
  }
  if (v) e = fca::launch_pack_v(v, s.vs, c->F, c->N, c->J, s.Npad, c->stream);
  if (e == hipSuccess && c->method == FCA_METHOD_AS && (lam || P_or_R)) {
    // lambda and P in one launch (a NULL one is skipped)
    e = fca::launch_copy3(s.lam, lam, lam ? (long long)c->F * c->J * c->I : 0, reinterpret_cast<float*>(s.P),
                          reinterpret_cast<const float*>(P_or_R), P_or_R ? 2LL * c->F * c->I * c->I : 0, nullptr,
                          nullptr, 0, c->stream);
  } else if (e == hipSuccess && P_or_R && c->method == FCA_METHOD_EM) {
    e = hipMemcpyAsync(s.R, P_or_R, sizeof(float2) * c->F * c->J * c->I * c->I, hipMemcpyDeviceToDevice, c->stream);
    if (e == hipSuccess) e = c->ks->em_rinv(s, c->stream);
  }
  if (e != hipSuccess) return hip_fail(c, e, "fca_set_params");
  return FCA_OK;
}

fca_status fca_set_option(fca_ctx* c, const char* key, long long value) {
  if (!c) return fail(nullptr, FCA_ERR_ARG, "NULL context");
  if (!key) return fail(c, FCA_ERR_ARG, "NULL key");
  if (!std::strcmp(key, "K")) {
    if (value < 1 || value > 64) return fail(c, FCA_ERR_ARG, "K must be in 1..64");
    if (c->s.K != (int)value) ++c->version;  // a recorded forward run no longer describes the iteration
    c->s.K = (int)value;
  } else if (!std::strcmp(key, "p_update")) {
    if (value < 0 || value > 4)
      return fail(c, FCA_ERR_ARG, "p_update must be 0 (fixed point), 1 (gradient), 2 (natural gradient), "
                                  "3 (Newton) or 4 (EM with P in the M-step)");
    if (c->method != FCA_METHOD_AS && value != 0) return fail(c, FCA_ERR_STATE, "p_update applies to FastFCA-AS contexts");
    if (c->s.p_update != (int)value) ++c->version;
    c->s.p_update = (int)value;
  } else if (!std::strcmp(key, "check_finite")) {
    if (value != 0 && value != 1) return fail(c, FCA_ERR_ARG, "check_finite must be 0 or 1");
    c->check_finite = (int)value;
  } else if (!std::strcmp(key, "path")) {
    if (value < 0 || value > 2) return fail(c, FCA_ERR_ARG, "path must be 0, 1 or 2");
    c->path = (int)value;
  } else if (!std::strcmp(key, "waves")) {
    if (value != 0 && value != 1 && value != 2 && value != 4)
      return fail(c, FCA_ERR_ARG, "waves must be 0 (auto), 1, 2 or 4");
    c->waves = (int)value;
  } else if (!std::strcmp(key, "bins_per_wg")) {
    if (value < 0 || value > 2) return fail(c, FCA_ERR_ARG, "bins_per_wg must be 0 (auto), 1 or 2");
    c->bpw = (int)value;
  } else if (!std::strcmp(key, "autotune")) {
    if (value != 0 && value != 1) return fail(c, FCA_ERR_ARG, "autotune must be 0 or 1");
    c->autotune = (int)value;
  } else if (!std::strcmp(key, "split_streams")) {
    if (value < 1 || value > 4) return fail(c, FCA_ERR_ARG, "split_streams must be in 1..4");
    c->split = (int)value;
  } else if (!std::strcmp(key, "sums_mfma")) {
    if (value < -1 || value > 2) return fail(c, FCA_ERR_ARG, "sums_mfma must be -1, 0, 1 or 2");
    if (c->s.sums_mfma != (int)value) ++c->version;  // a recorded forward run no longer describes the iteration
    c->s.sums_mfma = (int)value;
  } else {
    return fail(c, FCA_ERR_ARG, std::string("unknown option '") + key + "'");
  }
  return FCA_OK;
}

fca_status fca_get_option(fca_ctx* c, const char* key, long long* value) {
  if (!c) return fail(nullptr, FCA_ERR_ARG, "NULL context");
  if (!key || !value) return fail(c, FCA_ERR_ARG, "NULL key or value");
  if (!std::strcmp(key, "K")) *value = c->s.K;
  else if (!std::strcmp(key, "p_update")) *value = c->s.p_update;
  else if (!std::strcmp(key, "check_finite")) *value = c->check_finite;
  else if (!std::strcmp(key, "path")) *value = c->path;
  else if (!std::strcmp(key, "waves")) *value = c->waves;
  else if (!std::strcmp(key, "bins_per_wg")) *value = c->bpw;
  else if (!std::strcmp(key, "autotune")) *value = c->autotune;
  else if (!std::strcmp(key, "split_streams")) *value = c->split;
  else if (!std::strcmp(key, "sums_mfma")) *value = c->s.sums_mfma;
  else if (!std::strcmp(key, "last_waves")) *value = c->last_waves;
  else if (!std::strcmp(key, "last_bins_per_wg")) *value = c->last_bpw;
  else return fail(c, FCA_ERR_ARG, std::string("unknown option '") + key + "'");
  return FCA_OK;
}

fca_status fca_set_option_f64(fca_ctx* c, const char* key, double value) {
  if (!c) return fail(nullptr, FCA_ERR_ARG, "NULL context");
  if (!key) return fail(c, FCA_ERR_ARG, "NULL key");
  if (!std::strcmp(key, "p_step")) {
    if (!(value > 0.0 && value <= 1e3)) return fail(c, FCA_ERR_ARG, "p_step must be in (0, 1000]");
    if (c->s.p_step != (float)value) ++c->version;
    c->s.p_step = (float)value;
  } else {
    return fail(c, FCA_ERR_ARG, std::string("unknown real option '") + key + "'");
  }
  return FCA_OK;
}

fca_status fca_get_option_f64(fca_ctx* c, const char* key, double* value) {
  if (!c) return fail(nullptr, FCA_ERR_ARG, "NULL context");
  if (!key || !value) return fail(c, FCA_ERR_ARG, "NULL key or value");
  if (!std::strcmp(key, "p_step")) *value = c->s.p_step;
  else return fail(c, FCA_ERR_ARG, std::string("unknown real option '") + key + "'");
  return FCA_OK;
}

const char* fca_last_error(const fca_ctx* c) {
  if (c) return c->err.c_str();
  return g_init_error.c_str();
}

void fca_destroy(fca_ctx* c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  if (c->side[0]) {
    for (int k = 0; k < 3; ++k) {
      (void)hipStreamSynchronize(c->side[k]);
      (void)hipEventDestroy(c->ev_join[k]);
      (void)hipStreamDestroy(c->side[k]);
    }
    (void)hipEventDestroy(c->ev_fork);
  }
  if (c->arena) (void)hipFree(c->arena);
  if (c->tape) (void)hipFree(c->tape);
  delete c;
}

}  // extern "C"
