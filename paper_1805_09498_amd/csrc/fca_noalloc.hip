// Allocation-free FastFCA-AS run (C ABI, declared in include/fastfca.h):
// the iterations of fastfca_as_iterate on caller-owned parameters, with the
// library's working storage (the repacked mixture and v, the streaming
// kernels' per-tile partial sums, the log-likelihood partials) in one
// file-scope device array instead of device memory the library allocates.
//
// The array exists once per device and keeps the last call's contents.
// Nothing in it has to start at zero: the repacking kernels write every
// element they use (padding included) and the partial sums are written
// before they are read.  Calls that overlap on one device (two streams, two
// threads) share the array and race.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <string>

#include "fca_internal.h"

namespace {

__device__ __align__(256) char scratch[FCA_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
char* g_scratch[kMaxDevices];  // device address of `scratch` on each device (set on first use)

size_t up256(size_t v) { return (v + 255) / 256 * 256; }

struct Layout {
  size_t xs, vs, pA, pB, pL, llf, flag, total;
};

Layout layout(int F, int Npad, int I, int J, int nchunk, bool streaming) {
  Layout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) { const size_t at = off; off = up256(off + bytes); return at; };
  L.xs = take(sizeof(float) * (size_t)F * 2 * I * Npad);
  L.vs = take(sizeof(float) * (size_t)F * J * Npad);
  L.pA = streaming ? take(sizeof(float) * (size_t)F * nchunk * J * (I + 1)) : 0;
  L.pB = streaming ? take(sizeof(float) * (size_t)F * nchunk * I * I * I) : 0;
  L.pL = take(sizeof(double) * (size_t)F * nchunk);
  L.llf = take(sizeof(double) * (size_t)F);
  L.flag = take(sizeof(int));
  L.total = off;
  return L;
}

// The device address of this device's array, looked up once per device
// with that device current.
hipError_t scratch_base(char** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    if ((e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch))) != hipSuccess) return e;
    g_scratch[dev] = static_cast<char*>(p);
  }
  *out = g_scratch[dev];
  return hipSuccess;
}

}  // namespace

extern "C" fca_status fastfca_as_run_noalloc(int F, int N, int I, int J, const fca_c64* x, float* v, float* lam,
                                             fca_c64* P, int n_iter, double* loglik, void* hip_stream) {
  {
    std::string msg;
    const fca_status st = fca::validate_init(FCA_METHOD_AS, F, N, I, J, x, v, lam, P, nullptr, &msg);
    if (st != FCA_OK) return fca::ctx_fail(nullptr, st, msg);
  }
  if (n_iter < 0) return fca::ctx_fail(nullptr, FCA_ERR_ARG, "n_iter must be >= 0");
  if (loglik && (reinterpret_cast<uintptr_t>(loglik) % 8) != 0)
    return fca::ctx_fail(nullptr, FCA_ERR_ARG, "loglik must be an 8-byte aligned device pointer");
  const fca::KernelSet* ks = fca::kernel_set(I, J);
  if (!ks) return fca::ctx_fail(nullptr, FCA_ERR_UNSUPPORTED, "(I, J) not instantiated");

  // Launch shape: the first frequency-resident shape that holds N frames per
  // bin, else the streaming kernels on the caller's stream alone.
  static const int shapes[4][2] = {{4, 2}, {4, 1}, {2, 1}, {1, 1}};
  int waves = 0, bpw = 0;
  for (const auto& sh : shapes)
    if (ks->as_resident_fits(N, sh[0], sh[1])) { waves = sh[0]; bpw = sh[1]; break; }
  const bool streaming = waves == 0;
  const int Npad = (N + 63) / 64 * 64;
  const int nchunk = (N + fca::kChunk - 1) / fca::kChunk;
  const Layout L = layout(F, Npad, I, J, nchunk, streaming);
  if (L.total > (size_t)FCA_NOALLOC_SCRATCH_BYTES)
    return fca::ctx_fail(nullptr, FCA_ERR_ARG,
                         "the problem needs " + std::to_string(L.total) +
                             " bytes of working storage; the allocation-free entry point holds at most " +
                             std::to_string((unsigned long long)FCA_NOALLOC_SCRATCH_BYTES));

  char* base = nullptr;
  hipError_t e = scratch_base(&base);
  if (e != hipSuccess)
    return fca::ctx_fail(nullptr, FCA_ERR_HIP, std::string("hipGetSymbolAddress: ") + hipGetErrorString(e));

  fca::DevState s{};
  s.F = F; s.N = N; s.Npad = Npad;
  s.nchunk = nchunk; s.nchunk_em = (N + fca::kChunkEm - 1) / fca::kChunkEm;
  s.K = 1; s.p_update = 0; s.p_step = 0.1f;
  s.xs = reinterpret_cast<const float*>(base + L.xs);
  s.vs = reinterpret_cast<float*>(base + L.vs);
  s.lam = lam;
  s.P = reinterpret_cast<float2*>(P);
  s.R = nullptr; s.Rinv = nullptr;
  s.partA = streaming ? reinterpret_cast<float*>(base + L.pA) : nullptr;
  s.partB = streaming ? reinterpret_cast<float*>(base + L.pB) : nullptr;
  s.partE = nullptr;  // only the P updates other than the fixed point use it
  s.partL = reinterpret_cast<double*>(base + L.pL);
  s.llf = reinterpret_cast<double*>(base + L.llf);
  s.ll = loglik;
  s.flag = reinterpret_cast<int*>(base + L.flag);

  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  e = fca::launch_pack_x(reinterpret_cast<const float2*>(x), const_cast<float*>(s.xs), F, N, I, Npad, st);
  if (e == hipSuccess) e = fca::launch_pack_v(v, s.vs, F, N, J, Npad, st);
  for (int done = 0; done < n_iter && e == hipSuccess;) {
    if (streaming) {
      e = ks->as_iter_stream(s, st);
      ++done;
    } else {
      const int step = (n_iter - done) > 1024 ? 1024 : (n_iter - done);
      e = ks->as_iter_resident(s, st, step, waves, bpw);
      done += step;
    }
  }
  if (e == hipSuccess && loglik) e = ks->as_loglik(s, st);
  if (e == hipSuccess) e = fca::launch_unpack_v(s.vs, v, F, N, J, Npad, st);
  if (e == hipSuccess) e = hipGetLastError();
  if (e != hipSuccess) return fca::ctx_fail(nullptr, FCA_ERR_HIP, std::string("fastfca_as_run_noalloc: ") + hipGetErrorString(e));
  return FCA_OK;
}
