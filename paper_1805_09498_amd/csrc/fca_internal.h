// Internal definitions shared by the C ABI implementation files.
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include "fastfca.h"
#include "fca_state.h"

struct fca_ctx {
  fca_method method;
  int F, N, I, J;
  hipStream_t stream;
  const fca::KernelSet* ks;
  fca::DevState s;
  void* arena;
  int check_finite;
  int params_checked;  // with check_finite: the parameters passed the device check since fca_init / fca_set_params
  int path;   // 0 auto, 1 resident, 2 streaming
  int waves;  // 0 auto
  int bpw;    // bins per workgroup of the resident AS kernel, 0 auto
  int autotune;  // 1: time the candidate launch shapes once per (method, I, J, F, N)
  int split;     // streams over which streaming FastFCA-AS iterations split the bins (1..4)
  hipStream_t side[3];          // the split's extra streams (created on first use)
  hipEvent_t ev_fork, ev_join[3];
  float* backup;  // state copy used while tuning: vs, lam, P (AS) or vs, R (EM)
  int last_waves, last_bpw;  // launch shape of the last iterate call (waves 0: streaming)
  unsigned long long version;  // bumped by every call that changes the state
  // Recording of the last fastfca_as_forward, for fastfca_as_backward.
  void* tape;
  size_t tape_bytes;
  int tape_iters, tape_every;
  int tape_waves, tape_bpw;           // launch shape of the recorded iterations
  int tape_last_rec;                  // 1: the last segment's states are already in the tape
  unsigned long long tape_version;    // version right after the recording
  std::string err;
};

namespace fca {
// Three float-array device copies (n floats each; n = 0 skips one) in one
// launch (fca_common.hip).
hipError_t launch_copy3(float* d0, const float* s0, long long n0, float* d1, const float* s1, long long n1, float* d2,
                        const float* s2, long long n2, hipStream_t st);
// v packed as launch_pack_v does, and two float arrays copied, in one launch
hipError_t launch_pack_v_copy2(const float* v, float* vs, int F, int N, int J, int Npad, float* d1, const float* s1,
                               long long n1, float* d2, const float* s2, long long n2, hipStream_t st);

// Save the iterated state of a context to its backup region, or restore it.
hipError_t copy_state(fca_ctx* c, bool save);

// Error setters of the context (the message is kept for fca_last_error).
fca_status ctx_fail(fca_ctx* c, fca_status st, const std::string& msg);
fca_status ctx_hip_fail(fca_ctx* c, hipError_t e, const char* where);

// FastFCA-AS iterations of a context with its launch-shape choice (options,
// tuner); the shape used is returned in *waves, *bpw (waves 0: streaming).
fca_status as_iterate_chosen(fca_ctx* c, int n_iter, int* waves, int* bpw);
// The same, and where the chosen shape is frequency-resident the iterations
// run through the recording kernel into tr (*recorded = true).
fca_status as_iterate_chosen_trace(fca_ctx* c, int n_iter, const Trace& tr, int* waves, int* bpw, bool* recorded);
// n_iter FastFCA-AS iterations of the state view s (the context's x and
// scratch, any v / lambda / P) with a given launch shape.
hipError_t as_iterate_view(fca_ctx* c, const DevState& s, int waves, int bpw, int n_iter);
// Before the launches of an iterate call: with "check_finite", the device
// check of the parameters (once after fca_init / fca_set_params) and the
// clearing of the flag the iteration kernels report into.
fca_status pre_iterate(fca_ctx* c);
// After-launch checks of an iterate call (launch error; with "check_finite"
// a non-positive-definite solve or a non-finite parameter).
fca_status post_iterate(fca_ctx* c);

// The host-side argument checks of fca_init (no device access).
fca_status validate_init(fca_method method, int F, int N, int I, int J, const void* x, const void* v0,
                         const void* lam0, const void* P0, const void* R0, std::string* msg);

// Persistent launch-shape cache (fca_tunecache.cpp), active when the
// environment variable FASTFCA_TUNE_CACHE names a file.  Keys should start
// with tune_key_prefix() (device architecture, CU count, library build).
std::string tune_key_prefix();
bool tune_cache_get(const std::string& key, int* a, int* b);
void tune_cache_put(const std::string& key, int a, int b);
}  // namespace fca
