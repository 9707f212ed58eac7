// Differentiable unrolled FastFCA-AS (C ABI, declared in include/fastfca.h):
// a recorded forward run (iterations with a checkpoint of the state every
// k iterations, then the Wiener filter) and its reverse-mode pass.
//
// The backward pass walks the checkpoint segments from the last to the
// first: it rebuilds the states of a segment from its checkpoint with the
// same workgroup body and launch shape as the recorded run, then runs the
// adjoints of its iterations in reverse order in one launch (a workgroup
// carries its bin through the segment).  With the frequency-resident
// kernel one launch of its recording variant rebuilds a whole segment and
// also keeps the eq. 23 sums of every iteration for the adjoint; with the
// streaming kernels the segment is rebuilt one iteration at a time and the
// adjoint sums the eq. 23 terms again.  Memory is (checkpoints + k + 1)
// states of (v, lambda, P), k sets of eq. 23 sums and the adjoints.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <string>

#include "fca_internal.h"

using fca::AdjIter;
using fca::DevState;

namespace {

bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

// One (v, lambda, P) state inside the tape.
struct StateView {
  float* v;
  float* lam;
  float2* P;
};

struct TapeLayout {
  size_t state_floats;  // floats of one state (256-byte aligned parts)
  size_t v_off, lam_off, P_off;
  int n_ck, every;
  size_t ck_off, slot_off, S_off, vb_off, lb_off, Pb_off, xb_off, total_floats;
  size_t S_floats;  // eq. 23 sums of one iteration, [F][I][I*I]
};

size_t up64(size_t v) { return (v + 63) / 64 * 64; }  // 256 bytes of floats

TapeLayout layout(const fca_ctx* c, int n_iter, int every) {
  TapeLayout t{};
  const size_t fv = (size_t)c->F * c->J * c->s.Npad, fl = (size_t)c->F * c->J * c->I, fp = 2 * (size_t)c->F * c->I * c->I;
  t.v_off = 0;
  t.lam_off = up64(fv);
  t.P_off = t.lam_off + up64(fl);
  t.state_floats = t.P_off + up64(fp);
  t.every = every;
  t.n_ck = n_iter > 0 ? (n_iter + every - 1) / every : 0;
  const int slots = n_iter > 0 ? every + 1 : 0;
  t.ck_off = 0;
  t.slot_off = t.ck_off + (size_t)t.n_ck * t.state_floats;  // slot 0: work state; 1..k: rebuilt states
  t.S_floats = up64((size_t)c->F * c->I * c->I * c->I);
  t.S_off = t.slot_off + (size_t)slots * t.state_floats;
  t.vb_off = t.S_off + (size_t)(n_iter > 0 ? every : 0) * t.S_floats;
  t.lb_off = t.vb_off + 2 * up64(fv);
  t.Pb_off = t.lb_off + 2 * up64(fl);
  t.xb_off = t.Pb_off + 2 * up64(fp);
  t.total_floats = t.xb_off + up64((size_t)c->F * 2 * c->I * c->s.Npad);
  return t;
}

StateView state_at(const fca_ctx* c, const TapeLayout& t, size_t off) {
  float* base = static_cast<float*>(c->tape) + off;
  return StateView{base + t.v_off, base + t.lam_off, reinterpret_cast<float2*>(base + t.P_off)};
}

// One whole tape state (v, lambda, P and their padding) to another.
hipError_t copy_tape_state(const fca_ctx* c, const TapeLayout& t, size_t dst_off, size_t src_off) {
  float* base = static_cast<float*>(c->tape);
  return hipMemcpyAsync(base + dst_off, base + src_off, sizeof(float) * t.state_floats, hipMemcpyDeviceToDevice,
                        c->stream);
}

hipError_t copy_view(const fca_ctx* c, StateView dst, const float* v, const float* lam, const float2* P) {
  return fca::launch_copy3(dst.v, v, (long long)c->F * c->J * c->s.Npad, dst.lam, lam, (long long)c->F * c->J * c->I,
                           reinterpret_cast<float*>(dst.P), reinterpret_cast<const float*>(P),
                           2LL * c->F * c->I * c->I, c->stream);
}

DevState view_state(const fca_ctx* c, StateView v) {
  DevState s = c->s;
  s.vs = v.v;
  s.lam = v.lam;
  s.P = v.P;
  return s;
}

}  // namespace

extern "C" {

fca_status fastfca_as_forward(fca_ctx* c, int n_iter, int ckpt_every, fca_c64* out) {
  if (!c) return fca::ctx_fail(nullptr, FCA_ERR_ARG, "NULL context");
  if (c->method != FCA_METHOD_AS) return fca::ctx_fail(c, FCA_ERR_STATE, "fastfca_as_forward on an FCA EM context");
  if (n_iter < 0 || ckpt_every < 1) return fca::ctx_fail(c, FCA_ERR_ARG, "n_iter must be >= 0 and ckpt_every >= 1");
  if (out && !aligned(out, 8)) return fca::ctx_fail(c, FCA_ERR_ARG, "out must be an 8-byte aligned device pointer");
  if (c->s.K != 1 || c->s.p_update != 0)
    return fca::ctx_fail(c, FCA_ERR_UNSUPPORTED, "the recorded forward supports the fixed-point step with K = 1 only");
  const int every = ckpt_every < n_iter ? ckpt_every : (n_iter > 0 ? n_iter : 1);
  const TapeLayout t = layout(c, n_iter, every);
  const size_t bytes = sizeof(float) * t.total_floats;
  hipError_t e = hipSuccess;
  if (bytes > c->tape_bytes) {
    if (c->tape) {
      if ((e = hipStreamSynchronize(c->stream)) != hipSuccess) return fca::ctx_hip_fail(c, e, "hipStreamSynchronize");
      (void)hipFree(c->tape);
      c->tape = nullptr;
      c->tape_bytes = 0;
    }
    if ((e = hipMalloc(&c->tape, bytes)) != hipSuccess) {
      c->tape = nullptr;
      return fca::ctx_hip_fail(c, e, "tape allocation");
    }
    c->tape_bytes = bytes;
  }
  c->tape_version = ~0ULL;
  {
    fca_status pst = fca::pre_iterate(c);
    if (pst != FCA_OK) return pst;
  }
  int waves = 0, bpw = 0;
  bool last_rec = false;
  for (int k = 0; k < t.n_ck; ++k) {
    if ((e = copy_view(c, state_at(c, t, t.ck_off + (size_t)k * t.state_floats), c->s.vs, c->s.lam, c->s.P)) != hipSuccess)
      return fca::ctx_hip_fail(c, e, "checkpoint copy");
    const int steps = (n_iter - k * every) < every ? (n_iter - k * every) : every;
    int w = 0, b = 0;
    fca_status st;
    if (k == t.n_ck - 1) {
      // The last segment is the first one the backward pass needs: where the
      // shape is frequency-resident its states go straight into the tape.
      const StateView first = state_at(c, t, t.slot_off + t.state_floats);
      fca::Trace tr{first.v, first.lam, first.P, static_cast<float*>(c->tape) + t.S_off, (long long)t.state_floats,
                    (long long)t.S_floats};
      bool rec = false;
      st = fca::as_iterate_chosen_trace(c, steps, tr, &w, &b, &rec);
      last_rec = rec;
    } else {
      st = fca::as_iterate_chosen(c, steps, &w, &b);
    }
    if (st != FCA_OK) return st;
    if (k > 0 && (w != waves || b != bpw))
      return fca::ctx_fail(c, FCA_ERR_STATE, "the launch shape changed inside a recorded run");
    waves = w; bpw = b;
  }
  fca_status st = fca::post_iterate(c);
  if (st != FCA_OK) return st;
  if (out && (e = c->ks->as_wiener(c->s, c->stream, reinterpret_cast<float2*>(out))) != hipSuccess)
    return fca::ctx_hip_fail(c, e, "Wiener filter");
  c->tape_iters = n_iter;
  c->tape_every = every;
  c->tape_waves = waves;
  c->tape_bpw = bpw;
  c->tape_last_rec = last_rec ? 1 : 0;
  c->tape_version = c->version;
  return FCA_OK;
}

fca_status fastfca_as_backward(fca_ctx* c, const fca_c64* grad_out, fca_c64* grad_x, float* grad_v0,
                               float* grad_lam0, fca_c64* grad_P0) {
  if (!c) return fca::ctx_fail(nullptr, FCA_ERR_ARG, "NULL context");
  if (c->method != FCA_METHOD_AS) return fca::ctx_fail(c, FCA_ERR_STATE, "fastfca_as_backward on an FCA EM context");
  if (!c->tape || c->tape_version != c->version)
    return fca::ctx_fail(c, FCA_ERR_STATE, "no recorded forward run matches the current state");
  if (c->s.K != 1 || c->s.p_update != 0)
    return fca::ctx_fail(c, FCA_ERR_STATE, "the P-step options changed after the recorded forward run");
  if (!grad_out || !aligned(grad_out, 8) || (grad_x && !aligned(grad_x, 8)) || (grad_P0 && !aligned(grad_P0, 8)) ||
      (grad_v0 && !aligned(grad_v0, 4)) || (grad_lam0 && !aligned(grad_lam0, 4)))
    return fca::ctx_fail(c, FCA_ERR_ARG, "grad_out must be non-NULL; misaligned pointer");
  const int T = c->tape_iters, every = c->tape_every;
  const TapeLayout t = layout(c, T, every);
  float* tape = static_cast<float*>(c->tape);
  const size_t fv = up64((size_t)c->F * c->J * c->s.Npad), fl = up64((size_t)c->F * c->J * c->I),
               fp = up64(2 * (size_t)c->F * c->I * c->I);
  float* vb[2] = {tape + t.vb_off, tape + t.vb_off + fv};
  float* lb[2] = {tape + t.lb_off, tape + t.lb_off + fl};
  float2* Pb[2] = {reinterpret_cast<float2*>(tape + t.Pb_off), reinterpret_cast<float2*>(tape + t.Pb_off + fp)};
  float* xb = tape + t.xb_off;
  int cur = 0;
  hipError_t e;
  {
    AdjIter a{};
    a.vb_out = vb[cur]; a.lb_out = lb[cur]; a.Pb_out = Pb[cur]; a.xb = xb;
    if ((e = c->ks->adj_wiener(c->s, reinterpret_cast<const float2*>(grad_out), a, c->stream)) != hipSuccess)
      return fca::ctx_hip_fail(c, e, "Wiener adjoint");
  }
  const bool recorded = c->tape_waves > 0;  // frequency-resident: rebuild with the recording variant
  for (int k = t.n_ck - 1; k >= 0; --k) {
    const int t0 = k * every;
    const int len = (T - t0) < every ? (T - t0) : every;
    const size_t ck_at = t.ck_off + (size_t)k * t.state_floats;
    auto slot_at = [&](int j) { return j == 0 ? ck_at : t.slot_off + (size_t)j * t.state_floats; };
    if (recorded && k == t.n_ck - 1 && c->tape_last_rec) {
      // states recorded by the forward run
    } else if (recorded) {
      if ((e = copy_tape_state(c, t, t.slot_off, ck_at)) != hipSuccess) return fca::ctx_hip_fail(c, e, "segment restore");
      const StateView first = state_at(c, t, slot_at(1));
      fca::Trace tr{first.v, first.lam, first.P, tape + t.S_off, (long long)t.state_floats, (long long)t.S_floats};
      if ((e = c->ks->as_iter_resident_trace(view_state(c, state_at(c, t, t.slot_off)), c->stream, len, c->tape_waves,
                                             c->tape_bpw, tr)) != hipSuccess)
        return fca::ctx_hip_fail(c, e, "segment recompute");
    } else {
      for (int j = 0; j < len; ++j) {
        if ((e = copy_tape_state(c, t, slot_at(j + 1), slot_at(j))) != hipSuccess)
          return fca::ctx_hip_fail(c, e, "segment copy");
        if ((e = fca::as_iterate_view(c, view_state(c, state_at(c, t, slot_at(j + 1))), 0, 0, 1)) != hipSuccess)
          return fca::ctx_hip_fail(c, e, "segment recompute");
      }
    }
    // the segment's iteration adjoints, last first, in one launch
    fca::AdjSeg g{};
    g.tape = tape;
    g.ck = (long long)ck_at; g.slot0 = (long long)t.slot_off; g.stride = (long long)t.state_floats;
    g.v_off = (long long)t.v_off; g.lam_off = (long long)t.lam_off; g.P_off = (long long)t.P_off;
    g.S = recorded ? tape + t.S_off : nullptr;
    g.S_floats = (long long)t.S_floats;
    for (int k = 0; k < 2; ++k) { g.vb[k] = vb[k]; g.lb[k] = lb[k]; g.Pb[k] = Pb[k]; }
    g.xb = xb;
    g.len = len; g.cur = cur;
    if (len > 0 && (e = c->ks->adj_seg(c->s, g, c->stream)) != hipSuccess)
      return fca::ctx_hip_fail(c, e, "iteration adjoints");
    if (len & 1) cur = 1 - cur;
  }
  e = hipSuccess;
  if (grad_x) e = fca::launch_unpack_x(xb, reinterpret_cast<float2*>(grad_x), c->F, c->N, c->I, c->s.Npad, c->stream);
  if (e == hipSuccess && grad_v0) e = fca::launch_unpack_v(vb[cur], grad_v0, c->F, c->N, c->J, c->s.Npad, c->stream);
  if (e == hipSuccess && grad_lam0)
    e = hipMemcpyAsync(grad_lam0, lb[cur], sizeof(float) * (size_t)c->F * c->J * c->I, hipMemcpyDeviceToDevice, c->stream);
  if (e == hipSuccess && grad_P0)
    e = hipMemcpyAsync(grad_P0, Pb[cur], sizeof(float2) * (size_t)c->F * c->I * c->I, hipMemcpyDeviceToDevice, c->stream);
  if (e != hipSuccess) return fca::ctx_hip_fail(c, e, "gradient output");
  return FCA_OK;
}

}  // extern "C"
