// Device state shared by the kernels and the host-side launchers.
#pragma once

#include <hip/hip_runtime.h>

namespace fca {

// Streaming kernels: 256 lanes per workgroup, each lane owns kPts points of a
// tile; one tile covers kChunk consecutive frames of one frequency bin.
constexpr int kBlock = 256;
constexpr int kPts = 4;
constexpr int kChunk = kBlock * kPts;
constexpr int kChunkEm = kBlock;  // FCA EM: one point per lane
// Largest I whose frequency-resident FastFCA-AS kernel runs K > 1
// fixed-point steps or the gradient P step (both need the inverse of a
// matrix per lane); larger I with either uses the streaming kernels.
constexpr int kResMaxIK = 4;
// Largest I whose FastFCA-AS log-likelihood adds the bin's ln|det P| term in
// the first tile's workgroup; above, a lane-per-bin kernel writes per-bin
// totals into llf.
constexpr int kLoglikDetInTileMaxI = 4;

// Bits of DevState::flag, read by the host when the "check_finite" option is
// on (kernels set them with atomicOr; the host clears the flag first).
constexpr int kFlagNonFinite = 1;      // a NaN or Inf parameter after an update
constexpr int kFlagSingular = 2;       // a pivot <= 0 in an eq. 23 solve, a per-point C or a per-bin S_j
constexpr int kFlagNonPositive = 4;    // parameter check: v or lambda not positive and finite
constexpr int kFlagSingularParam = 8;  // parameter check: P(f) singular, or S_j not positive definite

// Internal layouts (library-owned):
//   xs   [F][2I][Npad]  split-complex mixture: plane i = Re x_i, plane I+i = Im x_i
//   vs   [F][J][Npad]   v_j(n,f), frames contiguous
//   lam  [F][J][I]      ABI layout
//   P    [F][I][I]      ABI layout (interleaved complex)
//   R    [F][J][I][I]   ABI layout; Rinv the same for S_j^-1 (EM only)
struct DevState {
  int F, N, Npad;
  int nchunk;     // tiles per bin of the AS streaming kernels
  int nchunk_em;  // tiles per bin of the EM kernels
  int K;          // fixed-point steps per hybrid iteration
  int p_update;   // P step: 0 fixed point (eq. 23), 1 gradient, 2 natural gradient, 3 Newton,
                  // 4 EM with P in the M-step
  float p_step;   // step size of the gradient-type P steps
  int sums_mfma;  // streaming pass B above I = 4: eq. 23 sums, 0 VALU, 1 / 2 matrix-core tiles, -1 by I
  const float* xs;
  float* vs;
  float* lam;
  float2* P;
  float2* R;
  float2* Rinv;
  float* partA;   // scratch per-tile partial sums
  float* partB;
  float* partE;   // EM with P in the M-step: per-tile sums [F][nchunk][J][I*I + I]
  double* partL;  // [F][max(nchunk, nchunk_em)]
  double* llf;    // [F]
  double* ll;     // [1]
  int* flag;      // [1] kFlag* bits
};

// Arguments of the adjoint kernels: the state before (t) and after (n) one
// iteration, the adjoints of the state after it (in) and of the state before
// it (out), and the mixture's adjoint xb [F][2I][Npad] (accumulated).
struct AdjIter {
  const float* S_t;   // eq. 23 sums of the iteration ([F][I][I*I] packed), or NULL: recomputed
  const float* v_t;
  const float* lam_t;
  const float2* P_t;
  const float* v_n;
  const float* lam_n;
  const float* vb_in;
  const float* lb_in;
  const float2* Pb_in;
  float* vb_out;
  float* lb_out;
  float2* Pb_out;
  float* xb;
};

// One checkpoint segment of the reverse pass in the tape (offsets in floats
// from tape): the state before iteration j at slot j (slot 0 = ck, slot j > 0
// at slot0 + j * stride), each state's v, lambda, P at v_off, lam_off,
// P_off; the eq. 23 sums of iteration j at S + j * S_floats (S NULL:
// recomputed); the adjoints of iterations len-1 .. 0 read buffer `cur` of
// vb / lb / Pb first and alternate.
struct AdjSeg {
  const float* tape;
  long long ck, slot0, stride, v_off, lam_off, P_off;
  const float* S;
  long long S_floats;
  float* vb[2];
  float* lb[2];
  float2* Pb[2];
  float* xb;
  int len, cur;
};

// Where a recording run of the frequency-resident FastFCA-AS kernel writes
// the state after each of its iterations: iteration it writes v, lambda and P
// at offset it * stride (floats) from v / lam / P (the layouts of DevState),
// and the eq. 23 sums S_c (packed Hermitian, [F][I][I*I]) at it * sstride
// from S.
struct Trace {
  float* v;
  float* lam;
  float2* P;
  float* S;
  long long stride;
  long long sstride;
};

// Host launchers of one (I, J) instantiation.
struct KernelSet {
  hipError_t (*as_iter_stream)(const DevState&, hipStream_t);
  hipError_t (*as_iter_resident)(const DevState&, hipStream_t, int n_iter, int waves, int bpw);
  int (*as_resident_fits)(int N, int waves, int bpw);
  hipError_t (*as_batch_resident)(const DevState* states, const int2* tiles, int ntiles, int n_max,
                                  hipStream_t, int n_iter, int waves, bool general,
                                  int* queue_counter,  // NULL: one workgroup per tile
                                  int* queued);        // out (may be NULL): 1 if the queue form ran
  hipError_t (*em_iter)(const DevState&, hipStream_t);
  hipError_t (*em_iter_resident)(const DevState&, hipStream_t, int n_iter, int waves);
  int (*em_resident_fits)(int N, int waves);
  hipError_t (*as_loglik)(const DevState&, hipStream_t);
  hipError_t (*em_loglik)(const DevState&, hipStream_t);
  hipError_t (*as_wiener)(const DevState&, hipStream_t, float2* out);
  hipError_t (*em_wiener)(const DevState&, hipStream_t, float2* out);
  hipError_t (*em_from_as)(const DevState&, hipStream_t);
  hipError_t (*em_rinv)(const DevState&, hipStream_t);
  hipError_t (*as_iter_resident_trace)(const DevState&, hipStream_t, int n_iter, int waves, int bpw,
                                       const Trace&);
  hipError_t (*adj_iter)(const DevState&, const AdjIter&, hipStream_t);
  hipError_t (*adj_seg)(const DevState&, const AdjSeg&, hipStream_t);
  hipError_t (*adj_wiener)(const DevState&, const float2* gout, const AdjIter&, hipStream_t);
  hipError_t (*check_matrices)(const DevState&, hipStream_t, int em);  // P(f) / S_j(f), kFlagSingularParam
};

// Non-templated kernels' launchers (fca_common.hip).
hipError_t launch_pack_x(const float2* x, float* xs, int F, int N, int I, int Npad, hipStream_t st);
hipError_t launch_pack_v(const float* v, float* vs, int F, int N, int J, int Npad, hipStream_t st);
hipError_t launch_unpack_v(const float* vs, float* v, int F, int N, int J, int Npad, hipStream_t st);
hipError_t launch_unpack_x(const float* xs, float2* x, int F, int N, int I, int Npad, hipStream_t st);
hipError_t launch_check_finite(const float* a, long long n, int* flag, hipStream_t st);
// v [F][J][Npad] (frames n < N) and lam (n_lam floats, may be NULL) positive
// and finite, else kFlagNonPositive.
hipError_t launch_check_positive(const float* vs, int F, int J, int N, int Npad, const float* lam, long long n_lam,
                                 int* flag, hipStream_t st);
// *flag = value, by a kernel (no memset node when a caller captures the stream).
hipError_t launch_set_flag(int* flag, int value, hipStream_t st);
hipError_t launch_sum_f(const double* llf, int F, double* out, hipStream_t st);
hipError_t launch_sum_chunks(const double* part, int F, int nchunk, double* out, hipStream_t st);

const KernelSet* kernel_set(int I, int J);  // NULL if not instantiated

}  // namespace fca
