// STFT front and back end (C ABI, declared in include/fastfca.h): the
// analysis and overlap-add synthesis of the experiments (Table 1 of the
// paper: 16 kHz, 1024-sample frames, shift 512, square root of a Hann window
// for analysis and synthesis), so that waveforms go in and separated
// waveforms come out.
//
// Framing: frame n covers samples n H - (W - H) .. n H - (W - H) + W - 1
// (zero outside the signal), N = floor((L - 1 + W - H) / H) + 1, so every
// sample lies in W / H frames; window w[t] = sin(pi t / W) (square root of
// the periodic Hann window); bins f = 0 .. W/2.  Synthesis multiplies each
// inverse-transformed frame by w and 2H / W and overlaps-and-adds, which
// inverts the analysis for H = W / R, R >= 2.
//
// Transforms: an in-LDS radix-2 decimation-in-time FFT, one workgroup per
// (frame, channel[, source]); twiddles from sincospif, written once per
// workgroup.  Overlap-add sums each output sample's frames in a fixed order.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "fca_internal.h"

namespace {

constexpr int kFftBlock = 256;

__device__ __forceinline__ unsigned bitrev(unsigned v, int bits) { return __brev(v) >> (32 - bits); }

// In-place transform of buf[W] (bit-reversed input), sign -1 (analysis) or +1.
__device__ void fft_lds(float2* buf, float2* tw, int W, int logW, float sign) {
  for (int k = threadIdx.x; k < W / 2; k += blockDim.x) {
    float s, c;
    sincospif(sign * 2.0f * (float)k / (float)W, &s, &c);
    tw[k] = make_float2(c, s);
  }
  __syncthreads();
  for (int st = 1; st <= logW; ++st) {
    const int half = 1 << (st - 1);
    for (int b = threadIdx.x; b < W / 2; b += blockDim.x) {
      const int pos = b & (half - 1);
      const int i0 = ((b >> (st - 1)) << st) + pos, i1 = i0 + half;
      const float2 w = tw[pos << (logW - st)];
      const float2 u = buf[i0], v = buf[i1];
      const float2 t = make_float2(w.x * v.x - w.y * v.y, w.x * v.y + w.y * v.x);
      buf[i0] = make_float2(u.x + t.x, u.y + t.y);
      buf[i1] = make_float2(u.x - t.x, u.y - t.y);
    }
    __syncthreads();
  }
}

// wav [C][L] -> X [F][N][C]; grid (N, C).
__global__ __launch_bounds__(kFftBlock) void k_stft(const float* __restrict__ wav, int C, int L, int W, int logW,
                                                    int H, int N, float2* __restrict__ X) {
  extern __shared__ float2 sm[];
  float2* buf = sm;
  float2* tw = sm + W;
  const int n = blockIdx.x, c = blockIdx.y;
  const long long first = (long long)n * H - (W - H);
  for (int t = threadIdx.x; t < W; t += blockDim.x) {
    const long long k = first + t;
    const float s = (k >= 0 && k < L) ? wav[(size_t)c * L + k] * sinpif((float)t / (float)W) : 0.f;
    buf[bitrev((unsigned)t, logW)] = make_float2(s, 0.f);
  }
  __syncthreads();
  fft_lds(buf, tw, W, logW, -1.f);
  const int F = W / 2 + 1;
  for (int f = threadIdx.x; f < F; f += blockDim.x) X[((size_t)f * N + n) * C + c] = buf[f];
}

// S [J][F][N][C] -> frames [J][C][N][W] (windowed, scaled); grid (N, C, J).
__global__ __launch_bounds__(kFftBlock) void k_istft_frames(const float2* __restrict__ S, int C, int N, int W,
                                                            int logW, float scale, float* __restrict__ frames) {
  extern __shared__ float2 sm[];
  float2* buf = sm;
  float2* tw = sm + W;
  const int n = blockIdx.x, c = blockIdx.y, j = blockIdx.z;
  const int F = W / 2 + 1;
  for (int t = threadIdx.x; t < W; t += blockDim.x) {
    const int f = t <= W / 2 ? t : W - t;
    float2 z = S[(((size_t)j * F + f) * N + n) * C + c];
    if (f == 0 || f == W / 2) z.y = 0.f;  // a real frame: only the real parts of these bins count
    if (t > W / 2) z.y = -z.y;            // Hermitian extension
    buf[bitrev((unsigned)t, logW)] = z;
  }
  __syncthreads();
  fft_lds(buf, tw, W, logW, 1.f);
  float* out = frames + (((size_t)j * C + c) * N + n) * W;
  for (int t = threadIdx.x; t < W; t += blockDim.x) out[t] = buf[t].x * scale * sinpif((float)t / (float)W);
}

// frames [JC][N][W] -> wav [JC][L]: each sample sums its frames in frame order.
__global__ void k_ola(const float* __restrict__ frames, int JC, int N, int W, int H, int L, float* __restrict__ wav) {
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= (long long)JC * L) return;
  const int jc = (int)(g / L), t = (int)(g % L);
  const int u = t + (W - H);                       // position in the padded signal
  int n_lo = u - W + 1 > 0 ? (u - W + 1 + H - 1) / H : 0;
  int n_hi = u / H;
  if (n_hi > N - 1) n_hi = N - 1;
  float acc = 0.f;
  for (int n = n_lo; n <= n_hi; ++n) acc += frames[((size_t)jc * N + n) * W + (u - n * H)];
  wav[g] = acc;
}

bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

fca_status check_frame(int W, int H, int* logW) {
  int lg = 0;
  while ((1 << lg) < W) ++lg;
  if (W < 16 || W > 4096 || (1 << lg) != W)
    return fca::ctx_fail(nullptr, FCA_ERR_ARG, "frame must be a power of two in 16..4096");
  if (H < 1 || W % H != 0 || W / H < 2)
    return fca::ctx_fail(nullptr, FCA_ERR_ARG, "hop must divide the frame and be at most half of it");
  *logW = lg;
  return FCA_OK;
}

}  // namespace

extern "C" {

fca_status fca_stft_shape(int L, int frame, int hop, int* F, int* N) {
  int lg;
  if (!F || !N || L < 1) return fca::ctx_fail(nullptr, FCA_ERR_ARG, "L must be positive and F, N non-NULL");
  fca_status st = check_frame(frame, hop, &lg);
  if (st != FCA_OK) return st;
  const long long n = ((long long)L - 1 + frame - hop) / hop + 1;
  if (n > (1 << 30)) return fca::ctx_fail(nullptr, FCA_ERR_ARG, "signal too long");
  *F = frame / 2 + 1;
  *N = (int)n;
  return FCA_OK;
}

fca_status fca_stft(const float* wav, int C, int L, int frame, int hop, fca_c64* X, void* hip_stream) {
  int F = 0, N = 0, lg = 0;
  fca_status st = fca_stft_shape(L, frame, hop, &F, &N);
  if (st != FCA_OK) return st;
  check_frame(frame, hop, &lg);
  if (C < 1 || !wav || !X || !aligned(wav, 4) || !aligned(X, 8))
    return fca::ctx_fail(nullptr, FCA_ERR_ARG, "C must be positive; wav and X non-NULL, aligned device pointers");
  if ((double)F * N * C >= 2147483648.0 || (double)C * L >= 2147483648.0)  // no overflow for any ints
    return fca::ctx_fail(nullptr, FCA_ERR_ARG, "signal too large");
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  const size_t lds = sizeof(float2) * (size_t)(frame + frame / 2);
  hipLaunchKernelGGL(k_stft, dim3(N, C), dim3(kFftBlock), lds, s, wav, C, L, frame, lg, hop, N,
                     reinterpret_cast<float2*>(X));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fca::ctx_hip_fail(nullptr, e, "fca_stft");
  return FCA_OK;
}

fca_status fca_istft(const fca_c64* S, int J, int C, int N, int frame, int hop, int L, float* wav, void* hip_stream) {
  int F = 0, Nl = 0, lg = 0;
  fca_status st = fca_stft_shape(L, frame, hop, &F, &Nl);
  if (st != FCA_OK) return st;
  check_frame(frame, hop, &lg);
  if (N != Nl) return fca::ctx_fail(nullptr, FCA_ERR_ARG, "N does not match the frame count of an L-sample signal");
  if (J < 1 || C < 1 || !S || !wav || !aligned(S, 8) || !aligned(wav, 4))
    return fca::ctx_fail(nullptr, FCA_ERR_ARG, "J, C must be positive; S and wav non-NULL, aligned device pointers");
  if ((double)J * C * N * frame >= 2147483648.0 || (double)J * C * L >= 2147483648.0)
    return fca::ctx_fail(nullptr, FCA_ERR_ARG, "signal too large");
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  float* frames = nullptr;
  hipError_t e = hipMallocAsync(reinterpret_cast<void**>(&frames), sizeof(float) * (size_t)J * C * N * frame, s);
  if (e != hipSuccess) return fca::ctx_hip_fail(nullptr, e, "fca_istft scratch");
  const float scale = 2.0f * (float)hop / ((float)frame * (float)frame);  // 1/W of the inverse DFT, 2H/W of the overlap
  const size_t lds = sizeof(float2) * (size_t)(frame + frame / 2);
  hipLaunchKernelGGL(k_istft_frames, dim3(N, C, J), dim3(kFftBlock), lds, s, reinterpret_cast<const float2*>(S), C,
                     N, frame, lg, scale, frames);
  e = hipGetLastError();
  if (e == hipSuccess) {
    const long long total = (long long)J * C * L;
    hipLaunchKernelGGL(k_ola, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, frames, J * C, N, frame, hop,
                       L, wav);
    e = hipGetLastError();
  }
  hipError_t e2 = hipFreeAsync(frames, s);
  if (e != hipSuccess) return fca::ctx_hip_fail(nullptr, e, "fca_istft");
  if (e2 != hipSuccess) return fca::ctx_hip_fail(nullptr, e2, "fca_istft scratch");
  return FCA_OK;
}

}  // extern "C"
