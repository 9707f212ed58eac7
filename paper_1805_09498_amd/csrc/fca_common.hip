// Layout conversion, finiteness check and the final log-likelihood sum.
#include "fca_state.h"

namespace fca {

// x [F][N][I] interleaved complex -> xs [F][2I][Npad] split planes (zero pad).
__global__ void k_pack_x(const float2* __restrict__ x, float* __restrict__ xs, int F, int N, int I, int Npad) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)F * Npad) return;
  const int f = (int)(t / Npad), n = (int)(t % Npad);
  float* dst = xs + (size_t)f * 2 * I * Npad + n;
  for (int i = 0; i < I; ++i) {
    const float2 z = (n < N) ? x[((size_t)f * N + n) * I + i] : make_float2(0.f, 0.f);
    dst[(size_t)i * Npad] = z.x;
    dst[(size_t)(I + i) * Npad] = z.y;
  }
}

// v [F][N][J] -> vs [F][J][Npad] (padding set to 1 so that unused lanes stay finite).
__global__ void k_pack_v(const float* __restrict__ v, float* __restrict__ vs, int F, int N, int J, int Npad) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)F * Npad) return;
  const int f = (int)(t / Npad), n = (int)(t % Npad);
  for (int j = 0; j < J; ++j)
    vs[((size_t)f * J + j) * Npad + n] = (n < N) ? v[((size_t)f * N + n) * J + j] : 1.f;
}

__global__ void k_unpack_v(const float* __restrict__ vs, float* __restrict__ v, int F, int N, int J, int Npad) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)F * N) return;
  const int f = (int)(t / N), n = (int)(t % N);
  for (int j = 0; j < J; ++j) v[((size_t)f * N + n) * J + j] = vs[((size_t)f * J + j) * Npad + n];
}

// xs [F][2I][Npad] -> x [F][N][I] (interleaved complex).
__global__ void k_unpack_x(const float* __restrict__ xs, float2* __restrict__ x, int F, int N, int I, int Npad) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)F * N) return;
  const int f = (int)(t / N), n = (int)(t % N);
  const float* src = xs + (size_t)f * 2 * I * Npad + n;
  for (int i = 0; i < I; ++i) x[((size_t)f * N + n) * I + i] = make_float2(src[(size_t)i * Npad], src[(size_t)(I + i) * Npad]);
}

// Up to three device-to-device copies of float arrays in one launch
// (blockIdx.y picks the array; 16-byte moves where both ends allow them).
struct Copy3 {
  float* dst[3];
  const float* src[3];
  long long n[3];
};

__global__ void k_copy3(Copy3 c) {
  const int a = blockIdx.y;
  float* d = c.dst[a];
  const float* s = c.src[a];
  const long long n = c.n[a];
  const long long stride = (long long)gridDim.x * blockDim.x;
  const long long t0 = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (((reinterpret_cast<unsigned long long>(d) | reinterpret_cast<unsigned long long>(s)) & 15) == 0) {
    const long long n4 = n / 4;
    for (long long i = t0; i < n4; i += stride) reinterpret_cast<float4*>(d)[i] = reinterpret_cast<const float4*>(s)[i];
    for (long long i = n4 * 4 + t0; i < n; i += stride) d[i] = s[i];
  } else {
    for (long long i = t0; i < n; i += stride) d[i] = s[i];
  }
}

// A parameter reset in one launch: blockIdx.y = 0 packs v as k_pack_v does
// (grid-stride over the F Npad frames), y = 1 and 2 copy lambda and P as
// k_copy3 does (n = 0 skips an array).
__global__ void k_pack_v_copy2(const float* __restrict__ v, float* __restrict__ vs, int F, int N, int J, int Npad,
                               Copy3 c) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  const long long t0 = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (blockIdx.y == 0) {
    for (long long t = t0; t < (long long)F * Npad; t += stride) {
      const int f = (int)(t / Npad), n = (int)(t % Npad);
      for (int j = 0; j < J; ++j)
        vs[((size_t)f * J + j) * Npad + n] = (n < N) ? v[((size_t)f * N + n) * J + j] : 1.f;
    }
    return;
  }
  const int a = blockIdx.y - 1;
  float* d = c.dst[a];
  const float* s = c.src[a];
  const long long n = c.n[a];
  if (((reinterpret_cast<unsigned long long>(d) | reinterpret_cast<unsigned long long>(s)) & 15) == 0) {
    const long long n4 = n / 4;
    for (long long i = t0; i < n4; i += stride) reinterpret_cast<float4*>(d)[i] = reinterpret_cast<const float4*>(s)[i];
    for (long long i = n4 * 4 + t0; i < n; i += stride) d[i] = s[i];
  } else {
    for (long long i = t0; i < n; i += stride) d[i] = s[i];
  }
}

__global__ void k_check_finite(const float* __restrict__ a, long long n, int* flag) {
  long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long stride = (long long)gridDim.x * blockDim.x;
  bool bad = false;
  for (; t < n; t += stride) bad = bad || !isfinite(a[t]);
  if (bad) atomicOr(flag, kFlagNonFinite);
}

// Deterministic sum of n doubles (the log-likelihood partials of every
// tile), one workgroup in a fixed order.
__global__ void k_sum_f(const double* __restrict__ part, int n, double* out) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int k = threadIdx.x; k < n; k += blockDim.x) acc += part[k];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int m = 128; m > 0; m >>= 1) {
    if ((int)threadIdx.x < m) red[threadIdx.x] += red[threadIdx.x + m];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

__global__ void k_check_positive(const float* __restrict__ vs, int F, int J, int N, int Npad,
                                 const float* __restrict__ lam, long long n_lam, int* flag) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  const long long t0 = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  bool bad = false;
  const long long nv = (long long)F * J * Npad;
  for (long long t = t0; t < nv; t += stride) {
    const float x = vs[t];
    bad = bad || ((t % Npad) < N && !(x > 0.f && isfinite(x)));
  }
  for (long long t = t0; t < n_lam; t += stride) {
    const float x = lam[t];
    bad = bad || !(x > 0.f && isfinite(x));
  }
  if (bad) atomicOr(flag, kFlagNonPositive);
}

__global__ void k_set_int(int* p, int value) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *p = value;
}

// Per-bin totals of per-tile partials: out[f] = sum_c part[f * nchunk + c],
// in tile order (one lane per bin).
__global__ void k_sum_chunks(const double* __restrict__ part, int F, int nchunk, double* __restrict__ out) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= F) return;
  double acc = 0.0;
  for (int c = 0; c < nchunk; ++c) acc += part[(size_t)f * nchunk + c];
  out[f] = acc;
}

static unsigned blocks_for(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

hipError_t launch_pack_x(const float2* x, float* xs, int F, int N, int I, int Npad, hipStream_t st) {
  hipLaunchKernelGGL(k_pack_x, dim3(blocks_for((long long)F * Npad, 256)), dim3(256), 0, st, x, xs, F, N, I, Npad);
  return hipGetLastError();
}
hipError_t launch_copy3(float* d0, const float* s0, long long n0, float* d1, const float* s1, long long n1, float* d2,
                        const float* s2, long long n2, hipStream_t st) {
  Copy3 c{{d0, d1, d2}, {s0, s1, s2}, {n0 > 0 ? n0 : 0, n1 > 0 ? n1 : 0, n2 > 0 ? n2 : 0}};
  long long mx = c.n[0] > c.n[1] ? c.n[0] : c.n[1];
  mx = mx > c.n[2] ? mx : c.n[2];
  if (mx == 0) return hipSuccess;
  long long bx = (mx / 4 + 255) / 256;
  bx = bx < 1 ? 1 : (bx > 1024 ? 1024 : bx);
  hipLaunchKernelGGL(k_copy3, dim3((unsigned)bx, 3), dim3(256), 0, st, c);
  return hipGetLastError();
}

hipError_t launch_pack_v_copy2(const float* v, float* vs, int F, int N, int J, int Npad, float* d1, const float* s1,
                               long long n1, float* d2, const float* s2, long long n2, hipStream_t st) {
  Copy3 c{{d1, d2, nullptr}, {s1, s2, nullptr}, {n1 > 0 ? n1 : 0, n2 > 0 ? n2 : 0, 0}};
  const long long frames = (long long)F * Npad;
  long long bx = (frames + 255) / 256;
  bx = bx < 1 ? 1 : (bx > 4096 ? 4096 : bx);
  hipLaunchKernelGGL(k_pack_v_copy2, dim3((unsigned)bx, 3), dim3(256), 0, st, v, vs, F, N, J, Npad, c);
  return hipGetLastError();
}

hipError_t launch_pack_v(const float* v, float* vs, int F, int N, int J, int Npad, hipStream_t st) {
  hipLaunchKernelGGL(k_pack_v, dim3(blocks_for((long long)F * Npad, 256)), dim3(256), 0, st, v, vs, F, N, J, Npad);
  return hipGetLastError();
}
hipError_t launch_unpack_v(const float* vs, float* v, int F, int N, int J, int Npad, hipStream_t st) {
  hipLaunchKernelGGL(k_unpack_v, dim3(blocks_for((long long)F * N, 256)), dim3(256), 0, st, vs, v, F, N, J, Npad);
  return hipGetLastError();
}
hipError_t launch_unpack_x(const float* xs, float2* x, int F, int N, int I, int Npad, hipStream_t st) {
  hipLaunchKernelGGL(k_unpack_x, dim3(blocks_for((long long)F * N, 256)), dim3(256), 0, st, xs, x, F, N, I, Npad);
  return hipGetLastError();
}
hipError_t launch_check_finite(const float* a, long long n, int* flag, hipStream_t st) {
  long long b = (n + 255) / 256;
  if (b > 4096) b = 4096;
  if (b < 1) b = 1;
  hipLaunchKernelGGL(k_check_finite, dim3((unsigned)b), dim3(256), 0, st, a, n, flag);
  return hipGetLastError();
}
hipError_t launch_sum_f(const double* llf, int F, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_sum_f, dim3(1), dim3(256), 0, st, llf, F, out);
  return hipGetLastError();
}
hipError_t launch_check_positive(const float* vs, int F, int J, int N, int Npad, const float* lam, long long n_lam,
                                 int* flag, hipStream_t st) {
  const long long n = (long long)F * J * Npad > n_lam ? (long long)F * J * Npad : n_lam;
  long long b = (n + 255) / 256;
  b = b < 1 ? 1 : (b > 4096 ? 4096 : b);
  hipLaunchKernelGGL(k_check_positive, dim3((unsigned)b), dim3(256), 0, st, vs, F, J, N, Npad, lam, n_lam, flag);
  return hipGetLastError();
}
hipError_t launch_set_flag(int* flag, int value, hipStream_t st) {
  hipLaunchKernelGGL(k_set_int, dim3(1), dim3(64), 0, st, flag, value);
  return hipGetLastError();
}
hipError_t launch_sum_chunks(const double* part, int F, int nchunk, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_sum_chunks, dim3(blocks_for(F, 64)), dim3(64), 0, st, part, F, nchunk, out);
  return hipGetLastError();
}

}  // namespace fca
