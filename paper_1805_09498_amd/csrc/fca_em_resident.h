// Frequency-resident conventional FCA EM (Section 3.3): the execution scheme
// of the resident FastFCA-AS kernel applied to the baseline.
#pragma once

#include "fca_kernels.h"
#include "fca_resident.h"

namespace fca {

// Frequency-resident conventional FCA EM (Section 3.3), the same execution
// scheme as k_as_resident: one workgroup per bin, the bin's x and v in
// registers, per iteration the summands of eq. 10 summed over the workgroup
// and S_j, S_j^-1 refreshed in LDS by lanes j < J of wave 0.
template <int I, int J>
constexpr bool em_resident_ok() { return J * I * I <= 64; }

template <int I, int J, int NPT>
__global__ __launch_bounds__(kResMaxBlock) void k_em_resident(DevState s, int n_iter) {
  constexpr int V = pad4(J * I * I);
  const int f = blockIdx.x;
  const int T = blockDim.x, nw = T / kWave;
  const int wbase = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave)) * kWave;
  __shared__ EmShared<I, J> sh;
  __shared__ float red[kResMaxWaves * V];
  em_load_shared<I, J>(s, f, sh);
  const float* xf = s.xs + (size_t)f * 2 * I * s.Npad;
  float* vf = s.vs + (size_t)f * J * s.Npad;
  float xr[NPT][I], xi[NPT][I], v[NPT][J];
#pragma unroll
  for (int k = 0; k < NPT; ++k) {
    const int n = threadIdx.x + k * T;
    const bool ok = n < s.N;
#pragma unroll
    for (int i = 0; i < I; ++i) {
      xr[k][i] = ok ? xf[(size_t)i * s.Npad + n] : 0.f;
      xi[k][i] = ok ? xf[(size_t)(I + i) * s.Npad + n] : 0.f;
    }
#pragma unroll
    for (int j = 0; j < J; ++j) v[k][j] = ok ? vf[(size_t)j * s.Npad + n] : 1.f;
  }
  __syncthreads();
  const float invN = 1.0f / float(s.N);
#pragma unroll 1
  for (int it = 0; it < n_iter; ++it) {
    // issue priority as in k_as_resident: the per-point sums low, the
    // cross-wave sums and the per-bin inversions (which every wave waits on)
    // high, so that two workgroups sharing a CU fill each other's gaps
    __builtin_amdgcn_s_setprio(0);
    float H[J][I * I];
#pragma unroll
    for (int j = 0; j < J; ++j)
#pragma unroll
      for (int q = 0; q < I * I; ++q) H[j][q] = 0.f;
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
      if (wbase + k * T < s.N) {
        const bool ok = threadIdx.x + k * T < s.N;
        if (!em_point<I, J>(sh, xr[k], xi[k], v[k], H, ok)) atomicOr(s.flag, kFlagSingular);
      }
    }
    float flat[J * I * I];
#pragma unroll
    for (int j = 0; j < J; ++j)
#pragma unroll
      for (int q = 0; q < I * I; ++q) flat[j * I * I + q] = H[j][q];
    __builtin_amdgcn_s_setprio(2);
    wave_totals_to_lds<J * I * I>(flat, red, V);
    __syncthreads();
    // S_j <- (1/N) sum_n Rhat_j / v_j (eq. 10), and S_j^-1 for eq. 9.
    if (wbase == 0 && threadIdx.x < J) {
      __builtin_amdgcn_s_setprio(3);
      const int j = threadIdx.x;
      float Rr[I][I], Ri[I][I], Xr[I][I], Xi[I][I];
      sum_waves<I * I>(red + j * I * I, V, nw, [&](int k, float t) {
        const int a = k / I, b = k % I;
        if (b >= a) Rr[a][b] = t * invN; else Ri[b][a] = t * invN;
      });
#pragma unroll
      for (int a = 0; a < I; ++a) {
        Ri[a][a] = 0.f;
#pragma unroll
        for (int b = a + 1; b < I; ++b) { Rr[b][a] = Rr[a][b]; Ri[b][a] = -Ri[a][b]; }
      }
      if (!herm_inv<I>(Rr, Ri, Xr, Xi)) atomicOr(s.flag, kFlagSingular);
#pragma unroll
      for (int a = 0; a < I; ++a)
#pragma unroll
        for (int b = 0; b < I; ++b) {
          sh.Rr[j][a][b] = Rr[a][b]; sh.Ri[j][a][b] = Ri[a][b];
          sh.Sr[j][a][b] = Xr[a][b]; sh.Si[j][a][b] = Xi[a][b];
        }
    }
    __syncthreads();
  }
#pragma unroll
  for (int k = 0; k < NPT; ++k) {
    const int n = threadIdx.x + k * T;
    if (n < s.N) {
#pragma unroll
      for (int j = 0; j < J; ++j) vf[(size_t)j * s.Npad + n] = v[k][j];
    }
  }
  for (int t = threadIdx.x; t < J * I * I; t += T) {
    const int j = t / (I * I), a = (t / I) % I, b = t % I;
    s.R[(size_t)f * J * I * I + t] = make_float2(sh.Rr[j][a][b], sh.Ri[j][a][b]);
    s.Rinv[(size_t)f * J * I * I + t] = make_float2(sh.Sr[j][a][b], sh.Si[j][a][b]);
  }
}

template <int I, int J>
int em_resident_fits(int N, int waves) {
  if constexpr (!em_resident_ok<I, J>()) {
    return 0;
  } else {
    if (waves != 1 && waves != 2 && waves != 4) return 0;
    return N <= 8 * waves * kWave ? 1 : 0;
  }
}

template <int I, int J>
hipError_t launch_em_iter_resident(const DevState& s, hipStream_t st, int n_iter, int waves) {
  if constexpr (!em_resident_ok<I, J>()) {
    return hipErrorInvalidValue;
  } else {
    const int T = waves * kWave;
    const int need = (s.N + T - 1) / T;
    dim3 grid(s.F), block(T);
    if (need <= 4)
      hipLaunchKernelGGL((k_em_resident<I, J, 4>), grid, block, 0, st, s, n_iter);
    else if (need <= 8)
      hipLaunchKernelGGL((k_em_resident<I, J, 8>), grid, block, 0, st, s, n_iter);
    else
      return hipErrorInvalidValue;
    return hipGetLastError();
  }
}

}  // namespace fca
