// Frequency-resident FastFCA-AS: one workgroup owns one frequency bin for a
// whole batch of hybrid iterations.
//
// Bins never interact (every sum of eq. 20 and eq. 23 runs over n at fixed
// f), so a workgroup can load its bin's mixture x(., f) and spectra v(., f)
// into registers once, run n_iter iterations entirely on chip, and write
// v, lambda and P back at the end.  Lane t of a workgroup with T lanes owns
// frames n = t, t + T, ..., t + (NPT-1) T (coalesced loads and stores).
//
// Per iteration:  phase A (per point, eq. 15-19) -> workgroup sum of the eq. 20
// summands -> lambda in LDS -> phase B (per point weights, eq. 23 sums) ->
// workgroup sums -> lanes 0..I-1 solve one column of eq. 23 each -> P in LDS.
#pragma once

#include "fca_kernels.h"

namespace fca {

constexpr int kResMaxBlock = 256;

// Sum a register vector over the workgroup; the totals land in dst (LDS),
// visible to every lane after the call.  scratch holds nwaves * V floats.
template <int V>
__device__ __forceinline__ void wg_sum_to_lds(float (&a)[V], float* scratch, float* dst, int nwaves) {
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
#pragma unroll
  for (int k = 0; k < V; ++k) {
    const float t = wave_sum(a[k]);
    if (lane == 0) scratch[wave * V + k] = t;
  }
  __syncthreads();
  for (int k = threadIdx.x; k < V; k += blockDim.x) {
    float t = 0.f;
    for (int w = 0; w < nwaves; ++w) t += scratch[w * V + k];
    dst[k] = t;
  }
  __syncthreads();
}

template <int I, int J, int NPT>
__global__ __launch_bounds__(kResMaxBlock) void k_as_resident(DevState s, int n_iter) {
  const int f = blockIdx.x;
  const int T = blockDim.x, nw = T / kWave;
  __shared__ float sPr[I][I], sPi[I][I];
  __shared__ float sLam[J * I];
  __shared__ float sQ[I * I * I];
  __shared__ float scratch[(kResMaxBlock / kWave) * (J * I > I * I ? J * I : I * I)];

  for (int t = threadIdx.x; t < I * I; t += T) {
    const float2 p = s.P[(size_t)f * I * I + t];
    sPr[t / I][t % I] = p.x; sPi[t / I][t % I] = p.y;
  }
  for (int t = threadIdx.x; t < J * I; t += T) sLam[t] = s.lam[(size_t)f * J * I + t];

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
    // ---- phase A: E-step statistics, v update, eq. 20 partial sums --------
    float Pr[I][I], Pi[I][I], lam[J][I], ilamI[J][I];
#pragma unroll
    for (int a = 0; a < I; ++a)
#pragma unroll
      for (int b = 0; b < I; ++b) { Pr[a][b] = sPr[a][b]; Pi[a][b] = sPi[a][b]; }
#pragma unroll
    for (int j = 0; j < J; ++j)
#pragma unroll
      for (int i = 0; i < I; ++i) {
        lam[j][i] = sLam[j * I + i];
        ilamI[j][i] = rcp(float(I) * lam[j][i]);
      }
    float S[J][I];
#pragma unroll
    for (int j = 0; j < J; ++j)
#pragma unroll
      for (int i = 0; i < I; ++i) S[j][i] = 0.f;
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
      if (k * T < s.N) {  // uniform: skip slots no lane of the block owns
        const bool ok = threadIdx.x + k * T < s.N;
        float y2[I];
        as_transform_pow<I>(Pr, Pi, xr[k], xi[k], y2);
        as_point_em<I, J>(y2, lam, ilamI, v[k], S, ok);
      }
    }
    float flat[J * I];
#pragma unroll
    for (int j = 0; j < J; ++j)
#pragma unroll
      for (int i = 0; i < I; ++i) flat[j * I + i] = S[j][i];
    wg_sum_to_lds<J * I>(flat, scratch, sLam, nw);  // sLam <- sums; scaled below
#pragma unroll
    for (int j = 0; j < J; ++j)
#pragma unroll
      for (int i = 0; i < I; ++i) lam[j][i] = sLam[j * I + i] * invN;  // eq. 20

    // ---- phase B: weighted covariances of eq. 23 --------------------------
    float w[NPT][I];
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
      const bool ok = threadIdx.x + k * T < s.N;
      float wk[I];
      as_point_weights<I, J>(lam, v[k], wk);
#pragma unroll
      for (int i = 0; i < I; ++i) w[k][i] = ok ? wk[i] : 0.f;
    }
#pragma unroll 1
    for (int i = 0; i < I; ++i) {
      float A[I * I];
#pragma unroll
      for (int q = 0; q < I * I; ++q) A[q] = 0.f;
#pragma unroll
      for (int k = 0; k < NPT; ++k)
        if (k * T < s.N) herm_rank1_acc<I>(A, w[k][i], xr[k], xi[k]);
      wg_sum_to_lds<I * I>(A, scratch, sQ + i * I * I, nw);
    }
    for (int t = threadIdx.x; t < J * I; t += T) sLam[t] *= invN;

    // ---- per-bin solve: lane i computes column i of eq. 23 ----------------
    const int i = threadIdx.x;
    float Lr[I][I], Li[I][I], dinv[I];
    if (i < I) {
      float Qr[I][I], Qi[I][I];
#pragma unroll
      for (int a = 0; a < I; ++a) {
        Qr[a][a] = sQ[i * I * I + a * I + a] * invN; Qi[a][a] = 0.f;
#pragma unroll
        for (int b = a + 1; b < I; ++b) {
          Qr[a][b] = sQ[i * I * I + a * I + b] * invN;
          Qi[a][b] = sQ[i * I * I + b * I + a] * invN;
        }
      }
      cholesky<I>(Qr, Qi, Lr, Li, dinv);
    }
#pragma unroll 1
    for (int kk = 0; kk < s.K; ++kk) {
      float pr[I], pi[I];
      if (i < I) {
        float Mr[I][I], Mi[I][I];
#pragma unroll
        for (int r = 0; r < I; ++r)
#pragma unroll
          for (int c = 0; c < I; ++c) { Mr[r][c] = sPr[c][r]; Mi[r][c] = -sPi[c][r]; }
#pragma unroll
        for (int r = 0; r < I; ++r) { pr[r] = (r == i) ? 1.f : 0.f; pi[r] = 0.f; }
        lu_solve<I>(Mr, Mi, pr, pi);
        cholesky_solve<I>(Lr, Li, dinv, pr, pi);
      }
      __syncthreads();
      if (i < I) {
#pragma unroll
        for (int a = 0; a < I; ++a) { sPr[a][i] = pr[a]; sPi[a][i] = pi[a]; }
      }
      __syncthreads();
    }
  }

  // ---- write the state back ------------------------------------------------
#pragma unroll
  for (int k = 0; k < NPT; ++k) {
    const int n = threadIdx.x + k * T;
    if (n < s.N) {
#pragma unroll
      for (int j = 0; j < J; ++j) vf[(size_t)j * s.Npad + n] = v[k][j];
    }
  }
  for (int t = threadIdx.x; t < I * I; t += T)
    s.P[(size_t)f * I * I + t] = make_float2(sPr[t / I][t % I], sPi[t / I][t % I]);
  if (n_iter > 0)
    for (int t = threadIdx.x; t < J * I; t += T) s.lam[(size_t)f * J * I + t] = sLam[t];
}

// Register budget of the resident kernel: NPT points of 2I + J floats each.
template <int I, int J>
constexpr int res_max_npt() {
  return (16 * (2 * I + J) <= 224) ? 16 : (8 * (2 * I + J) <= 224) ? 8 : 4;
}

template <int I, int J>
int as_resident_fits(int N, int waves) {
  if (waves < 1 || waves > kResMaxBlock / kWave) return 0;
  return N <= res_max_npt<I, J>() * waves * kWave ? 1 : 0;
}

template <int I, int J>
hipError_t launch_as_iter_resident(const DevState& s, hipStream_t st, int n_iter, int waves) {
  const int T = waves * kWave;
  const int need = (s.N + T - 1) / T;
  dim3 grid(s.F), block(T);
  if (need <= 4)
    hipLaunchKernelGGL((k_as_resident<I, J, 4>), grid, block, 0, st, s, n_iter);
  else if (need <= 8 && res_max_npt<I, J>() >= 8)
    hipLaunchKernelGGL((k_as_resident<I, J, 8>), grid, block, 0, st, s, n_iter);
  else if (need <= 16 && res_max_npt<I, J>() >= 16)
    hipLaunchKernelGGL((k_as_resident<I, J, 16>), grid, block, 0, st, s, n_iter);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace fca
