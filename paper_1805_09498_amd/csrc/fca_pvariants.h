// The P updates of Section 4.5 that replace the fixed-point step with a
// per-bin step of another kind, on the streaming path:
//
//  * Newton's method (p_update 3): one Newton step on L2 (eq. 14) in P alone,
//    v and lambda held at the values the EM step just produced.  Written
//    relative to the current P as P_new = P (1 + X): with G_i = P^H Q_i P the
//    weighted covariances of eq. 23 in the basis of y (the sums pass B
//    already forms) and Gamma's column i = G_i e_i, the Newton equations are
//      [G_1 X_1, ..., G_I X_I] + X^H = 1 - Gamma,
//    a real-linear system (X^H couples X_ai with X_ia).  L2 ignores the
//    phase of each column of P, so the imaginary diagonal of X is fixed at
//    0 and the matching equations (imaginary parts of the diagonal) are
//    dropped: 2I^2 - I real unknowns and equations, solved per bin by
//    Gaussian elimination with partial pivoting in LDS.
//
//  * EM with P in the M-step (p_update 4): the M-step raises the Q-function
//    (eq. 18) over P as well.  In the basis of y the posterior moments of
//    source j are mu~_j = g_j o y (g_ji = v_j lambda_ji / d_i) and the
//    diagonal phi~_j = v_j lambda_j (1 - g_j) (eq. 16-17); with the new v',
//    lambda', Q depends on A = P_old^-1 P through
//      2NJ ln|det A| - NJ sum_i a_i^H H_i a_i,
//      H_i = (1/(NJ)) sum_j (T_j + diag(Phi_j)) / lambda'_ji,
//      T_j = sum_n mu~_j mu~_j^H / v'_j,   Phi_j = sum_n phi~_j / v'_j.
//    k_as_pass_emp forms T_j and Phi_j per tile (before pass A overwrites v;
//    v' = v W is a per-point quantity), k_as_emp_step sweeps the columns:
//    a_i <- H_i^-1 [A^-H]_i scaled to a_i^H H_i a_i = 1 (each the maximiser
//    of Q over that column), then P_new = P_old A.
#pragma once

#include "fca_device.h"
#include "fca_point.h"
#include "fca_state.h"

namespace fca {

// ----------------------------------------------------------------------------
// EM with P in the M-step.
// ----------------------------------------------------------------------------
template <int I>
constexpr int kEmpV = I * I + I;  // per source: T_j (packed Hermitian) and Phi_j

// One tile (bin f = blockIdx.y, frames of chunk blockIdx.x) and one source
// j = blockIdx.z: the tile's sums of T_j and Phi_j.
template <int I, int J>
__global__ __launch_bounds__(kBlock) void k_as_pass_emp(DevState s) {
  const int f = blockIdx.y, chunk = blockIdx.x, j = blockIdx.z;
  constexpr int V = kEmpV<I>;
  constexpr int VP = pad4(V);
  __shared__ float2 sP[I * I];
  __shared__ float sLam[J * I];
  __shared__ float red[kBlock / kWave][VP];
  for (int t = threadIdx.x; t < I * I; t += kBlock) sP[t] = s.P[(size_t)f * I * I + t];
  for (int t = threadIdx.x; t < J * I; t += kBlock) sLam[t] = s.lam[(size_t)f * J * I + t];
  __syncthreads();
  float Pr[I][I], Pi[I][I], lam[J][I];
  load_P<I>(sP, Pr, Pi);
#pragma unroll
  for (int k = 0; k < J; ++k)
#pragma unroll
    for (int i = 0; i < I; ++i) lam[k][i] = sLam[k * I + i];
  const float* xf = s.xs + (size_t)f * 2 * I * s.Npad;
  const float* vf = s.vs + (size_t)f * J * s.Npad;
  float acc[V];
#pragma unroll
  for (int q = 0; q < V; ++q) acc[q] = 0.f;
#pragma unroll 1
  for (int p = 0; p < kPts; ++p) {
    const int n = chunk * kChunk + p * kBlock + threadIdx.x;
    if (n >= s.N) continue;
    float xr[I], xi[I], yr[I], yi[I], v[J];
#pragma unroll
    for (int i = 0; i < I; ++i) { xr[i] = xf[(size_t)i * s.Npad + n]; xi[i] = xf[(size_t)(I + i) * s.Npad + n]; }
#pragma unroll
    for (int k = 0; k < J; ++k) v[k] = vf[(size_t)k * s.Npad + n];
    as_transform<I>(Pr, Pi, xr, xi, yr, yi);
    // d_i, e_i = (|y_i|^2 / d_i - 1) / d_i, and W_j = v'_j / v_j (eq. 19)
    float rd[I], u = 0.f;
#pragma unroll
    for (int i = 0; i < I; ++i) {
      float d = 0.f;
#pragma unroll
      for (int k = 0; k < J; ++k) d = fmaf(v[k], lam[k][i], d);
      rd[i] = rcp(d);
      const float e = fmaf(fmaf(yr[i], yr[i], yi[i] * yi[i]), rd[i], -1.0f) * rd[i];
      u = fmaf(lam[j][i], e, u);
    }
    const float W = fmaf(v[j] * (1.0f / float(I)), u, 1.0f);
    const float iv = rcp(v[j] * W);  // 1 / v'_j
    float zr[I], zi[I];
#pragma unroll
    for (int i = 0; i < I; ++i) {
      const float vl = v[j] * lam[j][i];
      const float g = vl * rd[i];
      zr[i] = g * yr[i];
      zi[i] = g * yi[i];
      acc[I * I + i] = fmaf(vl * (1.0f - g), iv, acc[I * I + i]);  // phi~_ji / v'_j
    }
    float T[I * I];
#pragma unroll
    for (int q = 0; q < I * I; ++q) T[q] = acc[q];
    herm_rank1_acc<I>(T, iv, zr, zi);
#pragma unroll
    for (int q = 0; q < I * I; ++q) acc[q] = T[q];
  }
  wave_totals_to_lds<V>(acc, &red[0][0], VP);
  __syncthreads();
  float* out = s.partE + (((size_t)f * s.nchunk + chunk) * J + j) * V;
  for (int t = threadIdx.x; t < V; t += kBlock) {
    float w = 0.f;
#pragma unroll
    for (int k = 0; k < kBlock / kWave; ++k) w += red[k][t];
    out[t] = w;
  }
}

// One lane per bin: H_i from the tile sums and the new lambda (in s.lam
// after k_as_solve), the column sweep, P_new = P_old A.
template <int I, int J>
__global__ __launch_bounds__(64) void k_as_emp_step(DevState s) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= s.F) return;
  constexpr int V = kEmpV<I>;
  const float scale = 1.0f / (float(s.N) * float(J));
  float Ar[I][I], Ai[I][I];
#pragma unroll
  for (int a = 0; a < I; ++a)
#pragma unroll
    for (int b = 0; b < I; ++b) { Ar[a][b] = (a == b) ? 1.f : 0.f; Ai[a][b] = 0.f; }
  bool ok = true;
#pragma unroll 1
  for (int i = 0; i < I; ++i) {
    // H_i (upper triangle; packed slots as herm_rank1_acc)
    float Hq[I * I], Hd[I];
#pragma unroll
    for (int q = 0; q < I * I; ++q) Hq[q] = 0.f;
#pragma unroll
    for (int a = 0; a < I; ++a) Hd[a] = 0.f;
    for (int j = 0; j < J; ++j) {
      const float w = rcp(s.lam[((size_t)f * J + j) * I + i]);
      float Tq[V];
#pragma unroll
      for (int q = 0; q < V; ++q) Tq[q] = 0.f;
      for (int c = 0; c < s.nchunk; ++c) {
        const float* src = s.partE + (((size_t)f * s.nchunk + c) * J + j) * V;
#pragma unroll
        for (int q = 0; q < V; ++q) Tq[q] += src[q];
      }
#pragma unroll
      for (int q = 0; q < I * I; ++q) Hq[q] = fmaf(w, Tq[q], Hq[q]);
#pragma unroll
      for (int a = 0; a < I; ++a) Hd[a] = fmaf(w, Tq[I * I + a], Hd[a]);
    }
    float Hr[I][I], Hi[I][I];
#pragma unroll
    for (int a = 0; a < I; ++a) {
      Hr[a][a] = (Hq[a * I + a] + Hd[a]) * scale;
      Hi[a][a] = 0.f;
#pragma unroll
      for (int b = a + 1; b < I; ++b) {
        Hr[a][b] = Hq[a * I + b] * scale; Hi[a][b] = Hq[b * I + a] * scale;
        Hr[b][a] = Hr[a][b]; Hi[b][a] = -Hi[a][b];
      }
    }
    // z = A^-H e_i: solve A^H z = e_i
    float Mr[I][I], Mi[I][I], zr[I], zi[I];
#pragma unroll
    for (int a = 0; a < I; ++a) {
      zr[a] = (a == i) ? 1.f : 0.f; zi[a] = 0.f;
#pragma unroll
      for (int b = 0; b < I; ++b) { Mr[a][b] = Ar[b][a]; Mi[a][b] = -Ai[b][a]; }
    }
    ok = lu_solve<I>(Mr, Mi, zr, zi) && ok;
    ok = herm_solve<I>(Hr, Hi, zr, zi) && ok;  // a = H_i^-1 z
    // scale to a^H H_i a = 1 (the maximiser over the column)
    float q = 0.f;
#pragma unroll
    for (int a = 0; a < I; ++a) {
      float hr = 0.f, hi = 0.f;
#pragma unroll
      for (int b = 0; b < I; ++b) {
        hr = fmaf(Hr[a][b], zr[b], hr); hr = fmaf(-Hi[a][b], zi[b], hr);
        hi = fmaf(Hr[a][b], zi[b], hi); hi = fmaf(Hi[a][b], zr[b], hi);
      }
      q = fmaf(zr[a], hr, fmaf(zi[a], hi, q));
    }
    const float sc = __builtin_sqrtf(rcp(q));
#pragma unroll
    for (int a = 0; a < I; ++a) {
#pragma unroll
      for (int b = 0; b < I; ++b) {
        Ar[a][b] = (b == i) ? zr[a] * sc : Ar[a][b];
        Ai[a][b] = (b == i) ? zi[a] * sc : Ai[a][b];
      }
    }
  }
  if (!ok) atomicOr(s.flag, kFlagSingular);
  // P_new = P_old A
  float Pr[I][I], Pi[I][I];
  load_P<I>(s.P + (size_t)f * I * I, Pr, Pi);
#pragma unroll
  for (int a = 0; a < I; ++a)
#pragma unroll
    for (int c = 0; c < I; ++c) {
      float pr = 0.f, pi = 0.f;
#pragma unroll
      for (int b = 0; b < I; ++b) {
        pr = fmaf(Pr[a][b], Ar[b][c], pr); pr = fmaf(-Pi[a][b], Ai[b][c], pr);
        pi = fmaf(Pr[a][b], Ai[b][c], pi); pi = fmaf(Pi[a][b], Ar[b][c], pi);
      }
      s.P[(size_t)f * I * I + a * I + c] = make_float2(pr, pi);
    }
}

// ----------------------------------------------------------------------------
// Newton's method.
// ----------------------------------------------------------------------------
constexpr int kNewtonThreads = 256;

template <int I>
constexpr int kNewtonN = 2 * I * I - I;  // real unknowns and equations

// Unknown / equation index of the real part of entry (a, c) of X, and of
// the imaginary part of an off-diagonal entry (a != c).
template <int I>
__device__ __forceinline__ int nt_re(int a, int c) { return a * I + c; }
template <int I>
__device__ __forceinline__ int nt_im(int a, int c) { return I * I + a * (I - 1) + (c < a ? c : c - 1); }

// Entry (a, b) of G_i from the packed Hermitian S_i (real parts on and above
// the diagonal, imaginary parts of the upper triangle below it), times invN.
template <int I>
__device__ __forceinline__ float2 nt_G(const float* S, int a, int b, float invN) {
  if (a == b) return make_float2(S[a * I + a] * invN, 0.f);
  if (a < b) return make_float2(S[a * I + b] * invN, S[b * I + a] * invN);
  return make_float2(S[b * I + a] * invN, -S[a * I + b] * invN);
}

// One workgroup per bin: build the Newton system from the totals of the
// eq. 23 sums (left by k_as_solve in the bin's first tile slot of partB),
// eliminate with partial pivoting, back-substitute, P_new = P_old (1 + X).
template <int I, int J>
__global__ __launch_bounds__(kNewtonThreads) void k_as_newton(DevState s) {
  constexpr int n = kNewtonN<I>;
  constexpr int W = n + 1;  // augmented row
  const int f = blockIdx.x;
  __shared__ float M[n][W];
  __shared__ float S[I][I * I];
  __shared__ float xs[n];
  __shared__ int piv;
  __shared__ int bad;
  const float invN = 1.0f / float(s.N);
  const float* tot = s.partB + (size_t)f * s.nchunk * I * I * I;
  for (int t = threadIdx.x; t < I * I * I; t += blockDim.x) S[t / (I * I)][t % (I * I)] = tot[t];
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  // rows: real part of equation (a, i) for every (a, i), imaginary part for
  // a != i; equation (a, i): sum_b G_i(a,b) X(b,i) + conj(X(i,a)) = delta_ai - G_i(a,i)
  for (int r = threadIdx.x; r < n; r += blockDim.x) {
    for (int c = 0; c < W; ++c) M[r][c] = 0.f;
    const bool re = r < I * I;
    int a = r / I, i = r % I;
    if constexpr (I > 1) {
      if (!re) { const int o = r - I * I; a = o / (I - 1); const int k = o % (I - 1); i = k < a ? k : k + 1; }
    }
    for (int b = 0; b < I; ++b) {
      const float2 g = nt_G<I>(S[i], a, b, invN);
      if (re) {
        M[r][nt_re<I>(b, i)] += g.x;
        if (b != i) M[r][nt_im<I>(b, i)] -= g.y;
      } else {
        if (b != i) M[r][nt_im<I>(b, i)] += g.x;
        M[r][nt_re<I>(b, i)] += g.y;
      }
    }
    const float2 gai = nt_G<I>(S[i], a, i, invN);
    if (re) {
      M[r][nt_re<I>(i, a)] += 1.f;
      M[r][n] = ((a == i) ? 1.f : 0.f) - gai.x;
    } else {
      M[r][nt_im<I>(i, a)] -= 1.f;
      M[r][n] = -gai.y;
    }
  }
  __syncthreads();
  // elimination with partial pivoting
  for (int k = 0; k < n; ++k) {
    if (threadIdx.x < kWave) {
      float best = -1.f;
      int row = k;
      for (int r = k + threadIdx.x; r < n; r += kWave) {
        const float m = fabsf(M[r][k]);
        if (m > best) { best = m; row = r; }
      }
#pragma unroll
      for (int m = 32; m >= 1; m >>= 1) {
        const float ob = __shfl_xor(best, m, kWave);
        const int orow = __shfl_xor(row, m, kWave);
        if (ob > best || (ob == best && orow < row)) { best = ob; row = orow; }
      }
      if (threadIdx.x == 0) {
        piv = row;
        if (!(best > 0.f)) bad = 1;
      }
    }
    __syncthreads();
    const int p = piv;
    if (p != k)
      for (int c = k + threadIdx.x; c < W; c += blockDim.x) {
        const float t = M[k][c]; M[k][c] = M[p][c]; M[p][c] = t;
      }
    __syncthreads();
    const float ipiv = 1.0f / M[k][k];
    const int rows = n - k - 1, cols = W - k - 1;
    for (int t = threadIdx.x; t < rows * cols; t += blockDim.x) {
      const int r = k + 1 + t / cols, c = k + 1 + t % cols;
      M[r][c] = fmaf(-M[r][k] * ipiv, M[k][c], M[r][c]);
    }
    __syncthreads();
  }
  // back substitution: the first wave forms each unknown, the barrier
  // publishes it to the next row's dot product
  for (int k = n - 1; k >= 0; --k) {
    if (threadIdx.x < kWave) {
      float part = 0.f;
      for (int c = k + 1 + threadIdx.x; c < n; c += kWave) part = fmaf(M[k][c], xs[c], part);
#pragma unroll
      for (int m = 32; m >= 1; m >>= 1) part += __shfl_xor(part, m, kWave);
      if (threadIdx.x == 0) xs[k] = (M[k][n] - part) / M[k][k];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0 && bad) atomicOr(s.flag, kFlagSingular);
  // P_new = P_old (1 + X): entry (a, c) = P_ac + sum_b P_ab X_bc, formed in
  // LDS first (the row a is read by several threads before any write)
  __shared__ float2 Pn[I * I];
  const float2* Pf = s.P + (size_t)f * I * I;
  for (int t = threadIdx.x; t < I * I; t += blockDim.x) {
    const int a = t / I, c = t % I;
    float2 acc = Pf[a * I + c];
    for (int b = 0; b < I; ++b) {
      const float2 pb = Pf[a * I + b];
      const float xr = xs[nt_re<I>(b, c)], xi = (b == c) ? 0.f : xs[nt_im<I>(b, c)];
      acc.x = fmaf(pb.x, xr, fmaf(-pb.y, xi, acc.x));
      acc.y = fmaf(pb.x, xi, fmaf(pb.y, xr, acc.y));
    }
    Pn[t] = acc;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < I * I; t += blockDim.x) s.P[(size_t)f * I * I + t] = Pn[t];
}

}  // namespace fca
