// Per-point arithmetic of FastFCA-AS shared by the frequency-resident
// kernel (fca_resident.h), the streaming kernels (fca_kernels.h) and the
// adjoints: y = P^H x, the E-step with the v update and the eq. 20 summands,
// the eq. 23 weights, and packed Hermitian outer products.
#pragma once

#include "fca_device.h"
#include "fca_state.h"

namespace fca {

// ----------------------------------------------------------------------------
// Per-point arithmetic of FastFCA-AS.
// ----------------------------------------------------------------------------

// y = P^H x: y_i = sum_k conj(P_ki) x_k; returns |y_i|^2.
template <int I>
__device__ __forceinline__ void as_transform_pow(const float (&Pr)[I][I], const float (&Pi)[I][I],
                                                 const float (&xr)[I], const float (&xi)[I],
                                                 float (&y2)[I]) {
#pragma unroll
  for (int i = 0; i < I; ++i) {
    float yr = 0.f, yi = 0.f;
#pragma unroll
    for (int k = 0; k < I; ++k) {
      yr = fmaf(Pr[k][i], xr[k], yr);
      yr = fmaf(Pi[k][i], xi[k], yr);
      yi = fmaf(Pr[k][i], xi[k], yi);
      yi = fmaf(-Pi[k][i], xr[k], yi);
    }
    y2[i] = fmaf(yr, yr, yi * yi);
  }
}

template <int I>
__device__ __forceinline__ void as_transform(const float (&Pr)[I][I], const float (&Pi)[I][I],
                                             const float (&xr)[I], const float (&xi)[I],
                                             float (&yr)[I], float (&yi)[I]) {
#pragma unroll
  for (int i = 0; i < I; ++i) {
    float a = 0.f, b = 0.f;
#pragma unroll
    for (int k = 0; k < I; ++k) {
      a = fmaf(Pr[k][i], xr[k], a);
      a = fmaf(Pi[k][i], xi[k], a);
      b = fmaf(Pr[k][i], xi[k], b);
      b = fmaf(-Pi[k][i], xr[k], b);
    }
    yr[i] = a; yi[i] = b;
  }
}

// The part of as_point_em after e_i: W_j, the v update and the eq. 20 sums.
template <int I, int J>
__device__ __forceinline__ void as_point_em_e(const float (&e)[I], const float (&lamI)[J][I], float (&v)[J],
                                              float (&S0)[J], float (&S1)[J][I], bool take) {
#pragma unroll
  for (int j = 0; j < J; ++j) {
    float u = lamI[j][0] * e[0];
#pragma unroll
    for (int i = 1; i < I; ++i) u = fmaf(lamI[j][i], e[i], u);
    const float W = fmaf(v[j], u, 1.0f);
    // A lane that does not own a frame (take = false) keeps its v, so that
    // padded lanes stay finite over any number of iterations.
    const float rW = take ? rcp(W) : 0.f;
    const float m = v[j] * rW;
    S0[j] += rW;
#pragma unroll
    for (int i = 0; i < I; ++i) S1[j][i] = fmaf(m, e[i], S1[j][i]);
    v[j] = take ? v[j] * W : v[j];
  }
}

// E-step statistics and v update of one point, in a form with fewer
// operations that is algebraically identical to eq. 16-17, 19 and 20:
//   d_i = sum_j v_j lambda_ji,   g_ji = v_j lambda_ji / d_i  (diagonal Wiener gain),
//   (|mu~_ji|^2 + phi~_ji) / (v_j lambda_ji) = 1 - g_ji + g_ji |y_i|^2 / d_i
//                                            = 1 + v_j lambda_ji e_i =: r_ji,
//   with e_i = (|y_i|^2 / d_i - 1) / d_i;
//   v_j <- (1/I) sum_i v_j r_ji = v_j W_j,  W_j = 1 + v_j sum_i (lambda_ji / I) e_i  (eq. 19),
//   summand of eq. 20:  (|mu~|^2 + phi~)_ji / v_j(new) = lambda_ji r_ji / W_j
//                     = lambda_ji (1 / W_j + lambda_ji (v_j / W_j) e_i).
// The point adds 1 / W_j to S0[j] and (v_j / W_j) e_i to S1[j][i] (nothing
// when `take` is false) and updates v; after the frame sums the caller forms
// lambda_ji (S0_j + lambda_ji S1_ji) / N once per bin.  lamI = lambda / I.
template <int I, int J>
__device__ __forceinline__ void as_point_em(const float (&y2)[I], const float (&lam)[J][I],
                                            const float (&lamI)[J][I], float (&v)[J], float (&S0)[J],
                                            float (&S1)[J][I], bool take) {
  float e[I];
#pragma unroll
  for (int i = 0; i < I; ++i) {
    float d = v[0] * lam[0][i];
#pragma unroll
    for (int j = 1; j < J; ++j) d = fmaf(v[j], lam[j][i], d);
    const float t = rcp(d);
    e[i] = fmaf(y2[i], t, -1.0f) * t;
  }
  as_point_em_e<I, J>(e, lamI, v, S0, S1, take);
}

// The same with the reciprocals rd_i = 1 / d_i given (phase B of the
// previous iteration forms them as its eq. 23 weights, from the same v and
// lambda with the same operations, so the result is bitwise that of
// as_point_em).
template <int I, int J>
__device__ __forceinline__ void as_point_em_rd(const float (&y2)[I], const float (&rd)[I], const float (&lamI)[J][I],
                                               float (&v)[J], float (&S0)[J], float (&S1)[J][I], bool take) {
  float e[I];
#pragma unroll
  for (int i = 0; i < I; ++i) e[i] = fmaf(y2[i], rd[i], -1.0f) * rd[i];
  as_point_em_e<I, J>(e, lamI, v, S0, S1, take);
}

// Number of eq. 20 partial sums per bin or tile: S0 (J), then S1 (J x I).
template <int I, int J>
constexpr int kEq20Sums = J + J * I;

// lambda' = lambda (S0_j + lambda S1_ji) / N from the summed S0, S1 (eq. 20).
__device__ __forceinline__ float eq20_lambda(float lam, float s0, float s1, float invN) {
  return (lam * invN) * fmaf(lam, s1, s0);
}

// 1 / d_i with d_i = sum_j v_j lambda_ji (the weights of eq. 23).
template <int I, int J>
__device__ __forceinline__ void as_point_weights(const float (&lam)[J][I], const float (&v)[J],
                                                 float (&w)[I]) {
#pragma unroll
  for (int i = 0; i < I; ++i) {
    float d = 0.f;
#pragma unroll
    for (int j = 0; j < J; ++j) d = fmaf(v[j], lam[j][i], d);
    w[i] = rcp(d);
  }
}

// Packed Hermitian slot layout of an I x I matrix in I*I reals: slot (a, b)
// with a <= b holds Re A_ab, slot (b, a) with a < b holds Im A_ab.
// Adds w * x x^H, i.e. A_ab += w x_a conj(x_b).
// z = y y^H in the packed Hermitian layout of herm_rank1_acc.
template <int I>
__device__ __forceinline__ void herm_outer(float (&z)[I * I], const float (&yr)[I], const float (&yi)[I]) {
#pragma unroll
  for (int a = 0; a < I; ++a) {
    z[a * I + a] = fmaf(yr[a], yr[a], yi[a] * yi[a]);
#pragma unroll
    for (int b = a + 1; b < I; ++b) {
      z[a * I + b] = fmaf(yr[a], yr[b], yi[a] * yi[b]);
      z[b * I + a] = fmaf(yi[a], yr[b], -yr[a] * yi[b]);
    }
  }
}

template <int I>
__device__ __forceinline__ void herm_rank1_acc(float (&A)[I * I], float w, const float (&xr)[I],
                                               const float (&xi)[I]) {
#pragma unroll
  for (int a = 0; a < I; ++a) {
    A[a * I + a] = fmaf(w, fmaf(xr[a], xr[a], xi[a] * xi[a]), A[a * I + a]);
#pragma unroll
    for (int b = a + 1; b < I; ++b) {
      const float zr = fmaf(xr[a], xr[b], xi[a] * xi[b]);
      const float zi = fmaf(xi[a], xr[b], -xr[a] * xi[b]);
      A[a * I + b] = fmaf(w, zr, A[a * I + b]);
      A[b * I + a] = fmaf(w, zi, A[b * I + a]);
    }
  }
}

// Load the bin's P into registers from a staged copy.
template <int I>
__device__ __forceinline__ void load_P(const float2* __restrict__ Pg, float (&Pr)[I][I], float (&Pi)[I][I]) {
#pragma unroll
  for (int a = 0; a < I; ++a)
#pragma unroll
    for (int b = 0; b < I; ++b) {
      const float2 t = Pg[a * I + b];
      Pr[a][b] = t.x; Pi[a][b] = t.y;
    }
}

}  // namespace fca
