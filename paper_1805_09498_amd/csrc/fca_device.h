// Device building blocks shared by the libfastfca kernels (gfx950).
//
// Everything here is per-lane arithmetic on register arrays whose sizes are
// compile-time constants (I microphones, J sources), so loops unroll and the
// arrays stay in VGPRs.  Complex numbers are kept as separate re/im floats.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fca {

constexpr int kWave = 64;

__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// Full-precision reciprocal for the per-bin solves (off the per-point path).
__device__ __forceinline__ float rcp_exact(float x) { return 1.0f / x; }

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, kWave);
  return v;
}

__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, kWave);
  return v;
}

// ---------------------------------------------------------------------------
// Small dense complex linear algebra, one matrix per lane.
// ---------------------------------------------------------------------------

// Solve M z = rhs for one right-hand side by Gaussian elimination with
// partial pivoting (the pivot of column k is the largest-modulus entry at or
// below the diagonal).  M and rhs are destroyed.  Returns false when a pivot
// is exactly zero.
template <int I>
__device__ inline bool lu_solve(float (&Mr)[I][I], float (&Mi)[I][I], float (&br)[I], float (&bi)[I]) {
  bool ok = true;
#pragma unroll
  for (int k = 0; k < I; ++k) {
#pragma unroll
    for (int r = k + 1; r < I; ++r) {
      const float cur = Mr[k][k] * Mr[k][k] + Mi[k][k] * Mi[k][k];
      const float cand = Mr[r][k] * Mr[r][k] + Mi[r][k] * Mi[r][k];
      if (cand > cur) {
#pragma unroll
        for (int c = 0; c < I; ++c) {
          float t = Mr[k][c]; Mr[k][c] = Mr[r][c]; Mr[r][c] = t;
          t = Mi[k][c]; Mi[k][c] = Mi[r][c]; Mi[r][c] = t;
        }
        float t = br[k]; br[k] = br[r]; br[r] = t;
        t = bi[k]; bi[k] = bi[r]; bi[r] = t;
      }
    }
    const float pr = Mr[k][k], pi = Mi[k][k];
    const float den = pr * pr + pi * pi;
    ok = ok && (den > 0.0f);
    const float inv = rcp_exact(den);
    const float qr = pr * inv, qi = -pi * inv;  // 1 / pivot
#pragma unroll
    for (int r = k + 1; r < I; ++r) {
      const float lr = Mr[r][k] * qr - Mi[r][k] * qi;
      const float li = Mr[r][k] * qi + Mi[r][k] * qr;
#pragma unroll
      for (int c = k + 1; c < I; ++c) {
        Mr[r][c] -= lr * Mr[k][c] - li * Mi[k][c];
        Mi[r][c] -= lr * Mi[k][c] + li * Mr[k][c];
      }
      br[r] -= lr * br[k] - li * bi[k];
      bi[r] -= lr * bi[k] + li * br[k];
    }
  }
#pragma unroll
  for (int k = I - 1; k >= 0; --k) {
    float sr = br[k], si = bi[k];
#pragma unroll
    for (int c = k + 1; c < I; ++c) {
      sr -= Mr[k][c] * br[c] - Mi[k][c] * bi[c];
      si -= Mr[k][c] * bi[c] + Mi[k][c] * br[c];
    }
    const float pr = Mr[k][k], pi = Mi[k][k];
    const float inv = rcp_exact(pr * pr + pi * pi);
    br[k] = (sr * pr + si * pi) * inv;
    bi[k] = (si * pr - sr * pi) * inv;
  }
  return ok;
}

// ln|det M| by the same elimination (M destroyed).
template <int I>
__device__ inline float lu_logabsdet(float (&Mr)[I][I], float (&Mi)[I][I]) {
  float acc = 0.0f;
#pragma unroll
  for (int k = 0; k < I; ++k) {
#pragma unroll
    for (int r = k + 1; r < I; ++r) {
      const float cur = Mr[k][k] * Mr[k][k] + Mi[k][k] * Mi[k][k];
      const float cand = Mr[r][k] * Mr[r][k] + Mi[r][k] * Mi[r][k];
      if (cand > cur) {
#pragma unroll
        for (int c = 0; c < I; ++c) {
          float t = Mr[k][c]; Mr[k][c] = Mr[r][c]; Mr[r][c] = t;
          t = Mi[k][c]; Mi[k][c] = Mi[r][c]; Mi[r][c] = t;
        }
      }
    }
    const float pr = Mr[k][k], pi = Mi[k][k];
    const float den = pr * pr + pi * pi;
    acc += 0.5f * __logf(den);
    const float inv = rcp_exact(den);
    const float qr = pr * inv, qi = -pi * inv;
#pragma unroll
    for (int r = k + 1; r < I; ++r) {
      const float lr = Mr[r][k] * qr - Mi[r][k] * qi;
      const float li = Mr[r][k] * qi + Mi[r][k] * qr;
#pragma unroll
      for (int c = k + 1; c < I; ++c) {
        Mr[r][c] -= lr * Mr[k][c] - li * Mi[k][c];
        Mi[r][c] -= lr * Mi[k][c] + li * Mr[k][c];
      }
    }
  }
  return acc;
}

// Cholesky factor of a Hermitian positive-definite matrix given by its upper
// triangle: A = L L^H with L lower triangular and real positive diagonal.
// On return Lr/Li hold L (strictly-upper part unused) and dinv the
// reciprocal diagonal.  Returns false if A is not numerically PD.
template <int I>
__device__ inline bool cholesky(const float (&Ar)[I][I], const float (&Ai)[I][I],
                                float (&Lr)[I][I], float (&Li)[I][I], float (&dinv)[I]) {
  bool ok = true;
#pragma unroll
  for (int k = 0; k < I; ++k) {
    float s = Ar[k][k];
#pragma unroll
    for (int m = 0; m < k; ++m) s -= Lr[k][m] * Lr[k][m] + Li[k][m] * Li[k][m];
    ok = ok && (s > 0.0f);
    const float dk = __builtin_sqrtf(fmaxf(s, 1e-37f));
    const float ik = rcp_exact(dk);
    Lr[k][k] = dk; Li[k][k] = 0.0f; dinv[k] = ik;
#pragma unroll
    for (int r = k + 1; r < I; ++r) {
      // A[r][k] = conj(A[k][r]);  L[r][k] = (A[r][k] - sum_m L[r][m] conj(L[k][m])) / L[k][k]
      float sr = Ar[k][r], si = -Ai[k][r];
#pragma unroll
      for (int m = 0; m < k; ++m) {
        sr -= Lr[r][m] * Lr[k][m] + Li[r][m] * Li[k][m];
        si -= Li[r][m] * Lr[k][m] - Lr[r][m] * Li[k][m];
      }
      Lr[r][k] = sr * ik; Li[r][k] = si * ik;
    }
  }
  return ok;
}

// Solve (L L^H) z = b in place.
template <int I>
__device__ inline void cholesky_solve(const float (&Lr)[I][I], const float (&Li)[I][I],
                                      const float (&dinv)[I], float (&br)[I], float (&bi)[I]) {
#pragma unroll
  for (int k = 0; k < I; ++k) {
    float sr = br[k], si = bi[k];
#pragma unroll
    for (int m = 0; m < k; ++m) {
      sr -= Lr[k][m] * br[m] - Li[k][m] * bi[m];
      si -= Lr[k][m] * bi[m] + Li[k][m] * br[m];
    }
    br[k] = sr * dinv[k]; bi[k] = si * dinv[k];
  }
#pragma unroll
  for (int k = I - 1; k >= 0; --k) {
    float sr = br[k], si = bi[k];
#pragma unroll
    for (int m = k + 1; m < I; ++m) {
      // conj(L[m][k]) * b[m]
      sr -= Lr[m][k] * br[m] + Li[m][k] * bi[m];
      si -= Lr[m][k] * bi[m] - Li[m][k] * br[m];
    }
    br[k] = sr * dinv[k]; bi[k] = si * dinv[k];
  }
}

// Inverse of a Hermitian PD matrix (upper triangle in A) from its Cholesky
// factor: full matrix written to Xr/Xi.  Returns false if not PD.
template <int I>
__device__ inline bool herm_inverse(const float (&Ar)[I][I], const float (&Ai)[I][I],
                                    float (&Xr)[I][I], float (&Xi)[I][I]) {
  float Lr[I][I], Li[I][I], dinv[I];
  const bool ok = cholesky<I>(Ar, Ai, Lr, Li, dinv);
#pragma unroll
  for (int c = 0; c < I; ++c) {
    float br[I], bi[I];
#pragma unroll
    for (int k = 0; k < I; ++k) { br[k] = (k == c) ? 1.0f : 0.0f; bi[k] = 0.0f; }
    cholesky_solve<I>(Lr, Li, dinv, br, bi);
#pragma unroll
    for (int k = 0; k < I; ++k) { Xr[k][c] = br[k]; Xi[k][c] = bi[k]; }
  }
  return ok;
}

}  // namespace fca
