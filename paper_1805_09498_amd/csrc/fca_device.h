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

// Hardware reciprocal (v_rcp_f32, 1 ulp); used on every path, including the
// small per-bin solves.
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, kWave);
  return v;
}

// ---------------------------------------------------------------------------
// Transposed wave reduction (gfx950): V values per lane are summed over the
// 64 lanes with v_permlane32_swap / v_permlane16_swap (exchange of lane
// halves / quarters between two registers) and DPP row rotations, about 2V
// VALU operations in total instead of 6V cross-lane shuffles.
// On return out[m], in every lane of quarter Q = lane / 16, holds the wave
// total of value 4m + 2(Q & 1) + (Q >> 1).  V must be a multiple of 4.
// ---------------------------------------------------------------------------
template <int C>
__device__ __forceinline__ float dpp_row(float x) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), C, 0xF, 0xF, true));
}

__device__ __forceinline__ void swap_halves(float& a, float& b) {
  auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
  a = __uint_as_float(r[0]);
  b = __uint_as_float(r[1]);
}

__device__ __forceinline__ void swap_quarters(float& a, float& b) {
  auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false, false);
  a = __uint_as_float(r[0]);
  b = __uint_as_float(r[1]);
}

template <int V>
__device__ __forceinline__ void wave_reduce_t(const float (&a)[V], float (&out)[V / 4]) {
  static_assert(V % 4 == 0, "pad to a multiple of 4");
  float b[V / 2];
#pragma unroll
  for (int m = 0; m < V / 2; ++m) {
    float x = a[2 * m], y = a[2 * m + 1];
    swap_halves(x, y);  // x: [a2m lo | a2m+1 lo], y: [a2m hi | a2m+1 hi]
    b[m] = x + y;
  }
#pragma unroll
  for (int m = 0; m < V / 4; ++m) {
    float x = b[2 * m], y = b[2 * m + 1];
    swap_quarters(x, y);
    float c = x + y;
    c += dpp_row<0x128>(c);  // row_ror:8
    c += dpp_row<0x124>(c);  // row_ror:4
    c += dpp_row<0x122>(c);  // row_ror:2
    c += dpp_row<0x121>(c);  // row_ror:1
    out[m] = c;
  }
}

// Wave totals of V values written by lanes 0, 16, 32, 48 to
// part[wave * stride + k], k < V (stride >= pad4(V)).  Caller synchronises.
__host__ __device__ constexpr int pad4(int v) { return (v + 3) / 4 * 4; }

template <int V>
__device__ __forceinline__ void wave_totals_to_lds(const float (&a)[V], float* part, int stride) {
  constexpr int V4 = pad4(V);
  float p[V4];
#pragma unroll
  for (int k = 0; k < V4; ++k) p[k] = (k < V) ? a[k] : 0.f;
  float out[V4 / 4];
  wave_reduce_t<V4>(p, out);
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  if ((lane & 15) == 0) {
    const int q = lane >> 4;
    const int off = 2 * (q & 1) + (q >> 1);
#pragma unroll
    for (int m = 0; m < V4 / 4; ++m)
      if (4 * m + off < V) part[wave * stride + 4 * m + off] = out[m];
  }
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
    const float inv = rcp(den);
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
    const float inv = rcp(pr * pr + pi * pi);
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
    const float inv = rcp(den);
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
    const float ik = rcp(dk);
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

// ---------------------------------------------------------------------------
// Per-bin solves of eq. 23 for one column c (a per-lane runtime value).
// ---------------------------------------------------------------------------

// Column c of P^-H.  I <= 3: cofactors, (P^-H)_kc = conj(C_kc / det P) with
// C_kc the (k, c) cofactor of P; larger I: LU solve of P^H b = e_c.
template <int I>
__device__ __forceinline__ void pinvh_column(const float (&Pr)[I][I], const float (&Pi)[I][I], int c,
                                             float (&br)[I], float (&bi)[I]) {
  if constexpr (I <= 3) {
    float Cr[I][I], Ci[I][I];
#pragma unroll
    for (int k = 0; k < I; ++k)
#pragma unroll
      for (int l = 0; l < I; ++l) {
        if constexpr (I == 1) {
          Cr[k][l] = 1.f; Ci[k][l] = 0.f;
        } else if constexpr (I == 2) {
          const int r = 1 - k, q = 1 - l;
          const float sg = ((k + l) & 1) ? -1.f : 1.f;
          Cr[k][l] = sg * Pr[r][q]; Ci[k][l] = sg * Pi[r][q];
        } else {
          const int r0 = (k == 0) ? 1 : 0, r1 = (k == 2) ? 1 : 2;
          const int q0 = (l == 0) ? 1 : 0, q1 = (l == 2) ? 1 : 2;
          // m[r0][q0] m[r1][q1] - m[r0][q1] m[r1][q0]
          float dr = Pr[r0][q0] * Pr[r1][q1] - Pi[r0][q0] * Pi[r1][q1];
          float di = Pr[r0][q0] * Pi[r1][q1] + Pi[r0][q0] * Pr[r1][q1];
          dr -= Pr[r0][q1] * Pr[r1][q0] - Pi[r0][q1] * Pi[r1][q0];
          di -= Pr[r0][q1] * Pi[r1][q0] + Pi[r0][q1] * Pr[r1][q0];
          const float sg = ((k + l) & 1) ? -1.f : 1.f;
          Cr[k][l] = sg * dr; Ci[k][l] = sg * di;
        }
      }
    float detr = 0.f, deti = 0.f;  // expansion along column 0
#pragma unroll
    for (int k = 0; k < I; ++k) {
      detr += Pr[k][0] * Cr[k][0] - Pi[k][0] * Ci[k][0];
      deti += Pr[k][0] * Ci[k][0] + Pi[k][0] * Cr[k][0];
    }
    const float id = rcp(detr * detr + deti * deti);
    const float qr = detr * id, qi = -deti * id;  // 1 / det
#pragma unroll
    for (int k = 0; k < I; ++k) {
      float cr = Cr[k][0], ci = Ci[k][0];
#pragma unroll
      for (int l = 1; l < I; ++l) {
        cr = (c == l) ? Cr[k][l] : cr;
        ci = (c == l) ? Ci[k][l] : ci;
      }
      br[k] = cr * qr - ci * qi;       // conj(C / det)
      bi[k] = -(cr * qi + ci * qr);
    }
  } else {
    float Mr[I][I], Mi[I][I];
#pragma unroll
    for (int r = 0; r < I; ++r)
#pragma unroll
      for (int k = 0; k < I; ++k) { Mr[r][k] = Pr[k][r]; Mi[r][k] = -Pi[k][r]; }
#pragma unroll
    for (int r = 0; r < I; ++r) { br[r] = (r == c) ? 1.f : 0.f; bi[r] = 0.f; }
    lu_solve<I>(Mr, Mi, br, bi);
  }
}

// Solve Q p = b for a Hermitian positive-definite Q given by its upper
// triangle (Qr[a][b], Qi[a][b] for a <= b).  I <= 3: adjugate / determinant;
// larger I: Cholesky.  b is overwritten with p.
template <int I>
__device__ __forceinline__ void herm_solve(const float (&Qr)[I][I], const float (&Qi)[I][I],
                                           float (&br)[I], float (&bi)[I]) {
  if constexpr (I == 1) {
    const float iq = rcp(Qr[0][0]);
    br[0] *= iq; bi[0] *= iq;
  } else if constexpr (I == 2) {
    const float a = Qr[0][0], d = Qr[1][1], xr = Qr[0][1], xi = Qi[0][1];
    const float idet = rcp(a * d - (xr * xr + xi * xi));
    // adj = [[d, -x], [-conj(x), a]]
    const float p0r = d * br[0] - (xr * br[1] - xi * bi[1]);
    const float p0i = d * bi[0] - (xr * bi[1] + xi * br[1]);
    const float p1r = a * br[1] - (xr * br[0] + xi * bi[0]);
    const float p1i = a * bi[1] - (xr * bi[0] - xi * br[0]);
    br[0] = p0r * idet; bi[0] = p0i * idet; br[1] = p1r * idet; bi[1] = p1i * idet;
  } else if constexpr (I == 3) {
    // Q = [[a, x, y], [x*, d, z], [y*, z*, g]] with a, d, g real.
    const float a = Qr[0][0], d = Qr[1][1], g = Qr[2][2];
    const float xr = Qr[0][1], xi = Qi[0][1], yr = Qr[0][2], yi = Qi[0][2], zr = Qr[1][2], zi = Qi[1][2];
    const float x2 = xr * xr + xi * xi, y2 = yr * yr + yi * yi, z2 = zr * zr + zi * zi;
    // adjugate (Hermitian): diagonal and upper entries
    const float A00 = d * g - z2, A11 = a * g - y2, A22 = a * d - x2;
    // A01 = y conj(z) - x g
    const float A01r = (yr * zr + yi * zi) - xr * g, A01i = (yi * zr - yr * zi) - xi * g;
    // A02 = x z - y d
    const float A02r = (xr * zr - xi * zi) - yr * d, A02i = (xr * zi + xi * zr) - yi * d;
    // A12 = y conj(x) - a z
    const float A12r = (yr * xr + yi * xi) - a * zr, A12i = (yi * xr - yr * xi) - a * zi;
    // det = a A00 + 2 Re(x conj? ...) computed as a A00 + Re(x A10 + y A20) with A10 = conj(A01), A20 = conj(A02)
    const float det = a * A00 + (xr * A01r + xi * A01i) + (yr * A02r + yi * A02i);
    const float idet = rcp(det);
    const float b0r = br[0], b0i = bi[0], b1r = br[1], b1i = bi[1], b2r = br[2], b2i = bi[2];
    // p0 = A00 b0 + A01 b1 + A02 b2
    br[0] = (A00 * b0r + (A01r * b1r - A01i * b1i) + (A02r * b2r - A02i * b2i)) * idet;
    bi[0] = (A00 * b0i + (A01r * b1i + A01i * b1r) + (A02r * b2i + A02i * b2r)) * idet;
    // p1 = conj(A01) b0 + A11 b1 + A12 b2
    br[1] = ((A01r * b0r + A01i * b0i) + A11 * b1r + (A12r * b2r - A12i * b2i)) * idet;
    bi[1] = ((A01r * b0i - A01i * b0r) + A11 * b1i + (A12r * b2i + A12i * b2r)) * idet;
    // p2 = conj(A02) b0 + conj(A12) b1 + A22 b2
    br[2] = ((A02r * b0r + A02i * b0i) + (A12r * b1r + A12i * b1i) + A22 * b2r) * idet;
    bi[2] = ((A02r * b0i - A02i * b0r) + (A12r * b1i - A12i * b1r) + A22 * b2i) * idet;
  } else {
    float Lr[I][I], Li[I][I], dinv[I];
    cholesky<I>(Qr, Qi, Lr, Li, dinv);
    cholesky_solve<I>(Lr, Li, dinv, br, bi);
  }
}

// Inverse of a Hermitian positive-definite matrix given by its upper triangle
// (full result in Xr/Xi).  I <= 3: adjugate / determinant; larger I:
// Cholesky.
template <int I>
__device__ __forceinline__ void herm_inv(const float (&Ar)[I][I], const float (&Ai)[I][I],
                                         float (&Xr)[I][I], float (&Xi)[I][I]) {
  if constexpr (I == 1) {
    Xr[0][0] = rcp(Ar[0][0]); Xi[0][0] = 0.f;
  } else if constexpr (I == 2) {
    const float a = Ar[0][0], d = Ar[1][1], xr = Ar[0][1], xi = Ai[0][1];
    const float id = rcp(a * d - (xr * xr + xi * xi));
    Xr[0][0] = d * id; Xi[0][0] = 0.f; Xr[1][1] = a * id; Xi[1][1] = 0.f;
    Xr[0][1] = -xr * id; Xi[0][1] = -xi * id; Xr[1][0] = -xr * id; Xi[1][0] = xi * id;
  } else if constexpr (I == 3) {
    const float a = Ar[0][0], d = Ar[1][1], g = Ar[2][2];
    const float xr = Ar[0][1], xi = Ai[0][1], yr = Ar[0][2], yi = Ai[0][2], zr = Ar[1][2], zi = Ai[1][2];
    const float A00 = d * g - (zr * zr + zi * zi), A11 = a * g - (yr * yr + yi * yi), A22 = a * d - (xr * xr + xi * xi);
    const float A01r = (yr * zr + yi * zi) - xr * g, A01i = (yi * zr - yr * zi) - xi * g;
    const float A02r = (xr * zr - xi * zi) - yr * d, A02i = (xr * zi + xi * zr) - yi * d;
    const float A12r = (yr * xr + yi * xi) - a * zr, A12i = (yi * xr - yr * xi) - a * zi;
    const float id = rcp(a * A00 + (xr * A01r + xi * A01i) + (yr * A02r + yi * A02i));
    Xr[0][0] = A00 * id; Xi[0][0] = 0.f; Xr[1][1] = A11 * id; Xi[1][1] = 0.f; Xr[2][2] = A22 * id; Xi[2][2] = 0.f;
    Xr[0][1] = A01r * id; Xi[0][1] = A01i * id; Xr[1][0] = A01r * id; Xi[1][0] = -A01i * id;
    Xr[0][2] = A02r * id; Xi[0][2] = A02i * id; Xr[2][0] = A02r * id; Xi[2][0] = -A02i * id;
    Xr[1][2] = A12r * id; Xi[1][2] = A12i * id; Xr[2][1] = A12r * id; Xi[2][1] = -A12i * id;
  } else {
    herm_inverse<I>(Ar, Ai, Xr, Xi);
  }
}

}  // namespace fca
