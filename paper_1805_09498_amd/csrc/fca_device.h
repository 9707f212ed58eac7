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

// Scalar helpers of the per-bin solvers, which run in float or double.
template <typename T>
__device__ __forceinline__ T rcpT(T x);
template <>
__device__ __forceinline__ float rcpT<float>(float x) { return __builtin_amdgcn_rcpf(x); }
// Hardware estimate refined by two Newton steps r <- r + r (1 - x r) (each
// squares the relative error), instead of the longer IEEE division sequence.
template <>
__device__ __forceinline__ double rcpT<double>(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
  return __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
}
__device__ __forceinline__ float sqrtT(float x) { return __builtin_sqrtf(x); }
__device__ __forceinline__ double sqrtT(double x) { return __builtin_sqrt(x); }

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

// ---------------------------------------------------------------------------
// Small dense complex linear algebra, one matrix per lane.
// ---------------------------------------------------------------------------

// Solve M z = rhs for one right-hand side by Gaussian elimination with
// partial pivoting (the pivot of column k is the largest-modulus entry at or
// below the diagonal).  M and rhs are destroyed.  Returns false when a pivot
// is exactly zero.
template <int I, typename T = float>
__device__ inline bool lu_solve(T (&Mr)[I][I], T (&Mi)[I][I], T (&br)[I], T (&bi)[I]) {
  bool ok = true;
#pragma unroll
  for (int k = 0; k < I; ++k) {
#pragma unroll
    for (int r = k + 1; r < I; ++r) {
      const T cur = Mr[k][k] * Mr[k][k] + Mi[k][k] * Mi[k][k];
      const T cand = Mr[r][k] * Mr[r][k] + Mi[r][k] * Mi[r][k];
      if (cand > cur) {
#pragma unroll
        for (int c = 0; c < I; ++c) {
          T t = Mr[k][c]; Mr[k][c] = Mr[r][c]; Mr[r][c] = t;
          t = Mi[k][c]; Mi[k][c] = Mi[r][c]; Mi[r][c] = t;
        }
        T t = br[k]; br[k] = br[r]; br[r] = t;
        t = bi[k]; bi[k] = bi[r]; bi[r] = t;
      }
    }
    const T pr = Mr[k][k], pi = Mi[k][k];
    const T den = pr * pr + pi * pi;
    ok = ok && (den > T(0));
    const T inv = rcpT(den);
    const T qr = pr * inv, qi = -pi * inv;  // 1 / pivot
#pragma unroll
    for (int r = k + 1; r < I; ++r) {
      const T lr = Mr[r][k] * qr - Mi[r][k] * qi;
      const T li = Mr[r][k] * qi + Mi[r][k] * qr;
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
    T sr = br[k], si = bi[k];
#pragma unroll
    for (int c = k + 1; c < I; ++c) {
      sr -= Mr[k][c] * br[c] - Mi[k][c] * bi[c];
      si -= Mr[k][c] * bi[c] + Mi[k][c] * br[c];
    }
    const T pr = Mr[k][k], pi = Mi[k][k];
    const T inv = rcpT(pr * pr + pi * pi);
    br[k] = (sr * pr + si * pi) * inv;
    bi[k] = (si * pr - sr * pi) * inv;
  }
  return ok;
}

// Cholesky factor of a Hermitian positive-definite matrix given by its upper
// triangle: A = L L^H with L lower triangular and real positive diagonal.
// On return Lr/Li hold L (strictly-upper part unused) and dinv the
// reciprocal diagonal.  Returns false if a pivot is <= 0 (A not numerically
// positive definite).
template <int I, typename T = float>
__device__ inline bool cholesky(const T (&Ar)[I][I], const T (&Ai)[I][I],
                                T (&Lr)[I][I], T (&Li)[I][I], T (&dinv)[I]) {
  bool ok = true;
#pragma unroll
  for (int k = 0; k < I; ++k) {
    T s = Ar[k][k];
#pragma unroll
    for (int m = 0; m < k; ++m) s -= Lr[k][m] * Lr[k][m] + Li[k][m] * Li[k][m];
    ok = ok && !(s <= T(0));  // NaN passes: it is reported as a non-finite value instead
    const T dk = sqrtT(s > T(1e-37) ? s : T(1e-37));
    const T ik = rcpT(dk);
    Lr[k][k] = dk; Li[k][k] = T(0); dinv[k] = ik;
#pragma unroll
    for (int r = k + 1; r < I; ++r) {
      // A[r][k] = conj(A[k][r]);  L[r][k] = (A[r][k] - sum_m L[r][m] conj(L[k][m])) / L[k][k]
      T sr = Ar[k][r], si = -Ai[k][r];
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
template <int I, typename T = float>
__device__ inline void cholesky_solve(const T (&Lr)[I][I], const T (&Li)[I][I],
                                      const T (&dinv)[I], T (&br)[I], T (&bi)[I]) {
#pragma unroll
  for (int k = 0; k < I; ++k) {
    T sr = br[k], si = bi[k];
#pragma unroll
    for (int m = 0; m < k; ++m) {
      sr -= Lr[k][m] * br[m] - Li[k][m] * bi[m];
      si -= Lr[k][m] * bi[m] + Li[k][m] * br[m];
    }
    br[k] = sr * dinv[k]; bi[k] = si * dinv[k];
  }
#pragma unroll
  for (int k = I - 1; k >= 0; --k) {
    T sr = br[k], si = bi[k];
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
template <int I, typename T = float>
__device__ inline bool herm_inverse(const T (&Ar)[I][I], const T (&Ai)[I][I],
                                    T (&Xr)[I][I], T (&Xi)[I][I]) {
  T Lr[I][I], Li[I][I], dinv[I];
  const bool ok = cholesky<I, T>(Ar, Ai, Lr, Li, dinv);
#pragma unroll
  for (int c = 0; c < I; ++c) {
    T br[I], bi[I];
#pragma unroll
    for (int k = 0; k < I; ++k) { br[k] = (k == c) ? T(1) : T(0); bi[k] = T(0); }
    cholesky_solve<I, T>(Lr, Li, dinv, br, bi);
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
template <int I, typename T = float>
__device__ __forceinline__ void pinvh_column(const T (&Pr)[I][I], const T (&Pi)[I][I], int c,
                                             T (&br)[I], T (&bi)[I]) {
  if constexpr (I <= 3) {
    T Cr[I][I], Ci[I][I];
#pragma unroll
    for (int k = 0; k < I; ++k)
#pragma unroll
      for (int l = 0; l < I; ++l) {
        if constexpr (I == 1) {
          Cr[k][l] = T(1); Ci[k][l] = T(0);
        } else if constexpr (I == 2) {
          const int r = 1 - k, q = 1 - l;
          const T sg = ((k + l) & 1) ? -T(1) : T(1);
          Cr[k][l] = sg * Pr[r][q]; Ci[k][l] = sg * Pi[r][q];
        } else {
          const int r0 = (k == 0) ? 1 : 0, r1 = (k == 2) ? 1 : 2;
          const int q0 = (l == 0) ? 1 : 0, q1 = (l == 2) ? 1 : 2;
          // m[r0][q0] m[r1][q1] - m[r0][q1] m[r1][q0]
          T dr = Pr[r0][q0] * Pr[r1][q1] - Pi[r0][q0] * Pi[r1][q1];
          T di = Pr[r0][q0] * Pi[r1][q1] + Pi[r0][q0] * Pr[r1][q1];
          dr -= Pr[r0][q1] * Pr[r1][q0] - Pi[r0][q1] * Pi[r1][q0];
          di -= Pr[r0][q1] * Pi[r1][q0] + Pi[r0][q1] * Pr[r1][q0];
          const T sg = ((k + l) & 1) ? -T(1) : T(1);
          Cr[k][l] = sg * dr; Ci[k][l] = sg * di;
        }
      }
    T detr = T(0), deti = T(0);  // expansion along column 0
#pragma unroll
    for (int k = 0; k < I; ++k) {
      detr += Pr[k][0] * Cr[k][0] - Pi[k][0] * Ci[k][0];
      deti += Pr[k][0] * Ci[k][0] + Pi[k][0] * Cr[k][0];
    }
    const T id = rcpT(detr * detr + deti * deti);
    const T qr = detr * id, qi = -deti * id;  // 1 / det
#pragma unroll
    for (int k = 0; k < I; ++k) {
      T cr = Cr[k][0], ci = Ci[k][0];
#pragma unroll
      for (int l = 1; l < I; ++l) {
        cr = (c == l) ? Cr[k][l] : cr;
        ci = (c == l) ? Ci[k][l] : ci;
      }
      br[k] = cr * qr - ci * qi;       // conj(C / det)
      bi[k] = -(cr * qi + ci * qr);
    }
  } else {
    T Mr[I][I], Mi[I][I];
#pragma unroll
    for (int r = 0; r < I; ++r)
#pragma unroll
      for (int k = 0; k < I; ++k) { Mr[r][k] = Pr[k][r]; Mi[r][k] = -Pi[k][r]; }
#pragma unroll
    for (int r = 0; r < I; ++r) { br[r] = (r == c) ? T(1) : T(0); bi[r] = T(0); }
    lu_solve<I, T>(Mr, Mi, br, bi);
  }
}

// Column c of P^-H (c may differ between lanes) from single-precision P,
// computed in precision T.  Row c of P^-1 is the vector w with w^T P_l = 0
// for l != c and w^T P_c = 1 (bilinear, no conjugation), and [P^-H]_c is
// conj(w).  For I <= 3 the unnormalised w is the other column turned by a
// quarter (I = 2) or the cross product of the two other columns (I = 3);
// dividing by w^T P_c normalises it, whatever the order of the columns.  The
// columns are picked in single precision and widened afterwards.  Larger I:
// LU solve in T.
// A value the optimiser cannot trace back to the array element it came from:
// selects between such values stay register selects instead of becoming a
// lane-dependent index into a private (scratch) copy of the array.
__device__ __forceinline__ float opaque(float x) {
  asm("" : "+v"(x));
  return x;
}

template <int I, typename T>
__device__ __forceinline__ void pinvh_col(const float (&Pr)[I][I], const float (&Pi)[I][I], int c,
                                          T (&br)[I], T (&bi)[I]) {
  if constexpr (I == 1) {
    const T pr = Pr[0][0], pi = Pi[0][0];
    const T id = rcpT(pr * pr + pi * pi);
    br[0] = pr * id; bi[0] = pi * id;  // conj(1 / p) = p / |p|^2
  } else if constexpr (I <= 3) {
    float Mr[I][I], Mi[I][I];
#pragma unroll
    for (int a = 0; a < I; ++a)
#pragma unroll
      for (int b = 0; b < I; ++b) { Mr[a][b] = opaque(Pr[a][b]); Mi[a][b] = opaque(Pi[a][b]); }
    T pr[I], pi[I], wr[I], wi[I];
    if constexpr (I == 2) {
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        pr[k] = (c == 0) ? Mr[k][0] : Mr[k][1];
        pi[k] = (c == 0) ? Mi[k][0] : Mi[k][1];
      }
      const T a0r = (c == 0) ? Mr[0][1] : Mr[0][0], a0i = (c == 0) ? Mi[0][1] : Mi[0][0];
      const T a1r = (c == 0) ? Mr[1][1] : Mr[1][0], a1i = (c == 0) ? Mi[1][1] : Mi[1][0];
      wr[0] = a1r; wi[0] = a1i; wr[1] = -a0r; wi[1] = -a0i;
    } else {
      T ar[3], ai[3], er[3], ei[3];  // the two other columns, in index order
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        pr[k] = (c == 0) ? Mr[k][0] : ((c == 1) ? Mr[k][1] : Mr[k][2]);
        pi[k] = (c == 0) ? Mi[k][0] : ((c == 1) ? Mi[k][1] : Mi[k][2]);
        ar[k] = (c == 0) ? Mr[k][1] : Mr[k][0];
        ai[k] = (c == 0) ? Mi[k][1] : Mi[k][0];
        er[k] = (c == 2) ? Mr[k][1] : Mr[k][2];
        ei[k] = (c == 2) ? Mi[k][1] : Mi[k][2];
      }
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const int k1 = (k + 1) % 3, k2 = (k + 2) % 3;
        // w_k = a_k1 e_k2 - a_k2 e_k1
        wr[k] = (ar[k1] * er[k2] - ai[k1] * ei[k2]) - (ar[k2] * er[k1] - ai[k2] * ei[k1]);
        wi[k] = (ar[k1] * ei[k2] + ai[k1] * er[k2]) - (ar[k2] * ei[k1] + ai[k2] * er[k1]);
      }
    }
    T sr = T(0), si = T(0);  // s = w^T P_c
#pragma unroll
    for (int k = 0; k < I; ++k) {
      sr += wr[k] * pr[k] - wi[k] * pi[k];
      si += wr[k] * pi[k] + wi[k] * pr[k];
    }
    const T id = rcpT(sr * sr + si * si);
    const T qr = sr * id, qi = -si * id;  // 1 / s
#pragma unroll
    for (int k = 0; k < I; ++k) {
      br[k] = wr[k] * qr - wi[k] * qi;    // conj(w / s)
      bi[k] = -(wr[k] * qi + wi[k] * qr);
    }
  } else {
    T Pdr[I][I], Pdi[I][I];
#pragma unroll
    for (int a = 0; a < I; ++a)
#pragma unroll
      for (int b = 0; b < I; ++b) { Pdr[a][b] = Pr[a][b]; Pdi[a][b] = Pi[a][b]; }
    pinvh_column<I, T>(Pdr, Pdi, c, br, bi);
  }
}


// Solve Q p = b for a Hermitian positive-definite Q given by its upper
// triangle (Qr[a][b], Qi[a][b] for a <= b).  I <= 2: adjugate / determinant;
// I = 3: LDL^H; larger I: Cholesky.  b is overwritten with p.  Returns false
// when a pivot (or, for I = 2, the determinant) is <= 0: Q is not
// numerically positive definite.  A NaN pivot returns true (the result is
// reported as a non-finite value instead).
//
// Why not the 3x3 adjugate: near DC a diffuse field makes Q nearly rank one.
// The 2x2 minors of such a matrix cancel to O(lambda_1 lambda_2) from terms
// of O(lambda_1^2), and combining them cancels again, so the adjugate solve
// loses about cond(Q)^2 eps (1e-3 in single precision at cond ~ 1e3), while
// an LDL^H or Cholesky factorisation loses cond(Q) eps.  For I = 2 the
// adjugate entries are entries of Q and only the determinant cancels, which
// also costs cond(Q) eps.
template <int I, typename T = float>
__device__ __forceinline__ bool herm_solve(const T (&Qr)[I][I], const T (&Qi)[I][I],
                                           T (&br)[I], T (&bi)[I]) {
  if constexpr (I == 1) {
    const T iq = rcpT(Qr[0][0]);
    br[0] *= iq; bi[0] *= iq;
    return !(Qr[0][0] <= T(0));
  } else if constexpr (I == 2) {
    const T a = Qr[0][0], d = Qr[1][1], xr = Qr[0][1], xi = Qi[0][1];
    const T det = a * d - (xr * xr + xi * xi);
    const T idet = rcpT(det);
    // adj = [[d, -x], [-conj(x), a]]
    const T p0r = d * br[0] - (xr * br[1] - xi * bi[1]);
    const T p0i = d * bi[0] - (xr * bi[1] + xi * br[1]);
    const T p1r = a * br[1] - (xr * br[0] + xi * bi[0]);
    const T p1i = a * bi[1] - (xr * bi[0] - xi * br[0]);
    br[0] = p0r * idet; bi[0] = p0i * idet; br[1] = p1r * idet; bi[1] = p1i * idet;
    return !(a <= T(0) || det <= T(0));
  } else if constexpr (I == 3) {
    // Q = L D L^H, L unit lower triangular; with Q = [[a, x, y], [., d, z],
    // [., ., g]] the lower entries are conj(x), conj(y), conj(z).
    const T x_r = Qr[0][1], x_i = Qi[0][1], y_r = Qr[0][2], y_i = Qi[0][2];
    const T z_r = Qr[1][2], z_i = Qi[1][2];
    const T d0 = Qr[0][0], id0 = rcpT(d0);
    const T l10r = x_r * id0, l10i = -x_i * id0;  // L10 = conj(x) / d0
    const T l20r = y_r * id0, l20i = -y_i * id0;  // L20 = conj(y) / d0
    const T d1 = Qr[1][1] - d0 * (l10r * l10r + l10i * l10i), id1 = rcpT(d1);
    // L21 = (conj(z) - d0 L20 conj(L10)) / d1
    const T t_r = z_r - d0 * (l20r * l10r + l20i * l10i);
    const T t_i = -z_i - d0 * (l20i * l10r - l20r * l10i);
    const T l21r = t_r * id1, l21i = t_i * id1;
    const T d2 = Qr[2][2] - d0 * (l20r * l20r + l20i * l20i) - d1 * (l21r * l21r + l21i * l21i);
    const T id2 = rcpT(d2);
    // L w = b
    const T w0r = br[0], w0i = bi[0];
    const T w1r = br[1] - (l10r * w0r - l10i * w0i), w1i = bi[1] - (l10r * w0i + l10i * w0r);
    const T w2r = br[2] - (l20r * w0r - l20i * w0i) - (l21r * w1r - l21i * w1i);
    const T w2i = bi[2] - (l20r * w0i + l20i * w0r) - (l21r * w1i + l21i * w1r);
    // L^H p = D^-1 w
    const T p2r = w2r * id2, p2i = w2i * id2;
    const T p1r = w1r * id1 - (l21r * p2r + l21i * p2i), p1i = w1i * id1 - (l21r * p2i - l21i * p2r);
    br[0] = w0r * id0 - (l10r * p1r + l10i * p1i) - (l20r * p2r + l20i * p2i);
    bi[0] = w0i * id0 - (l10r * p1i - l10i * p1r) - (l20r * p2i - l20i * p2r);
    br[1] = p1r; bi[1] = p1i; br[2] = p2r; bi[2] = p2i;
    return !(d0 <= T(0) || d1 <= T(0) || d2 <= T(0));
  } else {
    T Lr[I][I], Li[I][I], dinv[I];
    const bool ok = cholesky<I, T>(Qr, Qi, Lr, Li, dinv);
    cholesky_solve<I, T>(Lr, Li, dinv, br, bi);
    return ok;
  }
}

// Inverse of a Hermitian positive-definite matrix given by its upper triangle
// (full result in Xr/Xi).  I <= 3: adjugate / determinant; larger I:
// Cholesky.  Returns false when the matrix is not numerically positive
// definite (a leading principal minor <= 0).
template <int I, typename T = float>
__device__ __forceinline__ bool herm_inv(const T (&Ar)[I][I], const T (&Ai)[I][I],
                                         T (&Xr)[I][I], T (&Xi)[I][I]) {
  if constexpr (I == 1) {
    Xr[0][0] = rcpT(Ar[0][0]); Xi[0][0] = T(0);
    return !(Ar[0][0] <= T(0));
  } else if constexpr (I == 2) {
    const T a = Ar[0][0], d = Ar[1][1], xr = Ar[0][1], xi = Ai[0][1];
    const T det = a * d - (xr * xr + xi * xi);
    const T id = rcpT(det);
    Xr[0][0] = d * id; Xi[0][0] = T(0); Xr[1][1] = a * id; Xi[1][1] = T(0);
    Xr[0][1] = -xr * id; Xi[0][1] = -xi * id; Xr[1][0] = -xr * id; Xi[1][0] = xi * id;
    return !(a <= T(0) || det <= T(0));
  } else if constexpr (I == 3) {
    const T a = Ar[0][0], d = Ar[1][1], g = Ar[2][2];
    const T xr = Ar[0][1], xi = Ai[0][1], yr = Ar[0][2], yi = Ai[0][2], zr = Ar[1][2], zi = Ai[1][2];
    const T A00 = d * g - (zr * zr + zi * zi), A11 = a * g - (yr * yr + yi * yi), A22 = a * d - (xr * xr + xi * xi);
    const T A01r = (yr * zr + yi * zi) - xr * g, A01i = (yi * zr - yr * zi) - xi * g;
    const T A02r = (xr * zr - xi * zi) - yr * d, A02i = (xr * zi + xi * zr) - yi * d;
    const T A12r = (yr * xr + yi * xi) - a * zr, A12i = (yi * xr - yr * xi) - a * zi;
    const T det = a * A00 + (xr * A01r + xi * A01i) + (yr * A02r + yi * A02i);
    const T id = rcpT(det);
    Xr[0][0] = A00 * id; Xi[0][0] = T(0); Xr[1][1] = A11 * id; Xi[1][1] = T(0); Xr[2][2] = A22 * id; Xi[2][2] = T(0);
    Xr[0][1] = A01r * id; Xi[0][1] = A01i * id; Xr[1][0] = A01r * id; Xi[1][0] = -A01i * id;
    Xr[0][2] = A02r * id; Xi[0][2] = A02i * id; Xr[2][0] = A02r * id; Xi[2][0] = -A02i * id;
    Xr[1][2] = A12r * id; Xi[1][2] = A12i * id; Xr[2][1] = A12r * id; Xi[2][1] = -A12i * id;
    return !(a <= T(0) || A22 <= T(0) || det <= T(0));
  } else {
    return herm_inverse<I, T>(Ar, Ai, Xr, Xi);
  }
}

}  // namespace fca
