// Reverse-mode derivatives (adjoints) of FastFCA-AS: one hybrid iteration
// (Section 4.3: eq. 15-20, then eq. 23) and the multichannel Wiener filter
// (eq. 3 with eq. 15).  Given dL/d(outputs) they produce dL/d(inputs) for a
// real loss L; a complex quantity z carries dL/dRe z + i dL/dIm z.
//
// One workgroup per frequency bin; the lanes stride over the bin's frames.
// The sums over n of the forward step become broadcasts here and the
// per-frame contributions to per-bin adjoints (lambda, P) are block sums.
//
// Iteration (forward in the basis of y = P^H x, A = P^-1 P_new):
//   q = v lambda, d = sum_j q, g = q / d, r = g^2 |y|^2 + q (1 - g)
//   v' = (1/I) sum_i r / lambda             lambda' = (1/N) sum_n r / v'
//   w = 1 / (sum_j v' lambda')              S_i = sum_n w_i y y^H
//   S_i a_i = N e_i                         P_new = P A
// Adjoint, with b_i = S_i^-1 (P^H Pbar_new)_i, alpha_i = a_i^H y,
// beta_i = b_i^H y:
//   Pbar = Pbar_new A^H + sum_n x ybar^H,   xbar = P ybar
//   wbar_i = -Re(conj(beta_i) alpha_i),     d'bar = -wbar w^2
//   lambda'bar += sum_n d'bar v',  v'bar += d'bar lambda' - (lambda'bar r) / (N v'^2)
//   rbar = lambda'bar / (N v') + v'bar / (I lambda)
//   ybar = -sum_i w_i (b_i alpha_i + a_i beta_i) + 2 (sum_j rbar dr/d|y|^2) y
// and the chain through r(q, d, |y|^2), q = v lambda, d = sum_j q.
#pragma once

#include "fca_kernels.h"

namespace fca {

// Lanes per bin.  Up to I = 3 the adjoint kernels need at most ~160 VGPRs
// (three waves per SIMD or more), so four waves per bin still keep all 513
// bins of a 513-bin problem (2052 waves) resident at once and halve the
// frames per lane; above, two waves per bin.
template <int I>
constexpr int kAdjBlock = (I <= 3) ? 256 : 128;

// Whether the frame loops of the iteration adjoint request the next frame's
// inputs ahead (more registers; above I = 5 it would cost a wave per SIMD).
template <int I>
constexpr bool kAdjPrefetch = (I <= 5);

// Pass 1 of the iteration adjoint forms alpha_i, beta_i, w_i and d'bar_i of
// every frame; where a bin's frames fit, it keeps them in LDS (6I floats per
// frame in float4 planes, plane-major so that lanes store consecutively) for
// pass 2, which would otherwise form them again.  The share of LDS is what
// three workgroups per CU leave each (their registers allow three).
template <int I>
constexpr int kAdjStashPlanes = (6 * I + 3) / 4;
constexpr int kAdjStashBytes = 52 * 1024;

template <int I, int J>
constexpr int adj_red_size() {
  constexpr int a = pad4((I * I * I <= 64) ? I * I * I : I * I);
  constexpr int b = pad4(J * I + 2 * I * I);
  return (a > b ? a : b) * (kAdjBlock<I> / kWave);
}

// Block sum of V per-lane values into out[V] (LDS or global): transposed wave
// sums, then the sum over the block's waves.  red holds
// pad4(V) * (waves per block) floats.  Ends with a barrier.
template <int V>
__device__ inline void block_sum_t(const float (&a)[V], float* out, float* red) {
  constexpr int S = pad4(V);
  wave_totals_to_lds<V>(a, red, S);
  __syncthreads();
  const int nw = blockDim.x / kWave;
  for (int k = threadIdx.x; k < V; k += blockDim.x) {
    float t = 0.f;
    for (int w = 0; w < nw; ++w) t += red[w * S + k];
    out[k] = t;
  }
  __syncthreads();
}

// Global accesses at a byte offset from a workgroup-uniform base: the base
// stays in scalar registers and every plane shares one 32-bit lane offset
// (instead of a 64-bit address per plane and lane).
__device__ __forceinline__ float ld_at(const float* base, unsigned byte_off) {
  return *reinterpret_cast<const float*>(reinterpret_cast<const char*>(base) + byte_off);
}
__device__ __forceinline__ void st_at(float* base, unsigned byte_off, float v) {
  *reinterpret_cast<float*>(reinterpret_cast<char*>(base) + byte_off) = v;
}
template <int I>
__device__ __forceinline__ void adj_load_x_at(const float* xf, int Npad, unsigned byte_off, float (&xr)[I],
                                              float (&xi)[I]) {
#pragma unroll
  for (int i = 0; i < I; ++i) {
    xr[i] = ld_at(xf + (size_t)i * Npad, byte_off);
    xi[i] = ld_at(xf + (size_t)(I + i) * Npad, byte_off);
  }
}

// ----------------------------------------------------------------------------
// Adjoint of one hybrid iteration (K = 1).
// ----------------------------------------------------------------------------
template <int I, int J, bool kStash>
__device__ __forceinline__ void adj_iter_body(const DevState& s, const AdjIter& a) {
  constexpr bool kOne = I * I * I <= 64;
  constexpr int SP = kAdjStashPlanes<I>;
  extern __shared__ float4 sStash[];  // [SP][N] when kStash
  constexpr int kB = kAdjBlock<I>, PH = kPH<I>;
  const int f = blockIdx.x, tid = threadIdx.x;
  const int N = s.N, Np = s.Npad;
  __shared__ float sPr[I][I], sPi[I][I];    // P_t
  __shared__ float sQr[I][I], sQi[I][I];    // Pbar of P_{t+1}
  __shared__ float sAr[I][I], sAi[I][I];    // column i: a_i
  __shared__ float4 sPc[I * PH];            // P_t by columns (y = P^H x)
  __shared__ float4 sPw[I * PH];            // P_t by rows (P ybar)
  __shared__ float4 sAB[I * I];             // (k, i): a_ki and b_ki (re, im, re, im)
  __shared__ float4 sPA[I * PH], sPB[I * PH];  // P A and P B by columns (alpha = (P a)^H x)
  __shared__ float4 sLm[J * I];             // (j, i): lambda_t, lambda', lambda'bar total, 1 / lambda_t
  __shared__ float sLb[J * I];
  __shared__ float sS[I][I * I];            // S_i, packed Hermitian
  __shared__ float sOut[J * I + 2 * I * I];
  __shared__ float red[adj_red_size<I, J>()];

  // Issue priority: two or three workgroups share a CU, and the per-bin
  // sections (set-up, solves, the block sums) that all waves of a workgroup
  // wait on issue ahead of another workgroup's frame passes, which fill the
  // gaps.
  __builtin_amdgcn_s_setprio(2);
  const float* xf = s.xs + (size_t)f * 2 * I * Np;
  const float* vt = a.v_t + (size_t)f * J * Np;
  const float* vn = a.v_n + (size_t)f * J * Np;
  const float* vbi = a.vb_in + (size_t)f * J * Np;
  float* vbo = a.vb_out + (size_t)f * J * Np;
  float* xb = a.xb + (size_t)f * 2 * I * Np;

  // Every frame loop below requests the next frame's inputs before it works
  // on the current one (one global-memory latency per pass instead of one
  // per frame); the first frame of pass 1 is requested here, before the
  // per-bin set-up.
  auto load1 = [&](int n, float (&xr)[I], float (&xi)[I], float (&vN)[J]) {
    unsigned u = 4u * n;
    asm volatile("" : "+v"(u));
    adj_load_x_at<I>(xf, Np, u, xr, xi);
#pragma unroll
    for (int j = 0; j < J; ++j) vN[j] = ld_at(vn + (size_t)j * Np, u);
  };
  float pxr[I], pxi[I], pvN[J];
  if (kAdjPrefetch<I> && tid < N) load1(tid, pxr, pxi, pvN);

  // The per-bin constants are read from LDS inside the frame loops (behind an
  // opaque zero offset, so they are not hoisted into registers): the
  // registers go to more waves per SIMD instead.
  const float2* Pt = a.P_t + (size_t)f * I * I;
  for (int t = tid; t < I * I; t += kB) {
    const float2 p = Pt[t], q = a.Pb_in[(size_t)f * I * I + t];
    sPr[t / I][t % I] = p.x; sPi[t / I][t % I] = p.y;
    sQr[t / I][t % I] = q.x; sQi[t / I][t % I] = q.y;
  }
  stage_P_columns<I>(Pt, sPc);
  for (int t = tid; t < I * PH; t += kB) {
    const int r = t / PH, k = 2 * (t % PH);
    const float2 p0 = Pt[r * I + k];
    const float2 p1 = (k + 1 < I) ? Pt[r * I + k + 1] : make_float2(0.f, 0.f);
    sPw[t] = make_float4(p0.x, p0.y, p1.x, p1.y);
  }
  for (int t = tid; t < J * I; t += kB) {
    const float lt = a.lam_t[(size_t)f * J * I + t];
    sLm[t] = make_float4(lt, a.lam_n[(size_t)f * J * I + t], a.lb_in[(size_t)f * J * I + t], rcp(lt));
  }
  if (a.S_t)
    for (int t = tid; t < I * I * I; t += kB) (&sS[0][0])[t] = a.S_t[(size_t)f * I * I * I + t];
  __syncthreads();

  // new weights w_i = 1 / sum_j v'_j lambda'_ji at a frame with v' = vN
  auto weights = [&](const float4* lm, const float (&vN)[J], float (&w)[I]) {
#pragma unroll
    for (int i = 0; i < I; ++i) {
      float d = 0.f;
#pragma unroll
      for (int j = 0; j < J; ++j) d = fmaf(vN[j], lm[j * I + i].y, d);
      w[i] = rcp(d);
    }
  };

  // ---- pass 0: S_i = sum_n w_i y y^H (recorded by the forward run, or
  // summed again here) ------------------------------------------------------
  if (a.S_t) {
    // staged above
  } else if constexpr (kOne) {
    float acc[I * I * I];
#pragma unroll
    for (int k = 0; k < I * I * I; ++k) acc[k] = 0.f;
    __builtin_amdgcn_s_setprio(0);  // frame pass
    for (int n = tid; n < N; n += kB) {
      int zo = 0;
      unsigned u = 4u * n;
      asm volatile("" : "+s"(zo), "+v"(u));
      float xr[I], xi[I], yr[I], yi[I], vN[J], w[I], z[I * I];
      adj_load_x_at<I>(xf, Np, u, xr, xi);
#pragma unroll
      for (int j = 0; j < J; ++j) vN[j] = ld_at(vn + (size_t)j * Np, u);
      as_transform_lds<I>(sPc + zo, xr, xi, yr, yi);
      weights(sLm + zo, vN, w);
      herm_outer<I>(z, yr, yi);
#pragma unroll
      for (int i = 0; i < I; ++i)
#pragma unroll
        for (int k = 0; k < I * I; ++k) acc[i * I * I + k] = fmaf(w[i], z[k], acc[i * I * I + k]);
    }
    __builtin_amdgcn_s_setprio(2);  // sums and per-bin work
    block_sum_t<I * I * I>(acc, &sS[0][0], red);
  } else {
#pragma unroll 1
    for (int i = 0; i < I; ++i) {
      float acc[I * I];
#pragma unroll
      for (int k = 0; k < I * I; ++k) acc[k] = 0.f;
      __builtin_amdgcn_s_setprio(0);  // frame pass
      for (int n = tid; n < N; n += kB) {
        int zo = 0;
        unsigned u = 4u * n;
        asm volatile("" : "+s"(zo), "+v"(u));
        float xr[I], xi[I], yr[I], yi[I], vN[J], w[I];
        adj_load_x_at<I>(xf, Np, u, xr, xi);
#pragma unroll
        for (int j = 0; j < J; ++j) vN[j] = ld_at(vn + (size_t)j * Np, u);
        as_transform_lds<I>(sPc + zo, xr, xi, yr, yi);
        weights(sLm + zo, vN, w);
        float wi = w[0];
#pragma unroll
        for (int k = 1; k < I; ++k) wi = (k == i) ? w[k] : wi;
        herm_rank1_acc<I>(acc, wi, yr, yi);
      }
      __builtin_amdgcn_s_setprio(2);  // sums and per-bin work
      block_sum_t<I * I>(acc, &sS[i][0], red);
    }
  }

  // ---- per bin: a_c = N S_c^-1 e_c and b_c = S_c^-1 (P^H Pbar_new)_c ------
  if (tid < I) {
    const int c = tid;
    float Sr[I][I], Si[I][I];
#pragma unroll
    for (int r = 0; r < I; ++r)
#pragma unroll
      for (int k = 0; k < I; ++k) {
        Sr[r][k] = sS[c][r * I + k];
        Si[r][k] = (k > r) ? sS[c][k * I + r] : 0.f;
      }
    float ar[I], ai[I], br[I], bi[I];
#pragma unroll
    for (int r = 0; r < I; ++r) {
      ar[r] = (r == c) ? float(N) : 0.f; ai[r] = 0.f;
      // (P^H Pbar_new)_rc = sum_k conj(P_kr) Pbar_kc
      float tr = 0.f, ti = 0.f;
#pragma unroll
      for (int k = 0; k < I; ++k) {
        const float qr = sQr[k][c], qi = sQi[k][c];
        tr = fmaf(sPr[k][r], qr, fmaf(sPi[k][r], qi, tr));
        ti = fmaf(sPr[k][r], qi, fmaf(-sPi[k][r], qr, ti));
      }
      br[r] = tr; bi[r] = ti;
    }
    herm_solve<I>(Sr, Si, ar, ai);
    herm_solve<I>(Sr, Si, br, bi);
#pragma unroll
    for (int r = 0; r < I; ++r) {
      sAr[r][c] = ar[r]; sAi[r][c] = ai[r];
      sAB[r * I + c] = make_float4(ar[r], ai[r], br[r], bi[r]);
    }
    // column c of P A and of P B, in the column staging of P
    float par[I], pai[I], pbr[I], pbi[I];
#pragma unroll
    for (int r = 0; r < I; ++r) {
      float t0 = 0.f, t1 = 0.f, t2 = 0.f, t3 = 0.f;
#pragma unroll
      for (int k = 0; k < I; ++k) {
        const float pr = sPr[r][k], pi = sPi[r][k];
        t0 = fmaf(pr, ar[k], fmaf(-pi, ai[k], t0));
        t1 = fmaf(pr, ai[k], fmaf(pi, ar[k], t1));
        t2 = fmaf(pr, br[k], fmaf(-pi, bi[k], t2));
        t3 = fmaf(pr, bi[k], fmaf(pi, br[k], t3));
      }
      par[r] = t0; pai[r] = t1; pbr[r] = t2; pbi[r] = t3;
    }
#pragma unroll
    for (int hh = 0; hh < PH; ++hh) {
      const int k = 2 * hh, k1 = (k + 1) % I;  // the second entry is zero past I
      const bool two = k + 1 < I;
      sPA[c * PH + hh] = make_float4(par[k], pai[k], two ? par[k1] : 0.f, two ? pai[k1] : 0.f);
      sPB[c * PH + hh] = make_float4(pbr[k], pbi[k], two ? pbr[k1] : 0.f, two ? pbi[k1] : 0.f);
    }
  }
  __syncthreads();

  // d'bar_i at frame n, with alpha_i = a_i^H y and beta_i = b_i^H y
  auto dprime_bar = [&](const float4* ab, const float (&yr)[I], const float (&yi)[I], const float (&w)[I],
                        float (&alr)[I], float (&ali)[I], float (&ber)[I], float (&bei)[I], float (&dpb)[I]) {
#pragma unroll
    for (int i = 0; i < I; ++i) {
      float a0 = 0.f, a1 = 0.f, b0 = 0.f, b1 = 0.f;
#pragma unroll
      for (int k = 0; k < I; ++k) {
        const float4 q = ab[k * I + i];
        a0 = fmaf(q.x, yr[k], fmaf(q.y, yi[k], a0));
        a1 = fmaf(q.x, yi[k], fmaf(-q.y, yr[k], a1));
        b0 = fmaf(q.z, yr[k], fmaf(q.w, yi[k], b0));
        b1 = fmaf(q.z, yi[k], fmaf(-q.w, yr[k], b1));
      }
      alr[i] = a0; ali[i] = a1; ber[i] = b0; bei[i] = b1;
      const float wbar = -fmaf(b0, a0, b1 * a1);  // -Re(conj(beta) alpha)
      dpb[i] = -wbar * w[i] * w[i];
    }
  };

  // the inputs of a pass-2 frame: x, v', v, v'bar-in and the xbar so far
  auto load2 = [&](int n, float (&xr)[I], float (&xi)[I], float (&vN)[J], float (&v)[J], float (&vb)[J],
                   float (&xbr)[I], float (&xbi)[I]) {
    unsigned u = 4u * n;
    asm volatile("" : "+v"(u));
    adj_load_x_at<I>(xf, Np, u, xr, xi);
#pragma unroll
    for (int j = 0; j < J; ++j) {
      vN[j] = ld_at(vn + (size_t)j * Np, u);
      v[j] = ld_at(vt + (size_t)j * Np, u);
      vb[j] = ld_at(vbi + (size_t)j * Np, u);
    }
    adj_load_x_at<I>(xb, Np, u, xbr, xbi);
  };
  float qxr[I], qxi[I], qvN[J], qv[J], qvb[J], qxbr[I], qxbi[I];

  // ---- pass 1: lambda'bar total = lambda'bar_in + sum_n d'bar v' ----------
  {
    float acc[J * I];
#pragma unroll
    for (int k = 0; k < J * I; ++k) acc[k] = 0.f;
    __builtin_amdgcn_s_setprio(0);  // frame pass
    for (int n = tid; n < N; n += kB) {
      float xr[I], xi[I], vN[J], w[I], alr[I], ali[I], ber[I], bei[I], dpb[I];
      if constexpr (kAdjPrefetch<I>) {
#pragma unroll
        for (int i = 0; i < I; ++i) { xr[i] = pxr[i]; xi[i] = pxi[i]; }
#pragma unroll
        for (int j = 0; j < J; ++j) vN[j] = pvN[j];
        if (n + kB < N) load1(n + kB, pxr, pxi, pvN);
      } else {
        load1(n, xr, xi, vN);
      }
      int zo = 0;
      asm volatile("" : "+s"(zo));
      // alpha_i = a_i^H y = (P a_i)^H x and beta_i = (P b_i)^H x: y itself is not needed here
      as_transform_lds<I>(sPA + zo, xr, xi, alr, ali);
      as_transform_lds<I>(sPB + zo, xr, xi, ber, bei);
      weights(sLm + zo, vN, w);
#pragma unroll
      for (int i = 0; i < I; ++i) {
        const float wbar = -fmaf(ber[i], alr[i], bei[i] * ali[i]);  // -Re(conj(beta) alpha)
        dpb[i] = -wbar * w[i] * w[i];
      }
#pragma unroll
      for (int j = 0; j < J; ++j)
#pragma unroll
        for (int i = 0; i < I; ++i) acc[j * I + i] = fmaf(dpb[i], vN[j], acc[j * I + i]);
      if constexpr (kStash) {
        float st[4 * SP];
#pragma unroll
        for (int i = 0; i < I; ++i) {
          st[i] = alr[i]; st[I + i] = ali[i]; st[2 * I + i] = ber[i];
          st[3 * I + i] = bei[i]; st[4 * I + i] = w[i]; st[5 * I + i] = dpb[i];
        }
#pragma unroll
        for (int k = 6 * I; k < 4 * SP; ++k) st[k] = 0.f;
#pragma unroll
        for (int q = 0; q < SP; ++q)
          sStash[q * N + n] = make_float4(st[4 * q], st[4 * q + 1], st[4 * q + 2], st[4 * q + 3]);
      }
    }
    if (kAdjPrefetch<I> && tid < N) load2(tid, qxr, qxi, qvN, qv, qvb, qxbr, qxbi);  // first frame of pass 2
    __builtin_amdgcn_s_setprio(2);  // sums and per-bin work
    block_sum_t<J * I>(acc, sLb, red);
    for (int t = tid; t < J * I; t += kB) sLm[t].z += sLb[t];
    __syncthreads();
  }

  // ---- pass 2: everything else ----------------------------------------------
  const float invN = 1.0f / float(N), invI = 1.0f / float(I);
  float acc[J * I + 2 * I * I];  // lambda-bar sums, then sum_n x ybar^H (re, im)
#pragma unroll
  for (int k = 0; k < J * I + 2 * I * I; ++k) acc[k] = 0.f;
  __builtin_amdgcn_s_setprio(0);  // frame pass
  for (int n = tid; n < N; n += kB) {
    float xr[I], xi[I], yr[I], yi[I], vN[J], w[I], alr[I], ali[I], ber[I], bei[I], dpb[I], v[J], vb[J];
    float xbr[I], xbi[I];
    if constexpr (kAdjPrefetch<I>) {
#pragma unroll
      for (int i = 0; i < I; ++i) { xr[i] = qxr[i]; xi[i] = qxi[i]; xbr[i] = qxbr[i]; xbi[i] = qxbi[i]; }
#pragma unroll
      for (int j = 0; j < J; ++j) { vN[j] = qvN[j]; v[j] = qv[j]; vb[j] = qvb[j]; }
      if (n + kB < N) load2(n + kB, qxr, qxi, qvN, qv, qvb, qxbr, qxbi);
    } else {
      load1(n, xr, xi, vN);
      unsigned u = 4u * n;
      asm volatile("" : "+v"(u));
#pragma unroll
      for (int j = 0; j < J; ++j) { v[j] = ld_at(vt + (size_t)j * Np, u); vb[j] = ld_at(vbi + (size_t)j * Np, u); }
    }
    int zo = 0;
    unsigned u = 4u * n;
    asm volatile("" : "+s"(zo), "+v"(u));
    as_transform_lds<I>(sPc + zo, xr, xi, yr, yi);
    if constexpr (kStash) {  // pass 1's values of this frame (same lane, written before the barrier)
      float st[4 * SP];
#pragma unroll
      for (int q = 0; q < SP; ++q) {
        const float4 t = sStash[q * N + n];
        st[4 * q] = t.x; st[4 * q + 1] = t.y; st[4 * q + 2] = t.z; st[4 * q + 3] = t.w;
      }
#pragma unroll
      for (int i = 0; i < I; ++i) {
        alr[i] = st[i]; ali[i] = st[I + i]; ber[i] = st[2 * I + i];
        bei[i] = st[3 * I + i]; w[i] = st[4 * I + i]; dpb[i] = st[5 * I + i];
      }
    } else {
      weights(sLm + zo, vN, w);
      dprime_bar(sAB + zo, yr, yi, w, alr, ali, ber, bei, dpb);
    }
    // with h_i = |y_i|^2 / d_i - 1 and q = v lambda, g = q / d:
    //   r = q (1 + g h),  dr/dq = 1 + 2 g h,  dr/dd = -g^2 (1 + 2 h),  dr/d|y|^2 = g^2
    float id[I], h[I], m2[I];  // 1 / d_i, h_i, -(1 + 2 h_i)
    asm volatile("" : "+s"(zo));
    const float4* lm = sLm + zo;
#pragma unroll
    for (int i = 0; i < I; ++i) {
      float t = 0.f;
#pragma unroll
      for (int j = 0; j < J; ++j) t = fmaf(v[j], lm[j * I + i].x, t);
      id[i] = rcp(t);
      h[i] = fmaf(fmaf(yr[i], yr[i], yi[i] * yi[i]), id[i], -1.f);
      m2[i] = fmaf(-2.f, h[i], -1.f);
    }
    // v'bar total and the rbar of every (j, i)
    float db2[I], eb[I], vbar[J];
#pragma unroll
    for (int i = 0; i < I; ++i) { db2[i] = 0.f; eb[i] = 0.f; }
#pragma unroll
    for (int j = 0; j < J; ++j) {
      asm volatile("" : "+s"(zo));
      lm = sLm + zo;
      const float ivn = rcp(vN[j]);
      float vbt = vb[j], rl = 0.f;
      float r[I], g[I];
#pragma unroll
      for (int i = 0; i < I; ++i) {
        const float4 L = lm[j * I + i];
        vbt = fmaf(dpb[i], L.y, vbt);
        const float q = v[j] * L.x;
        g[i] = q * id[i];
        r[i] = fmaf(q, g[i] * h[i], q);
        rl = fmaf(L.z, r[i], rl);
      }
      const float an = invN * ivn;
      vbt = fmaf(-rl * an, ivn, vbt);
      const float bv = vbt * invI;
      float vj = 0.f;
#pragma unroll
      for (int i = 0; i < I; ++i) {
        const float4 L = lm[j * I + i];
        const float rbar = fmaf(L.z, an, bv * L.w);
        acc[j * I + i] = fmaf(-bv * r[i], L.w * L.w, acc[j * I + i]);
        const float gi = g[i], g2 = gi * gi;
        const float qbar = rbar * fmaf(2.f * gi, h[i], 1.f);  // rbar dr/dq
        db2[i] = fmaf(rbar * g2, m2[i], db2[i]);             // rbar dr/dd
        eb[i] = fmaf(rbar, g2, eb[i]);                        // rbar dr/d|y|^2
        vj = fmaf(qbar, L.x, vj);
        acc[j * I + i] = fmaf(qbar, v[j], acc[j * I + i]);
      }
      vbar[j] = vj;
    }
    asm volatile("" : "+s"(zo));
    lm = sLm + zo;
#pragma unroll
    for (int j = 0; j < J; ++j) {
#pragma unroll
      for (int i = 0; i < I; ++i) {
        vbar[j] = fmaf(db2[i], lm[j * I + i].x, vbar[j]);
        acc[j * I + i] = fmaf(db2[i], v[j], acc[j * I + i]);
      }
      st_at(vbo + (size_t)j * Np, u, vbar[j]);
    }
    // ybar = -sum_i w_i (b_i alpha_i + a_i beta_i) + 2 eb y
    asm volatile("" : "+s"(zo));
    const float4* ab = sAB + zo;
    float ybr[I], ybi[I];
#pragma unroll
    for (int k = 0; k < I; ++k) {
      float tr = 2.f * eb[k] * yr[k], ti = 2.f * eb[k] * yi[k];
#pragma unroll
      for (int i = 0; i < I; ++i) {
        // b_ki alpha_i + a_ki beta_i
        const float4 q = ab[k * I + i];
        const float ur = (q.z * alr[i] - q.w * ali[i]) + (q.x * ber[i] - q.y * bei[i]);
        const float ui = (q.z * ali[i] + q.w * alr[i]) + (q.x * bei[i] + q.y * ber[i]);
        tr = fmaf(-w[i], ur, tr);
        ti = fmaf(-w[i], ui, ti);
      }
      ybr[k] = tr; ybi[k] = ti;
    }
    // xbar += P ybar;  sum_n x ybar^H
    asm volatile("" : "+s"(zo));
    const float4* pw = sPw + zo;
#pragma unroll
    for (int r = 0; r < I; ++r) {
      float tr = 0.f, ti = 0.f;
#pragma unroll
      for (int h = 0; h < PH; ++h) {
        const float4 q = pw[r * PH + h];
        const int k = 2 * h;
        tr = fmaf(q.x, ybr[k], fmaf(-q.y, ybi[k], tr));
        ti = fmaf(q.x, ybi[k], fmaf(q.y, ybr[k], ti));
        if (k + 1 < I) {
          tr = fmaf(q.z, ybr[k + 1], fmaf(-q.w, ybi[k + 1], tr));
          ti = fmaf(q.z, ybi[k + 1], fmaf(q.w, ybr[k + 1], ti));
        }
      }
      if constexpr (!kAdjPrefetch<I>) {  // xbar so far, read late to keep it out of the frame's registers
        xbr[r] = ld_at(xb + (size_t)r * Np, u);
        xbi[r] = ld_at(xb + (size_t)(I + r) * Np, u);
      }
      st_at(xb + (size_t)r * Np, u, xbr[r] + tr);
      st_at(xb + (size_t)(I + r) * Np, u, xbi[r] + ti);
#pragma unroll
      for (int k = 0; k < I; ++k) {
        // x_r conj(ybar_k)
        acc[J * I + r * I + k] = fmaf(xr[r], ybr[k], fmaf(xi[r], ybi[k], acc[J * I + r * I + k]));
        acc[J * I + I * I + r * I + k] = fmaf(xi[r], ybr[k], fmaf(-xr[r], ybi[k], acc[J * I + I * I + r * I + k]));
      }
    }
  }
  __builtin_amdgcn_s_setprio(2);  // sums and per-bin work
  block_sum_t<J * I + 2 * I * I>(acc, sOut, red);
  for (int t = tid; t < J * I; t += kB) a.lb_out[(size_t)f * J * I + t] = sOut[t];
  for (int t = tid; t < I * I; t += kB) {
    const int r = t / I, c = t % I;
    // (Pbar_new A^H)_rc = sum_k Pbar_rk conj(A_ck)
    float tr = sOut[J * I + t], ti = sOut[J * I + I * I + t];
#pragma unroll
    for (int k = 0; k < I; ++k) {
      tr = fmaf(sQr[r][k], sAr[c][k], fmaf(sQi[r][k], sAi[c][k], tr));
      ti = fmaf(sQi[r][k], sAr[c][k], fmaf(-sQr[r][k], sAi[c][k], ti));
    }
    a.Pb_out[(size_t)f * I * I + t] = make_float2(tr, ti);
  }
}

template <int I, int J, bool kStash>
__global__ __launch_bounds__(kAdjBlock<I>) void k_adj_iter(DevState s, AdjIter a) {
  adj_iter_body<I, J, kStash>(s, a);
}

// The inputs and outputs of the adjoint of iteration j of a segment whose
// adjoints alternate between the two buffers, `cur` being read at j.
__host__ __device__ inline AdjIter adj_seg_iter(const AdjSeg& g, int j, int cur) {
  const long long st = j == 0 ? g.ck : g.slot0 + j * g.stride;
  const long long sn = g.slot0 + (j + 1) * g.stride;
  AdjIter a;
  a.S_t = g.S ? g.S + j * g.S_floats : nullptr;
  a.v_t = g.tape + st + g.v_off;
  a.lam_t = g.tape + st + g.lam_off;
  a.P_t = reinterpret_cast<const float2*>(g.tape + st + g.P_off);
  a.v_n = g.tape + sn + g.v_off;
  a.lam_n = g.tape + sn + g.lam_off;
  a.vb_in = g.vb[cur]; a.lb_in = g.lb[cur]; a.Pb_in = g.Pb[cur];
  a.vb_out = g.vb[1 - cur]; a.lb_out = g.lb[1 - cur]; a.Pb_out = g.Pb[1 - cur];
  a.xb = g.xb;
  return a;
}

// The adjoints of iterations len-1 .. 0 of one checkpoint segment in one
// launch.  Bins never interact, so a workgroup takes its bin through the
// whole segment: what one iteration's adjoint hands the next (v'bar,
// lambda'bar, P'bar, xbar of this bin) goes through global memory, written
// and read by this workgroup only, ordered by the barrier between them.
template <int I, int J, bool kStash>
__global__ __launch_bounds__(kAdjBlock<I>) void k_adj_seg(DevState s, AdjSeg g) {
  int cur = g.cur;
#pragma unroll 1
  for (int j = g.len - 1; j >= 0; --j) {
    adj_iter_body<I, J, kStash>(s, adj_seg_iter(g, j, cur));
    cur = 1 - cur;
    __syncthreads();  // this bin's outputs before the next iteration reads them
  }
}

// ----------------------------------------------------------------------------
// Adjoint of the Wiener filter s_j = P^-H (g_j o y), g_ji = v_j lambda_ji / d_i
// (B = P^-H is formed in the workgroup).  gout [J][F][N][I]; writes vb_out, lb_out, Pb_out
// and initialises xb.
// ----------------------------------------------------------------------------
template <int I, int J>
__global__ __launch_bounds__(kAdjBlock<I>) void k_adj_wiener(DevState s, const float2* __restrict__ gout, AdjIter a) {
  constexpr int kB = kAdjBlock<I>, PH = kPH<I>;
  const int f = blockIdx.x, tid = threadIdx.x;
  const int N = s.N, Np = s.Npad, F = s.F;
  __shared__ float sBr[I][I], sBi[I][I];
  __shared__ float4 sPc[I * PH];  // P by columns (y = P^H x)
  __shared__ float4 sPw[I * PH];  // P by rows (P ybar)
  __shared__ float4 sBc[I * PH];  // B by columns (zbar = B^H sbar)
  __shared__ float sL[J * I];
  __shared__ float sOut[J * I + 4 * I * I];
  __shared__ float red[pad4(J * I + 4 * I * I) * (kB / kWave)];
  const float2* Pf = s.P + (size_t)f * I * I;
  if (tid < I) {  // B = P^-H, formed here: lane c solves P^H b = e_c for column c
    const int c = tid;
    float Mr[I][I], Mi[I][I], br[I], bi[I];
#pragma unroll
    for (int r = 0; r < I; ++r)
#pragma unroll
      for (int k = 0; k < I; ++k) {
        const float2 p = Pf[k * I + r];
        Mr[r][k] = p.x; Mi[r][k] = -p.y;
      }
#pragma unroll
    for (int r = 0; r < I; ++r) { br[r] = (r == c) ? 1.f : 0.f; bi[r] = 0.f; }
    lu_solve<I>(Mr, Mi, br, bi);
#pragma unroll
    for (int r = 0; r < I; ++r) { sBr[r][c] = br[r]; sBi[r][c] = bi[r]; }
  }
  stage_P_columns<I>(Pf, sPc);
  for (int t = tid; t < I * PH; t += kB) {
    const int r = t / PH, k = 2 * (t % PH);
    const float2 p0 = Pf[r * I + k];
    const float2 p1 = (k + 1 < I) ? Pf[r * I + k + 1] : make_float2(0.f, 0.f);
    sPw[t] = make_float4(p0.x, p0.y, p1.x, p1.y);
  }
  for (int t = tid; t < J * I; t += kB) sL[t] = s.lam[(size_t)f * J * I + t];
  __syncthreads();
  for (int t = tid; t < I * PH; t += kB) {  // B by columns, from the solve above
    const int i = t / PH, k = 2 * (t % PH), k1 = (k + 1) % I;
    const bool two = k + 1 < I;
    sBc[t] = make_float4(sBr[k][i], sBi[k][i], two ? sBr[k1][i] : 0.f, two ? sBi[k1][i] : 0.f);
  }
  __syncthreads();
  const float* xf = s.xs + (size_t)f * 2 * I * Np;
  const float* vf = s.vs + (size_t)f * J * Np;
  float* vbo = a.vb_out + (size_t)f * J * Np;
  float* xb = a.xb + (size_t)f * 2 * I * Np;
  // lambda-bar sums, sum_n sum_j sbar_j z_j^H (re, im), sum_n x ybar^H (re, im)
  float acc[J * I + 4 * I * I];
#pragma unroll
  for (int k = 0; k < J * I + 4 * I * I; ++k) acc[k] = 0.f;
  for (int n = tid; n < N; n += kB) {
    // per-bin constants come from LDS behind opaque zero offsets (fresh per
    // use, so no read is kept live across the frame); one 32-bit lane offset
    // serves every plane
    int zo = 0;
    unsigned u = 4u * n;
    asm volatile("" : "+s"(zo), "+v"(u));
    float xr[I], xi[I], yr[I], yi[I], v[J], d[I];
    adj_load_x_at<I>(xf, Np, u, xr, xi);
    as_transform_lds<I>(sPc + zo, xr, xi, yr, yi);
#pragma unroll
    for (int j = 0; j < J; ++j) v[j] = ld_at(vf + (size_t)j * Np, u);
    asm volatile("" : "+s"(zo));
    const float* lam = sL + zo;
#pragma unroll
    for (int i = 0; i < I; ++i) {
      float t = 0.f;
#pragma unroll
      for (int j = 0; j < J; ++j) t = fmaf(v[j], lam[j * I + i], t);
      d[i] = t;
    }
    float ybr[I], ybi[I], dbar[I], id[I];
#pragma unroll
    for (int i = 0; i < I; ++i) { ybr[i] = 0.f; ybi[i] = 0.f; dbar[i] = 0.f; id[i] = rcp(d[i]); }
    float qb[J][I];
#pragma unroll
    for (int j = 0; j < J; ++j) {
      float sr[I], si[I];
      // s_j at frame n: I interleaved complex values at byte offset 2 I u
      const float* gp = reinterpret_cast<const float*>(gout + ((size_t)j * F + f) * N * I);
#pragma unroll
      for (int i = 0; i < I; ++i) { sr[i] = ld_at(gp + 2 * i, u * (2 * I)); si[i] = ld_at(gp + 2 * i + 1, u * (2 * I)); }
      asm volatile("" : "+s"(zo));
      const float4* bc = sBc + zo;
      lam = sL + zo;
#pragma unroll
      for (int i = 0; i < I; ++i) {
        const float q = v[j] * lam[j * I + i], g = q * id[i];
        // zbar_i = (B^H sbar)_i = sum_k conj(B_ki) sbar_k
        float zr = 0.f, zi = 0.f;
#pragma unroll
        for (int h = 0; h < PH; ++h) {
          const float4 b = bc[i * PH + h];
          const int k = 2 * h;
          zr = fmaf(b.x, sr[k], fmaf(b.y, si[k], zr));
          zi = fmaf(b.x, si[k], fmaf(-b.y, sr[k], zi));
          if (k + 1 < I) {
            zr = fmaf(b.z, sr[k + 1], fmaf(b.w, si[k + 1], zr));
            zi = fmaf(b.z, si[k + 1], fmaf(-b.w, sr[k + 1], zi));
          }
        }
        const float gbar = fmaf(yr[i], zr, yi[i] * zi);   // Re(conj(y) zbar)
        ybr[i] = fmaf(g, zr, ybr[i]);
        ybi[i] = fmaf(g, zi, ybi[i]);
        qb[j][i] = gbar * id[i];
        dbar[i] = fmaf(-gbar * q, id[i] * id[i], dbar[i]);
        // sbar_k conj(z_i), z_i = g y_i
        const float zzr = g * yr[i], zzi = g * yi[i];
#pragma unroll
        for (int k = 0; k < I; ++k) {
          acc[J * I + k * I + i] = fmaf(sr[k], zzr, fmaf(si[k], zzi, acc[J * I + k * I + i]));
          acc[J * I + I * I + k * I + i] = fmaf(si[k], zzr, fmaf(-sr[k], zzi, acc[J * I + I * I + k * I + i]));
        }
      }
    }
    asm volatile("" : "+s"(zo));
    lam = sL + zo;
#pragma unroll
    for (int j = 0; j < J; ++j) {
      float vb = 0.f;
#pragma unroll
      for (int i = 0; i < I; ++i) {
        const float t = qb[j][i] + dbar[i];
        vb = fmaf(t, lam[j * I + i], vb);
        acc[j * I + i] = fmaf(t, v[j], acc[j * I + i]);
      }
      st_at(vbo + (size_t)j * Np, u, vb);
    }
    asm volatile("" : "+s"(zo));
    const float4* pw = sPw + zo;
#pragma unroll
    for (int r = 0; r < I; ++r) {
      float tr = 0.f, ti = 0.f;
#pragma unroll
      for (int h = 0; h < PH; ++h) {
        const float4 q = pw[r * PH + h];
        const int k = 2 * h;
        tr = fmaf(q.x, ybr[k], fmaf(-q.y, ybi[k], tr));
        ti = fmaf(q.x, ybi[k], fmaf(q.y, ybr[k], ti));
        if (k + 1 < I) {
          tr = fmaf(q.z, ybr[k + 1], fmaf(-q.w, ybi[k + 1], tr));
          ti = fmaf(q.z, ybi[k + 1], fmaf(q.w, ybr[k + 1], ti));
        }
      }
      st_at(xb + (size_t)r * Np, u, tr);
      st_at(xb + (size_t)(I + r) * Np, u, ti);
#pragma unroll
      for (int k = 0; k < I; ++k) {
        acc[J * I + 2 * I * I + r * I + k] = fmaf(xr[r], ybr[k], fmaf(xi[r], ybi[k], acc[J * I + 2 * I * I + r * I + k]));
        acc[J * I + 3 * I * I + r * I + k] = fmaf(xi[r], ybr[k], fmaf(-xr[r], ybi[k], acc[J * I + 3 * I * I + r * I + k]));
      }
    }
  }
  block_sum_t<J * I + 4 * I * I>(acc, sOut, red);
  for (int t = tid; t < J * I; t += kB) a.lb_out[(size_t)f * J * I + t] = sOut[t];
  for (int t = tid; t < I * I; t += kB) {
    const int r = t / I, c = t % I;
    // -(B Bbar^H B)_rc + (sum_n x ybar^H)_rc
    float tr = sOut[J * I + 2 * I * I + t], ti = sOut[J * I + 3 * I * I + t];
#pragma unroll
    for (int l = 0; l < I; ++l) {
      // (B Bbar^H)_rl = sum_k B_rk conj(Bbar_lk)
      float mr = 0.f, mi = 0.f;
#pragma unroll
      for (int k = 0; k < I; ++k) {
        const float br = sOut[J * I + l * I + k], bi = sOut[J * I + I * I + l * I + k];
        mr = fmaf(sBr[r][k], br, fmaf(sBi[r][k], bi, mr));
        mi = fmaf(sBi[r][k], br, fmaf(-sBr[r][k], bi, mi));
      }
      tr -= mr * sBr[l][c] - mi * sBi[l][c];
      ti -= mr * sBi[l][c] + mi * sBr[l][c];
    }
    a.Pb_out[(size_t)f * I * I + t] = make_float2(tr, ti);
  }
}

template <int I, int J>
hipError_t launch_adj_iter(const DevState& s, const AdjIter& a, hipStream_t st) {
  const size_t stash = sizeof(float4) * kAdjStashPlanes<I> * (size_t)s.N;
  if (stash <= (size_t)kAdjStashBytes)
    hipLaunchKernelGGL((k_adj_iter<I, J, true>), dim3(s.F), dim3(kAdjBlock<I>), stash, st, s, a);
  else
    hipLaunchKernelGGL((k_adj_iter<I, J, false>), dim3(s.F), dim3(kAdjBlock<I>), 0, st, s, a);
  return hipGetLastError();
}

// One launch for the segment when every bin's workgroup is resident at once
// (a workgroup that had to wait for another to finish its whole segment
// would double the time); otherwise one launch per iteration.
template <int I, int J, bool kStash>
hipError_t launch_adj_seg_k(const DevState& s, const AdjSeg& g, hipStream_t st, size_t shm) {
  int per_cu = 0, dev = 0, cus = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_adj_seg<I, J, kStash>, kAdjBlock<I>, shm);
  if (e == hipSuccess) e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  if ((long long)per_cu * cus >= s.F) {
    hipLaunchKernelGGL((k_adj_seg<I, J, kStash>), dim3(s.F), dim3(kAdjBlock<I>), shm, st, s, g);
    return hipGetLastError();
  }
  int cur = g.cur;
  for (int j = g.len - 1; j >= 0; --j) {
    if ((e = launch_adj_iter<I, J>(s, adj_seg_iter(g, j, cur), st)) != hipSuccess) return e;
    cur = 1 - cur;
  }
  return hipSuccess;
}

template <int I, int J>
hipError_t launch_adj_seg(const DevState& s, const AdjSeg& g, hipStream_t st) {
  const size_t stash = sizeof(float4) * kAdjStashPlanes<I> * (size_t)s.N;
  return stash <= (size_t)kAdjStashBytes ? launch_adj_seg_k<I, J, true>(s, g, st, stash)
                                         : launch_adj_seg_k<I, J, false>(s, g, st, 0);
}

template <int I, int J>
hipError_t launch_adj_wiener(const DevState& s, const float2* gout, const AdjIter& a, hipStream_t st) {
  hipLaunchKernelGGL((k_adj_wiener<I, J>), dim3(s.F), dim3(kAdjBlock<I>), 0, st, s, gout, a);
  return hipGetLastError();
}

}  // namespace fca
