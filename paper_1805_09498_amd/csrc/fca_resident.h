// Frequency-resident FastFCA-AS: one workgroup owns one frequency bin for a
// whole batch of hybrid iterations.
//
// Bins never interact (every sum of eq. 20 and eq. 23 runs over n at fixed
// f), so a workgroup loads its bin's mixture x(., f) and spectra v(., f) into
// registers once, runs n_iter iterations entirely on chip, and writes v,
// lambda and P back at the end.  Lane t of a workgroup with T lanes owns
// frames n = t, t + T, ..., t + (NPT-1) T (coalesced loads and stores).
//
// Per iteration:  phase A (per point y = P^H x, eq. 15-19) -> transposed
// wave sums of the eq. 20 summands -> LDS -> lambda (eq. 20) in every lane ->
// phase B (per point weights and the weighted sums of y y^H) -> transposed
// wave sums -> LDS -> lanes 0..I-1 of wave 0 each solve one column of eq. 23
// in the basis of y -> P in LDS.
//
// Eq. 23 in the basis of y.  With y = P^H x the weighted covariance of
// eq. 23 is Q_i = P^-H G_i P^-1, G_i = (1/N) sum_n y y^H / d_i, so the
// update p_i = Q_i^-1 [P^-H]_i equals P G_i^-1 e_i exactly: column i of
// A = P_old^-1 P_new solves G_i a = e_i and P_new = P_old A.  Near DC a
// diffuse field makes Q_i nearly singular (condition ~1e4), and rounding its
// single-precision sums costs ~1e-4 in P; P has already absorbed that
// structure, so G_i stays well conditioned and no inverse of P is needed.
// Further fixed-point steps (K > 1) iterate the same map on A from A = 1.
#pragma once

#include <type_traits>

#include "fca_point.h"

namespace fca {

constexpr int kResMaxBlock = 256;
constexpr int kResMaxWaves = kResMaxBlock / kWave;

// Up to I = 4 the workgroup keeps x in registers next to y = P^H x; beyond,
// it reads x again each iteration, which leaves room for more frames per lane
// (the largest configurations spend ~I^3 flops per point and byte of x).
template <int I>
constexpr bool kResXInRegs = (I <= 4);

// Above I = 4 the eq. 23 sums of the resident kernel take several passes
// over the points, CPP columns each (I^2 accumulators per column, a point's
// y y^H formed once per pass).  Where the kernel runs one wave per SIMD
// whatever CPP (8 frames per lane at I = 6; and at I = 5 with J >= 5), it
// takes the fewest passes that fit; elsewhere two columns per pass keep two
// waves per SIMD.
template <int I, int J, int NPT>
constexpr int kResColsPerPass = (I == 5) ? ((NPT >= 8 && J >= 5) ? 5 : 2) : (I == 6) ? (NPT >= 8 ? 3 : 2) : 1;

// use(k, t_k) for k < V, t_k the sum of the per-wave partials
// part[w * stride + k] over the nw waves (nw in {1, 2, 4}, uniform), summed in
// wave order.  One uniform test selects the wave count for all V values (a
// test per value costs a branch each), and each total is consumed as it is
// formed, so no array of V totals stays live.
template <int V, typename Use>
__device__ __forceinline__ void sum_waves(const float* part, int stride, int nw, Use&& use) {
  if (nw == 1) {
#pragma unroll
    for (int k = 0; k < V; ++k) use(k, part[k]);
  } else if (nw == 2) {
#pragma unroll
    for (int k = 0; k < V; ++k) use(k, part[k] + part[stride + k]);
  } else {
#pragma unroll
    for (int k = 0; k < V; ++k)
      use(k, ((part[k] + part[stride + k]) + part[2 * stride + k]) + part[3 * stride + k]);
  }
}

// The body of one frequency-resident workgroup: bins f0 .. f0 + nb - 1 of the
// problem s (nb in {1, 2}), n_iter hybrid iterations.  kGen = false compiles
// the plain step only (K = 1, fixed-point P update), which keeps the
// registers and branches of the other P updates off the common path.
template <int I, int J, int NPT, bool kTrace = false, bool kGen = true>
__device__ __forceinline__ void as_resident_body(const DevState& s, int f0, int nb, int n_iter,
                                                 const Trace& tr = Trace{}) {
  const int p_update = kGen ? s.p_update : 0;
  const int n_fp = kGen ? s.K : 1;  // fixed-point steps per iteration
  constexpr int VS = pad4(kEq20Sums<I, J>);
  constexpr bool kOnePass = I * I * I <= 64;       // all I weighted sums in one sweep
  constexpr int VQ = kOnePass ? pad4(I * I * I) : pad4(I * I);
  constexpr int QSTRIDE = kOnePass ? VQ : I * VQ;  // per-wave stride of the Q partials
  constexpr bool kXReg = kResXInRegs<I>;
  // A workgroup of W waves owns nb bins with W / nb waves each; the waves of
  // one bin are consecutive.
  const int W = blockDim.x / kWave;
  const int nw = W / nb;                                   // waves per bin
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
  const int bin = wave / nw, wl = wave % nw;               // bin in the workgroup, wave in the bin
  const int f = f0 + bin;
  const int T = nw * kWave;                                // lanes per bin
  const int tb = wl * kWave + (int)(threadIdx.x & (kWave - 1));  // lane index within the bin
  const int lane = (int)(threadIdx.x & (kWave - 1));
  const int c = lane % I;                                  // the column of eq. 23 this lane solves
  // first frame of this wave's slot 0; a slot k is skipped by the whole wave
  // when wbase + k T >= N (a scalar branch)
  const int wbase = wl * kWave;
  __shared__ float sPr[2][I][I], sPi[2][I][I];
  __shared__ float sLam[2][J * I];
  __shared__ float redS[kResMaxWaves * VS];
  __shared__ float redQ[kResMaxWaves * QSTRIDE];
  const float* binS = redS + bin * nw * VS;                // this bin's wave partials
  const float* binQ = redQ + bin * nw * QSTRIDE;

  for (int t = tb; t < I * I; t += T) {
    const float2 p = s.P[(size_t)f * I * I + t];
    sPr[bin][t / I][t % I] = p.x; sPi[bin][t / I][t % I] = p.y;
  }
  for (int t = tb; t < J * I; t += T) sLam[bin][t] = s.lam[(size_t)f * J * I + t];

  const float* xf = s.xs + (size_t)f * 2 * I * s.Npad;
  float* vf = s.vs + (size_t)f * J * s.Npad;
  float xr[kXReg ? NPT : 1][I], xi[kXReg ? NPT : 1][I], v[NPT][J];
  float yr[NPT][I], yi[NPT][I];  // y = P^H x of the current iteration (phase A -> B)
  // Where the registers allow, phase B keeps its eq. 23 weights 1 / d_i
  // (from the updated v and lambda) for the next iteration's phase A, whose
  // d_i are the same sums: the E-step then forms no d_i and no reciprocal.
  // (not in the recording variant, whose trace addresses take those
  // registers: there it would cost the second workgroup per CU).
  constexpr bool kKeepRd = kOnePass && NPT <= 8 && !kGen && !kTrace;
  float rdk[kKeepRd ? NPT : 1][I];
  // The same kernels compile a second form of phases A and B for waves whose
  // slots all hold frames (see phase_a); in the recording variant only up to
  // 7 slots (at 8 its registers would leave one workgroup per CU).
  constexpr bool kDense = kOnePass && !kGen && (kTrace ? NPT <= 7 : NPT <= 8);
#pragma unroll
  for (int k = 0; k < NPT; ++k) {
    const int n = tb + k * T;
    const bool ok = n < s.N;
    if constexpr (kXReg) {
#pragma unroll
      for (int i = 0; i < I; ++i) {
        xr[k][i] = ok ? xf[(size_t)i * s.Npad + n] : 0.f;
        xi[k][i] = ok ? xf[(size_t)(I + i) * s.Npad + n] : 0.f;
      }
    }
#pragma unroll
    for (int j = 0; j < J; ++j) v[k][j] = ok ? vf[(size_t)j * s.Npad + n] : 1.f;
  }
  __syncthreads();
  const float invN = 1.0f / float(s.N);
  if constexpr (kKeepRd) {
    float lam0[J][I];
#pragma unroll
    for (int j = 0; j < J; ++j)
#pragma unroll
      for (int i = 0; i < I; ++i) lam0[j][i] = sLam[bin][j * I + i];
#pragma unroll
    for (int k = 0; k < NPT; ++k)
      if (wbase + k * T < s.N) as_point_weights<I, J>(lam0, v[k], rdk[k]);
  }

#pragma unroll 1
  for (int it = 0; it < n_iter; ++it) {
    float Pr[I][I], Pi[I][I], lam[J][I];
#pragma unroll
    for (int a = 0; a < I; ++a)
#pragma unroll
      for (int b = 0; b < I; ++b) { Pr[a][b] = sPr[bin][a][b]; Pi[a][b] = sPi[bin][a][b]; }
#pragma unroll
    for (int j = 0; j < J; ++j)
#pragma unroll
      for (int i = 0; i < I; ++i) lam[j][i] = sLam[bin][j * I + i];

    // ---- phase A: E-step statistics, v update, eq. 20 summands ------------
    // Issue priority: where the waves of two workgroups share a SIMD (the CU
    // that holds an odd bin out, the batch kernels), the sections that every
    // wave of a workgroup waits on -- the cross-wave sums, lambda, the
    // per-bin solve -- issue ahead of the other workgroup's per-frame phases,
    // which fill the gaps.  (One workgroup per CU: no effect.)
    __builtin_amdgcn_s_setprio(0);
    {
      float S0[J], S1[J][I], lamI[J][I];
#pragma unroll
      for (int j = 0; j < J; ++j) {
        S0[j] = 0.f;
#pragma unroll
        for (int i = 0; i < I; ++i) { S1[j][i] = 0.f; lamI[j][i] = lam[j][i] * (1.0f / float(I)); }
      }
      // every = true: all NPT slots of the wave hold frames, no slot is
      // tested and the compiler interleaves the slots' dependency chains
      // (one basic block); otherwise each slot is tested (wave-uniform).
      auto phase_a = [&](auto every) {
#pragma unroll
      for (int k = 0; k < NPT; ++k) {
        if (decltype(every)::value || wbase + k * T < s.N) {
          const bool ok = tb + k * T < s.N;
          if constexpr (kXReg) {
            as_transform<I>(Pr, Pi, xr[k], xi[k], yr[k], yi[k]);
          } else {
            // x is read again each iteration (cached; it never changes).  The
            // slot starts below N at a multiple of 64 and Npad is a multiple of
            // 64, so every lane reads inside the zero-padded plane: no select.
            // The zero offset is opaque to the optimiser: otherwise it keeps
            // the addresses of every point's loads alive across iterations.
            float xr1[I], xi1[I];
            int zoff = 0;
            asm volatile("" : "+s"(zoff));
            const float* xl = xf + zoff + tb + k * T;
#pragma unroll
            for (int i = 0; i < I; ++i) {
              xr1[i] = xl[(size_t)i * s.Npad];
              xi1[i] = xl[(size_t)(I + i) * s.Npad];
            }
            as_transform<I>(Pr, Pi, xr1, xi1, yr[k], yi[k]);
          }
          float y2[I];
#pragma unroll
          for (int i = 0; i < I; ++i) y2[i] = fmaf(yr[k][i], yr[k][i], yi[k][i] * yi[k][i]);
          if constexpr (kKeepRd) {
            // one form for every slot: a copy without the per-lane selects
            // for the full slots cost more in register copies than it saved
            as_point_em_rd<I, J>(y2, rdk[k], lamI, v[k], S0, S1, ok);
          } else {
            // a slot every lane of the wave owns skips the per-lane selects
            if (wbase + k * T + kWave <= s.N)
              as_point_em<I, J>(y2, lam, lamI, v[k], S0, S1, true);
            else
              as_point_em<I, J>(y2, lam, lamI, v[k], S0, S1, ok);
          }
        }
      }
      };
      if (kDense && wbase + (NPT - 1) * T < s.N)
        phase_a(std::true_type{});
      else
        phase_a(std::false_type{});
      float flat[kEq20Sums<I, J>];
#pragma unroll
      for (int j = 0; j < J; ++j) {
        flat[j] = S0[j];
#pragma unroll
        for (int i = 0; i < I; ++i) flat[J + j * I + i] = S1[j][i];
      }
      __builtin_amdgcn_s_setprio(2);
      wave_totals_to_lds<kEq20Sums<I, J>>(flat, redS, VS);  // slot of wave `wave`
    }
    __syncthreads();
    // eq. 20: lambda (S0_j + lambda S1_ji) / N with the old lambda
    {
      float s0[J], s1[J][I];
      sum_waves<kEq20Sums<I, J>>(binS, VS, nw, [&](int k, float t) {
        if (k < J) s0[k] = t; else s1[(k - J) / I][(k - J) % I] = t;
      });
#pragma unroll
      for (int j = 0; j < J; ++j)
#pragma unroll
        for (int i = 0; i < I; ++i) lam[j][i] = eq20_lambda(lam[j][i], s0[j], s1[j][i], invN);
    }

    // ---- phase B: the weighted sums N G_i of y y^H (eq. 23) ----------------
    __builtin_amdgcn_s_setprio(0);
    if constexpr (kOnePass) {
      float A[I][I * I];
#pragma unroll
      for (int i = 0; i < I; ++i)
#pragma unroll
        for (int q = 0; q < I * I; ++q) A[i][q] = 0.f;
      auto phase_b = [&](auto every) {
#pragma unroll
      for (int k = 0; k < NPT; ++k) {
        if (decltype(every)::value || wbase + k * T < s.N) {
          // lanes past N hold y = 0 and their initial v (kept by phase A), so
          // their weight is finite and they add nothing
          float w[I], z[I * I];
          as_point_weights<I, J>(lam, v[k], w);
          herm_outer<I>(z, yr[k], yi[k]);
          if constexpr (kKeepRd) {
#pragma unroll
            for (int a = 0; a < I; ++a) rdk[k][a] = w[a];
          }
#pragma unroll
          for (int i = 0; i < I; ++i)
#pragma unroll
            for (int q = 0; q < I * I; ++q) A[i][q] = fmaf(w[i], z[q], A[i][q]);
        }
      }
      };
      if (kDense && wbase + (NPT - 1) * T < s.N)
        phase_b(std::true_type{});
      else
        phase_b(std::false_type{});
      float flat[I * I * I];
#pragma unroll
      for (int i = 0; i < I; ++i)
#pragma unroll
        for (int q = 0; q < I * I; ++q) flat[i * I * I + q] = A[i][q];
      __builtin_amdgcn_s_setprio(2);
      wave_totals_to_lds<I * I * I>(flat, redQ, QSTRIDE);
    } else {
      // one pass over the points per CPP columns: a point's y y^H is formed
      // once per pass and its weights 1 / d_i in the pass (rather than kept for
      // all points: registers)
      constexpr int CPP = kResColsPerPass<I, J, NPT>;
      if constexpr (CPP == 1) {
#pragma unroll
        for (int i = 0; i < I; ++i) {
          float A[I * I];
#pragma unroll
          for (int q = 0; q < I * I; ++q) A[q] = 0.f;
#pragma unroll
          for (int k = 0; k < NPT; ++k)
            if (wbase + k * T < s.N) {
              float d = 0.f;  // y = 0 and v kept past N: finite, adds nothing
#pragma unroll
              for (int j = 0; j < J; ++j) d = fmaf(v[k][j], lam[j][i], d);
              herm_rank1_acc<I>(A, rcp(d), yr[k], yi[k]);
            }
          wave_totals_to_lds<I * I>(A, redQ + i * VQ, QSTRIDE);
        }
      } else {
#pragma unroll
      for (int i0 = 0; i0 < I; i0 += CPP) {
        float A[CPP][I * I];
#pragma unroll
        for (int ci = 0; ci < CPP; ++ci)
#pragma unroll
          for (int q = 0; q < I * I; ++q) A[ci][q] = 0.f;
#pragma unroll
        for (int k = 0; k < NPT; ++k)
          if (wbase + k * T < s.N) {
            float z[I * I];
            herm_outer<I>(z, yr[k], yi[k]);
#pragma unroll
            for (int ci = 0; ci < CPP; ++ci) {
              if (i0 + ci < I) {
                float d = 0.f;  // y = 0 and v kept past N: finite, adds nothing
#pragma unroll
                for (int j = 0; j < J; ++j) d = fmaf(v[k][j], lam[j][i0 + ci], d);
                const float w = rcp(d);
#pragma unroll
                for (int q = 0; q < I * I; ++q) A[ci][q] = fmaf(w, z[q], A[ci][q]);
              }
            }
          }
#pragma unroll
        for (int ci = 0; ci < CPP; ++ci)
          if (i0 + ci < I) wave_totals_to_lds<I * I>(A[ci], redQ + (i0 + ci) * VQ, QSTRIDE);
      }
      }
    }
    __builtin_amdgcn_s_setprio(2);
    __syncthreads();

    // ---- per-bin solve: lane c < I computes column c of eq. 23 ------------
    if (tb == 0) {
#pragma unroll
      for (int q = 0; q < J * I; ++q) sLam[bin][q] = lam[q / I][q % I];
    }
    // One wave of the bin solves (lane c: column c); the other waves go
    // straight to the barrier that publishes the new P.  The solving wave
    // rotates with the iteration, so that on a CU whose SIMDs host waves of
    // two workgroups the serial solves land on every SIMD in turn.
    if (wl == (it & (nw - 1))) {  // nw is 1, 2 or 4
      __builtin_amdgcn_s_setprio(3);  // every wave of the workgroup waits on this one
      // P_old for p_c = P_old a_c, requested before the solve's chain
      float Por[I][I], Poi[I][I];
#pragma unroll
      for (int a = 0; a < I; ++a)
#pragma unroll
        for (int b = 0; b < I; ++b) { Por[a][b] = sPr[bin][a][b]; Poi[a][b] = sPi[bin][a][b]; }
      // S_c = N G_c (upper triangle); column c of A solves S_c a = N e_c.
      // packed: real parts on and above, imaginary parts below the diagonal
      float Sr[I][I], Si[I][I];
      sum_waves<I * I>(binQ + (kOnePass ? c * I * I : c * VQ), QSTRIDE, nw, [&](int k, float t) {
        const int a = k / I, b = k % I;
        if (b >= a) Sr[a][b] = t; else Si[b][a] = t;
      });
#pragma unroll
      for (int a = 0; a < I; ++a) Si[a][a] = 0.f;
      if constexpr (kTrace) {
        if (lane < I) {  // S_c packed: real parts on and above, imaginary parts below the diagonal
          float* dst = tr.S + (size_t)it * tr.sstride + ((size_t)f * I + c) * I * I;
#pragma unroll
          for (int a = 0; a < I; ++a)
#pragma unroll
            for (int b = 0; b < I; ++b) dst[a * I + b] = (b >= a) ? Sr[a][b] : Si[b][a];
        }
      }
      const float fN = float(s.N);
      float ar[I], ai[I], pnr[I], pni[I];
      // gamma_c = S_c e_c / N (column c of G_c), for the gradient-type steps
      float gr[I], gi[I];
      if (p_update != 0) {
#pragma unroll
        for (int a = 0; a < I; ++a) {
          float r = 0.f, m = 0.f;  // a select chain keeps every index a constant
#pragma unroll
          for (int cc = 0; cc < I; ++cc) {  // entry (a, cc) of S_c: conj of (cc, a) below the diagonal
            r = (c == cc) ? ((a <= cc) ? Sr[a][cc] : Sr[cc][a]) : r;
            m = (c == cc) ? ((a == cc) ? 0.f : (a < cc) ? Si[a][cc] : -Si[cc][a]) : m;
          }
          gr[a] = r * invN;
          gi[a] = m * invN;
        }
      }
      if (p_update == 2) {  // natural gradient: A = 1 + mu (1 - Gamma)
#pragma unroll
        for (int a = 0; a < I; ++a) {
          ar[a] = ((a == c) ? 1.f + s.p_step : 0.f) - s.p_step * gr[a];
          ai[a] = -s.p_step * gi[a];
        }
      } else {
#pragma unroll
        for (int a = 0; a < I; ++a) { ar[a] = (a == c) ? fN : 0.f; ai[a] = 0.f; }
        if (!herm_solve<I>(Sr, Si, ar, ai) && lane < I) atomicOr(s.flag, kFlagSingular);
      }
      // K > 1: further fixed-point steps a_c = G_c^-1 [A^-H]_c; lane b holds
      // column b of the current A, gathered with readlane (no LDS, no
      // barrier: only the bin's first wave takes part).  Compiled up to
      // I = kResMaxIK only (the inverse of A costs registers that larger I
      // cannot spare); the host sends K > 1 at larger I to the streaming
      // kernels.
#pragma unroll 1
      for (int kk = 1; kk < ((I <= kResMaxIK && p_update == 0) ? n_fp : 1); ++kk) {
        float A2r[I][I], A2i[I][I];
#pragma unroll
        for (int a = 0; a < I; ++a)
#pragma unroll
          for (int b = 0; b < I; ++b) {
            A2r[a][b] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(ar[a]), b));
            A2i[a][b] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(ai[a]), b));
          }
        pinvh_col<I, float>(A2r, A2i, c, ar, ai);
#pragma unroll
        for (int a = 0; a < I; ++a) { ar[a] *= fN; ai[a] *= fN; }
        if (!herm_solve<I>(Sr, Si, ar, ai) && lane < I) atomicOr(s.flag, kFlagSingular);
      }
      // p_c = P_old a_c (P_old read from LDS above: the copy in registers
      // from phase A is not kept alive through phase B).  Lane c < I writes
      // column c of the LDS copy below, after every lane has read it.
#pragma unroll
      for (int a = 0; a < I; ++a) {
        float pr = 0.f, pi = 0.f;
#pragma unroll
        for (int b = 0; b < I; ++b) {
          const float qr = Por[a][b], qi = Poi[a][b];
          pr = fmaf(qr, ar[b], pr);
          pr = fmaf(-qi, ai[b], pr);
          pi = fmaf(qr, ai[b], pi);
          pi = fmaf(qi, ar[b], pi);
        }
        pnr[a] = pr; pni[a] = pi;
      }
      if constexpr (I <= kResMaxIK) {
        if (p_update == 1) {
          // gradient: p_c + mu P^-H (e_c - gamma_c); lane b forms column b of
          // P^-H, the matrix is gathered with readlane (wave 0 only)
          float Pr2[I][I], Pi2[I][I], br[I], bi[I];
#pragma unroll
          for (int a = 0; a < I; ++a)
#pragma unroll
            for (int b = 0; b < I; ++b) { Pr2[a][b] = sPr[bin][a][b]; Pi2[a][b] = sPi[bin][a][b]; }
          pinvh_col<I, float>(Pr2, Pi2, c, br, bi);
#pragma unroll
          for (int a = 0; a < I; ++a) { pnr[a] = sPr[bin][a][c]; pni[a] = sPi[bin][a][c]; }
#pragma unroll
          for (int b = 0; b < I; ++b) {
            const float dr = ((b == c) ? 1.f : 0.f) - gr[b];  // e_c - gamma_c
            const float di = -gi[b];
#pragma unroll
            for (int a = 0; a < I; ++a) {
              const float Br = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(br[a]), b));
              const float Bi = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(bi[a]), b));
              pnr[a] = fmaf(s.p_step, Br * dr - Bi * di, pnr[a]);
              pni[a] = fmaf(s.p_step, Br * di + Bi * dr, pni[a]);
            }
          }
        }
      }
      if (lane < I) {
#pragma unroll
        for (int a = 0; a < I; ++a) { sPr[bin][a][c] = pnr[a]; sPi[bin][a][c] = pni[a]; }
      }
    }
    __syncthreads();
    if constexpr (kTrace) {  // the state after this iteration
      const size_t off = (size_t)it * tr.stride;
#pragma unroll
      for (int k = 0; k < NPT; ++k) {
        const int n = tb + k * T;
        if (n < s.N) {
#pragma unroll
          for (int j = 0; j < J; ++j) tr.v[off + ((size_t)f * J + j) * s.Npad + n] = v[k][j];
        }
      }
      float2* Pit = reinterpret_cast<float2*>(reinterpret_cast<float*>(tr.P) + off);
      for (int t = tb; t < I * I; t += T)
        Pit[(size_t)f * I * I + t] = make_float2(sPr[bin][t / I][t % I], sPi[bin][t / I][t % I]);
      for (int t = tb; t < J * I; t += T) tr.lam[off + (size_t)f * J * I + t] = sLam[bin][t];
    }
  }

  // ---- write the state back ------------------------------------------------
#pragma unroll
  for (int k = 0; k < NPT; ++k) {
    const int n = tb + k * T;
    if (n < s.N) {
#pragma unroll
      for (int j = 0; j < J; ++j) vf[(size_t)j * s.Npad + n] = v[k][j];
    }
  }
  for (int t = tb; t < I * I; t += T)
    s.P[(size_t)f * I * I + t] = make_float2(sPr[bin][t / I][t % I], sPi[bin][t / I][t % I]);
  for (int t = tb; t < J * I; t += T) s.lam[(size_t)f * J * I + t] = sLam[bin][t];
}

// One problem: workgroup g owns bins g*bpw .. (the last may own fewer).
template <int I, int J, int NPT, bool kGen>
__global__ __launch_bounds__(kResMaxBlock) void k_as_resident(DevState s, int n_iter, int bpw) {
  const int f0 = blockIdx.x * bpw;
  const int nb = (s.F - f0 < bpw) ? (s.F - f0) : bpw;
  as_resident_body<I, J, NPT, false, kGen>(s, f0, nb, n_iter);
}

// The same as k_as_resident (plain step only), recording the state after
// every iteration.
template <int I, int J, int NPT>
__global__ __launch_bounds__(kResMaxBlock) void k_as_resident_trace(DevState s, int n_iter, int bpw, Trace tr) {
  const int f0 = blockIdx.x * bpw;
  const int nb = (s.F - f0 < bpw) ? (s.F - f0) : bpw;
  as_resident_body<I, J, NPT, true, false>(s, f0, nb, n_iter, tr);
}

// Many problems of the same (I, J): workgroup g takes tile g = (problem,
// bin) of a table the host sorts by decreasing N, so the hardware dispatcher
// hands the longest tiles out first.
template <int I, int J, int NPT, bool kGen>
__global__ __launch_bounds__(kResMaxBlock) void k_as_resident_batch(const DevState* __restrict__ states,
                                                                    const int2* __restrict__ tiles,
                                                                    int n_iter) {
  const int2 t = tiles[blockIdx.x];
  const DevState s = states[t.x];
  // one bin per workgroup, passed as a value the optimiser cannot see: with
  // the constant, the I = 6 kernels came out at 512 registers plus scratch
  // spills (389 and none with the run-time value)
  int nb = 1;
  asm volatile("" : "+s"(nb));
  as_resident_body<I, J, NPT, false, kGen>(s, t.y, nb, n_iter);
}

// The same with a work queue: a grid of as many workgroups as fit on the
// device at once, each taking the next tile from a device counter (which
// the host resets to zero before the launch) until the table is exhausted.
// Every workgroup leaves once the counter passes the table's end.
template <int I, int J, int NPT, bool kGen>
__global__ __launch_bounds__(kResMaxBlock) void k_as_resident_batch_q(const DevState* __restrict__ states,
                                                                      const int2* __restrict__ tiles, int ntiles,
                                                                      int n_iter, int* __restrict__ counter) {
  __shared__ int next;
  for (;;) {
    if (threadIdx.x == 0) next = atomicAdd(counter, 1);
    __syncthreads();
    const int k = next;
    __syncthreads();  // every lane has read `next` before lane 0 takes another tile
    if (k >= ntiles) break;
    const int2 t = tiles[k];
    const DevState s = states[t.x];
    int nb = 1;
    asm volatile("" : "+s"(nb));
    as_resident_body<I, J, NPT, false, kGen>(s, t.y, nb, n_iter);
    __syncthreads();  // the tile's last LDS reads before the next tile's writes
  }
}

// Register budget of the resident kernel: NPT points of y (2I), v (J), the
// eq. 23 weights (I) and, up to I = 4, x (2I) per lane.
template <int I, int J>
constexpr int res_max_npt() {
  constexpr int per = (kResXInRegs<I> ? 5 * I : 3 * I) + J;
  return (16 * per <= 224) ? 16 : (12 * per <= 224) ? 12 : (8 * per <= 224) ? 8 : 4;
}

template <int I, int J>
int as_resident_fits(int N, int waves, int bpw) {
  if (waves != 1 && waves != 2 && waves != 4) return 0;
  if (bpw != 1 && bpw != 2) return 0;
  if (bpw == 2 && waves < 2) return 0;
  return N <= res_max_npt<I, J>() * (waves / bpw) * kWave ? 1 : 0;
}

// Batched launch: tiles of problems whose N are at most n_max, one workgroup
// of `waves` waves per tile; `general` when any member takes K > 1 or another
// P update.
// One tile per workgroup in table order, or (counter != NULL) the work-queue
// form with as many workgroups as fit on the device.  Where the queue
// kernel's registers overflow to scratch memory (the tile loop keeps a few
// more values live than the one-tile kernel, which the largest bodies do not
// have to spare) the one-tile form is launched instead.  *queued (when not
// NULL) tells which form ran.
template <int I, int J, int NPT, bool kGen>
hipError_t launch_as_batch_npt(const DevState* states, const int2* tiles, int ntiles, hipStream_t st, int n_iter,
                               int T, int* counter, int* queued) {
  static const int q_scratch = [] {
    hipFuncAttributes a{};
    if (hipFuncGetAttributes(&a, reinterpret_cast<const void*>(k_as_resident_batch_q<I, J, NPT, kGen>)) !=
        hipSuccess)
      return 1;
    return a.localSizeBytes > 0 ? 1 : 0;
  }();
  if (queued) *queued = (counter && !q_scratch) ? 1 : 0;
  if (!counter || q_scratch) {
    hipLaunchKernelGGL((k_as_resident_batch<I, J, NPT, kGen>), dim3(ntiles), dim3(T), 0, st, states, tiles, n_iter);
    return hipGetLastError();
  }
  int per_cu = 0, dev = 0, cus = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_as_resident_batch_q<I, J, NPT, kGen>, T, 0);
  if (e == hipSuccess) e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  long long g = (long long)(per_cu > 0 ? per_cu : 1) * (cus > 0 ? cus : 1);
  g = g < ntiles ? g : ntiles;
  if ((e = launch_set_flag(counter, 0, st)) != hipSuccess) return e;
  hipLaunchKernelGGL((k_as_resident_batch_q<I, J, NPT, kGen>), dim3((unsigned)g), dim3(T), 0, st, states, tiles,
                     ntiles, n_iter, counter);
  return hipGetLastError();
}

template <int I, int J, bool kGen>
hipError_t launch_as_batch_g(const DevState* states, const int2* tiles, int ntiles, int n_max, hipStream_t st,
                             int n_iter, int waves, int* counter, int* queued) {
  const int T = waves * kWave;
  const int need = (n_max + T - 1) / T;
  constexpr int mx = res_max_npt<I, J>();
  if (ntiles <= 0) return hipSuccess;
  if (need <= 4) return launch_as_batch_npt<I, J, 4, kGen>(states, tiles, ntiles, st, n_iter, T, counter, queued);
  if (need <= 8 && mx >= 8)
    return launch_as_batch_npt<I, J, (mx >= 8 ? 8 : 4), kGen>(states, tiles, ntiles, st, n_iter, T, counter,
                                                              queued);
  if (need <= 12 && mx >= 12)
    return launch_as_batch_npt<I, J, (mx >= 12 ? 12 : 4), kGen>(states, tiles, ntiles, st, n_iter, T, counter,
                                                                queued);
  if (need <= 16 && mx >= 16)
    return launch_as_batch_npt<I, J, (mx >= 16 ? 16 : 4), kGen>(states, tiles, ntiles, st, n_iter, T, counter,
                                                                queued);
  return hipErrorInvalidValue;
}

template <int I, int J>
hipError_t launch_as_batch_resident(const DevState* states, const int2* tiles, int ntiles, int n_max,
                                    hipStream_t st, int n_iter, int waves, bool general, int* counter,
                                    int* queued) {
  return general ? launch_as_batch_g<I, J, true>(states, tiles, ntiles, n_max, st, n_iter, waves, counter, queued)
                 : launch_as_batch_g<I, J, false>(states, tiles, ntiles, n_max, st, n_iter, waves, counter, queued);
}

template <int I, int J, bool kGen>
hipError_t launch_as_resident_g(const DevState& s, hipStream_t st, int n_iter, int waves, int bpw) {
  const int T = (waves / bpw) * kWave;  // lanes per bin when the workgroup is full
  const int need = (s.N + T - 1) / T;
  constexpr int mx = res_max_npt<I, J>();
  dim3 grid((s.F + bpw - 1) / bpw), block(waves * kWave);
  auto go = [&](auto npt) {
    hipLaunchKernelGGL((k_as_resident<I, J, decltype(npt)::value, kGen>), grid, block, 0, st, s, n_iter, bpw);
  };
  // The plain step at I <= 4 takes the exact slot count below 8 (where the
  // registers allow it), so that the waves of the full workgroups run the
  // form of phases A and B without a test per slot.
  constexpr bool kE = !kGen && I <= 4, kE8 = kE && mx >= 8;
  using std::integral_constant;
  if (kE && need == 1) go(integral_constant<int, kE ? 1 : 4>{});
  else if (kE && need == 2) go(integral_constant<int, kE ? 2 : 4>{});
  else if (kE && need == 3) go(integral_constant<int, kE ? 3 : 4>{});
  else if (need <= 4) go(integral_constant<int, 4>{});
  else if (kE8 && need == 5) go(integral_constant<int, kE8 ? 5 : 4>{});
  else if (kE8 && need == 6) go(integral_constant<int, kE8 ? 6 : 4>{});
  else if (kE8 && need == 7) go(integral_constant<int, kE8 ? 7 : 4>{});
  else if (need <= 8 && mx >= 8) go(integral_constant<int, (mx >= 8 ? 8 : 4)>{});
  else if (need <= 12 && mx >= 12) go(integral_constant<int, (mx >= 12 ? 12 : 4)>{});
  else if (need <= 16 && mx >= 16) go(integral_constant<int, (mx >= 16 ? 16 : 4)>{});
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

template <int I, int J>
hipError_t launch_as_iter_resident(const DevState& s, hipStream_t st, int n_iter, int waves, int bpw) {
  return (s.K > 1 || s.p_update != 0) ? launch_as_resident_g<I, J, true>(s, st, n_iter, waves, bpw)
                                      : launch_as_resident_g<I, J, false>(s, st, n_iter, waves, bpw);
}

// The recording kernel runs the plain step only (K = 1, fixed-point P update).
template <int I, int J>
hipError_t launch_as_iter_resident_trace(const DevState& s, hipStream_t st, int n_iter, int waves, int bpw,
                                         const Trace& tr) {
  if (s.K != 1 || s.p_update != 0) return hipErrorInvalidValue;
  const int T = (waves / bpw) * kWave;
  const int need = (s.N + T - 1) / T;
  constexpr int mx = res_max_npt<I, J>();
  dim3 grid((s.F + bpw - 1) / bpw), block(waves * kWave);
  auto go = [&](auto npt) {
    hipLaunchKernelGGL((k_as_resident_trace<I, J, decltype(npt)::value>), grid, block, 0, st, s, n_iter, bpw, tr);
  };
  // exact slot counts below 8 at I <= 4, as the plain kernel's launcher
  constexpr bool kE = I <= 4, kE8 = kE && mx >= 8;
  using std::integral_constant;
  if (kE && need == 1) go(integral_constant<int, kE ? 1 : 4>{});
  else if (kE && need == 2) go(integral_constant<int, kE ? 2 : 4>{});
  else if (kE && need == 3) go(integral_constant<int, kE ? 3 : 4>{});
  else if (kE8 && need == 5) go(integral_constant<int, kE8 ? 5 : 4>{});
  else if (kE8 && need == 6) go(integral_constant<int, kE8 ? 6 : 4>{});
  else if (kE8 && need == 7) go(integral_constant<int, kE8 ? 7 : 4>{});
  else if (need <= 4)
    hipLaunchKernelGGL((k_as_resident_trace<I, J, 4>), grid, block, 0, st, s, n_iter, bpw, tr);
  else if (need <= 8 && mx >= 8)
    hipLaunchKernelGGL((k_as_resident_trace<I, J, (mx >= 8 ? 8 : 4)>), grid, block, 0, st, s, n_iter, bpw, tr);
  else if (need <= 12 && mx >= 12)
    hipLaunchKernelGGL((k_as_resident_trace<I, J, (mx >= 12 ? 12 : 4)>), grid, block, 0, st, s, n_iter, bpw, tr);
  else if (need <= 16 && mx >= 16)
    hipLaunchKernelGGL((k_as_resident_trace<I, J, (mx >= 16 ? 16 : 4)>), grid, block, 0, st, s, n_iter, bpw, tr);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace fca
