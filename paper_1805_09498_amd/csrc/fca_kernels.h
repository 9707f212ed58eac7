// Templated kernels of libfastfca, instantiated per (I, J) by fca_inst_I*.hip.
//
// FastFCA-AS iteration (Section 4.3 of the paper), streaming form, three
// launches per hybrid iteration:
//   as_pass_a  per point: y = P^H x, d_i = sum_j v_j lambda_ji, diagonal
//              posterior statistics (eq. 16-17), v update (eq. 19); per tile
//              the partial sums of eq. 20.
//   as_pass_b  lambda update (eq. 20) from the tile partials; per point the
//              new d_i; per tile the partial weighted covariances of eq. 23.
//   as_solve   per bin and column: P^-H column by LU, Cholesky solve of eq. 23.
// The frequency-resident form (fca_resident.h) runs whole iterations inside
// one workgroup per bin with the bin's data kept in registers.
#pragma once

#include "fca_device.h"
#include "fca_point.h"
#include "fca_pvariants.h"
#include "fca_state.h"

namespace fca {

// ----------------------------------------------------------------------------
// FastFCA-AS streaming kernels.
// ----------------------------------------------------------------------------
// Tiles are (bin, chunk of kChunk frames): lane t of a 256-lane workgroup
// takes frames chunk*kChunk + p*256 + t, p < kPts.  Up to I = 4 the bin's P
// sits in registers; above, every lane reads it from LDS for each frame (a
// broadcast read), which keeps the registers for more waves per SIMD.
template <int I>
constexpr bool kStreamPinLds = (I >= 5);

// P staged in LDS by columns: entry i * PH + h holds P[2h][i] and
// P[2h + 1][i] (re, im, re, im; zero past I), so that y_i = (P^H x)_i reads
// column i with 128-bit broadcast loads.
template <int I>
constexpr int kPH = (I + 1) / 2;

template <int I>
__device__ __forceinline__ void stage_P_columns(const float2* __restrict__ P, float4* sPt) {
  for (int t = threadIdx.x; t < I * kPH<I>; t += blockDim.x) {
    const int i = t / kPH<I>, k = 2 * (t % kPH<I>);
    const float2 p0 = P[k * I + i];
    const float2 p1 = (k + 1 < I) ? P[(k + 1) * I + i] : make_float2(0.f, 0.f);
    sPt[t] = make_float4(p0.x, p0.y, p1.x, p1.y);
  }
}

// y = P^H x with P read from its column staging in LDS.
template <int I>
__device__ __forceinline__ void as_transform_lds(const float4* sPt, const float (&xr)[I], const float (&xi)[I],
                                                 float (&yr)[I], float (&yi)[I]) {
#pragma unroll
  for (int i = 0; i < I; ++i) {
    float a = 0.f, b = 0.f;
#pragma unroll
    for (int h = 0; h < kPH<I>; ++h) {
      const float4 q = sPt[i * kPH<I> + h];
      const int k = 2 * h;
      a = fmaf(q.x, xr[k], a);
      a = fmaf(q.y, xi[k], a);
      b = fmaf(q.x, xi[k], b);
      b = fmaf(-q.y, xr[k], b);
      if (k + 1 < I) {
        a = fmaf(q.z, xr[k + 1], a);
        a = fmaf(q.w, xi[k + 1], a);
        b = fmaf(q.z, xi[k + 1], b);
        b = fmaf(-q.w, xr[k + 1], b);
      }
    }
    yr[i] = a; yi[i] = b;
  }
}

// Per-workgroup totals of V per-lane values: transposed wave sums, then the
// waves' totals summed in wave order by the first V lanes, stored to out.
template <int V>
__device__ __forceinline__ void block_totals_store(const float (&a)[V], float* __restrict__ out, float* lds) {
  constexpr int V4 = pad4(V);
  wave_totals_to_lds<V>(a, lds, V4);
  __syncthreads();
  const int nw = blockDim.x / kWave;
  for (int k = threadIdx.x; k < V; k += blockDim.x) {
    float t = lds[k];
    for (int w = 1; w < nw; ++w) t += lds[w * V4 + k];
    out[k] = t;
  }
}

// Pass A: y = P^H x, E-step and v update per frame (eq. 15-19, the form of
// as_point_em), and the tile's sums of the eq. 20 summands.
template <int I, int J>
__global__ __launch_bounds__(kBlock) void k_as_pass_a(DevState s) {
  const int f = blockIdx.y, chunk = blockIdx.x;
  __shared__ float4 sPt[I * kPH<I>];
  __shared__ float sLam[J * I];
  constexpr int V = kEq20Sums<I, J>;
  __shared__ float red[(kBlock / kWave) * pad4(V)];
  stage_P_columns<I>(s.P + (size_t)f * I * I, sPt);
  for (int t = threadIdx.x; t < J * I; t += kBlock) sLam[t] = s.lam[(size_t)f * J * I + t];
  __syncthreads();
  float lam[J][I], lamI[J][I];
#pragma unroll
  for (int j = 0; j < J; ++j)
#pragma unroll
    for (int i = 0; i < I; ++i) { lam[j][i] = sLam[j * I + i]; lamI[j][i] = lam[j][i] * (1.0f / float(I)); }
  float Pr[kStreamPinLds<I> ? 1 : I][kStreamPinLds<I> ? 1 : I], Pi[kStreamPinLds<I> ? 1 : I][kStreamPinLds<I> ? 1 : I];
  if constexpr (!kStreamPinLds<I>) {
#pragma unroll
    for (int i = 0; i < I; ++i)
#pragma unroll
      for (int h = 0; h < kPH<I>; ++h) {
        const float4 q = sPt[i * kPH<I> + h];
        Pr[2 * h][i] = q.x; Pi[2 * h][i] = q.y;
        if (2 * h + 1 < I) { Pr[2 * h + 1][i] = q.z; Pi[2 * h + 1][i] = q.w; }
      }
  }
  float S0[J], S1[J][I];
#pragma unroll
  for (int j = 0; j < J; ++j) {
    S0[j] = 0.f;
#pragma unroll
    for (int i = 0; i < I; ++i) S1[j][i] = 0.f;
  }

  const float* xf = s.xs + (size_t)f * 2 * I * s.Npad;
  float* vf = s.vs + (size_t)f * J * s.Npad;
  // (loading frame p + 1 ahead of frame p costs the registers of a third
  // wave per SIMD at I = 8, and is slower there)
#pragma unroll kStreamPinLds<I> ? 1 : kPts
  for (int p = 0; p < kPts; ++p) {
    const int n = chunk * kChunk + p * kBlock + threadIdx.x;
    const bool ok = n < s.N;
    const int nn = ok ? n : 0;  // frames past N read frame 0 and add nothing
    float xr[I], xi[I], v[J], yr[I], yi[I], y2[I];
#pragma unroll
    for (int i = 0; i < I; ++i) { xr[i] = xf[(size_t)i * s.Npad + nn]; xi[i] = xf[(size_t)(I + i) * s.Npad + nn]; }
#pragma unroll
    for (int j = 0; j < J; ++j) v[j] = vf[(size_t)j * s.Npad + nn];
    if constexpr (kStreamPinLds<I>) {
      // an offset opaque to the optimiser keeps P's reads inside the loop
      // (hoisted, they would hold all of P in registers)
      int zo = 0;
      asm volatile("" : "+s"(zo));
      as_transform_lds<I>(sPt + zo, xr, xi, yr, yi);
    } else {
      as_transform<I>(Pr, Pi, xr, xi, yr, yi);
    }
#pragma unroll
    for (int i = 0; i < I; ++i) y2[i] = fmaf(yr[i], yr[i], yi[i] * yi[i]);
    as_point_em<I, J>(y2, lam, lamI, v, S0, S1, ok);
    if (ok) {
#pragma unroll
      for (int j = 0; j < J; ++j) vf[(size_t)j * s.Npad + n] = v[j];
    }
  }
  float flat[V];
#pragma unroll
  for (int j = 0; j < J; ++j) {
    flat[j] = S0[j];
#pragma unroll
    for (int i = 0; i < I; ++i) flat[J + j * I + i] = S1[j][i];
  }
  block_totals_store<V>(flat, s.partA + ((size_t)f * s.nchunk + chunk) * V, red);
}

// lambda' of eq. 20 for entry t = j I + i of bin f from the tiles' S0, S1.
template <int I, int J>
__device__ __forceinline__ float eq20_from_tiles(const DevState& s, int f, int t, float lam, float invN) {
  constexpr int V = kEq20Sums<I, J>;
  const float* base = s.partA + (size_t)f * s.nchunk * V;
  float s0 = 0.f, s1 = 0.f;
  int c = 0;
  // four tiles' values loaded before any is added (in flight together),
  // then added in tile order
  for (; c + 4 <= s.nchunk; c += 4) {
    float l0[4], l1[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      l0[u] = base[(size_t)(c + u) * V + t / I];
      l1[u] = base[(size_t)(c + u) * V + J + t];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) { s0 += l0[u]; s1 += l1[u]; }
  }
  for (; c < s.nchunk; ++c) {
    s0 += base[(size_t)c * V + t / I];
    s1 += base[(size_t)c * V + J + t];
  }
  return eq20_lambda(lam, s0, s1, invN);
}

// Pass B: lambda (eq. 20) from the tile sums of pass A, then the tile's
// weighted sums of eq. 23 in the basis of y: for every column c,
// sum_n w_c y y^H with w_c = 1 / sum_j v_j lambda_jc, stored packed (slot
// (a, b), a <= b: Re, slot (b, a), a < b: Im) at partB[tile][c][I*I].
//
// Up to I = 4 a lane accumulates all I^3 sums of its own frames.  Above, the
// I^3 sums per frame exceed the registers, so the tile is staged in LDS: each
// lane writes its frame's w (I values) and y y^H (I^2 values) as one record,
// then lane (g, a) of group g accumulates row a of the packed y y^H times
// every w_c over the frames g, g + G, ... of the stage (I^2 sums per lane, I
// lanes per frame), and the groups' sums are added at the end of the tile.
// A record keeps slot (a, b) of y y^H at position b * I + a, so that the I
// lanes of a group read consecutive words, and its stride is odd, so that
// the lanes writing records (one each) and the groups reading them fall on
// different LDS banks.
template <int I>
struct PassBLayout {
  static constexpr bool kLds = I >= 5;
  // lanes = frames per stage: 2 waves, so that more workgroups share a CU
  // and wait at their stage barriers independently
  static constexpr int kThreads = kLds ? 128 : kBlock;
  static constexpr int kStages = kChunk / kThreads;
  static constexpr int kRec = I * I + I;                // y y^H, then w
  static constexpr int kStride = kRec | 1;              // odd record stride (LDS banks)
  static constexpr int kGroups = kThreads / I;          // frames accumulated side by side
  static constexpr int kFloats = kLds ? kThreads * kStride : 1;
  static_assert(!kLds || kGroups * I * I * I <= kThreads * kStride, "group sums reuse the records");
  static_assert(kChunk % kThreads == 0, "stages tile a chunk");
};

// The matrix-core form of pass B's sums above I = 4 (option "sums_mfma" = 1;
// slower than the VALU form above at I = 6 and I = 8).  Each stage's frames
// are staged in LDS as planes (plane q < I^2: entry q of the packed y y^H of
// every frame of the stage; plane I^2 + c: the weight w_c), a frame per
// column, and the stage's sums sum_n w_c(n) z_q(n) -- a contraction over the
// frames, W^T Z with W = [w_c(n)] and Z = [z_q(n)] -- run on the FP32
// 16x16x4 MFMA: rows c (I of the 16 used), 16 columns q per tile, 4 frames
// per instruction, each of the two waves over its half of the stage's
// frames.  A plane stride of 2 mod 32 words keeps both the writes (a frame
// per lane) and the operand reads (lane (k, n): frame k, column n) on
// distinct LDS banks; a last plane of zeros feeds the operand lanes past I
// rows or I^2 columns.
template <int I>
struct PassBMfma {
  static constexpr int kThreads = 128;                 // frames per stage: 2 waves
  static constexpr int kStages = kChunk / kThreads;
  static constexpr int kPlanes = I * I + I;            // then the zero plane
  static constexpr int kPlane = kThreads + 2;
  static constexpr int kNT = (I * I + 15) / 16;        // 16-column tiles of the I^2 sums
  static constexpr int kFloats = (kPlanes + 1) * kPlane;
  static_assert(kNT * 4 * kWave <= kPlanes * kPlane, "wave 1's partial sums reuse the planes");
  static_assert(kChunk % kThreads == 0, "stages tile a chunk");
};

// The same sums on the 16-block 4x4x1 FP32 MFMA (option "sums_mfma" = 2,
// 5 <= I <= 8): block b of an instruction holds columns q = 4b .. 4b + 3
// and rows c = 4h .. 4h + 3 (h = 0 .. ceil(I/4) - 1, an instruction each), one
// frame per instruction, so lane l feeds plane q = l and the weight plane of
// row 4h + l % 4, and every lane's column q is used while I^2 = 64.  Planes
// are 16-byte aligned with a stride of 4 mod 32 words, so a lane's 128-bit
// read of four consecutive frames and the eight lanes served together fall
// on distinct banks.  Four accumulators per row group (one per frame of
// four) keep each summation chain at the 16x16x4 form's length.
template <int I>
struct PassBMfma4 {
  static constexpr int kThreads = 128;                 // frames per stage: 2 waves
  static constexpr int kStages = kChunk / kThreads;
  static constexpr int kPlanes = I * I + I;            // then the zero plane
  static constexpr int kPlane = kThreads + 4;
  static constexpr int kNH = (I + 3) / 4;              // row groups (instructions per frame)
  static constexpr int kFloats = (kPlanes + 1) * kPlane;
  static_assert(I * I <= kWave, "a lane per column q");
  static_assert(kPlane % 32 == 4, "bank spread of the 128-bit operand reads");
  static_assert(kNH * 4 * kWave <= kPlanes * kPlane, "wave 1's partial sums reuse the planes");
  static_assert(kChunk % kThreads == 0, "stages tile a chunk");
};

template <int I, int J, int kMf = 0>
__global__ __launch_bounds__(PassBLayout<I>::kThreads) void k_as_pass_b(DevState s) {
  using L = PassBLayout<I>;
  using M = PassBMfma<I>;
  using M4 = PassBMfma4<I < 5 ? 5 : I>;
  static_assert(kMf == 0 || (L::kLds && L::kThreads == M::kThreads && L::kThreads == M4::kThreads),
                "matrix-core forms: above I = 4");
  const int f = blockIdx.y, chunk = blockIdx.x;
  __shared__ float sLam[J * I];
  __shared__ float4 sPt[I * kPH<I>];
  __shared__ __align__(16) float sRec[kMf == 2 ? M4::kFloats : kMf == 1 ? M::kFloats
                                    : L::kLds ? L::kFloats : (kBlock / kWave) * pad4(I * I * I)];
  const float invN = 1.0f / float(s.N);
  for (int t = threadIdx.x; t < J * I; t += L::kThreads)
    sLam[t] = eq20_from_tiles<I, J>(s, f, t, s.lam[(size_t)f * J * I + t], invN);  // eq. 20
  stage_P_columns<I>(s.P + (size_t)f * I * I, sPt);  // the old P (k_as_solve replaces it after this pass)
  __syncthreads();
  const float* xf = s.xs + (size_t)f * 2 * I * s.Npad;
  const float* vf = s.vs + (size_t)f * J * s.Npad;
  float* out = s.partB + ((size_t)f * s.nchunk + chunk) * I * I * I;

  // frame n of this lane: y, the weights w (0 past N) and y y^H (packed)
  auto frame = [&](int p, const float (&lam)[J][I], float (&w)[I], float (&z)[I * I]) {
    const int n = chunk * kChunk + p * kBlock + threadIdx.x;
    const bool ok = n < s.N;
    const int nn = ok ? n : 0;
    float xr[I], xi[I], v[J], yr[I], yi[I];
#pragma unroll
    for (int i = 0; i < I; ++i) { xr[i] = xf[(size_t)i * s.Npad + nn]; xi[i] = xf[(size_t)(I + i) * s.Npad + nn]; }
#pragma unroll
    for (int j = 0; j < J; ++j) v[j] = vf[(size_t)j * s.Npad + nn];
    int zo = 0;  // opaque offset: P is read from LDS per frame, not hoisted into registers
    asm volatile("" : "+s"(zo));
    as_transform_lds<I>(sPt + zo, xr, xi, yr, yi);
    as_point_weights<I, J>(lam, v, w);
#pragma unroll
    for (int i = 0; i < I; ++i) w[i] = ok ? w[i] : 0.f;
    herm_outer<I>(z, yr, yi);
  };

  if constexpr (!L::kLds) {
    float lam[J][I];
#pragma unroll
    for (int j = 0; j < J; ++j)
#pragma unroll
      for (int i = 0; i < I; ++i) lam[j][i] = sLam[j * I + i];
    float A[I][I * I];
#pragma unroll
    for (int c = 0; c < I; ++c)
#pragma unroll
      for (int q = 0; q < I * I; ++q) A[c][q] = 0.f;
#pragma unroll
    for (int p = 0; p < kPts; ++p) {
      float w[I], z[I * I];
      frame(p, lam, w, z);
#pragma unroll
      for (int c = 0; c < I; ++c)
#pragma unroll
        for (int q = 0; q < I * I; ++q) A[c][q] = fmaf(w[c], z[q], A[c][q]);
    }
    float flat[I * I * I];
#pragma unroll
    for (int c = 0; c < I; ++c)
#pragma unroll
      for (int q = 0; q < I * I; ++q) flat[c * I * I + q] = A[c][q];
    block_totals_store<I * I * I>(flat, out, sRec);
  } else if constexpr (kMf == 2) {
    typedef float v4f __attribute__((ext_vector_type(4)));
    constexpr int P = M4::kPlane, NH = M4::kNH;
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    for (int t = threadIdx.x; t < P; t += M4::kThreads) sRec[M4::kPlanes * P + t] = 0.f;  // the zero plane
    v4f acc[NH][4];
#pragma unroll
    for (int h = 0; h < NH; ++h)
#pragma unroll
      for (int u = 0; u < 4; ++u) acc[h][u] = v4f{0.f, 0.f, 0.f, 0.f};
    float xr[I], xi[I], v[J], xrn[I], xin[I], vnx[J];
    auto load = [&](int p) {
      const int n = chunk * kChunk + p * M4::kThreads + threadIdx.x;
      const int nn = n < s.N ? n : 0;  // frames past N read frame 0 (weight 0)
#pragma unroll
      for (int i = 0; i < I; ++i) {
        xrn[i] = xf[(size_t)i * s.Npad + nn];
        xin[i] = xf[(size_t)(I + i) * s.Npad + nn];
      }
#pragma unroll
      for (int j = 0; j < J; ++j) vnx[j] = vf[(size_t)j * s.Npad + nn];
    };
    load(0);
    // operand planes: B (lane l: column q = l) and A of row group h (lane l:
    // row 4h + l % 4); lanes past I^2 columns or I rows read the zero plane
    const int pb = (lane < I * I ? lane : M4::kPlanes) * P;
    int pa[NH];
#pragma unroll
    for (int h = 0; h < NH; ++h) pa[h] = (4 * h + (lane & 3) < I ? I * I + 4 * h + (lane & 3) : M4::kPlanes) * P;
#pragma unroll 1
    for (int p = 0; p < M4::kStages; ++p) {
#pragma unroll
      for (int i = 0; i < I; ++i) { xr[i] = xrn[i]; xi[i] = xin[i]; }
#pragma unroll
      for (int j = 0; j < J; ++j) v[j] = vnx[j];
      if (p + 1 < M4::kStages) load(p + 1);
      {
        // this lane's frame: column threadIdx.x of every plane
        const bool ok = chunk * kChunk + p * M4::kThreads + (int)threadIdx.x < s.N;
        int zo = 0;
        asm volatile("" : "+s"(zo));
        float yr[I], yi[I];
        as_transform_lds<I>(sPt + zo, xr, xi, yr, yi);
        float* col = sRec + threadIdx.x;
#pragma unroll
        for (int a2 = 0; a2 < I; ++a2) {
          col[(a2 * I + a2) * P] = fmaf(yr[a2], yr[a2], yi[a2] * yi[a2]);
#pragma unroll
          for (int b = a2 + 1; b < I; ++b) {  // packed: Re at (a, b), Im at (b, a)
            col[(a2 * I + b) * P] = fmaf(yr[a2], yr[b], yi[a2] * yi[b]);
            col[(b * I + a2) * P] = fmaf(yi[a2], yr[b], -yr[a2] * yi[b]);
          }
        }
        const float* lamz = sLam + zo;
#pragma unroll
        for (int c = 0; c < I; ++c) {
          float d = v[0] * lamz[c];
#pragma unroll
          for (int j = 1; j < J; ++j) d = fmaf(v[j], lamz[j * I + c], d);
          col[(I * I + c) * P] = ok ? rcp(d) : 0.f;
        }
      }
      __syncthreads();
      {
        const float* fr = sRec + wv * kWave;  // this wave's 64 frames of the stage
#pragma unroll 4
        for (int st = 0; st < kWave / 4; ++st) {
          const float4 b4 = *reinterpret_cast<const float4*>(fr + pb + 4 * st);
          float4 a4[NH];
#pragma unroll
          for (int h = 0; h < NH; ++h) a4[h] = *reinterpret_cast<const float4*>(fr + pa[h] + 4 * st);
#pragma unroll
          for (int h = 0; h < NH; ++h) {
            acc[h][0] = __builtin_amdgcn_mfma_f32_4x4x1f32(a4[h].x, b4.x, acc[h][0], 0, 0, 0);
            acc[h][1] = __builtin_amdgcn_mfma_f32_4x4x1f32(a4[h].y, b4.y, acc[h][1], 0, 0, 0);
            acc[h][2] = __builtin_amdgcn_mfma_f32_4x4x1f32(a4[h].z, b4.z, acc[h][2], 0, 0, 0);
            acc[h][3] = __builtin_amdgcn_mfma_f32_4x4x1f32(a4[h].w, b4.w, acc[h][3], 0, 0, 0);
          }
        }
      }
      __syncthreads();  // the planes are rewritten by the next stage
    }
    // lane l holds, in register r of row group h, the sum for (c, q) =
    // (4h + r, l); wave 1 stores its sums, wave 0 adds them and writes
    v4f tot[NH];
#pragma unroll
    for (int h = 0; h < NH; ++h) tot[h] = (acc[h][0] + acc[h][1]) + (acc[h][2] + acc[h][3]);
    if (wv == 1) {
#pragma unroll
      for (int h = 0; h < NH; ++h)
#pragma unroll
        for (int r = 0; r < 4; ++r) sRec[(h * 4 + r) * kWave + lane] = tot[h][r];
    }
    __syncthreads();
    if (wv == 0 && lane < I * I) {
#pragma unroll
      for (int h = 0; h < NH; ++h)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int c = 4 * h + r;
          if (c < I) out[c * I * I + lane] = tot[h][r] + sRec[(h * 4 + r) * kWave + lane];
        }
    }
  } else if constexpr (kMf == 1) {
    typedef float v4f __attribute__((ext_vector_type(4)));
    constexpr int P = M::kPlane, NT = M::kNT;
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    const int kq = lane >> 4, n16 = lane & 15;  // operand row k (frame of 4) and column n of a tile
    for (int t = threadIdx.x; t < P; t += M::kThreads) sRec[M::kPlanes * P + t] = 0.f;  // the zero plane
    v4f acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = v4f{0.f, 0.f, 0.f, 0.f};
    float xr[I], xi[I], v[J], xrn[I], xin[I], vnx[J];
    auto load = [&](int p) {
      const int n = chunk * kChunk + p * M::kThreads + threadIdx.x;
      const int nn = n < s.N ? n : 0;  // frames past N read frame 0 (weight 0)
#pragma unroll
      for (int i = 0; i < I; ++i) {
        xrn[i] = xf[(size_t)i * s.Npad + nn];
        xin[i] = xf[(size_t)(I + i) * s.Npad + nn];
      }
#pragma unroll
      for (int j = 0; j < J; ++j) vnx[j] = vf[(size_t)j * s.Npad + nn];
    };
    load(0);
    // operand offsets: A (lane: row n16 = c, frame kq) reads plane I^2 + c,
    // B (lane: frame kq, column n16 of tile t) plane 16 t + n16; lanes past
    // I (or I^2) read the zero plane
    const int pa = ((n16 < I) ? I * I + n16 : M::kPlanes) * P;
    int pb[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) pb[t] = ((16 * t + n16 < I * I) ? 16 * t + n16 : M::kPlanes) * P;
#pragma unroll 1
    for (int p = 0; p < M::kStages; ++p) {
#pragma unroll
      for (int i = 0; i < I; ++i) { xr[i] = xrn[i]; xi[i] = xin[i]; }
#pragma unroll
      for (int j = 0; j < J; ++j) v[j] = vnx[j];
      if (p + 1 < M::kStages) load(p + 1);
      {
        // this lane's frame: column threadIdx.x of every plane
        const bool ok = chunk * kChunk + p * M::kThreads + (int)threadIdx.x < s.N;
        int zo = 0;
        asm volatile("" : "+s"(zo));
        float yr[I], yi[I];
        as_transform_lds<I>(sPt + zo, xr, xi, yr, yi);
        float* col = sRec + threadIdx.x;
#pragma unroll
        for (int a2 = 0; a2 < I; ++a2) {
          col[(a2 * I + a2) * P] = fmaf(yr[a2], yr[a2], yi[a2] * yi[a2]);
#pragma unroll
          for (int b = a2 + 1; b < I; ++b) {  // packed: Re at (a, b), Im at (b, a)
            col[(a2 * I + b) * P] = fmaf(yr[a2], yr[b], yi[a2] * yi[b]);
            col[(b * I + a2) * P] = fmaf(yi[a2], yr[b], -yr[a2] * yi[b]);
          }
        }
        const float* lamz = sLam + zo;
#pragma unroll
        for (int c = 0; c < I; ++c) {
          float d = v[0] * lamz[c];
#pragma unroll
          for (int j = 1; j < J; ++j) d = fmaf(v[j], lamz[j * I + c], d);
          col[(I * I + c) * P] = ok ? rcp(d) : 0.f;
        }
      }
      __syncthreads();
      {
        const float* fr = sRec + wv * kWave + kq;  // frame 64 wv + 4 st + kq: column fr + 4 st
#pragma unroll 4
        for (int st = 0; st < kWave / 4; ++st) {
          const float a = fr[pa + 4 * st];
#pragma unroll
          for (int t = 0; t < NT; ++t)
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, fr[pb[t] + 4 * st], acc[t], 0, 0, 0);
        }
      }
      __syncthreads();  // the planes are rewritten by the next stage
    }
    // the two waves' sums: wave 1 stores its tiles, wave 0 adds them and
    // writes entry (c, q) = (4 kq + r, 16 t + n16) of the tile's sums
    if (wv == 1) {
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) sRec[(t * 4 + r) * kWave + lane] = acc[t][r];
    }
    __syncthreads();
    if (wv == 0) {
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int c = 4 * kq + r, q = 16 * t + n16;
          if (c < I && q < I * I) out[c * I * I + q] = acc[t][r] + sRec[(t * 4 + r) * kWave + lane];
        }
    }
  } else {
    const int a = threadIdx.x % I, g = threadIdx.x / I;  // row a of group g (g >= kGroups: idle)
    float acc[I][I];                                     // [c][b]: row a, column b of S_c (packed)
#pragma unroll
    for (int c = 0; c < I; ++c)
#pragma unroll
      for (int b = 0; b < I; ++b) acc[c][b] = 0.f;
    // the frame of the next stage is loaded while this one is summed
    float xr[I], xi[I], v[J], xrn[I], xin[I], vnx[J];
    auto load = [&](int p) {
      const int n = chunk * kChunk + p * L::kThreads + threadIdx.x;
      const int nn = n < s.N ? n : 0;  // frames past N read frame 0 (weight 0)
#pragma unroll
      for (int i = 0; i < I; ++i) {
        xrn[i] = xf[(size_t)i * s.Npad + nn];
        xin[i] = xf[(size_t)(I + i) * s.Npad + nn];
      }
#pragma unroll
      for (int j = 0; j < J; ++j) vnx[j] = vf[(size_t)j * s.Npad + nn];
    };
    load(0);
#pragma unroll 1
    for (int p = 0; p < L::kStages; ++p) {
#pragma unroll
      for (int i = 0; i < I; ++i) { xr[i] = xrn[i]; xi[i] = xin[i]; }
#pragma unroll
      for (int j = 0; j < J; ++j) v[j] = vnx[j];
      if (p + 1 < L::kStages) load(p + 1);
      {
        // this lane's record: y y^H and w, each value stored as it is formed;
        // lambda is read from LDS (in registers it would sit beside the sums)
        const bool ok = chunk * kChunk + p * L::kThreads + (int)threadIdx.x < s.N;
        int zo = 0;
        asm volatile("" : "+s"(zo));
        float yr[I], yi[I];
        as_transform_lds<I>(sPt + zo, xr, xi, yr, yi);
        float* rec = sRec + threadIdx.x * L::kStride;
#pragma unroll
        for (int a2 = 0; a2 < I; ++a2) {
          rec[a2 * I + a2] = fmaf(yr[a2], yr[a2], yi[a2] * yi[a2]);
#pragma unroll
          for (int b = a2 + 1; b < I; ++b) {  // slot (a, b) at b * I + a (see below)
            rec[b * I + a2] = fmaf(yr[a2], yr[b], yi[a2] * yi[b]);
            rec[a2 * I + b] = fmaf(yi[a2], yr[b], -yr[a2] * yi[b]);
          }
        }
        const float* lamz = sLam + zo;
#pragma unroll
        for (int c = 0; c < I; ++c) {
          float d = v[0] * lamz[c];
#pragma unroll
          for (int j = 1; j < J; ++j) d = fmaf(v[j], lamz[j * I + c], d);
          rec[I * I + c] = ok ? rcp(d) : 0.f;
        }
      }
      __syncthreads();
      if (g < L::kGroups) {
#pragma unroll 2
        for (int m = g; m < L::kThreads; m += L::kGroups) {
          const float* rec = sRec + m * L::kStride;
          float w[I], z[I];
#pragma unroll
          for (int c = 0; c < I; ++c) w[c] = rec[I * I + c];
#pragma unroll
          for (int b = 0; b < I; ++b) z[b] = rec[b * I + a];
#pragma unroll
          for (int c = 0; c < I; ++c)
#pragma unroll
            for (int b = 0; b < I; ++b) acc[c][b] = fmaf(w[c], z[b], acc[c][b]);
        }
      }
      __syncthreads();  // the records are rewritten by the next stage
    }
    // the groups' sums, added in group order
    if (g < L::kGroups) {
#pragma unroll
      for (int c = 0; c < I; ++c)
#pragma unroll
        for (int b = 0; b < I; ++b) sRec[g * I * I * I + c * I * I + a * I + b] = acc[c][b];
    }
    __syncthreads();
    for (int o = threadIdx.x; o < I * I * I; o += L::kThreads) {
      float t = sRec[o];
      for (int gg = 1; gg < L::kGroups; ++gg) t += sRec[gg * I * I * I + o];
      out[o] = t;
    }
  }
}

// One lane per (bin, column); 8 bins per 64-lane workgroup.  Eq. 23 in the
// basis of y = P^H x (as in the resident kernel): column i of
// A = P_old^-1 P_new solves S_i a = N e_i with S_i = N G_i the tile sums of
// pass B, K > 1 iterates a_i = N S_i^-1 [A^-H]_i from A = 1, and
// P_new = P_old A.
template <int I, int J>
__global__ __launch_bounds__(64) void k_as_solve(DevState s) {
  const int fl = threadIdx.x / 8, i = threadIdx.x % 8;
  const int f = blockIdx.x * 8 + fl;
  const bool act = (f < s.F) && (i < I);
  __shared__ float sAr[8][I][I], sAi[8][I][I];
  const float invN = 1.0f / float(s.N), fN = float(s.N);
  float Sr[I][I], Si[I][I], Pr[I][I], Pi[I][I];
  if (act) {
    // the old P (every lane of a bin reads it before any lane writes)
#pragma unroll
    for (int a = 0; a < I; ++a)
#pragma unroll
      for (int b = 0; b < I; ++b) {
        const float2 t = s.P[(size_t)f * I * I + a * I + b];
        Pr[a][b] = t.x; Pi[a][b] = t.y;
      }
    // S_i from the tile partials (EM with P in the M-step uses other sums),
    // requested before the lambda stores below; four tiles' values loaded
    // before any is added, then added in tile order
    float A[I * I];
#pragma unroll
    for (int k = 0; k < I * I; ++k) A[k] = 0.f;
    {
      const int nc = s.p_update == 4 ? 0 : s.nchunk;
      const float* base = s.partB + (size_t)f * s.nchunk * I * I * I + i * I * I;
      int c = 0;
      for (; c + 4 <= nc; c += 4) {
        float l4[4][I * I];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int k = 0; k < I * I; ++k) l4[u][k] = base[(size_t)(c + u) * I * I * I + k];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int k = 0; k < I * I; ++k) A[k] += l4[u][k];
      }
      for (; c < nc; ++c) {
#pragma unroll
        for (int k = 0; k < I * I; ++k) A[k] += base[(size_t)c * I * I * I + k];
      }
    }
    // lambda update (eq. 20): column i of every Lambda_j.
#pragma unroll
    for (int j = 0; j < J; ++j) {
      float* l = s.lam + (size_t)f * J * I + j * I + i;
      *l = eq20_from_tiles<I, J>(s, f, j * I + i, *l, invN);  // eq. 20
    }
    if (s.p_update == 3) {  // Newton's step: the totals go to the first tile's slot for k_as_newton
      float* dst = s.partB + (size_t)f * s.nchunk * I * I * I + i * I * I;
#pragma unroll
      for (int k = 0; k < I * I; ++k) dst[k] = A[k];
    }
#pragma unroll
    for (int a = 0; a < I; ++a) {
      Sr[a][a] = A[a * I + a]; Si[a][a] = 0.f;
#pragma unroll
      for (int b = a + 1; b < I; ++b) {
        Sr[a][b] = A[a * I + b]; Si[a][b] = A[b * I + a];
        Sr[b][a] = Sr[a][b]; Si[b][a] = -Si[a][b];
      }
    }
  }
  if (s.p_update >= 3) return;  // Newton / EM with P in the M-step: k_as_newton / k_as_emp_step
  // gamma_i = S_i e_i / N (column i of G_i) for the gradient-type P steps
  float gr[I], gi[I];
#pragma unroll
  for (int a = 0; a < I; ++a) { gr[a] = 0.f; gi[a] = 0.f; }
  if (act && s.p_update != 0) {
#pragma unroll
    for (int a = 0; a < I; ++a)
#pragma unroll
      for (int b = 0; b < I; ++b) {
        gr[a] = (b == i) ? Sr[a][b] / fN : gr[a];
        gi[a] = (b == i) ? Si[a][b] / fN : gi[a];
      }
  }
  const int steps = s.p_update == 0 ? s.K : 1;
  for (int kk = 0; kk < steps; ++kk) {
    float ar[I], ai[I];
    if (act) {
      if (s.p_update == 2) {  // natural gradient: A = 1 + mu (1 - Gamma)
#pragma unroll
        for (int a = 0; a < I; ++a) {
          ar[a] = ((a == i) ? 1.f + s.p_step : 0.f) - s.p_step * gr[a];
          ai[a] = -s.p_step * gi[a];
        }
      } else if (kk == 0) {
#pragma unroll
        for (int a = 0; a < I; ++a) { ar[a] = (a == i) ? fN : 0.f; ai[a] = 0.f; }
        if (!herm_solve<I>(Sr, Si, ar, ai)) atomicOr(s.flag, kFlagSingular);
      } else {
        float Ar[I][I], Ai[I][I];
#pragma unroll
        for (int a = 0; a < I; ++a)
#pragma unroll
          for (int b = 0; b < I; ++b) { Ar[a][b] = sAr[fl][a][b]; Ai[a][b] = sAi[fl][a][b]; }
        pinvh_col<I, float>(Ar, Ai, i, ar, ai);   // column i of A^-H
#pragma unroll
        for (int a = 0; a < I; ++a) { ar[a] *= fN; ai[a] *= fN; }
        if (!herm_solve<I>(Sr, Si, ar, ai)) atomicOr(s.flag, kFlagSingular);
      }
    }
    __syncthreads();
    if (act) {
#pragma unroll
      for (int a = 0; a < I; ++a) { sAr[fl][a][i] = ar[a]; sAi[fl][a][i] = ai[a]; }
    }
    __syncthreads();
  }
  if (s.p_update == 1) {
    // gradient: p_i + mu P^-H (e_i - gamma_i); the columns of P^-H go
    // through the same LDS tile
    float br[I], bi[I];
    if (act) pinvh_col<I, float>(Pr, Pi, i, br, bi);
    __syncthreads();
    if (act) {
#pragma unroll
      for (int a = 0; a < I; ++a) { sAr[fl][a][i] = br[a]; sAi[fl][a][i] = bi[a]; }
    }
    __syncthreads();
    if (act) {
#pragma unroll
      for (int a = 0; a < I; ++a) {
        float pr = 0.f, pi = 0.f;
#pragma unroll
        for (int b = 0; b < I; ++b) { pr = (b == i) ? Pr[a][b] : pr; pi = (b == i) ? Pi[a][b] : pi; }
#pragma unroll
        for (int b = 0; b < I; ++b) {
          const float dr = ((b == i) ? 1.f : 0.f) - gr[b], di = -gi[b];
          pr = fmaf(s.p_step, sAr[fl][a][b] * dr - sAi[fl][a][b] * di, pr);
          pi = fmaf(s.p_step, sAr[fl][a][b] * di + sAi[fl][a][b] * dr, pi);
        }
        s.P[(size_t)f * I * I + a * I + i] = make_float2(pr, pi);
      }
    }
  } else if (act) {
    // column i of P_new = P_old A
#pragma unroll
    for (int a = 0; a < I; ++a) {
      float pr = 0.f, pi = 0.f;
#pragma unroll
      for (int b = 0; b < I; ++b) {
        pr = fmaf(Pr[a][b], sAr[fl][b][i], pr);
        pr = fmaf(-Pi[a][b], sAi[fl][b][i], pr);
        pi = fmaf(Pr[a][b], sAi[fl][b][i], pi);
        pi = fmaf(Pi[a][b], sAr[fl][b][i], pi);
      }
      s.P[(size_t)f * I * I + a * I + i] = make_float2(pr, pi);
    }
  }
}

// The plain step at I >= 5: one wave per bin, lane (i, r) holding row r of
// S_i.  The I lanes of a column's group factorise S_i = L L^H together
// (right-looking Cholesky: the pivot and column k of L reach the group's
// other lanes by lane shuffles), then solve L L^H a_i = N e_i by columns, so
// that the dependent chain of one factorisation is spread over I lanes
// instead of lying on one (k_as_solve).  Lane (i, r) then forms entry (r, i)
// of P_new = P_old A.
template <int I, int J>
__global__ __launch_bounds__(kWave) void k_as_solve_rows(DevState s) {
  static_assert(I * I <= kWave, "a bin's rows fit one wave");
  const int f = blockIdx.x, lane = threadIdx.x;
  const bool act = lane < I * I;
  const int i = act ? lane / I : 0, r = act ? lane % I : 0;
  const int base = i * I;  // the group's first lane
  const float invN = 1.0f / float(s.N), fN = float(s.N);
  __shared__ float sLr[I][I][I], sLi[I][I][I];  // [i][row][col] of L_i
  // P_old row r, requested before the sums
  float Por[I], Poi[I];
#pragma unroll
  for (int b = 0; b < I; ++b) {
    const float2 p = s.P[(size_t)f * I * I + r * I + b];
    Por[b] = p.x; Poi[b] = p.y;
  }
  // row r of S_i from the tiles' packed sums (slot (a, b), a <= b: Re,
  // (b, a), a < b: Im), each slot summed over the tiles in tile order.
  // Requested before the eq. 20 update below, whose store to lambda the
  // compiler would otherwise keep ahead of these loads (one more memory
  // round trip on the solve's path).
  float Sr[I], Si[I];
#pragma unroll
  for (int c = 0; c < I; ++c) { Sr[c] = 0.f; Si[c] = 0.f; }
  {
    float ra[I], rb[I];
#pragma unroll
    for (int c = 0; c < I; ++c) { ra[c] = 0.f; rb[c] = 0.f; }
    const float* base = s.partB + (size_t)f * s.nchunk * I * I * I + i * I * I;
    int ch = 0;
    // four tiles' rows loaded before any is added (in flight together), then
    // added in tile order
    for (; ch + 4 <= s.nchunk; ch += 4) {
      float la[4][I], lb[4][I];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const float* src = base + (size_t)(ch + u) * I * I * I;
#pragma unroll
        for (int c = 0; c < I; ++c) { la[u][c] = src[r * I + c]; lb[u][c] = src[c * I + r]; }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int c = 0; c < I; ++c) { ra[c] += la[u][c]; rb[c] += lb[u][c]; }
    }
    for (; ch < s.nchunk; ++ch) {
      const float* src = base + (size_t)ch * I * I * I;
#pragma unroll
      for (int c = 0; c < I; ++c) { ra[c] += src[r * I + c]; rb[c] += src[c * I + r]; }
    }
#pragma unroll
    for (int c = 0; c < I; ++c) {
      Sr[c] = (c >= r) ? ra[c] : rb[c];
      Si[c] = (c > r) ? rb[c] : ((c < r) ? -ra[c] : 0.f);
    }
  }
  // eq. 20
  for (int t = lane; t < J * I; t += kWave) {
    float* l = s.lam + (size_t)f * J * I + t;
    *l = eq20_from_tiles<I, J>(s, f, t, *l, invN);
  }
  // Cholesky: row r of the working matrix becomes row r of L
  bool pd = true;
  float dself = 1.f;  // 1 / L_rr
#pragma unroll
  for (int k = 0; k < I; ++k) {
    const float skk = __shfl(Sr[k], base + k, kWave);
    pd = pd && !(skk <= 0.f);
    const float dk = sqrtT(skk > 1e-37f ? skk : 1e-37f);
    const float ik = rcpT(dk);
    if (r > k) { Sr[k] *= ik; Si[k] *= ik; }
    if (r == k) { Sr[k] = dk; Si[k] = 0.f; dself = ik; }
#pragma unroll
    for (int c = k + 1; c < I; ++c) {
      const float lr = __shfl(Sr[k], base + c, kWave), li = __shfl(Si[k], base + c, kWave);  // L_ck
      if (r > k && c <= r) {  // S_rc -= L_rk conj(L_ck)
        Sr[c] -= Sr[k] * lr + Si[k] * li;
        Si[c] -= Si[k] * lr - Sr[k] * li;
      }
    }
  }
  if (act && r == 0 && !pd) atomicOr(s.flag, kFlagSingular);
  if (act) {
#pragma unroll
    for (int c = 0; c < I; ++c) { sLr[i][r][c] = Sr[c]; sLi[i][r][c] = Si[c]; }
  }
  // L z = N e_i, by columns: lane r accumulates N delta_ri - sum_k L_rk z_k
  float zr = (r == i) ? fN : 0.f, zi = 0.f;
#pragma unroll
  for (int k = 0; k < I; ++k) {
    if (r == k) { zr *= dself; zi *= dself; }
    const float tr = __shfl(zr, base + k, kWave), ti = __shfl(zi, base + k, kWave);
    if (r > k) {
      zr -= Sr[k] * tr - Si[k] * ti;
      zi -= Sr[k] * ti + Si[k] * tr;
    }
  }
  __builtin_amdgcn_wave_barrier();  // rows of L in LDS (one wave: in order)
  // L^H a = z, by columns from the last: lane r subtracts conj(L_kr) a_k
  float ar = zr, ai = zi;
#pragma unroll
  for (int k = I - 1; k >= 0; --k) {
    if (r == k) { ar *= dself; ai *= dself; }
    const float tr = __shfl(ar, base + k, kWave), ti = __shfl(ai, base + k, kWave);
    if (r < k) {
      const float lr = sLr[i][k][r], li = sLi[i][k][r];
      ar -= lr * tr + li * ti;
      ai -= lr * ti - li * tr;
    }
  }
  // entry (r, i) of P_new = P_old A: a_i gathered from the group
  float pr = 0.f, pi = 0.f;
#pragma unroll
  for (int b = 0; b < I; ++b) {
    const float br = __shfl(ar, base + b, kWave), bi = __shfl(ai, base + b, kWave);
    pr = fmaf(Por[b], br, pr);
    pr = fmaf(-Poi[b], bi, pr);
    pi = fmaf(Por[b], bi, pi);
    pi = fmaf(Poi[b], br, pi);
  }
  if (act) s.P[(size_t)f * I * I + r * I + i] = make_float2(pr, pi);
}

template <int I, int J>
hipError_t launch_as_iter_stream(const DevState& s, hipStream_t st) {
  dim3 grid(s.nchunk, s.F);
  // EM with P in the M-step: its sums need the v before pass A overwrites it
  if (s.p_update == 4) hipLaunchKernelGGL((k_as_pass_emp<I, J>), dim3(s.nchunk, s.F, J), dim3(kBlock), 0, st, s);
  hipLaunchKernelGGL((k_as_pass_a<I, J>), grid, dim3(kBlock), 0, st, s);
  if (s.p_update != 4) {
    if constexpr (I >= 5) {
      // default (-1): the 4x4x1 matrix-core form where it measured faster (I = 8)
      const int form = s.sums_mfma < 0 ? (I == 8 ? 2 : 0) : s.sums_mfma;
      if (form == 2 && I <= 8)
        hipLaunchKernelGGL((k_as_pass_b<I, J, (I <= 8 ? 2 : 1)>), grid, dim3(PassBLayout<I>::kThreads), 0, st, s);
      else if (form == 1)
        hipLaunchKernelGGL((k_as_pass_b<I, J, 1>), grid, dim3(PassBLayout<I>::kThreads), 0, st, s);
      else
        hipLaunchKernelGGL((k_as_pass_b<I, J>), grid, dim3(PassBLayout<I>::kThreads), 0, st, s);
    } else {
      hipLaunchKernelGGL((k_as_pass_b<I, J>), grid, dim3(PassBLayout<I>::kThreads), 0, st, s);
    }
  }
  if constexpr (I >= 5) {
    if (s.p_update == 0 && s.K == 1)
      hipLaunchKernelGGL((k_as_solve_rows<I, J>), dim3(s.F), dim3(kWave), 0, st, s);
    else
      hipLaunchKernelGGL((k_as_solve<I, J>), dim3((s.F + 7) / 8), dim3(64), 0, st, s);
  } else {
    hipLaunchKernelGGL((k_as_solve<I, J>), dim3((s.F + 7) / 8), dim3(64), 0, st, s);
  }
  if (s.p_update == 3) hipLaunchKernelGGL((k_as_newton<I, J>), dim3(s.F), dim3(kNewtonThreads), 0, st, s);
  if (s.p_update == 4) hipLaunchKernelGGL((k_as_emp_step<I, J>), dim3((s.F + 63) / 64), dim3(64), 0, st, s);
  return hipGetLastError();
}

// ----------------------------------------------------------------------------
// Log-likelihood (eq. 14 for AS, eq. 5 for EM).
// ----------------------------------------------------------------------------
__device__ inline void block_sum_store_d(double a, double* out, double* lds) {
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const double t = wave_sum_d(a);
  if (lane == 0) lds[wave] = t;
  __syncthreads();
  if (threadIdx.x == 0) {
    double u = 0.0;
    for (int w = 0; w < (int)(blockDim.x / kWave); ++w) u += lds[w];
    *out = u;
  }
}

// Up to I = 4 the bin's ln|det P| (one LU by one lane) is cheap enough to
// sit in its first tile's workgroup; above, a lane-per-bin kernel forms it.
template <int I>
constexpr bool kLoglikDetInTile = (I <= kLoglikDetInTileMaxI);

// Per point: -sum_i ln d_i - sum_i |(P^H x)_i|^2 / d_i   (the n-dependent part of L2).
template <int I, int J>
__global__ __launch_bounds__(kBlock) void k_as_loglik(DevState s) {
  const int f = blockIdx.y, chunk = blockIdx.x;
  __shared__ float2 sP[I * I];
  __shared__ float sLam[J * I];
  __shared__ double red[kBlock / kWave];
  for (int t = threadIdx.x; t < I * I; t += kBlock) sP[t] = s.P[(size_t)f * I * I + t];
  for (int t = threadIdx.x; t < J * I; t += kBlock) sLam[t] = s.lam[(size_t)f * J * I + t];
  __syncthreads();
  float Pr[I][I], Pi[I][I], lam[J][I];
  load_P<I>(sP, Pr, Pi);
#pragma unroll
  for (int j = 0; j < J; ++j)
#pragma unroll
    for (int i = 0; i < I; ++i) lam[j][i] = sLam[j * I + i];
  const float* xf = s.xs + (size_t)f * 2 * I * s.Npad;
  const float* vf = s.vs + (size_t)f * J * s.Npad;
  double acc = 0.0;
#pragma unroll
  for (int p = 0; p < kPts; ++p) {
    const int n = chunk * kChunk + p * kBlock + threadIdx.x;
    if (n < s.N) {
      float xr[I], xi[I], v[J], y2[I];
#pragma unroll
      for (int i = 0; i < I; ++i) { xr[i] = xf[(size_t)i * s.Npad + n]; xi[i] = xf[(size_t)(I + i) * s.Npad + n]; }
#pragma unroll
      for (int j = 0; j < J; ++j) v[j] = vf[(size_t)j * s.Npad + n];
      as_transform_pow<I>(Pr, Pi, xr, xi, y2);
      float t = 0.f;
#pragma unroll
      for (int i = 0; i < I; ++i) {
        float d = 0.f;
#pragma unroll
        for (int j = 0; j < J; ++j) d = fmaf(v[j], lam[j][i], d);
        t -= __logf(d) + y2[i] / d;
      }
      acc += (double)t;
    }
  }
  if constexpr (kLoglikDetInTile<I>) {
    if (chunk == 0 && threadIdx.x == 0) {  // the bin's N (2 ln|det P| - I ln pi), once
      float Mr[I][I], Mi[I][I];
#pragma unroll
      for (int a = 0; a < I; ++a)
#pragma unroll
        for (int b = 0; b < I; ++b) { Mr[a][b] = sP[a * I + b].x; Mi[a][b] = sP[a * I + b].y; }
      const double lad = (double)lu_logabsdet<I>(Mr, Mi);
      acc += (double)s.N * (2.0 * lad - (double)I * 1.1447298858494002);
    }
  }
  block_sum_store_d(acc, s.partL + (size_t)f * s.nchunk + chunk, red);
}

// Above I = 4: per bin, one lane per bin, the sum of the tiles + N (2 ln|det P| - I ln pi).
template <int I>
__global__ __launch_bounds__(64) void k_as_loglik_bin(DevState s) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= s.F) return;
  float Mr[I][I], Mi[I][I];
#pragma unroll
  for (int a = 0; a < I; ++a)
#pragma unroll
    for (int b = 0; b < I; ++b) {
      const float2 t = s.P[(size_t)f * I * I + a * I + b];
      Mr[a][b] = t.x; Mi[a][b] = t.y;
    }
  const double lad = (double)lu_logabsdet<I>(Mr, Mi);
  double acc = 0.0;
  for (int c = 0; c < s.nchunk; ++c) acc += s.partL[(size_t)f * s.nchunk + c];
  s.llf[f] = acc + (double)s.N * (2.0 * lad - (double)I * 1.1447298858494002);
}

// L2 into s.ll: the tiles' partials, then one workgroup sums them (or, above
// I = 4, the per-bin totals) in a fixed order.
template <int I, int J>
hipError_t launch_as_loglik(const DevState& s, hipStream_t st) {
  hipLaunchKernelGGL((k_as_loglik<I, J>), dim3(s.nchunk, s.F), dim3(kBlock), 0, st, s);
  if constexpr (kLoglikDetInTile<I>) {
    return launch_sum_f(s.partL, s.F * s.nchunk, s.ll, st);
  } else {
    hipLaunchKernelGGL((k_as_loglik_bin<I>), dim3((s.F + 63) / 64), dim3(64), 0, st, s);
    return launch_sum_f(s.llf, s.F, s.ll, st);
  }
}

// ----------------------------------------------------------------------------
// Wiener filter (eq. 3; AS form x_j = P^-H (g_j o y) from eq. 15-16).
// ----------------------------------------------------------------------------
// Output-bound: 8IJ bytes written per point.  A wave's 64 consecutive frames
// of one source are 64 I contiguous complex values in [J][F][N][I]; each
// lane's I values go to a wave-private LDS tile and come back as
// consecutive 16-byte chunks (8-byte ones for odd I or an output not
// 16-byte aligned), so every store instruction writes whole cache lines.
// Up to I = 6 P and B = P^-H sit in registers; above, they are read from LDS
// at each use (their 2 x 128 values in registers left one wave per SIMD).
template <int I>
constexpr bool kWienerPinLds = (I >= 7);
using v4f = float __attribute__((ext_vector_type(4)));
using v2f = float __attribute__((ext_vector_type(2)));

template <int I, int J, bool kVec4>
__global__ __launch_bounds__(kBlock) void k_as_wiener(DevState s, float2* __restrict__ out) {
  const int f = blockIdx.y, chunk = blockIdx.x;
  __shared__ float2 sP[I * I], sB[I * I];
  __shared__ float sLam[J * I];
  __shared__ float2 sOut[kBlock / kWave][kWave * I];
  for (int t = threadIdx.x; t < I * I; t += kBlock) sP[t] = s.P[(size_t)f * I * I + t];
  for (int t = threadIdx.x; t < J * I; t += kBlock) sLam[t] = s.lam[(size_t)f * J * I + t];
  __syncthreads();
  if (threadIdx.x < I) {  // B = P^-H, lane c solves P^H b = e_c for column c
    const int c = threadIdx.x;
    float Mr[I][I], Mi[I][I], br[I], bi[I];
#pragma unroll
    for (int r = 0; r < I; ++r)
#pragma unroll
      for (int k = 0; k < I; ++k) { Mr[r][k] = sP[k * I + r].x; Mi[r][k] = -sP[k * I + r].y; }
#pragma unroll
    for (int r = 0; r < I; ++r) { br[r] = (r == c) ? 1.f : 0.f; bi[r] = 0.f; }
    lu_solve<I>(Mr, Mi, br, bi);
#pragma unroll
    for (int r = 0; r < I; ++r) sB[r * I + c] = make_float2(br[r], bi[r]);
  }
  __syncthreads();
  constexpr bool kLds = kWienerPinLds<I>;
  float Pr[kLds ? 1 : I][I], Pi[kLds ? 1 : I][I], Br[kLds ? 1 : I][I], Bi[kLds ? 1 : I][I];
  if constexpr (!kLds) {
    load_P<I>(sP, Pr, Pi);
    load_P<I>(sB, Br, Bi);
  }
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  float2* tile = sOut[wave];
  const float* xf = s.xs + (size_t)f * 2 * I * s.Npad;
  const float* vf = s.vs + (size_t)f * J * s.Npad;
#pragma unroll 1
  for (int p = 0; p < kPts; ++p) {
    const int n0 = chunk * kChunk + p * kBlock + wave * kWave;  // the wave's first frame
    if (n0 >= s.N) break;                                       // wave-uniform
    const int n = n0 + lane;
    const bool ok = n < s.N;
    const int nn = ok ? n : n0;
    float xr[I], xi[I], v[J], yr[I], yi[I], id[I];
#pragma unroll
    for (int i = 0; i < I; ++i) { xr[i] = xf[(size_t)i * s.Npad + nn]; xi[i] = xf[(size_t)(I + i) * s.Npad + nn]; }
#pragma unroll
    for (int j = 0; j < J; ++j) v[j] = vf[(size_t)j * s.Npad + nn];
    if constexpr (kLds) {
#pragma unroll
      for (int i = 0; i < I; ++i) {
        float a = 0.f, b = 0.f;
#pragma unroll
        for (int k = 0; k < I; ++k) {
          const float2 pk = sP[k * I + i];
          a = fmaf(pk.x, xr[k], a); a = fmaf(pk.y, xi[k], a);
          b = fmaf(pk.x, xi[k], b); b = fmaf(-pk.y, xr[k], b);
        }
        yr[i] = a; yi[i] = b;
      }
    } else {
      as_transform<I>(Pr, Pi, xr, xi, yr, yi);
    }
#pragma unroll
    for (int i = 0; i < I; ++i) {
      float d = 0.f;
#pragma unroll
      for (int j = 0; j < J; ++j) d = fmaf(v[j], sLam[j * I + i], d);
      id[i] = 1.0f / d;
    }
    const int rows = (s.N - n0 < kWave ? s.N - n0 : kWave) * I;  // valid complex values of the wave
#pragma unroll 1
    for (int j = 0; j < J; ++j) {
      // v_j and lambda_j by selection and from LDS (a uniform address): a
      // register array indexed by the loop counter is placed in scratch memory
      float vj = v[0];
#pragma unroll
      for (int q = 1; q < J; ++q) vj = (j == q) ? v[q] : vj;
      float ur[I], ui[I];
#pragma unroll
      for (int i = 0; i < I; ++i) {
        const float g = vj * sLam[j * I + i] * id[i];
        ur[i] = g * yr[i]; ui[i] = g * yi[i];
      }
#pragma unroll
      for (int a = 0; a < I; ++a) {
        float sr = 0.f, si = 0.f;
#pragma unroll
        for (int i = 0; i < I; ++i) {
          float br, bi;
          if constexpr (kLds) { const float2 b = sB[a * I + i]; br = b.x; bi = b.y; }
          else { br = Br[a][i]; bi = Bi[a][i]; }
          sr = fmaf(br, ur[i], sr); sr = fmaf(-bi, ui[i], sr);
          si = fmaf(br, ui[i], si); si = fmaf(bi, ur[i], si);
        }
        tile[lane * I + a] = make_float2(sr, si);
      }
      __builtin_amdgcn_wave_barrier();
      float2* o = out + (((size_t)j * s.F + f) * s.N + n0) * I;
      if constexpr (kVec4) {
        const float4* t4 = reinterpret_cast<const float4*>(tile);
        float4* o4 = reinterpret_cast<float4*>(o);
#pragma unroll
        for (int r = 0; r < I / 2; ++r) {
          const int q = lane + r * kWave;
          if (2 * q < rows) {
            // streamed out, never re-read: non-temporal stores where they
            // measured faster (I = 6: 187 -> 168 us at the 60 s shape; at I = 8
            // they took 374 -> 394 us, so there the stores stay ordinary)
            if constexpr (!kLds)
              __builtin_nontemporal_store(reinterpret_cast<const v4f*>(t4)[q], reinterpret_cast<v4f*>(o4) + q);
            else
              o4[q] = t4[q];
          }
        }
      } else {
#pragma unroll
        for (int r = 0; r < I; ++r) {
          const int q = lane + r * kWave;
          if (q < rows) {
            if constexpr (!kLds)
              __builtin_nontemporal_store(reinterpret_cast<const v2f*>(tile)[q], reinterpret_cast<v2f*>(o) + q);
            else
              o[q] = tile[q];
          }
        }
      }
      __builtin_amdgcn_wave_barrier();
    }
  }
}

template <int I, int J>
hipError_t launch_as_wiener(const DevState& s, hipStream_t st, float2* out) {
  const bool vec4 = (I % 2 == 0) && ((reinterpret_cast<uintptr_t>(out) & 15) == 0);
  if (vec4)
    hipLaunchKernelGGL((k_as_wiener<I, J, true>), dim3(s.nchunk, s.F), dim3(kBlock), 0, st, s, out);
  else
    hipLaunchKernelGGL((k_as_wiener<I, J, false>), dim3(s.nchunk, s.F), dim3(kBlock), 0, st, s, out);
  return hipGetLastError();
}

// ----------------------------------------------------------------------------
// Conventional FCA EM (Section 3.3).
// ----------------------------------------------------------------------------
template <int I, int J>
struct EmShared {
  float Rr[J][I][I], Ri[J][I][I];  // S_j
  float Sr[J][I][I], Si[J][I][I];  // S_j^-1
};

template <int I, int J>
__device__ inline void em_load_shared(const DevState& s, int f, EmShared<I, J>& sh) {
  for (int t = threadIdx.x; t < J * I * I; t += blockDim.x) {
    const int j = t / (I * I), a = (t / I) % I, b = t % I;
    const float2 r = s.R[(size_t)f * J * I * I + t];
    const float2 q = s.Rinv[(size_t)f * J * I * I + t];
    sh.Rr[j][a][b] = r.x; sh.Ri[j][a][b] = r.y;
    sh.Sr[j][a][b] = q.x; sh.Si[j][a][b] = q.y;
  }
}

// C = sum_j v_j S_j (upper triangle).
template <int I, int J>
__device__ __forceinline__ void em_model_cov(const EmShared<I, J>& sh, const float (&v)[J],
                                             float (&Cr)[I][I], float (&Ci)[I][I]) {
#pragma unroll
  for (int a = 0; a < I; ++a)
#pragma unroll
    for (int b = a; b < I; ++b) {
      float cr = 0.f, ci = 0.f;
#pragma unroll
      for (int j = 0; j < J; ++j) { cr = fmaf(v[j], sh.Rr[j][a][b], cr); ci = fmaf(v[j], sh.Ri[j][a][b], ci); }
      Cr[a][b] = cr; Ci[a][b] = ci;
    }
}

// One FCA EM point: E-step (eq. 7-8) for every source with one Hermitian
// inverse C^-1 and two I x I products per source (S_j C^-1 and (S_j C^-1) S_j),
// the v update (eq. 9, current S_j) and the summand of eq. 10 (new v_j),
// Rhat_j / v_j in packed Hermitian slots, added to H[j] (nothing if !ok).
// Returns false for a point (with ok) whose C is not numerically positive
// definite.
template <int I, int J>
__device__ __forceinline__ bool em_point(const EmShared<I, J>& sh, const float (&xr)[I],
                                         const float (&xi)[I], float (&v)[J], float (&H)[J][I * I],
                                         bool ok) {
  float Cr[I][I], Ci[I][I], Xr[I][I], Xi[I][I];
  em_model_cov<I, J>(sh, v, Cr, Ci);
  const bool pd = herm_inv<I>(Cr, Ci, Xr, Xi);  // C^-1 (one inversion per point)
#pragma unroll
  for (int j = 0; j < J; ++j) {
    // K = S_j C^-1 (first product); W_j = v_j K.
    float Kr[I][I], Ki[I][I];
#pragma unroll
    for (int a = 0; a < I; ++a)
#pragma unroll
      for (int b = 0; b < I; ++b) {
        float kr = 0.f, ki = 0.f;
#pragma unroll
        for (int c = 0; c < I; ++c) {
          kr = fmaf(sh.Rr[j][a][c], Xr[c][b], kr); kr = fmaf(-sh.Ri[j][a][c], Xi[c][b], kr);
          ki = fmaf(sh.Rr[j][a][c], Xi[c][b], ki); ki = fmaf(sh.Ri[j][a][c], Xr[c][b], ki);
        }
        Kr[a][b] = kr; Ki[a][b] = ki;
      }
    const float vj = v[j];
    // mu_j = v_j K x  (eq. 7)
    float mr[I], mi[I];
#pragma unroll
    for (int a = 0; a < I; ++a) {
      float sr = 0.f, si = 0.f;
#pragma unroll
      for (int c = 0; c < I; ++c) {
        sr = fmaf(Kr[a][c], xr[c], sr); sr = fmaf(-Ki[a][c], xi[c], sr);
        si = fmaf(Kr[a][c], xi[c], si); si = fmaf(Ki[a][c], xr[c], si);
      }
      mr[a] = vj * sr; mi[a] = vj * si;
    }
    // Rhat = mu mu^H + v_j S_j - v_j^2 K S_j  (eq. 8, second product), upper triangle.
    float Hr[I][I], Hi[I][I];
    const float vj2 = vj * vj;
#pragma unroll
    for (int a = 0; a < I; ++a)
#pragma unroll
      for (int b = a; b < I; ++b) {
        float kr = 0.f, ki = 0.f;
#pragma unroll
        for (int c = 0; c < I; ++c) {
          kr = fmaf(Kr[a][c], sh.Rr[j][c][b], kr); kr = fmaf(-Ki[a][c], sh.Ri[j][c][b], kr);
          ki = fmaf(Kr[a][c], sh.Ri[j][c][b], ki); ki = fmaf(Ki[a][c], sh.Rr[j][c][b], ki);
        }
        const float mmr = fmaf(mr[a], mr[b], mi[a] * mi[b]);
        const float mmi = fmaf(mi[a], mr[b], -mr[a] * mi[b]);
        Hr[a][b] = mmr + fmaf(vj, sh.Rr[j][a][b], -vj2 * kr);
        Hi[a][b] = (a == b) ? 0.f : mmi + fmaf(vj, sh.Ri[j][a][b], -vj2 * ki);
      }
    // v_j <- Re tr(S_j^-1 Rhat) / I  (eq. 9, with the current S_j)
    float tr = 0.f;
#pragma unroll
    for (int a = 0; a < I; ++a) {
      tr = fmaf(sh.Sr[j][a][a], Hr[a][a], tr);
#pragma unroll
      for (int b = a + 1; b < I; ++b)
        tr = fmaf(2.f, fmaf(sh.Sr[j][a][b], Hr[a][b], sh.Si[j][a][b] * Hi[a][b]), tr);
    }
    const float vn = tr * (1.0f / float(I));
    v[j] = ok ? vn : v[j];
    const float iv = ok ? rcp(vn) : 0.f;
#pragma unroll
    for (int a = 0; a < I; ++a)
#pragma unroll
      for (int b = a; b < I; ++b) {
        H[j][a * I + b] = fmaf(Hr[a][b], iv, H[j][a * I + b]);
        if (b > a) H[j][b * I + a] = fmaf(Hi[a][b], iv, H[j][b * I + a]);
      }
  }
  return pd || !ok;
}

// Streaming FCA EM pass: one point per lane; per source the summands of
// eq. 10 are summed over the wave (transposed reduction) into the wave's LDS
// slot, then over the waves into the tile partial.
template <int I, int J>
__global__ __launch_bounds__(kBlock) void k_em_pass(DevState s) {
  constexpr int V = pad4(I * I);
  const int f = blockIdx.y, chunk = blockIdx.x;
  __shared__ EmShared<I, J> sh;
  __shared__ float acc[kBlock / kWave][J][V];
  em_load_shared<I, J>(s, f, sh);
  __syncthreads();
  const int wave = threadIdx.x / kWave;
  const int n = chunk * kChunkEm + threadIdx.x;
  const bool ok = n < s.N;
  const int nn = ok ? n : 0;
  const float* xf = s.xs + (size_t)f * 2 * I * s.Npad;
  float* vf = s.vs + (size_t)f * J * s.Npad;
  float xr[I], xi[I], v[J];
#pragma unroll
  for (int i = 0; i < I; ++i) { xr[i] = xf[(size_t)i * s.Npad + nn]; xi[i] = xf[(size_t)(I + i) * s.Npad + nn]; }
#pragma unroll
  for (int j = 0; j < J; ++j) v[j] = ok ? vf[(size_t)j * s.Npad + nn] : 1.f;
  float H[J][I * I];
#pragma unroll
  for (int j = 0; j < J; ++j)
#pragma unroll
    for (int q = 0; q < I * I; ++q) H[j][q] = 0.f;
  if (!em_point<I, J>(sh, xr, xi, v, H, ok)) atomicOr(s.flag, kFlagSingular);
  if (ok) {
#pragma unroll
    for (int j = 0; j < J; ++j) vf[(size_t)j * s.Npad + n] = v[j];
  }
#pragma unroll
  for (int j = 0; j < J; ++j) wave_totals_to_lds<I * I>(H[j], &acc[0][j][0], J * V);
  __syncthreads();
  float* out = s.partA + ((size_t)f * s.nchunk_em + chunk) * J * I * I;
  for (int t = threadIdx.x; t < J * I * I; t += kBlock) {
    const int j = t / (I * I), q = t % (I * I);
    float u = 0.f;
#pragma unroll
    for (int w = 0; w < kBlock / kWave; ++w) u += acc[w][j][q];
    out[t] = u;
  }
}

// S_j <- (1/N) sum over tiles (eq. 10), exactly Hermitian; S_j^-1 for the next
// v update.  One lane per (bin, source).
template <int I, int J>
__global__ __launch_bounds__(64) void k_em_finalize(DevState s) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int f = t / J, j = t % J;
  if (f >= s.F) return;
  float A[I * I];
#pragma unroll
  for (int k = 0; k < I * I; ++k) A[k] = 0.f;
  for (int c = 0; c < s.nchunk_em; ++c) {
    const float* src = s.partA + ((size_t)f * s.nchunk_em + c) * J * I * I + j * I * I;
#pragma unroll
    for (int k = 0; k < I * I; ++k) A[k] += src[k];
  }
  const float invN = 1.0f / float(s.N);
  float Rr[I][I], Ri[I][I], Xr[I][I], Xi[I][I];
#pragma unroll
  for (int a = 0; a < I; ++a) {
    Rr[a][a] = A[a * I + a] * invN; Ri[a][a] = 0.f;
#pragma unroll
    for (int b = a + 1; b < I; ++b) {
      Rr[a][b] = A[a * I + b] * invN; Ri[a][b] = A[b * I + a] * invN;
      Rr[b][a] = Rr[a][b]; Ri[b][a] = -Ri[a][b];
    }
  }
  if (!herm_inv<I>(Rr, Ri, Xr, Xi)) atomicOr(s.flag, kFlagSingular);
  float2* R = s.R + ((size_t)f * J + j) * I * I;
  float2* X = s.Rinv + ((size_t)f * J + j) * I * I;
#pragma unroll
  for (int a = 0; a < I; ++a)
#pragma unroll
    for (int b = 0; b < I; ++b) {
      R[a * I + b] = make_float2(Rr[a][b], Ri[a][b]);
      X[a * I + b] = make_float2(Xr[a][b], Xi[a][b]);
    }
}

template <int I, int J>
hipError_t launch_em_iter(const DevState& s, hipStream_t st) {
  hipLaunchKernelGGL((k_em_pass<I, J>), dim3(s.nchunk_em, s.F), dim3(kBlock), 0, st, s);
  hipLaunchKernelGGL((k_em_finalize<I, J>), dim3((s.F * J + 63) / 64), dim3(64), 0, st, s);
  return hipGetLastError();
}

// S_j = P^-H diag(lambda_j) P^-1 (eq. 12) and S_j^-1 = P diag(1/lambda_j) P^H,
// one lane per (bin, source): the EM starting point equal to an AS state.
template <int I, int J>
__global__ __launch_bounds__(64) void k_em_from_as(DevState s) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int f = t / J, j = t % J;
  if (f >= s.F) return;
  float Pr[I][I], Pi[I][I], Ur[I][I], Ui[I][I];  // U = P^-1
  load_P<I>(s.P + (size_t)f * I * I, Pr, Pi);
#pragma unroll
  for (int c = 0; c < I; ++c) {
    float Mr[I][I], Mi[I][I], br[I], bi[I];
#pragma unroll
    for (int a = 0; a < I; ++a) {
#pragma unroll
      for (int b = 0; b < I; ++b) { Mr[a][b] = Pr[a][b]; Mi[a][b] = Pi[a][b]; }
      br[a] = (a == c) ? 1.f : 0.f; bi[a] = 0.f;
    }
    lu_solve<I>(Mr, Mi, br, bi);
#pragma unroll
    for (int a = 0; a < I; ++a) { Ur[a][c] = br[a]; Ui[a][c] = bi[a]; }
  }
  float lam[I];
#pragma unroll
  for (int i = 0; i < I; ++i) lam[i] = s.lam[((size_t)f * J + j) * I + i];
  float2* R = s.R + ((size_t)f * J + j) * I * I;
  float2* X = s.Rinv + ((size_t)f * J + j) * I * I;
#pragma unroll
  for (int a = 0; a < I; ++a)
#pragma unroll
    for (int b = 0; b < I; ++b) {
      // (U^H diag(lam) U)_ab = sum_k conj(U_ka) lam_k U_kb
      float rr = 0.f, ri = 0.f, xr = 0.f, xi = 0.f;
#pragma unroll
      for (int k = 0; k < I; ++k) {
        const float ar = Ur[k][a] * lam[k], ai = -Ui[k][a] * lam[k];
        rr += ar * Ur[k][b] - ai * Ui[k][b];
        ri += ar * Ui[k][b] + ai * Ur[k][b];
        // (P diag(1/lam) P^H)_ab = sum_k P_ak / lam_k conj(P_bk)
        const float pr = Pr[a][k] / lam[k], pi = Pi[a][k] / lam[k];
        xr += pr * Pr[b][k] + pi * Pi[b][k];
        xi += pi * Pr[b][k] - pr * Pi[b][k];
      }
      R[a * I + b] = make_float2(rr, ri);
      X[a * I + b] = make_float2(xr, xi);
    }
}

template <int I, int J>
hipError_t launch_em_from_as(const DevState& s, hipStream_t st) {
  hipLaunchKernelGGL((k_em_from_as<I, J>), dim3((s.F * J + 63) / 64), dim3(64), 0, st, s);
  return hipGetLastError();
}

// S_j^-1 of caller-given S_j (its upper triangle; the stored S_j is made
// exactly Hermitian from it).
template <int I, int J>
__global__ __launch_bounds__(64) void k_em_rinv(DevState s) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int f = t / J, j = t % J;
  if (f >= s.F) return;
  float2* R = s.R + ((size_t)f * J + j) * I * I;
  float Rr[I][I], Ri[I][I], Xr[I][I], Xi[I][I];
#pragma unroll
  for (int a = 0; a < I; ++a)
#pragma unroll
    for (int b = a; b < I; ++b) {
      const float2 r = R[a * I + b];
      Rr[a][b] = r.x; Ri[a][b] = (a == b) ? 0.f : r.y;
      Rr[b][a] = r.x; Ri[b][a] = -Ri[a][b];
    }
  herm_inv<I>(Rr, Ri, Xr, Xi);
  float2* X = s.Rinv + ((size_t)f * J + j) * I * I;
#pragma unroll
  for (int a = 0; a < I; ++a)
#pragma unroll
    for (int b = 0; b < I; ++b) {
      R[a * I + b] = make_float2(Rr[a][b], Ri[a][b]);
      X[a * I + b] = make_float2(Xr[a][b], Xi[a][b]);
    }
}

template <int I, int J>
hipError_t launch_em_rinv(const DevState& s, hipStream_t st) {
  hipLaunchKernelGGL((k_em_rinv<I, J>), dim3((s.F * J + 63) / 64), dim3(64), 0, st, s);
  return hipGetLastError();
}

// L1 per point: -ln det C - x^H C^-1 x (Cholesky of C).
template <int I, int J>
__global__ __launch_bounds__(kBlock) void k_em_loglik(DevState s) {
  const int f = blockIdx.y, chunk = blockIdx.x;
  __shared__ EmShared<I, J> sh;
  __shared__ double red[kBlock / kWave];
  em_load_shared<I, J>(s, f, sh);
  __syncthreads();
  const float* xf = s.xs + (size_t)f * 2 * I * s.Npad;
  const float* vf = s.vs + (size_t)f * J * s.Npad;
  const int n = chunk * kChunkEm + threadIdx.x;
  double acc = 0.0;
  if (n < s.N) {
    float xr[I], xi[I], v[J];
#pragma unroll
    for (int i = 0; i < I; ++i) { xr[i] = xf[(size_t)i * s.Npad + n]; xi[i] = xf[(size_t)(I + i) * s.Npad + n]; }
#pragma unroll
    for (int j = 0; j < J; ++j) v[j] = vf[(size_t)j * s.Npad + n];
    float Cr[I][I], Ci[I][I], Lr[I][I], Li[I][I], dinv[I];
    em_model_cov<I, J>(sh, v, Cr, Ci);
    cholesky<I>(Cr, Ci, Lr, Li, dinv);
    float t = 0.f;
#pragma unroll
    for (int k = 0; k < I; ++k) {
      float sr = xr[k], si = xi[k];
#pragma unroll
      for (int m = 0; m < k; ++m) {
        sr -= Lr[k][m] * xr[m] - Li[k][m] * xi[m];
        si -= Lr[k][m] * xi[m] + Li[k][m] * xr[m];
      }
      xr[k] = sr * dinv[k]; xi[k] = si * dinv[k];
      t -= 2.f * __logf(Lr[k][k]) + xr[k] * xr[k] + xi[k] * xi[k];
    }
    acc = (double)t;
  }
  if (chunk == 0 && threadIdx.x == 0) acc -= (double)s.N * (double)I * 1.1447298858494002;  // the bin's -N I ln pi
  block_sum_store_d(acc, s.partL + (size_t)f * s.nchunk_em + chunk, red);
}

// L1 = the sum of all tiles' partials (one workgroup, fixed order) into s.ll.
template <int I, int J>
hipError_t launch_em_loglik(const DevState& s, hipStream_t st) {
  hipLaunchKernelGGL((k_em_loglik<I, J>), dim3(s.nchunk_em, s.F), dim3(kBlock), 0, st, s);
  return launch_sum_f(s.partL, s.F * s.nchunk_em, s.ll, st);
}

// x_j = v_j S_j C^-1 x (eq. 3).
template <int I, int J>
__global__ __launch_bounds__(kBlock) void k_em_wiener(DevState s, float2* __restrict__ out) {
  const int f = blockIdx.y, chunk = blockIdx.x;
  __shared__ EmShared<I, J> sh;
  em_load_shared<I, J>(s, f, sh);
  __syncthreads();
  const int n = chunk * kChunkEm + threadIdx.x;
  if (n >= s.N) return;
  const float* xf = s.xs + (size_t)f * 2 * I * s.Npad;
  const float* vf = s.vs + (size_t)f * J * s.Npad;
  float xr[I], xi[I], v[J];
#pragma unroll
  for (int i = 0; i < I; ++i) { xr[i] = xf[(size_t)i * s.Npad + n]; xi[i] = xf[(size_t)(I + i) * s.Npad + n]; }
#pragma unroll
  for (int j = 0; j < J; ++j) v[j] = vf[(size_t)j * s.Npad + n];
  float Cr[I][I], Ci[I][I], Lr[I][I], Li[I][I], dinv[I];
  em_model_cov<I, J>(sh, v, Cr, Ci);
  cholesky<I>(Cr, Ci, Lr, Li, dinv);
  cholesky_solve<I>(Lr, Li, dinv, xr, xi);  // z = C^-1 x
#pragma unroll
  for (int j = 0; j < J; ++j) {
    float2* o = out + (((size_t)j * s.F + f) * s.N + n) * I;
#pragma unroll
    for (int a = 0; a < I; ++a) {
      float sr = 0.f, si = 0.f;
#pragma unroll
      for (int c = 0; c < I; ++c) {
        sr = fmaf(sh.Rr[j][a][c], xr[c], sr); sr = fmaf(-sh.Ri[j][a][c], xi[c], sr);
        si = fmaf(sh.Rr[j][a][c], xi[c], si); si = fmaf(sh.Ri[j][a][c], xr[c], si);
      }
      o[a] = make_float2(v[j] * sr, v[j] * si);
    }
  }
}

template <int I, int J>
hipError_t launch_em_wiener(const DevState& s, hipStream_t st, float2* out) {
  hipLaunchKernelGGL((k_em_wiener<I, J>), dim3(s.nchunk_em, s.F), dim3(kBlock), 0, st, s, out);
  return hipGetLastError();
}

// ----------------------------------------------------------------------------
// Parameter check (option "check_finite"): the model needs v > 0, lambda > 0
// and a non-singular P(f) (Section 3.1 and eq. 12), or S_j(f) positive
// definite for FCA.  v and lambda are checked by k_check_positive
// (fca_common.hip); this kernel checks the matrices, one lane per bin (AS)
// or per (bin, source) (EM), and sets kFlagSingularParam.
// ----------------------------------------------------------------------------
template <int I, int J>
__global__ __launch_bounds__(64) void k_check_matrices(DevState s, int em) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (!em) {
    if (t >= s.F) return;
    // Gaussian elimination with partial pivoting on P(f): singular when a
    // pivot's modulus falls to I * 2^-23 of the largest entry's (P is
    // singular to working precision) or is NaN.
    float Mr[I][I], Mi[I][I], big = 0.f;
#pragma unroll
    for (int a = 0; a < I; ++a)
#pragma unroll
      for (int b = 0; b < I; ++b) {
        const float2 z = s.P[(size_t)t * I * I + a * I + b];
        Mr[a][b] = z.x; Mi[a][b] = z.y;
        big = fmaxf(big, z.x * z.x + z.y * z.y);
      }
    const float tol = float(I) * float(I) * 1.42108547e-14f * big;  // (I 2^-23)^2 |max|^2
    bool ok = big > 0.f;
#pragma unroll
    for (int k = 0; k < I; ++k) {
#pragma unroll
      for (int r = k + 1; r < I; ++r) {
        const float cur = Mr[k][k] * Mr[k][k] + Mi[k][k] * Mi[k][k];
        const float cand = Mr[r][k] * Mr[r][k] + Mi[r][k] * Mi[r][k];
        if (cand > cur) {
#pragma unroll
          for (int c = 0; c < I; ++c) {
            float u = Mr[k][c]; Mr[k][c] = Mr[r][c]; Mr[r][c] = u;
            u = Mi[k][c]; Mi[k][c] = Mi[r][c]; Mi[r][c] = u;
          }
        }
      }
      const float pr = Mr[k][k], pi = Mi[k][k];
      const float den = pr * pr + pi * pi;
      ok = ok && (den > tol);
      const float inv = rcp(den > tol ? den : 1.f);
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
    if (!ok) atomicOr(s.flag, kFlagSingularParam);
  } else {
    if (t >= s.F * J) return;
    float Ar[I][I], Ai[I][I], Lr[I][I], Li[I][I], dinv[I];
    const float2* R = s.R + (size_t)t * I * I;
    bool fin = true;
#pragma unroll
    for (int a = 0; a < I; ++a)
#pragma unroll
      for (int b = 0; b < I; ++b) {
        const float2 z = R[a * I + b];
        Ar[a][b] = z.x; Ai[a][b] = z.y;
        fin = fin && isfinite(z.x) && isfinite(z.y);
      }
    if (!fin || !cholesky<I>(Ar, Ai, Lr, Li, dinv)) atomicOr(s.flag, kFlagSingularParam);
  }
}

template <int I, int J>
hipError_t launch_check_matrices(const DevState& s, hipStream_t st, int em) {
  const int n = em ? s.F * J : s.F;
  hipLaunchKernelGGL((k_check_matrices<I, J>), dim3((n + 63) / 64), dim3(64), 0, st, s, em);
  return hipGetLastError();
}

}  // namespace fca
